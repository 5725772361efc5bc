"""Thin Python binding of libpb.so (include/pb.h).

Argument marshalling only: torch provides device memory and the stream, every step of the
computation runs in the library's HIP kernels. The functions keep the C names. If the
library is not built, importing this module raises — there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpb.so")

PB_OK, PB_EINVAL, PB_ENOMEM, PB_EDEVICE, PB_ECAPACITY, PB_ENOCONV, PB_EGEOM = 0, -1, -2, -3, -4, -5, -6
PB_REG_TANGENT_GUARDED, PB_REG_TANGENT, PB_REG_EUCLIDEAN = 0, 1, 2
PB_LS_VDW, PB_LS_SES = 0, 1
PB_FP64, PB_MIXED, PB_TREE = 0, 1, 2
PB_X0_ZERO, PB_X0_DIAG, PB_X0_USER, PB_X0_LEARNED = 0, 1, 2, 3
PB_PRECOND_NONE, PB_PRECOND_LEARNED = 0, 1
PB_GRAD_CENTRAL, PB_GRAD_WENO = 0, 1
PB_JAC_ONE, PB_JAC_FULL = 0, 1
PB_AVG_FLAT, PB_AVG_CURVED = 0, 1
KCAL_PER_UNIT = 4.0 * np.pi * 332.0637

EXPORTS = [
    "pb_create", "pb_destroy", "pb_last_error", "pb_default_params", "pb_default_solve_opts",
    "pb_grid_for_atoms", "pb_build_levelset", "pb_narrowband_compact", "pb_ibim_rhs", "pb_ibim_matvec",
    "pb_ibim_solve", "pb_solvation_energy", "pb_set_timing", "pb_kernel_time", "pb_tree_info", "pb_ibim_solve_batched",
    "pb_nn_create", "pb_nn_destroy", "pb_nn_param_count", "pb_nn_get_params", "pb_nn_set_params", "pb_nn_prepare",
    "pb_nn_apply", "pb_nn_train_step", "pb_nn_geometry", "pb_far_kernel", "pb_solvation_energy_noalloc",
]


class pb_params(C.Structure):
    _fields_ = [("eps_in", C.c_double), ("eps_out", C.c_double), ("kappa", C.c_double), ("probe", C.c_double),
                ("h", C.c_double), ("band_k", C.c_double), ("tau_k", C.c_double), ("cfl", C.c_double),
                ("near_k", C.c_double), ("tree_theta", C.c_double), ("reg_metric", C.c_int), ("ls_mode", C.c_int), ("reinit_steps", C.c_int),
                ("grad_scheme", C.c_int), ("jacobian", C.c_int), ("tree_degree", C.c_int), ("reg_avg", C.c_int)]


class pb_grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("origin", C.c_double * 3), ("h", C.c_double)]


class pb_band(C.Structure):
    _fields_ = [("n", C.c_int64), ("capacity", C.c_int64)] + \
               [(f, C.c_void_p) for f in ("px", "py", "pz", "nx", "ny", "nz", "phi", "w", "gidx", "curv")]


class pb_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("restart", C.c_int), ("precision", C.c_int),
                ("x0", C.c_int), ("precond", C.c_int), ("max_outer", C.c_int), ("nn", C.c_void_p)]


class pb_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("converged", C.c_int), ("fallback_used", C.c_int),
                ("matvecs_fp64", C.c_int), ("matvecs_mixed", C.c_int), ("true_relres", C.c_double),
                ("t_total_s", C.c_double), ("t_matvec_s", C.c_double), ("pairs", C.c_double)]


class pb_batch_stats(C.Structure):
    _fields_ = [("t_total_s", C.c_double), ("t_p50_s", C.c_double), ("t_p99_s", C.c_double), ("pairs", C.c_double),
                ("graph_replays", C.c_int), ("far_tile", C.c_int), ("far_tpl", C.c_int), ("n_items", C.c_int),
                ("outer", C.c_int), ("far_symmetric", C.c_int)]


class pb_energy(C.Structure):
    _fields_ = [("g_pol", C.c_double), ("g_pol_kcal", C.c_double), ("area", C.c_double)]


class PBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pb status {status}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (no CPU fallback exists)")
    L = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    L.pb_create.argtypes = [P(vp), C.c_int, vp]
    L.pb_destroy.argtypes = [vp]
    L.pb_destroy.restype = None
    L.pb_last_error.argtypes = [vp]
    L.pb_last_error.restype = C.c_char_p
    L.pb_default_params.argtypes = [P(pb_params)]
    L.pb_default_params.restype = None
    L.pb_default_solve_opts.argtypes = [P(pb_solve_opts)]
    L.pb_default_solve_opts.restype = None
    L.pb_grid_for_atoms.argtypes = [vp, C.c_int, P(pb_params), P(pb_grid)]
    L.pb_build_levelset.argtypes = [vp, vp, C.c_int, P(pb_params), P(pb_grid), vp, C.c_size_t, P(C.c_size_t)]
    L.pb_narrowband_compact.argtypes = [vp, P(pb_grid), vp, P(pb_params), P(pb_band)]
    L.pb_ibim_rhs.argtypes = [vp, P(pb_band), vp, C.c_int, P(pb_params), vp]
    L.pb_ibim_matvec.argtypes = [vp, P(pb_band), P(pb_params), C.c_int, vp, vp]
    L.pb_ibim_solve.argtypes = [vp, P(pb_band), vp, C.c_int, P(pb_params), P(pb_solve_opts), vp, P(pb_solve_stats)]
    L.pb_solvation_energy.argtypes = [vp, P(pb_band), vp, C.c_int, P(pb_params), vp, P(pb_energy), vp]
    L.pb_solvation_energy_noalloc.argtypes = [vp, P(pb_band), vp, C.c_int, P(pb_params), vp, vp, vp]
    L.pb_ibim_solve_batched.argtypes = [vp, C.c_int, P(pb_band), P(vp), P(C.c_int), P(pb_params), P(pb_solve_opts),
                                        P(vp), P(pb_solve_stats), P(pb_batch_stats)]
    L.pb_nn_create.argtypes = [vp, C.c_uint64, P(vp)]
    L.pb_nn_destroy.argtypes = [vp]
    L.pb_nn_destroy.restype = None
    L.pb_nn_param_count.argtypes = []
    L.pb_nn_param_count.restype = C.c_int64
    L.pb_nn_get_params.argtypes = [vp, vp, vp, vp]
    L.pb_nn_set_params.argtypes = [vp, vp, vp]
    L.pb_nn_prepare.argtypes = [vp, P(pb_band), P(pb_params)]
    L.pb_nn_apply.argtypes = [vp, vp, P(pb_band), P(pb_params), vp, vp]
    L.pb_nn_train_step.argtypes = [vp, vp, P(pb_band), P(pb_params), vp, vp, C.c_float, P(C.c_double)]
    L.pb_nn_geometry.argtypes = [vp, P(pb_band), vp, vp]
    L.pb_set_timing.argtypes = [vp, C.c_int]
    L.pb_kernel_time.argtypes = [vp, C.c_char_p, P(C.c_double), P(C.c_int64)]
    L.pb_far_kernel.argtypes = [vp, C.c_int64, P(C.c_int)]
    L.pb_tree_info.argtypes = [vp, P(C.c_int64)]
    for name in EXPORTS:
        if name not in ("pb_destroy", "pb_last_error", "pb_default_params", "pb_default_solve_opts", "pb_nn_destroy",
                        "pb_nn_param_count"):
            getattr(L, name).restype = C.c_int
    return L


lib = load()


def params(h=0.5, **kw) -> pb_params:
    p = pb_params()
    lib.pb_default_params(C.byref(p))
    p.h = h
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def solve_opts(**kw) -> pb_solve_opts:
    o = pb_solve_opts()
    lib.pb_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous() and t.dtype in (torch.float64, torch.int64), "device f64/i64 tensor"
    return C.c_void_p(t.data_ptr())


class Context:
    """pb_ctx on one device, bound to torch's current stream at creation."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.handle = C.c_void_p()
        st = lib.pb_create(C.byref(self.handle), device, C.c_void_p(self.stream.cuda_stream))
        if st != PB_OK:
            raise PBError(st, "pb_create failed")

    def check(self, st: int):
        if st != PB_OK:
            raise PBError(st, lib.pb_last_error(self.handle).decode())
        return st

    def close(self):
        if self.handle:
            lib.pb_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, level):
        """0/False off, 1/True every kernel family, 2 the far-field families only."""
        self.check(lib.pb_set_timing(self.handle, int(level)))

    def kernel_time(self, name: str):
        ms, cnt = C.c_double(), C.c_int64()
        self.check(lib.pb_kernel_time(self.handle, name.encode(), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def tree_info(self) -> dict:
        info = (C.c_int64 * 6)()
        self.check(lib.pb_tree_info(self.handle, info))
        keys = ("batches", "clusters", "proxy_items", "direct_pairs", "proxy_interactions", "near_pairs")
        return dict(zip(keys, [int(v) for v in info]))

    def far_kernel(self, n: int) -> int:
        cfg = C.c_int()
        self.check(lib.pb_far_kernel(self.handle, int(n), C.byref(cfg)))
        return cfg.value


@dataclass
class Band:
    """Device SoA of the band; keeps the tensors alive behind the pb_band struct."""
    n: int
    px: torch.Tensor
    py: torch.Tensor
    pz: torch.Tensor
    nx: torch.Tensor
    ny: torch.Tensor
    nz: torch.Tensor
    phi: torch.Tensor
    w: torch.Tensor
    gidx: torch.Tensor
    curv: torch.Tensor | None = None  # κ1 + κ2 at x* (written by the compaction)

    def struct(self) -> pb_band:
        b = pb_band()
        b.n = self.n
        b.capacity = self.px.numel()
        for f in ("px", "py", "pz", "nx", "ny", "nz", "phi", "w", "gidx"):
            setattr(b, f, getattr(self, f).data_ptr())
        b.curv = self.curv.data_ptr() if self.curv is not None else None
        return b

    def table(self) -> np.ndarray:
        """Host n × 8 table (x*, y*, z*, n_x, n_y, n_z, φ, ω) in band order."""
        cols = [getattr(self, f)[: self.n] for f in ("px", "py", "pz", "nx", "ny", "nz", "phi", "w")]
        return torch.stack(cols, 1).cpu().numpy()

    @staticmethod
    def alloc(capacity: int, device) -> "Band":
        z = lambda dt=torch.float64: torch.zeros(max(capacity, 1), dtype=dt, device=device)
        return Band(0, z(), z(), z(), z(), z(), z(), z(), z(), z(torch.int64), z())


def pb_grid_for_atoms(atoms: np.ndarray, prm: pb_params) -> pb_grid:
    a = np.ascontiguousarray(atoms, dtype=np.float64)
    g = pb_grid()
    st = lib.pb_grid_for_atoms(a.ctypes.data_as(C.c_void_p), len(a), C.byref(prm), C.byref(g))
    if st != PB_OK:
        raise PBError(st, "pb_grid_for_atoms")
    return g


def grid_shape(g: pb_grid):
    return (g.nx, g.ny, g.nz)


def pb_build_levelset(ctx: Context, atoms: torch.Tensor, prm: pb_params, grid: pb_grid,
                      phi: torch.Tensor | None = None) -> torch.Tensor:
    """φ on the grid. Without phi, the size comes from the library's size query (phi = NULL)."""
    if phi is None:
        need = C.c_size_t()
        ctx.check(lib.pb_build_levelset(ctx.handle, None, 0, C.byref(prm), C.byref(grid), None, 0, C.byref(need)))
        phi = torch.empty(need.value, dtype=torch.float64, device=atoms.device)
    assert phi.dtype == torch.float64 and phi.is_contiguous()
    ctx.check(lib.pb_build_levelset(ctx.handle, _ptr(atoms), atoms.shape[0], C.byref(prm), C.byref(grid), _ptr(phi),
                                    phi.numel(), None))
    return phi


def pb_narrowband_compact(ctx: Context, grid: pb_grid, phi: torch.Tensor, prm: pb_params,
                          band: Band | None = None) -> Band:
    if band is None:
        probe = pb_band()
        probe.capacity = 0
        st = lib.pb_narrowband_compact(ctx.handle, C.byref(grid), _ptr(phi), C.byref(prm), C.byref(probe))
        if st not in (PB_ECAPACITY, PB_OK):
            ctx.check(st)
        band = Band.alloc(int(probe.n), phi.device)
    s = band.struct()
    ctx.check(lib.pb_narrowband_compact(ctx.handle, C.byref(grid), _ptr(phi), C.byref(prm), C.byref(s)))
    band.n = int(s.n)
    return band


def pb_ibim_rhs(ctx: Context, band: Band, atoms: torch.Tensor, prm: pb_params, g: torch.Tensor | None = None):
    if g is None:
        g = torch.empty(2 * band.n, dtype=torch.float64, device=atoms.device)
    s = band.struct()
    ctx.check(lib.pb_ibim_rhs(ctx.handle, C.byref(s), _ptr(atoms), atoms.shape[0], C.byref(prm), _ptr(g)))
    return g


def pb_ibim_matvec(ctx: Context, band: Band, prm: pb_params, p: torch.Tensor, precision: int = PB_FP64,
                   y: torch.Tensor | None = None) -> torch.Tensor:
    if y is None:
        y = torch.empty_like(p)
    s = band.struct()
    ctx.check(lib.pb_ibim_matvec(ctx.handle, C.byref(s), C.byref(prm), precision, _ptr(p), _ptr(y)))
    return y


def pb_ibim_solve(ctx: Context, band: Band, atoms: torch.Tensor, prm: pb_params, opts: pb_solve_opts | None = None,
                  p: torch.Tensor | None = None, allow_noconv: bool = False):
    if opts is None:
        opts = solve_opts()
    if p is None:
        p = torch.zeros(2 * band.n, dtype=torch.float64, device=atoms.device)
    s = band.struct()
    stats = pb_solve_stats()
    st = lib.pb_ibim_solve(ctx.handle, C.byref(s), _ptr(atoms), atoms.shape[0], C.byref(prm), C.byref(opts), _ptr(p),
                           C.byref(stats))
    if not (allow_noconv and st == PB_ENOCONV):
        ctx.check(st)
    return p, stats


def pb_ibim_solve_batched(ctx: Context, bands: list, atoms: list, prm: pb_params, opts: pb_solve_opts | None = None,
                          ps: list | None = None, allow_noconv: bool = False):
    """Batched mixed-precision solve of several molecules. Returns (list of p, list of stats, batch stats)."""
    n = len(bands)
    if opts is None:
        opts = solve_opts(precision=PB_MIXED)
    if ps is None:
        ps = [torch.zeros(2 * b.n, dtype=torch.float64, device=a.device) for b, a in zip(bands, atoms)]
    barr = (pb_band * n)(*[b.struct() for b in bands])
    aarr = (C.c_void_p * n)(*[a.data_ptr() for a in atoms])
    narr = (C.c_int * n)(*[a.shape[0] for a in atoms])
    parr = (C.c_void_p * n)(*[q.data_ptr() for q in ps])
    stats = (pb_solve_stats * n)()
    bst = pb_batch_stats()
    st = lib.pb_ibim_solve_batched(ctx.handle, n, barr, aarr, narr, C.byref(prm), C.byref(opts), parr, stats,
                                   C.byref(bst))
    if not (allow_noconv and st == PB_ENOCONV):
        ctx.check(st)
    return ps, list(stats), bst


def pb_solvation_energy(ctx: Context, band: Band, atoms: torch.Tensor, prm: pb_params, p: torch.Tensor,
                        psi_rxn: torch.Tensor | None = None) -> pb_energy:
    out = pb_energy()
    s = band.struct()
    ctx.check(lib.pb_solvation_energy(ctx.handle, C.byref(s), _ptr(atoms), atoms.shape[0], C.byref(prm), _ptr(p),
                                      C.byref(out), _ptr(psi_rxn) if psi_rxn is not None else None))
    return out


def pb_solvation_energy_noalloc(ctx: Context, band: Band, atoms: torch.Tensor, prm: pb_params, p: torch.Tensor,
                                out: torch.Tensor, psi_rxn: torch.Tensor | None = None) -> torch.Tensor:
    """out (device, 3 doubles) receives (g_pol, g_pol_kcal, area) on the context stream; no
    allocation, no synchronization."""
    assert out.dtype == torch.float64 and out.numel() >= 3
    s = band.struct()
    ctx.check(lib.pb_solvation_energy_noalloc(ctx.handle, C.byref(s), _ptr(atoms), atoms.shape[0], C.byref(prm),
                                              _ptr(p), _ptr(out), _ptr(psi_rxn) if psi_rxn is not None else None))
    return out


# ---------------------------------------------------------------- learned preconditioner

NN_FORMAT = 1
NN_LAYERS = ((256, 64), (1024, 64), (1024, 64), (1024, 16))  # (K, Cout) per layer


class Net:
    """pb_nn handle: the point-convolution network on the device."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        self.handle = C.c_void_p()
        ctx.check(lib.pb_nn_create(ctx.handle, seed, C.byref(self.handle)))

    @staticmethod
    def param_count() -> int:
        return int(lib.pb_nn_param_count())

    def close(self):
        if self.handle:
            lib.pb_nn_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.param_count(), dtype=np.float32)
        self.ctx.check(lib.pb_nn_get_params(self.ctx.handle, self.handle, out.ctypes.data_as(C.c_void_p), None))
        return out

    def grads(self) -> np.ndarray:
        out = np.empty(self.param_count(), dtype=np.float32)
        self.ctx.check(lib.pb_nn_get_params(self.ctx.handle, self.handle, None, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.param_count()
        self.ctx.check(lib.pb_nn_set_params(self.ctx.handle, self.handle, w.ctypes.data_as(C.c_void_p)))

    def save(self, path: str):
        """Weights file: format version, layer shapes, FP32 parameters and their SHA-256."""
        import hashlib
        w = self.params()
        np.savez(path, format=np.int64(NN_FORMAT), layers=np.array(NN_LAYERS, dtype=np.int64), params=w,
                 sha256=np.frombuffer(hashlib.sha256(w.tobytes()).digest(), dtype=np.uint8))

    def load(self, path: str):
        import hashlib
        z = np.load(path, allow_pickle=False)
        if int(z["format"]) != NN_FORMAT or tuple(map(tuple, z["layers"])) != NN_LAYERS:
            raise ValueError(f"{path}: unsupported network format")
        w = z["params"].astype(np.float32)
        if hashlib.sha256(w.tobytes()).digest() != z["sha256"].tobytes():
            raise ValueError(f"{path}: parameter hash mismatch")
        self.set_params(w)


def pb_nn_prepare(ctx: Context, band: Band, prm: pb_params):
    s = band.struct()
    ctx.check(lib.pb_nn_prepare(ctx.handle, C.byref(s), C.byref(prm)))


def pb_nn_apply(ctx: Context, net: Net, band: Band, prm: pb_params, v: torch.Tensor,
                out: torch.Tensor | None = None) -> torch.Tensor:
    if out is None:
        out = torch.empty_like(v)
    s = band.struct()
    ctx.check(lib.pb_nn_apply(ctx.handle, net.handle, C.byref(s), C.byref(prm), _ptr(v), _ptr(out)))
    return out


def pb_nn_train_step(ctx: Context, net: Net, band: Band, prm: pb_params, v: torch.Tensor, u: torch.Tensor,
                     lr: float) -> float:
    s = band.struct()
    loss = C.c_double()
    ctx.check(lib.pb_nn_train_step(ctx.handle, net.handle, C.byref(s), C.byref(prm), _ptr(v), _ptr(u), lr,
                                   C.byref(loss)))
    return loss.value


def pb_nn_geometry(ctx: Context, band: Band):
    nbr = np.empty((band.n, 16), dtype=np.int32)
    feat = np.empty((band.n, 5), dtype=np.float32)
    s = band.struct()
    ctx.check(lib.pb_nn_geometry(ctx.handle, C.byref(s), nbr.ctypes.data_as(C.c_void_p),
                                 feat.ctypes.data_as(C.c_void_p)))
    return nbr, feat
