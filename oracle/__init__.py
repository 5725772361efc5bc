"""Plain FP64 CPU oracle of the implicit boundary integral method (arXiv:1709.08070).

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline leg of
``bench.py`` use it to check the GPU library; the product path never imports it. The C
source (``pbo.c``) shares no code with the GPU library. This module only marshals numpy
arrays into the C routines; every piece of arithmetic sits in ``pbo.c``.

Parameter vector indices follow ``pbo.h`` (PBO_*). Node table rows are
(x*, y*, z*, n_x, n_y, n_z, φ, ω).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libpbo.so")

EPS_IN, EPS_OUT, KAPPA, H, BAND, TAU, METRIC, PROBE, CFL, REINIT, AVG = range(11)
NPRM = 11
AVG_FLAT, AVG_CURVED = 0, 1
METRIC_GUARDED, METRIC_TANGENT, METRIC_EUCLID = 0, 1, 2


def build() -> str:
    """Compile pbo.c into libpbo.so (gcc, -O2, OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-o", _SO, os.path.join(_HERE, "pbo.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(os.path.join(_HERE, "pbo.c")):
            build()
        L = C.CDLL(_SO)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_long)
        L.pbo_grid.argtypes = [dp, C.c_int, C.c_double, C.c_double, ip, dp]
        L.pbo_vdw.argtypes = [ip, dp, C.c_double, dp, C.c_int, dp]
        L.pbo_eikonal.argtypes = [ip, C.c_double, dp, C.c_double, C.c_double]
        L.pbo_cavity.argtypes = [ip, C.c_double, dp, C.c_double, C.c_void_p]
        L.pbo_cavity.restype = C.c_long
        L.pbo_reinit.argtypes = [ip, C.c_double, dp, C.c_int, C.c_double]
        L.pbo_ses.argtypes = [ip, dp, dp, C.c_int, dp, dp]
        L.pbo_ses.restype = C.c_long
        L.pbo_weno_grad.argtypes = [ip, C.c_double, dp, C.c_long, dp, dp]
        L.pbo_band.argtypes = [ip, dp, C.c_double, dp, C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
        L.pbo_jacobian.argtypes = [ip, C.c_double, dp, C.c_long, dp]
        L.pbo_jacobian.restype = C.c_double
        L.pbo_band.restype = C.c_long
        L.pbo_delta.argtypes = [C.c_double, C.c_double]
        L.pbo_delta.restype = C.c_double
        L.pbo_pair.argtypes = [dp, dp, dp, dp, dp, C.c_double, dp]
        L.pbo_matvec.argtypes = [C.c_long, dp, dp, C.c_void_p, dp, dp]
        L.pbo_matvec_rows.argtypes = [C.c_long, dp, dp, C.c_void_p, dp, lp, C.c_long, dp, dp]
        L.pbo_dense.argtypes = [C.c_long, dp, dp, C.c_void_p, dp]
        L.pbo_curvature.argtypes = [ip, C.c_double, dp, C.c_long, dp]
        L.pbo_curvature.restype = C.c_double
        L.pbo_rhs.argtypes = [C.c_long, dp, dp, C.c_int, dp, dp]
        L.pbo_gmres.argtypes = [C.c_long, dp, dp, C.c_void_p, dp, dp, C.c_double, C.c_int, C.c_int, ip, dp]
        L.pbo_gmres.restype = C.c_int
        L.pbo_area.argtypes = [C.c_long, dp, C.c_double]
        L.pbo_area.restype = C.c_double
        L.pbo_energy.argtypes = [C.c_long, dp, dp, C.c_int, dp, dp, dp]
        L.pbo_energy.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(h, eps_in=1.0, eps_out=80.0, kappa=0.1257, band_k=2.0, tau_k=1.0, metric=METRIC_GUARDED,
           probe=1.4, cfl=0.3, reinit_steps=0, avg=AVG_FLAT):
    """Parameter vector: ε = band_k·h, τ = tau_k·h (the experiments use ε = 2h, τ ∈ {h, h/2});
    avg: disc averages of the regularized pairs (the paper's, or curvature-corrected)."""
    p = np.zeros(NPRM)
    p[EPS_IN], p[EPS_OUT], p[KAPPA], p[H] = eps_in, eps_out, kappa, h
    p[BAND], p[TAU], p[METRIC] = band_k * h, tau_k * h, metric
    p[PROBE], p[CFL], p[REINIT], p[AVG] = probe, cfl, reinit_steps, avg
    return p


def _cv(curv, n):
    if curv is None:
        return None, None
    c = _f64(curv)
    assert c.shape == (n,)
    return c, c.ctypes.data_as(C.c_void_p)


def grid(atoms, h, margin):
    atoms = _f64(atoms)
    dims = (C.c_int * 3)()
    origin = (C.c_double * 3)()
    lib().pbo_grid(_d(atoms), len(atoms), h, margin, dims, origin)
    return tuple(dims), tuple(origin)


def vdw(dims, origin, h, atoms):
    atoms = _f64(atoms)
    phi = np.empty(int(np.prod(dims)))
    lib().pbo_vdw((C.c_int * 3)(*dims), (C.c_double * 3)(*origin), h, _d(atoms), len(atoms), _d(phi))
    return phi


def eikonal(dims, h, phi, t_end, cfl=0.3):
    phi = _f64(phi).copy()
    lib().pbo_eikonal((C.c_int * 3)(*dims), h, _d(phi), t_end, cfl)
    return phi


def cavity(dims, h, phi, eps):
    phi = _f64(phi).copy()
    outside = np.zeros(len(phi), dtype=np.uint8)
    nset = lib().pbo_cavity((C.c_int * 3)(*dims), h, _d(phi), eps, outside.ctypes.data_as(C.c_void_p))
    return phi, outside, nset


def reinit(dims, h, phi, steps, cfl=0.3):
    phi = _f64(phi).copy()
    lib().pbo_reinit((C.c_int * 3)(*dims), h, _d(phi), steps, cfl)
    return phi


def ses(dims, origin, atoms, prm):
    atoms, prm = _f64(atoms), _f64(prm)
    phi = np.empty(int(np.prod(dims)))
    ncav = lib().pbo_ses((C.c_int * 3)(*dims), (C.c_double * 3)(*origin), _d(atoms), len(atoms), _d(prm), _d(phi))
    return phi, ncav


def weno_grad(dims, h, phi, node):
    phi = _f64(phi)
    m, p = (C.c_double * 3)(), (C.c_double * 3)()
    lib().pbo_weno_grad((C.c_int * 3)(*dims), h, _d(phi), node, m, p)
    return np.array(m[:]), np.array(p[:])


GRAD_CENTRAL, GRAD_WENO = 0, 1


def band(dims, origin, h, phi, eps, grad_scheme=GRAD_WENO, jacobian=False):
    """Returns (nodes [n×8], gidx [n]); raises if a band node touches the grid edge.
    grad_scheme: the WENO5 average (default, as in the paper's simulations) or central
    differences; jacobian: ω carries the explicit J."""
    phi = _f64(phi)
    d3, o3 = (C.c_int * 3)(*dims), (C.c_double * 3)(*origin)
    n = lib().pbo_band(d3, o3, h, _d(phi), eps, grad_scheme, int(jacobian), None, None)
    if n < 0:
        raise ValueError("band touches the grid boundary")
    nodes = np.empty((n, 8))
    gidx = np.empty(n, dtype=np.int64)
    lib().pbo_band(d3, o3, h, _d(phi), eps, grad_scheme, int(jacobian), nodes.ctypes.data_as(C.c_void_p),
                   gidx.ctypes.data_as(C.c_void_p))
    return nodes, gidx


def jacobian(dims, h, phi, node, n):
    """Explicit J at one interior grid node with unit normal n."""
    return lib().pbo_jacobian((C.c_int * 3)(*dims), h, _d(_f64(phi)), int(node), _d(_f64(n)))


def curvature(dims, h, phi, gidx, nodes):
    """κ1 + κ2 of the surface at each band node's projection (nodes: the band table, gidx: grid indices)."""
    phi = _f64(phi)
    d3 = (C.c_int * 3)(*dims)
    L = lib()
    return np.array([L.pbo_curvature(d3, h, _d(phi), int(g), _d(_f64(nd[3:6]))) for g, nd in zip(gidx, nodes)])


def delta(eta, eps):
    return lib().pbo_delta(float(eta), float(eps))


def pair(x, nx, y, ny, prm, curv_x=0.0):
    K = np.empty(4)
    lib().pbo_pair(_d(_f64(x)), _d(_f64(nx)), _d(_f64(y)), _d(_f64(ny)), _d(_f64(prm)), float(curv_x), _d(K))
    return K


def matvec(nodes, prm, p, curv=None):
    nodes, prm, p = _f64(nodes), _f64(prm), _f64(p)
    c, cp = _cv(curv, len(nodes))
    y = np.empty(2 * len(nodes))
    lib().pbo_matvec(len(nodes), _d(nodes), _d(prm), cp, _d(p), _d(y))
    return y


def matvec_rows(nodes, prm, p, rows, curv=None):
    nodes, prm, p = _f64(nodes), _f64(prm), _f64(p)
    c, cp = _cv(curv, len(nodes))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y1, y2 = np.empty(len(rows)), np.empty(len(rows))
    lib().pbo_matvec_rows(len(nodes), _d(nodes), _d(prm), cp, _d(p), rows.ctypes.data_as(C.POINTER(C.c_long)),
                          len(rows), _d(y1), _d(y2))
    return y1, y2


def dense(nodes, prm, curv=None):
    nodes, prm = _f64(nodes), _f64(prm)
    c, cp = _cv(curv, len(nodes))
    A = np.empty((2 * len(nodes), 2 * len(nodes)))
    lib().pbo_dense(len(nodes), _d(nodes), _d(prm), cp, _d(A))
    return A


def rhs(nodes, atoms, prm):
    nodes, atoms, prm = _f64(nodes), _f64(atoms), _f64(prm)
    g = np.empty(2 * len(nodes))
    lib().pbo_rhs(len(nodes), _d(nodes), _d(atoms), len(atoms), _d(prm), _d(g))
    return g


def lam(prm):
    """Diagonal of Λ: ½(1+ε_E/ε_I) and ½(1+ε_I/ε_E)."""
    return 0.5 * (1 + prm[EPS_OUT] / prm[EPS_IN]), 0.5 * (1 + prm[EPS_IN] / prm[EPS_OUT])


def gmres(nodes, prm, g, x0=None, tol=1e-8, max_iter=500, restart=200, curv=None):
    """GMRES from x0 (default Λ⁻¹g, the paper's diagonal initial guess). Returns (x, iters, relres, ok)."""
    nodes, prm, g = _f64(nodes), _f64(prm), _f64(g)
    n = len(nodes)
    c, cp = _cv(curv, n)
    if x0 is None:
        l1, l2 = lam(prm)
        x = np.concatenate([g[:n] / l1, g[n:] / l2])
    else:
        x = _f64(x0).copy()
    it, rr = C.c_int(), C.c_double()
    ok = lib().pbo_gmres(n, _d(nodes), _d(prm), cp, _d(g), _d(x), tol, max_iter, restart, C.byref(it),
                         C.byref(rr))
    return x, it.value, rr.value, bool(ok)


def area(nodes, h):
    nodes = _f64(nodes)
    return lib().pbo_area(len(nodes), _d(nodes), h)


def energy(nodes, atoms, prm, p):
    """Returns (G_pol in paper units e²/(ε0·Å), ψ_rxn at each atom)."""
    nodes, atoms, prm, p = _f64(nodes), _f64(atoms), _f64(prm), _f64(p)
    psi = np.empty(len(atoms))
    G = lib().pbo_energy(len(nodes), _d(nodes), _d(atoms), len(atoms), _d(prm), _d(p), _d(psi))
    return G, psi


KCAL_PER_UNIT = 4.0 * math.pi * 332.0637  # e²/(ε0·Å) in kcal/mol


def grid_margin(atoms, h, band_k=2.0, probe=1.4, ses=True):
    """Margin around the atoms: r_max + ρ0 (SES only) + ε + 4h + 1 Å."""
    rmax = float(np.max(np.asarray(atoms)[:, 3]))
    return rmax + (probe if ses else 0.0) + band_k * h + 4 * h + 1.0


def pipeline(atoms, h, ses=True, tau_k=1.0, grad_scheme=GRAD_WENO, jacobian=False, **kw):
    """Stage 1 + Stage 2 on the CPU: returns dims, origin, phi, nodes, gidx, prm."""
    prm = params(h, tau_k=tau_k, **kw)
    dims, origin = grid(atoms, h, grid_margin(atoms, h, prm[BAND] / h, prm[PROBE], ses))
    if ses:
        phi, _ = ses_fn(dims, origin, atoms, prm)
    else:
        phi = vdw(dims, origin, h, atoms)
    nodes, gidx = band(dims, origin, h, phi, prm[BAND], grad_scheme, jacobian)
    return dims, origin, phi, nodes, gidx, prm


ses_fn = ses
