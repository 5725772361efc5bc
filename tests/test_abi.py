"""The C-ABI library loads on the CPU and exports every function include/pb.h declares.

No device work is done here: only the host-only helpers (default parameters, grid
construction) are called, and their results are checked against the oracle's grid.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(pb_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_hot_path_calls():
    d = _declared()
    for name in ("pb_build_levelset", "pb_narrowband_compact", "pb_ibim_matvec", "pb_ibim_solve",
                 "pb_solvation_energy"):
        assert name in d


def test_library_exports_every_declared_symbol():
    from paper_1709_08070_amd import pb

    lib = C.CDLL(pb.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(pb.EXPORTS) <= _declared()


def test_default_params_are_the_papers():
    from paper_1709_08070_amd import pb

    p = pb.params()
    assert (p.eps_in, p.eps_out, p.kappa, p.band_k, p.tau_k, p.probe) == (1.0, 80.0, 0.1257, 2.0, 1.0, 1.4)
    assert (p.grad_scheme, p.jacobian) == (pb.PB_GRAD_WENO, pb.PB_JAC_ONE)
    # the C struct is no larger than its ctypes mirror: bytes past it stay untouched
    import ctypes as C

    size = C.sizeof(pb.pb_params)
    buf = (C.c_ubyte * (size + 64))(*([0xA5] * (size + 64)))
    pb.lib.pb_default_params(C.cast(buf, C.POINTER(pb.pb_params)))
    assert bytes(buf[size:]) == b"\xa5" * 64
    q = C.cast(buf, C.POINTER(pb.pb_params)).contents
    assert (q.jacobian, q.grad_scheme, q.reinit_steps, q.h) == (0, 1, 0, 0.5)
    o = pb.solve_opts()
    assert o.x0 == pb.PB_X0_DIAG and o.precision == pb.PB_FP64


@pytest.mark.parametrize("ses", [False, True])
def test_grid_for_atoms_matches_oracle_grid(ses):
    from paper_1709_08070_amd import pb, synth

    atoms = synth.globule(30, 4)
    for h in (0.25, 0.5):
        prm = pb.params(h, ls_mode=pb.PB_LS_SES if ses else pb.PB_LS_VDW)
        g = pb.pb_grid_for_atoms(atoms, prm)
        dims, origin = oracle.grid(atoms, h, oracle.grid_margin(atoms, h, ses=ses))
        assert (g.nx, g.ny, g.nz) == dims
        assert np.allclose(list(g.origin), origin, atol=1e-12, rtol=0)


def test_grid_for_atoms_rejects_bad_input():
    from paper_1709_08070_amd import pb

    prm = pb.params(0.5)
    bad = np.array([[0.0, 0.0, np.nan, 1.0, 0.0]])
    with pytest.raises(pb.PBError):
        pb.pb_grid_for_atoms(bad, prm)
