"""GPU parity of every operator path on the parameter cases the workloads do not reach: no
screening (κ = 0, the Laplace limit, where Gκ = G0 and the FP32 kernels take their
unscreened branch) and other dielectric constants (ε_I = 2, ε_E = 40), on the Born ion
(3281 nodes, all rows) against the FP64 oracle. Bars as elsewhere: FP64 operator 1e-12
relative (2-norm), mixed 1e-5, treecode 1e-5.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1709_08070_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_08070_amd import pb

    return pb


CASES = {"laplace": dict(kappa=0.0), "dielectrics": dict(eps_in=2.0, eps_out=40.0, kappa=0.7)}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("path", ["fp64_tiled", "fp64_sym", "mixed_tiled", "mixed_sym", "tree"])
def test_operator_paths(pbm, case, path):
    import torch

    kw = CASES[case]
    say(f"case: Born ion R=2 h=0.25, {case} {kw}, path {path}")
    env = {"fp64_tiled": ("PB_F64_CFG", "0"), "fp64_sym": ("PB_F64_CFG", "1"), "mixed_tiled": ("PB_FAR_CFG", "2"),
           "mixed_sym": ("PB_FAR_CFG", "4")}.get(path)
    if env:
        os.environ[env[0]] = env[1]
    try:
        ctx = pbm.Context(0)
        atoms = synth.born_ion()
        prm = pbm.params(0.25, ls_mode=pbm.PB_LS_VDW, **kw)
        grid = pbm.pb_grid_for_atoms(atoms, prm)
        at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
        phi = pbm.pb_build_levelset(ctx, at, prm, grid)
        band = pbm.pb_narrowband_compact(ctx, grid, phi, prm)
        p = torch.tensor(np.random.default_rng(31).normal(size=2 * band.n), device="cuda")
        prec = pbm.PB_FP64 if path.startswith("fp64") else (pbm.PB_TREE if path == "tree" else pbm.PB_MIXED)
        y = pbm.pb_ibim_matvec(ctx, band, prm, p, prec).cpu().numpy()
        ctx.close()
    finally:
        if env:
            del os.environ[env[0]]
    ref = oracle.matvec(band.table(), oracle.params(0.25, **kw), p.cpu().numpy())
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"  n={band.n}: {path} vs oracle {rel:.3e}")
    assert rel < (1e-12 if path.startswith("fp64") else 1e-5)
