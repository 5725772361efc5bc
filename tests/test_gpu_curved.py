"""GPU parity of the curvature-corrected disc averages (reg_avg = PB_AVG_CURVED) against the
FP64 oracle: the band's curvature κ1 + κ2 at x* (Born ion, exact distance, and a 40-atom SES
globule), every operator path on the Born ion with the GPU's band, and the FP64 solve's
energy against the oracle's and the closed form. Bars: curvature 1e-10 absolute; FP64
operator 1e-12 relative (2-norm); mixed and treecode 1e-5; energy 1e-8 relative to the
oracle and within 0.5 % of the Born closed form (τ = h, h = 0.25). Plus the argument checks:
the curved averages need band->curv; the batched solve refuses them.
"""
import math
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


@pytest.fixture(scope="module")
def ctx(pbm):
    return pbm.Context(0)


def _case(pbm, ctx, atoms, h, ses):
    import torch

    prm = pbm.params(h, ls_mode=pbm.PB_LS_SES if ses else pbm.PB_LS_VDW, reg_avg=pbm.PB_AVG_CURVED)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    band = pbm.pb_narrowband_compact(ctx, grid, phi, prm)
    return prm, grid, at, phi, band


@pytest.fixture(scope="module")
def born(pbm, ctx):
    say("case: curved disc averages, Born ion R=2 h=0.25")
    return _case(pbm, ctx, synth.born_ion(), 0.25, False)


@pytest.mark.parametrize("name", ["born", "globule40"])
def test_band_curvature_matches_oracle(pbm, ctx, born, name):
    if name == "born":
        prm, grid, at, phi, band = born
        h = 0.25
    else:
        say("case: curvature, globule 40 atoms seed 9 h=0.5 SES")
        prm, grid, at, phi, band = _case(pbm, ctx, synth.globule(40, 9), 0.5, True)
        h = 0.5
    dims = (grid.nx, grid.ny, grid.nz)
    nodes = band.table()
    ref = oracle.curvature(dims, h, phi.cpu().numpy(), band.gidx[: band.n].cpu().numpy(), nodes)
    got = band.curv[: band.n].cpu().numpy()
    say(f"  n={band.n}: max |Δcurv| {np.max(np.abs(got - ref)):.3e}")
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10)
    if name == "born":
        assert np.max(np.abs(got - 1.0)) < 6e-3  # 2/R


@pytest.mark.parametrize("path", ["fp64", "mixed", "tree"])
def test_curved_operator_matches_oracle(pbm, ctx, born, path):
    import torch

    prm, grid, at, phi, band = born
    p = torch.tensor(np.random.default_rng(41).normal(size=2 * band.n), device="cuda")
    prec = {"fp64": pbm.PB_FP64, "mixed": pbm.PB_MIXED, "tree": pbm.PB_TREE}[path]
    y = pbm.pb_ibim_matvec(ctx, band, prm, p, prec).cpu().numpy()
    ref = oracle.matvec(band.table(), oracle.params(0.25, avg=oracle.AVG_CURVED), p.cpu().numpy(),
                        curv=band.curv[: band.n].cpu().numpy())
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    say(f"  {path}: vs oracle {rel:.3e}")
    assert rel < (1e-12 if path == "fp64" else 1e-5)


def test_curved_solve_energy(pbm, ctx, born):
    prm, grid, at, phi, band = born
    q, st = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(tol=1e-10, precision=pbm.PB_FP64))
    assert st.converged
    e = pbm.pb_solvation_energy(ctx, band, at, prm, q).g_pol
    nodes, curv = band.table(), band.curv[: band.n].cpu().numpy()
    oprm = oracle.params(0.25, avg=oracle.AVG_CURVED)
    ox, *_ = oracle.gmres(nodes, oprm, oracle.rhs(nodes, synth.born_ion(), oprm), tol=1e-10, curv=curv)
    oe, _ = oracle.energy(nodes, synth.born_ion(), oprm, ox)
    Gs = 1.0 / (16 * math.pi) * (1.0 / (80 * (1 + 0.1257 * 2)) - 1.0)
    say(f"  G_pol GPU {e:.12e} oracle {oe:.12e}; vs Born closed form {(e - Gs) / Gs:+.5f}")
    assert e == pytest.approx(oe, rel=1e-8)
    assert 0.0 < (e - Gs) / Gs < 0.005


def test_curved_argument_checks(pbm, ctx, born):
    import torch

    prm, grid, at, phi, band = born
    p = torch.zeros(2 * band.n, dtype=torch.float64, device="cuda")
    no_curv = pbm.Band(band.n, band.px, band.py, band.pz, band.nx, band.ny, band.nz, band.phi, band.w, band.gidx)
    with pytest.raises(Exception) as e:
        pbm.pb_ibim_matvec(ctx, no_curv, prm, p, pbm.PB_FP64)
    assert "curv" in str(e.value)
    with pytest.raises(Exception) as e:
        pbm.pb_ibim_solve_batched(ctx, [band], [at], prm, pbm.solve_opts(tol=1e-6, precision=pbm.PB_MIXED))
    assert "disc averages" in str(e.value)
