"""GPU cavity stress cases against the FP64 oracle: a closed shell of atoms around a void
that the 1.4 Å probe cannot reach (section "Cavities removal"), empty and with a charged ion
inside the void. The void must be filled: no band node inside the shell, including around
the inner ion, whose own surface lies in the excluded region. The GPU level set must equal
the oracle's (1e-10 absolute), the band bit-exact, and the mixed solve's energy must match
the FP64 oracle solve on the same band (1e-6 relative).
"""
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


@pytest.mark.parametrize("inner_ion", [False, True], ids=["empty_void", "ion_in_void"])
def test_shell_cavity(pbm, inner_ion):
    import torch

    atoms = synth.shell(6.0, 1.6, 2.2)
    if inner_ion:
        atoms = np.vstack([atoms, [[0.1, -0.05, 0.2, 1.5, 1.0]]])
    say(f"case: closed shell R=6 of {len(atoms)} atoms, h=0.5, ion inside: {inner_ion}")
    ctx = pbm.Context(0)
    h = 0.5
    prm = pbm.params(h, ls_mode=pbm.PB_LS_SES)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    dims, origin = (grid.nx, grid.ny, grid.nz), tuple(grid.origin)
    ophi, ncav = oracle.ses(dims, origin, atoms, oracle.params(h))
    assert ncav > 0
    d = np.max(np.abs(phi.cpu().numpy() - ophi))
    say(f"  cavity nodes set by the oracle {ncav}; level set max |Δφ| {d:.3e}")
    assert d <= 1e-10
    band = pbm.pb_narrowband_compact(ctx, grid, phi, prm)
    onodes, ogidx = oracle.band(dims, origin, h, ophi, 2 * h)
    assert band.n == len(onodes)
    np.testing.assert_array_equal(band.gidx[: band.n].cpu().numpy(), ogidx)
    t = band.table()
    assert np.min(np.linalg.norm(t[:, :3], axis=1)) > 6.0  # nothing left inside the shell
    q, st = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(tol=1e-8, precision=pbm.PB_MIXED))
    assert st.converged
    e = pbm.pb_solvation_energy(ctx, band, at, prm, q).g_pol
    oprm = oracle.params(h)
    ox, *_ = oracle.gmres(t, oprm, oracle.rhs(t, atoms, oprm), tol=1e-9)
    oe, _ = oracle.energy(t, atoms, oprm, ox)
    say(f"  n={band.n}: energy GPU mixed {e:.10e} oracle {oe:.10e}")
    assert e == pytest.approx(oe, rel=1e-6)
    ctx.close()


def test_cli_on_a_pqr_file(pbm, tmp_path):
    """The command-line driver on a PQR file equals the same pipeline called directly, and
    its energy matches the oracle's solve on the same band."""
    import os

    import torch

    from paper_1709_08070_amd import cli, pqr

    path = str(tmp_path / "glob.pqr")
    atoms = synth.globule(30, 77)
    pqr.write_pqr(path, atoms)
    say("case: cli on a 30-atom PQR file, h=0.5, fp64, tol 1e-9")
    out = cli.run(path, h=0.5, precision="fp64", tol=1e-9)
    assert out["converged"] and out["true_relres"] <= 1e-9
    back = pqr.read_pqr(path)
    ctx = pbm.Context(0)
    prm = pbm.params(0.5, ls_mode=pbm.PB_LS_SES)
    grid = pbm.pb_grid_for_atoms(back, prm)
    at = torch.tensor(back, dtype=torch.float64, device="cuda")
    band = pbm.pb_narrowband_compact(ctx, grid, pbm.pb_build_levelset(ctx, at, prm, grid), prm)
    assert band.n == out["band_nodes"]
    t = band.table()
    oprm = oracle.params(0.5)
    ox, *_ = oracle.gmres(t, oprm, oracle.rhs(t, back, oprm), tol=1e-10)
    oe, _ = oracle.energy(t, back, oprm, ox)
    say(f"  n={band.n}: cli G_pol {out['g_pol']:.10e} oracle {oe:.10e}")
    assert out["g_pol"] == pytest.approx(oe, rel=1e-8)
    assert out["area"] == pytest.approx(oracle.area(t, 0.5), rel=1e-12)
    ctx.close()
