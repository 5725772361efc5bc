"""GPU: the symmetric kernels (each unordered pair evaluated once for both directions) —
the FP32 far field forced with PB_FAR_CFG=4 and the FP64 operator forced with
PB_F64_CFG=1 — against the FP64 oracle and the one-directional kernels.

Cases: the Born ion (3281 nodes: chunks of one 512-node sub-block, a ragged last chunk,
near pairs inside diagonal and off-diagonal chunk pairs), the 500-atom globule at h = 0.5
(36,033 nodes, sampled rows), a batch through the batched solve, and repeated launches
(bitwise reproducible). Bars as for the mixed operator: 1e-5 relative against the oracle
(2-norm over the rows compared), 1e-6 relative between the two FP32 kernels; for the FP64
operator as for the FP64 path: 1e-12 relative (2-norm) and 1e-10 of max|y| elementwise
against the oracle, under each regularization metric (the tangent-plane test is taken per
direction).
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


def _mixed(pbm, cfg, band, prm, p):
    """Mixed operator with the far-field kernel fixed to cfg (fresh context: fresh autotune cache)."""
    os.environ["PB_FAR_CFG"] = str(cfg)
    try:
        ctx = pbm.Context(0)
        y = pbm.pb_ibim_matvec(ctx, band, prm, p, pbm.PB_MIXED).cpu().numpy()
        y2 = pbm.pb_ibim_matvec(ctx, band, prm, p, pbm.PB_MIXED).cpu().numpy()
        ctx.close()
    finally:
        del os.environ["PB_FAR_CFG"]
    assert np.array_equal(y, y2), "repeated launches differ"
    return y


def _pipeline(pbm, ctx, atoms, h, ses):
    import torch

    prm = pbm.params(h, ls_mode=pbm.PB_LS_SES if ses else pbm.PB_LS_VDW)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    return prm, at, pbm.pb_narrowband_compact(ctx, grid, phi, prm)


@pytest.mark.parametrize("case", ["born", "globule500"])
def test_symmetric_matches_oracle_and_tiled(pbm, case):
    import torch

    ctx = pbm.Context(0)
    if case == "born":
        say("case: symmetric far field, Born ion R=2 h=0.25 (all rows)")
        atoms, h, ses = synth.born_ion(), 0.25, False
    else:
        say("case: symmetric far field, globule 500 atoms seed 500 h=0.5 (64 sampled rows)")
        atoms, h, ses = synth.globule(500, 500), 0.5, True
    prm, at, band = _pipeline(pbm, ctx, atoms, h, ses)
    n = band.n
    p = torch.tensor(np.random.default_rng(5).normal(size=2 * n), device="cuda")
    ys = _mixed(pbm, 4, band, prm, p)
    yt = _mixed(pbm, 2, band, prm, p)
    rel_t = np.linalg.norm(ys - yt) / np.linalg.norm(yt)
    nodes = band.table()
    rows = np.arange(n) if case == "born" else np.random.default_rng(6).choice(n, 64, replace=False)
    y1, y2 = oracle.matvec_rows(nodes, oracle.params(h), p.cpu().numpy(), rows)
    ref = np.concatenate([y1, y2])
    got = np.concatenate([ys[rows], ys[n + rows]])
    rel_o = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"n={n}: symmetric vs tiled {rel_t:.3e}, symmetric vs oracle {rel_o:.3e}")
    assert rel_t < 1e-6
    assert rel_o < 1e-5
    ctx.close()


def test_symmetric_multi_subblock_chunks(pbm):
    """A band above 51,200 nodes, where a chunk of the symmetric kernels holds several 512-node
    sub-blocks (target sub-blocks keep their forward sums in registers over the chunk's
    sources, reverse slots are stored by the first target sub-block and added to by the
    later ones) and the last chunk is ragged; most sub-block pairs take the FP64 kernel's far
    path. FP32 symmetric vs one-directional on every row (1e-6), FP64 symmetric vs
    one-directional on every row (1e-13), both against the oracle on 64 sampled rows."""
    import torch

    say("case: symmetric kernels with multi-sub-block chunks, globule 1200 atoms seed 1200 h=0.5")
    ctx = pbm.Context(0)
    prm, at, band = _pipeline(pbm, ctx, synth.globule(1200, 1200), 0.5, True)
    n = band.n
    nsub = -(-n // (100 * 512))
    say(f"  n={n}, sub-blocks per chunk {nsub}")
    assert nsub >= 2 and n % (512 * nsub) != 0
    p = torch.tensor(np.random.default_rng(11).normal(size=2 * n), device="cuda")
    ys, yt = _mixed(pbm, 4, band, prm, p), _mixed(pbm, 2, band, prm, p)
    zs, zt = _fp64(pbm, 1, band, prm, p), _fp64(pbm, 0, band, prm, p)
    rel32 = np.linalg.norm(ys - yt) / np.linalg.norm(yt)
    rel64 = np.linalg.norm(zs - zt) / np.linalg.norm(zt)
    rows = np.random.default_rng(12).choice(n, 64, replace=False)
    y1, y2 = oracle.matvec_rows(band.table(), oracle.params(0.5), p.cpu().numpy(), rows)
    ref = np.concatenate([y1, y2])
    o32 = np.linalg.norm(np.concatenate([ys[rows], ys[n + rows]]) - ref) / np.linalg.norm(ref)
    got64 = np.concatenate([zs[rows], zs[n + rows]])
    o64 = np.max(np.abs(got64 - ref)) / np.max(np.abs(ref))
    say(f"  FP32 sym vs tiled {rel32:.3e}, vs oracle rows {o32:.3e}; FP64 sym vs tiled {rel64:.3e}, "
        f"vs oracle rows (max) {o64:.3e}")
    assert rel32 < 1e-6 and o32 < 1e-5
    assert rel64 < 1e-13 and o64 < 1e-10
    ctx.close()


def test_symmetric_in_batched_solve(pbm):
    say("case: batched solve with the symmetric FP32 far field and FP64 operator, 3 globules (25/60/110 atoms), "
        "h=0.5, tol 1e-8")
    ctx = pbm.Context(0)
    mols = [_pipeline(pbm, ctx, synth.globule(na, s), 0.5, True) for na, s in ((25, 7300), (60, 7301), (110, 7302))]
    prm = mols[0][0]
    bands, ats = [b for _, _, b in mols], [a for _, a, _ in mols]
    opts = pbm.solve_opts(tol=1e-8, precision=pbm.PB_MIXED)
    os.environ["PB_FAR_CFG"] = "4"
    os.environ["PB_F64_CFG"] = "1"
    try:
        bctx = pbm.Context(0)
        ps, stats, bst = pbm.pb_ibim_solve_batched(bctx, bands, ats, prm, opts)
        ps2, _, _ = pbm.pb_ibim_solve_batched(bctx, bands, ats, prm, opts)
    finally:
        del os.environ["PB_FAR_CFG"]
        del os.environ["PB_F64_CFG"]
    assert bst.far_symmetric == 1
    for i, (b, at) in enumerate(zip(bands, ats)):
        assert stats[i].converged and stats[i].true_relres <= 1e-8
        assert np.array_equal(ps[i].cpu().numpy(), ps2[i].cpu().numpy())
        q, st = pbm.pb_ibim_solve(ctx, b, at, prm, pbm.solve_opts(tol=1e-8, precision=pbm.PB_FP64))
        e_b = pbm.pb_solvation_energy(ctx, b, at, prm, ps[i]).g_pol
        e_1 = pbm.pb_solvation_energy(ctx, b, at, prm, q).g_pol
        say(f"  mol {i}: n={b.n} iters {stats[i].iters} energy batch {e_b:.10e} FP64 {e_1:.10e}")
        assert e_b == pytest.approx(e_1, rel=1e-7)
    bctx.close()
    ctx.close()


def _fp64(pbm, cfg, band, prm, p):
    os.environ["PB_F64_CFG"] = str(cfg)
    try:
        ctx = pbm.Context(0)
        y = pbm.pb_ibim_matvec(ctx, band, prm, p, pbm.PB_FP64).cpu().numpy()
        y2 = pbm.pb_ibim_matvec(ctx, band, prm, p, pbm.PB_FP64).cpu().numpy()
        ctx.close()
    finally:
        del os.environ["PB_F64_CFG"]
    assert np.array_equal(y, y2), "repeated launches differ"
    return y


@pytest.mark.parametrize("tau_k,metric", [(1.0, 0), (0.5, 0), (1.0, 1), (1.0, 2)])
def test_symmetric_fp64_born(pbm, tau_k, metric):
    import torch

    say(f"case: symmetric FP64 operator, Born ion R=2 h=0.25, tau_k={tau_k} metric={metric} (all rows)")
    ctx = pbm.Context(0)
    atoms = synth.born_ion()
    prm = pbm.params(0.25, ls_mode=pbm.PB_LS_VDW, tau_k=tau_k, reg_metric=metric)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    band = pbm.pb_narrowband_compact(ctx, grid, phi, prm)
    n = band.n
    p = torch.tensor(np.random.default_rng(7).normal(size=2 * n), device="cuda")
    ys = _fp64(pbm, 1, band, prm, p)
    yt = _fp64(pbm, 0, band, prm, p)
    ref = oracle.matvec(band.table(), oracle.params(0.25, tau_k=tau_k, metric=metric), p.cpu().numpy())
    rel = np.linalg.norm(ys - ref) / np.linalg.norm(ref)
    say(f"n={n}: symmetric vs oracle {rel:.3e} (max {np.max(np.abs(ys - ref)) / np.max(np.abs(ref)):.3e}), "
        f"vs tiled {np.linalg.norm(ys - yt) / np.linalg.norm(yt):.3e}")
    assert rel < 1e-12
    assert np.max(np.abs(ys - ref)) < 1e-10 * np.max(np.abs(ref))
    ctx.close()


def test_symmetric_fp64_globule500(pbm):
    import torch

    say("case: symmetric FP64 operator, globule 500 atoms seed 500 h=0.5 (64 sampled rows)")
    ctx = pbm.Context(0)
    prm, at, band = _pipeline(pbm, ctx, synth.globule(500, 500), 0.5, True)
    n = band.n
    p = torch.tensor(np.random.default_rng(8).normal(size=2 * n), device="cuda")
    ys = _fp64(pbm, 1, band, prm, p)
    rows = np.random.default_rng(9).choice(n, 64, replace=False)
    y1, y2 = oracle.matvec_rows(band.table(), oracle.params(0.5), p.cpu().numpy(), rows)
    ref = np.concatenate([y1, y2])
    got = np.concatenate([ys[rows], ys[n + rows]])
    say(f"n={n}: symmetric FP64 vs oracle rows {np.linalg.norm(got - ref) / np.linalg.norm(ref):.3e}")
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))
    ctx.close()


@pytest.mark.parametrize("cfg", ["far0", "far1", "far2", "far3", "far4", "f64_0", "f64_1"])
def test_band_smaller_than_one_tile(pbm, cfg):
    """A single 0.8 Å sphere at h = 0.5: a band of 195 nodes, below one 256-node group (the
    tiled kernels run one partial tile and one partial bounding-box group; the symmetric
    kernels a single, partial diagonal chunk). Every operator variant against the oracle
    on all rows."""
    import torch

    ctx = pbm.Context(0)
    atoms = synth.born_ion(0.8)
    prm = pbm.params(0.5, ls_mode=pbm.PB_LS_VDW)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    band = pbm.pb_narrowband_compact(ctx, grid, phi, prm)
    n = band.n
    say(f"case: small band ({cfg}), sphere R=0.8 h=0.5, n={n}")
    assert n < 256
    p = torch.tensor(np.random.default_rng(10).normal(size=2 * n), device="cuda")
    ref = oracle.matvec(band.table(), oracle.params(0.5), p.cpu().numpy())
    kind, k = cfg.split("_") if "_" in cfg else ("far", cfg[3:])
    if kind == "far":
        y = _mixed(pbm, int(k), band, prm, p)
        rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        say(f"  mixed vs oracle {rel:.3e}")
        assert rel < 1e-5
    else:
        y = _fp64(pbm, int(k), band, prm, p)
        rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        say(f"  FP64 vs oracle {rel:.3e}")
        assert rel < 1e-12
    ctx.close()
