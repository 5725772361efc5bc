"""GPU: the batched mixed-precision solve (persistent far-field launch, captured Arnoldi-step
graph) against independent single-molecule solves and, for the smallest molecule, the oracle.

Seeded globules of uneven size (atom counts log-uniform), h = 0.5, SES. Bar: every molecule
converges to the requested FP64 residual and its energy matches the single-molecule FP64
solve to 1e-6 relative (both sides solve the same discrete system to 1e-9).
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


def _prepare(pb, ctx, atoms_list, h):
    import torch

    prm = pb.params(h, ls_mode=pb.PB_LS_SES)
    bands, ats = [], []
    for atoms in atoms_list:
        grid = pb.pb_grid_for_atoms(atoms, prm)
        at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
        phi = pb.pb_build_levelset(ctx, at, prm, grid)
        bands.append(pb.pb_narrowband_compact(ctx, grid, phi, prm))
        ats.append(at)
    return prm, bands, ats


def test_batched_matches_single_solves(pbm):
    ctx = pbm.Context(0)
    sizes = synth.batch_sizes(6, seed0=7100, lo=15, hi=200)
    atoms_list = [synth.globule(n, 7100 + i) for i, n in enumerate(sizes)]
    say(f"case: batch of {len(sizes)} globules, atoms {sizes}, h=0.5")
    prm, bands, ats = _prepare(pbm, ctx, atoms_list, 0.5)
    say("band nodes", [b.n for b in bands])
    opts = pbm.solve_opts(tol=1e-9, precision=pbm.PB_MIXED)
    ps, stats, bst = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, opts)
    say(f"batch: replays={bst.graph_replays} outer={bst.outer} tile={bst.far_tile}x{bst.far_tpl} "
        f"items={bst.n_items} p50={bst.t_p50_s:.4f}s p99={bst.t_p99_s:.4f}s total={bst.t_total_s:.3f}s")
    assert bst.graph_replays > 0 and bst.t_p50_s > 0 and bst.t_p99_s >= bst.t_p50_s
    for i, (b, at, p, st) in enumerate(zip(bands, ats, ps, stats)):
        assert st.converged and st.true_relres <= 1e-9, (i, st.true_relres)
        e_b = pbm.pb_solvation_energy(ctx, b, at, prm, p).g_pol
        q, st1 = pbm.pb_ibim_solve(ctx, b, at, prm, pbm.solve_opts(tol=1e-9, precision=pbm.PB_FP64))
        e_1 = pbm.pb_solvation_energy(ctx, b, at, prm, q).g_pol
        say(f"mol {i}: n={b.n} iters={st.iters} e_batch={e_b:.10e} e_single={e_1:.10e}")
        assert e_b == pytest.approx(e_1, rel=1e-6)
    # the smallest molecule against the oracle (same band)
    i = int(np.argmin([b.n for b in bands]))
    nodes = bands[i].table()
    oprm = oracle.params(0.5)
    ox, *_ = oracle.gmres(nodes, oprm, oracle.rhs(nodes, atoms_list[i], oprm), tol=1e-10)
    oG, _ = oracle.energy(nodes, atoms_list[i], oprm, ox)
    assert pbm.pb_solvation_energy(ctx, bands[i], ats[i], prm, ps[i]).g_pol == pytest.approx(oG, rel=1e-6)
    # a second call reuses the cached tile shape and gives the same answers bitwise
    ps2, stats2, bst2 = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, opts)
    for p, p2 in zip(ps, ps2):
        assert np.array_equal(p.cpu().numpy(), p2.cpu().numpy())
    ctx.close()


@pytest.mark.parametrize("x0", ["zero", "diag"])
def test_batched_application_count(pbm, x0):
    """The batched refinement's bookkeeping, as the single solve's: the first pass runs on the
    mixed operator from the initial guess (its residual from one mixed application, none from a
    zero start); with restart 400 every inner cycle ends on its residual estimate, so a molecule
    spends one mixed application per Arnoldi step beyond that first residual, and one FP64
    application per pass it takes (at least one, at most the batch's passes)."""
    ctx = pbm.Context(0)
    sizes = synth.batch_sizes(3, seed0=7300, lo=15, hi=120)
    atoms_list = [synth.globule(n, 7300 + i) for i, n in enumerate(sizes)]
    say(f"case: batch of {len(sizes)} globules, atoms {sizes}, h=0.5, tol 1e-9, restart 400, x0 {x0}")
    prm, bands, ats = _prepare(pbm, ctx, atoms_list, 0.5)
    mode = pbm.PB_X0_ZERO if x0 == "zero" else pbm.PB_X0_DIAG
    opts = pbm.solve_opts(tol=1e-9, precision=pbm.PB_MIXED, restart=400, max_iter=400, x0=mode)
    ps, stats, bst = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, opts)
    for i, st in enumerate(stats):
        say(f"  mol {i}: n={bands[i].n} iters {st.iters}, mixed {st.matvecs_mixed}, FP64 {st.matvecs_fp64}, "
            f"batch passes {bst.outer}")
        assert st.converged and st.true_relres <= 1e-9
        assert 1 <= st.matvecs_fp64 <= bst.outer
        assert st.matvecs_mixed == st.iters + (0 if x0 == "zero" else 1)
    ctx.close()


def test_batch64_full_size_sampled(pbm):
    """The benchmark's batch at full size (64 globules, atom counts log-uniform over 50–2000,
    seeds 64000 + m, h = 0.5, mixed solve to 1e-6 in one batched call). For the smallest,
    the median and the largest molecule the oracle recomputes, from the batch's solution, the
    residual on 64 sampled operator rows (1e-5 relative) and the energy (1e-10)."""
    ctx = pbm.Context(0)
    sizes = synth.batch_sizes(64, 64000)
    atoms_list = [synth.globule(n, 64000 + m) for m, n in enumerate(sizes)]
    say(f"case: batch64, atoms {min(sizes)}-{max(sizes)}, h=0.5, tol 1e-6")
    prm, bands, ats = _prepare(pbm, ctx, atoms_list, 0.5)
    ns = [b.n for b in bands]
    say(f"  band nodes {min(ns)}-{max(ns)}, {sum(ns)} in total")
    ps, stats, bst = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, pbm.solve_opts(tol=1e-6,
                                                                                     precision=pbm.PB_MIXED))
    say(f"  replays={bst.graph_replays} outer={bst.outer} items={bst.n_items} p50={bst.t_p50_s:.3f}s "
        f"p99={bst.t_p99_s:.3f}s")
    assert all(st.converged and st.true_relres <= 1e-6 for st in stats)
    oprm = oracle.params(0.5)
    order = np.argsort(ns)
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        nodes = bands[i].table()
        n = len(nodes)
        s = ps[i].cpu().numpy()
        rows = np.random.default_rng(i).choice(n, 64, replace=False)
        g = oracle.rhs(nodes, atoms_list[i], oprm)
        a1, a2 = oracle.matvec_rows(nodes, oprm, s, rows)
        res = np.concatenate([a1 - g[rows], a2 - g[n + rows]])
        rel = np.linalg.norm(res) / np.linalg.norm(np.concatenate([g[rows], g[n + rows]]))
        e_gpu = pbm.pb_solvation_energy(ctx, bands[i], ats[i], prm, ps[i]).g_pol
        oE, _ = oracle.energy(nodes, atoms_list[i], oprm, s)
        say(f"  mol {i}: n={n} iters={stats[i].iters} sampled residual {rel:.2e}, energy {e_gpu:.10e} "
            f"oracle {oE:.10e}")
        assert rel < 1e-5
        assert e_gpu == pytest.approx(oE, rel=1e-10)
    # the same batch with the committed network as x0 and right preconditioner
    import os

    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1709_08070_amd",
                         "weights", "learned_mixh.npz")
    if os.path.exists(wpath):
        net = pbm.Net(ctx, seed=1)
        net.load(wpath)
        lopts = pbm.solve_opts(tol=1e-6, precision=pbm.PB_MIXED, x0=pbm.PB_X0_LEARNED,
                               precond=pbm.PB_PRECOND_LEARNED, nn=net.handle)
        lps, lstats, lbst = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, lopts)
        say(f"  learned: replays={lbst.graph_replays} (plain {bst.graph_replays}), "
            f"fallbacks {sum(st.fallback_used for st in lstats)}")
        assert all(st.converged and st.true_relres <= 1e-6 and not st.fallback_used for st in lstats)
        assert lbst.graph_replays < bst.graph_replays
        for i in range(len(bands)):
            e_l = pbm.pb_solvation_energy(ctx, bands[i], ats[i], prm, lps[i]).g_pol
            e_p = pbm.pb_solvation_energy(ctx, bands[i], ats[i], prm, ps[i]).g_pol
            assert e_l == pytest.approx(e_p, rel=1e-6)
        i = int(order[-1])
        nodes = bands[i].table()
        oE, _ = oracle.energy(nodes, atoms_list[i], oprm, lps[i].cpu().numpy())
        assert pbm.pb_solvation_energy(ctx, bands[i], ats[i], prm, lps[i]).g_pol == pytest.approx(oE, rel=1e-10)
    ctx.close()


def test_batched_rejects_bad_input(pbm):
    import torch

    ctx = pbm.Context(0)
    prm, bands, ats = _prepare(pbm, ctx, [synth.globule(20, 3)], 0.5)
    with pytest.raises(pbm.PBError) as e:
        pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, pbm.solve_opts(precision=pbm.PB_FP64))
    assert e.value.status == pbm.PB_EINVAL
    lit = pbm.params(0.5, ls_mode=pbm.PB_LS_SES, reg_metric=pbm.PB_REG_TANGENT)
    with pytest.raises(pbm.PBError) as e:
        pbm.pb_ibim_solve_batched(ctx, bands, ats, lit, pbm.solve_opts(precision=pbm.PB_MIXED))
    assert e.value.status == pbm.PB_EINVAL
    ctx.close()
