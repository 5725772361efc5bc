"""GPU: the learned preconditioner's BF16 MFMA kernels against the FP64 CPU reference
(oracle/nn_ref.py), its training, and what it gains over the method without it.

Bars: neighbour lists bit-exact; features 1e-6; M(v) and the parameter gradients within
1e-2 relative of the reference evaluated with the same BF16 roundings (BF16 operands,
FP32 accumulation in another order); training lowers the loss; the learned solve never ends
worse than plain GMRES (plain GMRES is the fallback, for the learned x0 alone as for the
preconditioner, within the one iteration budget) and reaches the same energy.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import nn_ref
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


def _band(pbm, ctx, atoms, h=0.5):
    import torch

    prm = pbm.params(h, ls_mode=pbm.PB_LS_SES)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    return prm, at, pbm.pb_narrowband_compact(ctx, grid, phi, prm)


@pytest.fixture(scope="module")
def small(pbm, ctx):
    say("case: nn geometry, globule 12 atoms seed 21 h=0.5")
    atoms = synth.globule(12, 21)
    prm, at, band = _band(pbm, ctx, atoms)
    pbm.pb_nn_prepare(ctx, band, prm)
    nodes = band.table()
    ref_nbr = nn_ref.knn(nodes[:, :3])
    return dict(atoms=atoms, prm=prm, at=at, band=band, nodes=nodes, ref_nbr=ref_nbr)


def test_neighbours_and_features(pbm, ctx, small):
    nbr, feat = pbm.pb_nn_geometry(ctx, small["band"])
    say(f"n={small['band'].n}")
    np.testing.assert_array_equal(nbr, small["ref_nbr"])
    ref = nn_ref.features(small["nodes"], small["ref_nbr"], 1.0)
    np.testing.assert_allclose(feat, ref, rtol=0, atol=2e-6)


def _random_params(pbm, seed, scale_last=0.05):
    rng = np.random.default_rng(seed)
    w = np.zeros(pbm.Net.param_count(), dtype=np.float32)
    off = 0
    for K, C in nn_ref.layer_shapes():
        a = np.sqrt(6.0 / K) * (scale_last if C == 16 else 1.0)
        w[off:off + K * C] = rng.uniform(-a, a, K * C)
        off += K * C
        w[off:off + C] = rng.normal(0, 0.05, C)
        off += C
    return w


def test_apply_matches_reference(pbm, ctx, small):
    import torch

    net = pbm.Net(ctx, seed=1)
    w = _random_params(pbm, 2, scale_last=1.0)
    net.set_params(w)
    n = small["band"].n
    v = np.random.default_rng(3).normal(size=2 * n)
    p = pbm.pb_nn_apply(ctx, net, small["band"], small["prm"], torch.tensor(v, device="cuda")).cpu().numpy()
    feat = nn_ref.features(small["nodes"], small["ref_nbr"], 1.0).astype(np.float32)
    ref = nn_ref.apply(small["nodes"], small["ref_nbr"], feat, v, w, (40.5, 0.50625), 1.0)
    diag = np.concatenate([v[:n] / 40.5, v[n:] / 0.50625])
    err = np.linalg.norm(p - ref) / np.linalg.norm(ref - diag)
    say(f"apply: correction rel err {err:.3e}")
    assert err < 1e-2
    # an untrained network is exactly the diagonal solve
    net0 = pbm.Net(ctx, seed=5)
    p0 = pbm.pb_nn_apply(ctx, net0, small["band"], small["prm"], torch.tensor(v, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(p0, diag, rtol=1e-15)


def test_gradients_match_reference(pbm, ctx, small):
    import torch

    net = pbm.Net(ctx, seed=1)
    w = _random_params(pbm, 7, scale_last=1.0)
    net.set_params(w)
    n = small["band"].n
    rng = np.random.default_rng(8)
    v, u = rng.normal(size=2 * n), rng.normal(size=2 * n)
    loss = pbm.pb_nn_train_step(ctx, net, small["band"], small["prm"], torch.tensor(v, device="cuda"),
                                torch.tensor(u, device="cuda"), 0.0)
    g = net.grads().astype(np.float64)
    feat = nn_ref.features(small["nodes"], small["ref_nbr"], 1.0).astype(np.float32)
    rl, rg = nn_ref.loss_and_grads(small["nodes"], small["ref_nbr"], feat, v, u, w, (40.5, 0.50625), 1.0)
    say(f"loss gpu {loss:.6e} ref {rl:.6e}")
    assert loss == pytest.approx(rl, rel=1e-2)
    off = 0
    for K, C in nn_ref.layer_shapes():
        for size in (K * C, C):
            a, b = g[off:off + size], rg[off:off + size]
            err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            say(f"grad block {off}:{off + size} rel err {err:.3e}")
            assert err < 1e-2
            off += size


def _training_set(pbm, ctx, seeds, sizes):
    import torch

    data = []
    for s, na in zip(seeds, sizes):
        atoms = synth.globule(na, s)
        prm, at, band = _band(pbm, ctx, atoms)
        g = pbm.pb_ibim_rhs(ctx, band, at, prm)
        u, st = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(tol=1e-8, precision=pbm.PB_MIXED))
        data.append((prm, at, band, g, u))
    return data


@pytest.fixture(scope="module")
def trained(pbm, ctx):
    say("case: nn training on 12 globules (40-120 atoms)")
    rng = np.random.default_rng(11)
    train = _training_set(pbm, ctx, list(range(9100, 9112)), list(rng.integers(40, 121, 12)))
    net = pbm.Net(ctx, seed=3)
    losses = []
    for epoch in range(25):
        for prm, at, band, g, u in train:
            pbm.pb_nn_prepare(ctx, band, prm)
            losses.append(pbm.pb_nn_train_step(ctx, net, band, prm, g, u, 2e-3))
    return net, losses


def test_training_and_gain(pbm, ctx, trained):
    net, losses = trained
    first, last = np.mean(losses[:12]), np.mean(losses[-12:])
    say(f"loss first epoch {first:.4f} last epoch {last:.4f}")
    assert last < 0.7 * first
    gains = []
    for s in (9900, 9901):
        atoms = synth.globule(150, s)
        prm, at, band = _band(pbm, ctx, atoms)
        base, st0 = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(tol=1e-6, precision=pbm.PB_MIXED))
        q, st1 = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(
            tol=1e-6, precision=pbm.PB_MIXED, x0=pbm.PB_X0_LEARNED, precond=pbm.PB_PRECOND_LEARNED, nn=net.handle))
        e0 = pbm.pb_solvation_energy(ctx, band, at, prm, base).g_pol
        e1 = pbm.pb_solvation_energy(ctx, band, at, prm, q).g_pol
        say(f"held-out {s}: plain iters {st0.iters} learned iters {st1.iters} fallback {st1.fallback_used} "
            f"energies {e0:.8e} {e1:.8e}")
        assert st1.converged and st1.true_relres <= 1e-6
        assert e1 == pytest.approx(e0, rel=1e-5)
        gains.append(st0.iters - st1.iters)
    assert min(gains) >= 0


def test_batched_learned_matches_single(pbm, ctx, trained):
    """The batched solve with the learned x0 and preconditioner (network over the
    concatenated batch, applied inside the captured Arnoldi step) against single learned
    solves and plain solves of the same molecules: same convergence, energies within the
    tolerance, iteration counts within a few steps of the single learned solves (the
    per-molecule RMS normalisation sums in another order, and the single solve's first pass
    runs on g rather than on the FP64 residual), fewer steps than plain."""
    net, _ = trained
    say("case: batched learned solve, held-out globules 150/110/70 atoms seeds 9900-9902, h=0.5, tol 1e-6 and 1e-9")
    mols = [_band(pbm, ctx, synth.globule(na, s)) for na, s in ((150, 9900), (110, 9901), (70, 9902))]
    bands = [b for _, _, b in mols]
    ats = [a for _, a, _ in mols]
    prm = mols[0][0]
    for tol in (1e-6, 1e-9):
        lopts = pbm.solve_opts(tol=tol, precision=pbm.PB_MIXED, x0=pbm.PB_X0_LEARNED,
                               precond=pbm.PB_PRECOND_LEARNED, nn=net.handle)
        ps, stats, bst = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, lopts)
        ps0, stats0, bst0 = pbm.pb_ibim_solve_batched(ctx, bands, ats, prm, pbm.solve_opts(tol=tol, precision=pbm.PB_MIXED))
        say(f"tol {tol:g}: learned replays {bst.graph_replays} outer {bst.outer}; plain replays {bst0.graph_replays}")
        for i, (b, at) in enumerate(zip(bands, ats)):
            st, st0 = stats[i], stats0[i]
            q, st1 = pbm.pb_ibim_solve(ctx, b, at, prm, lopts)
            e_b = pbm.pb_solvation_energy(ctx, b, at, prm, ps[i]).g_pol
            e_1 = pbm.pb_solvation_energy(ctx, b, at, prm, q).g_pol
            e_0 = pbm.pb_solvation_energy(ctx, b, at, prm, ps0[i]).g_pol
            say(f"  mol {i}: n={b.n} batch learned iters {st.iters} fallback {st.fallback_used} relres "
                f"{st.true_relres:.2e}; single learned iters {st1.iters}; batch plain iters {st0.iters}; "
                f"energies {e_b:.10e} {e_1:.10e} {e_0:.10e}")
            assert st.converged and st.true_relres <= tol and not st.fallback_used
            assert e_b == pytest.approx(e_1, rel=max(10 * tol, 1e-8))
            assert e_b == pytest.approx(e_0, rel=max(10 * tol, 1e-8))
            assert abs(st.iters - st1.iters) <= max(3, 0.15 * st1.iters)
        assert bst.graph_replays < bst0.graph_replays


def _nan_net(pbm, ctx):
    """A network whose output is not finite: finite parameters of magnitude 1e30 with random
    signs (the library refuses non-finite parameters), so the second layer's activations
    overflow FP32 and the sums of opposite infinities give NaN."""
    net = pbm.Net(ctx, seed=9)
    signs = np.where(np.random.default_rng(12).random(pbm.Net.param_count()) < 0.5, -1.0, 1.0)
    net.set_params((1e30 * signs).astype(np.float32))
    return net


def test_batched_learned_fallback(pbm, ctx, small):
    """A useless network: the batched learned run misses the tolerance and every molecule is
    finished by plain GMRES from its last iterate, reported as fallback, within the batch's
    iteration budget."""
    net = pbm.Net(ctx, seed=9)
    net.set_params(_random_params(pbm, 10, scale_last=1.0) * 40.0)
    say("case: batched learned fallback, globules 12/30 atoms seeds 21/22, useless network, tol 1e-8")
    m2 = _band(pbm, ctx, synth.globule(30, 22))
    bands, ats = [small["band"], m2[2]], [small["at"], m2[1]]
    ps, stats, bst = pbm.pb_ibim_solve_batched(ctx, bands, ats, small["prm"], pbm.solve_opts(
        tol=1e-8, precision=pbm.PB_MIXED, precond=pbm.PB_PRECOND_LEARNED, nn=net.handle, max_iter=300))
    for i, st in enumerate(stats):
        say(f"  mol {i}: fallback {st.fallback_used} iters {st.iters} relres {st.true_relres:.2e}")
        assert st.fallback_used == 1
        assert st.converged and st.true_relres <= 1e-8


def test_batched_learned_x0_nonfinite_fallback(pbm, ctx, small):
    """x0 = M(g) alone with a network that returns NaN: every molecule restarts from Λ⁻¹g
    without the network and converges, reported as fallback."""
    net = _nan_net(pbm, ctx)
    say("case: batched learned x0 only, NaN network, globules 12/30 atoms seeds 21/22, tol 1e-8")
    m2 = _band(pbm, ctx, synth.globule(30, 22))
    bands, ats = [small["band"], m2[2]], [small["at"], m2[1]]
    ps, stats, bst = pbm.pb_ibim_solve_batched(ctx, bands, ats, small["prm"], pbm.solve_opts(
        tol=1e-8, precision=pbm.PB_MIXED, x0=pbm.PB_X0_LEARNED, nn=net.handle, max_iter=300))
    for i, st in enumerate(stats):
        say(f"  mol {i}: fallback {st.fallback_used} iters {st.iters} relres {st.true_relres:.2e}")
        assert st.fallback_used == 1
        assert st.converged and st.true_relres <= 1e-8 and np.isfinite(ps[i].cpu().numpy()).all()


def test_fallback_to_plain_gmres(pbm, ctx, small):
    """A useless preconditioner: the solve is finished by plain GMRES from the last iterate,
    reported as fallback, and the two passes together stay within max_iter."""
    net = pbm.Net(ctx, seed=9)
    w = _random_params(pbm, 10, scale_last=1.0) * 40.0  # a useless network
    net.set_params(w)
    q, st = pbm.pb_ibim_solve(ctx, small["band"], small["at"], small["prm"], pbm.solve_opts(
        tol=1e-8, precision=pbm.PB_MIXED, precond=pbm.PB_PRECOND_LEARNED, nn=net.handle, max_iter=300))
    say(f"fallback: used={st.fallback_used} iters={st.iters} relres={st.true_relres:.2e}")
    assert st.fallback_used == 1
    assert st.converged and st.true_relres <= 1e-8 and st.iters <= 300


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_x0_nonfinite_fallback(pbm, ctx, small, precision):
    """x0 = M(g) alone (no preconditioner) with a network that returns NaN: the solve restarts
    from Λ⁻¹g without the network and converges within the same budget, reported as
    fallback; with a budget too small to converge it still returns a finite iterate."""
    net = _nan_net(pbm, ctx)
    prec = pbm.PB_FP64 if precision == "fp64" else pbm.PB_MIXED
    say(f"case: learned x0 only, NaN network, {precision}, globule 12 atoms, tol 1e-8")
    base, st0 = pbm.pb_ibim_solve(ctx, small["band"], small["at"], small["prm"],
                                  pbm.solve_opts(tol=1e-8, precision=prec))
    q, st = pbm.pb_ibim_solve(ctx, small["band"], small["at"], small["prm"], pbm.solve_opts(
        tol=1e-8, precision=prec, x0=pbm.PB_X0_LEARNED, nn=net.handle, max_iter=200))
    say(f"  plain iters {st0.iters}; learned-x0 fallback={st.fallback_used} iters={st.iters} "
        f"relres={st.true_relres:.2e}")
    assert st.fallback_used == 1 and st.converged and st.true_relres <= 1e-8 and st.iters <= 200
    e0 = pbm.pb_solvation_energy(ctx, small["band"], small["at"], small["prm"], base).g_pol
    e1 = pbm.pb_solvation_energy(ctx, small["band"], small["at"], small["prm"], q).g_pol
    assert e1 == pytest.approx(e0, rel=1e-7)
    q2, st2 = pbm.pb_ibim_solve(ctx, small["band"], small["at"], small["prm"], pbm.solve_opts(
        tol=1e-12, precision=prec, x0=pbm.PB_X0_LEARNED, nn=net.handle, max_iter=3), allow_noconv=True)
    say(f"  budget 3: fallback={st2.fallback_used} iters={st2.iters} relres={st2.true_relres:.2e}")
    assert st2.fallback_used == 1 and not st2.converged and st2.iters <= 3
    assert np.isfinite(st2.true_relres) and np.isfinite(q2.cpu().numpy()).all()


def test_committed_network_on_heldout_globule(pbm, ctx):
    """The committed network (trained on 200–1500-atom globules) on a held-out 5000-atom
    globule (seed 200000, never in training; about 158k band nodes at h = 0.5), as x0 and
    right preconditioner of the mixed solve to 1e-6: no fallback, fewer iterations than the
    plain mixed solve, and the oracle recomputes the residual on 64 sampled operator rows
    (1e-5 relative) and the energy (1e-10) from the learned solution."""
    import os

    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1709_08070_amd",
                         "weights", "learned_mixh.npz")
    if not os.path.exists(wpath):
        pytest.skip("no committed network")
    say("case: committed network, held-out globule 5000 atoms seed 200000 h=0.5, tol 1e-6")
    atoms = synth.globule(5000, 200000)
    prm, at, band = _band(pbm, ctx, atoms)
    n = band.n
    net = pbm.Net(ctx, seed=1)
    net.load(wpath)
    _, st0 = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(tol=1e-6, precision=pbm.PB_MIXED))
    sol, st = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(
        tol=1e-6, precision=pbm.PB_MIXED, x0=pbm.PB_X0_LEARNED, precond=pbm.PB_PRECOND_LEARNED, nn=net.handle))
    say(f"  n={n}: plain mixed {st0.iters} iterations, learned {st.iters} (fallback {st.fallback_used})")
    assert st.converged and st.true_relres <= 1e-6 and not st.fallback_used
    assert st.iters < st0.iters
    nodes = band.table()
    oprm = oracle.params(0.5)
    g = oracle.rhs(nodes, atoms, oprm)
    rows = np.random.default_rng(17).choice(n, 64, replace=False)
    s = sol.cpu().numpy()
    a1, a2 = oracle.matvec_rows(nodes, oprm, s, rows)
    rel = np.linalg.norm(np.concatenate([a1 - g[rows], a2 - g[n + rows]])) / np.linalg.norm(
        np.concatenate([g[rows], g[n + rows]]))
    e_gpu = pbm.pb_solvation_energy(ctx, band, at, prm, sol).g_pol
    oE, _ = oracle.energy(nodes, atoms, oprm, s)
    say(f"  sampled residual {rel:.2e}; energy {e_gpu:.12e} oracle {oE:.12e}")
    assert rel < 1e-5
    assert e_gpu == pytest.approx(oE, rel=1e-10)
