"""GPU: the per-family event timers behind bench.py's roofline figures.

Level 2 of pb_set_timing times the far-field families only; level 1 every family; other
levels are rejected. A GMRES step that the host enqueued after the convergence test was met
does no work, and its timers are dropped: over a whole mixed solve the far-field timer
counts exactly the mixed operator applications the solve reports, and the treecode timer
those of a treecode solve.
"""
import sys

import numpy as np
import pytest

from paper_1709_08070_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_08070_amd import pb

    say("case: timers, globule 60 atoms seed 7301 h=0.5 SES")
    ctx = pb.Context(0)
    atoms = synth.globule(60, 7301)
    prm = pb.params(0.5, ls_mode=pb.PB_LS_SES)
    grid = pb.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pb.pb_build_levelset(ctx, at, prm, grid)
    band = pb.pb_narrowband_compact(ctx, grid, phi, prm)
    p = torch.tensor(np.random.default_rng(11).normal(size=2 * band.n), device="cuda")
    yield pb, ctx, prm, at, band, p
    ctx.close()


def test_timing_levels(setup):
    pb, ctx, prm, at, band, p = setup
    pb.pb_ibim_matvec(ctx, band, prm, p, pb.PB_MIXED)  # plan and autotuner outside the timers
    ctx.set_timing(2)
    pb.pb_ibim_matvec(ctx, band, prm, p, pb.PB_MIXED)
    ms, n_far = ctx.kernel_time("p2p_f32")
    _, n_near = ctx.kernel_time("near_f64")
    say(f"  level 2: p2p_f32 {n_far} launch(es) {ms:.3f} ms, near_f64 {n_near}")
    assert n_far == 1 and ms > 0.0 and n_near == 0
    ctx.set_timing(1)
    pb.pb_ibim_matvec(ctx, band, prm, p, pb.PB_MIXED)
    assert ctx.kernel_time("p2p_f32")[1] == 1 and ctx.kernel_time("near_f64")[1] == 1
    ctx.set_timing(0)
    for bad in (3, -1):
        with pytest.raises(RuntimeError):
            ctx.set_timing(bad)


@pytest.mark.parametrize("precision", ["mixed", "tree"])
def test_skipped_steps_are_not_timed(setup, precision):
    pb, ctx, prm, at, band, p = setup
    prec = pb.PB_MIXED if precision == "mixed" else pb.PB_TREE
    opts = pb.solve_opts(tol=1e-8, precision=prec, restart=7)  # several cycles
    pb.pb_ibim_solve(ctx, band, at, prm, opts)  # warm: plans and autotuner
    ctx.set_timing(2)
    _, st = pb.pb_ibim_solve(ctx, band, at, prm, opts)
    n_dense = ctx.kernel_time("p2p_f32")[1]
    n_tree = ctx.kernel_time("tree_f32")[1]
    n_fp64 = ctx.kernel_time("p2p_f64")[1]
    ctx.set_timing(0)
    say(f"  {precision}: {st.iters} iterations, {st.outer} outer steps; applications reported: "
        f"{st.matvecs_mixed} inner/residual, {st.matvecs_fp64} FP64; timed launches: dense {n_dense}, "
        f"treecode {n_tree}, FP64 {n_fp64}")
    assert st.converged
    # inner and residual applications together (at this tolerance the treecode solve takes its
    # refinement residuals from the FP64 operator)
    assert n_dense + n_tree == st.matvecs_mixed
    assert n_fp64 == st.matvecs_fp64
    if precision == "mixed":
        assert n_tree == 0
