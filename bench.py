"""Benchmark of the IBIM hot path on one MI355X.

One step = the whole path over one synthetic molecule, inputs resident in HBM:
level set of the SES (pb_build_levelset) → band compaction (pb_narrowband_compact) →
GMRES to ‖g − Ap‖/‖g‖ ≤ 1e-6 (pb_ibim_solve, which also forms the right-hand side): by
default mixed precision with FP64 iterative refinement and the learned x0 and right
preconditioner (the committed network), --step-solve mixed without the network → area and
polarization energy (pb_solvation_energy).

The default workload is the largest single-GPU configuration: the 5000-atom synthetic
globule at h = 0.25 Å (638,391 band nodes).

value = pair-interactions evaluated by the operator during the K timed steps ÷ their wall
time (one pair-interaction = one ordered (target, source) evaluation of the 2×2 kernel
block, n² per dense operator application).

Extra fields: the dominant kernel's roofline (the FP32 far-field kernel, HIP-event timed
over the timed region; algorithmic FLOPs of the dense definition, with the executed counts
of the committed counter summary beside them); GMRES time-to-1e-6 of plain FP64, mixed,
learned + mixed, treecode and learned + treecode solves on the same band; the same on one
held-out 5000-atom molecule at h = 0.5 (the learned-preconditioner configuration); one
batched solve of 64 molecules with its per-molecule p50/p99 times; and the FP64 CPU oracle
timed on the host on a bounded sample.

Other workloads: globule500 (the same step at 500 atoms, h = 0.5), batch64 (64 molecules
per step through the batched solve, plain and learned), heldout5000 (time to 1e-6 on up to
8 held-out 5000-atom molecules at h = 0.5).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 61  # algorithmic FP32 FLOPs per pair-interaction (FMA = 2)
PEAK_FP32 = 157.3e12  # MI355X FP32 vector peak, FLOP/s

METRIC = "BIM pair-interactions/s; GMRES time-to-1e-6 (learned+mixed vs plain FP64)"

WORKLOADS = {
    # name: (atoms, seed, h); batch64 is 64 globules with atom counts log-uniform over 50-2000;
    # heldout5000 is 8 globules of 5000 atoms, seeds 200000+i (never used in training)
    "globule5000": (5000, 5000, 0.25),
    "globule500": (500, 500, 0.5),
    "batch64": (None, 64000, 0.5),
    "heldout5000": (5000, 200000, 0.5),
}

WEIGHTS = os.path.join(ROOT, "paper_1709_08070_amd", "weights", "learned_mixh.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def one_thread_rate(oracle, nodes, oprm, x, cores: int):
    """The oracle's pair rate on one host thread: 256 operator rows against every source,
    with the OpenMP runtime the oracle library runs on set to one thread for the sample."""
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    import numpy as np

    rows = np.arange(min(len(nodes), 256))
    gomp.omp_set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.matvec_rows(nodes, oprm, x, rows)
        dt = time.perf_counter() - t1
    finally:
        gomp.omp_set_num_threads(cores)
    return {"value": len(rows) * float(len(nodes)) / dt, "unit": "pair-interactions/s", "cores": 1,
            "sample": f"{len(rows)} operator rows x {len(nodes)} sources, {dt:.2f} s"}


def kernel_source_hash(path: str) -> str:
    """Hash of the source file that holds the kernel and every device function it inlines."""
    import hashlib

    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel's source has changed since the counters were taken (or none were taken)."""
    path = os.path.join(ROOT, "profiles", f"{kernel.replace('k_', '')}_{workload}_hbm.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, kv.get("source", ""))
    try:
        if kernel_source_hash(src) != kv.get("source_sha256_16"):
            return None
    except OSError:
        return None
    return float(kv["traffic_bytes"])


def load_net(ctx, args):
    """(net, record) from --learned-train, else from the weights file; (None, None) if neither."""
    from paper_1709_08070_amd import pb

    if args.learned_train > 0:
        from paper_1709_08070_amd import learn

        net = pb.Net(ctx, seed=1)
        info = learn.train(ctx, net, n_mol=args.learned_train, epochs=args.learned_epochs, log=log)
        rec = {k: info[k] for k in ("molecules", "epochs", "t_data_s", "t_train_s")}
        rec["final_loss"] = info["loss"][-1]
        rec["source"] = "trained in this run"
        return net, rec
    path = args.learned_weights
    if not path or not os.path.exists(path):
        return None, None
    net = pb.Net(ctx, seed=1)
    net.load(path)
    rec = {"source": os.path.relpath(path, ROOT)}
    meta = path.rsplit(".", 1)[0] + ".json"
    if os.path.exists(meta):
        info = json.load(open(meta))
        rec.update({k: info.get(k) for k in ("molecules", "epochs", "t_data_s", "t_train_s")})
        rec["final_loss"] = info["loss"][-1] if info.get("loss") else None
    return net, rec


def timed_solve(ctx, band, at, prm, opts, q, warm=True, warm_tol=None):
    """Wall time of one solve from x0; returns (seconds, stats). warm: one untimed solve
    first (it warms the caches, the workspace and the far-field autotuner), to warm_tol if
    given (a loose tolerance: the same set-up for a fraction of the iterations)."""
    import torch

    from paper_1709_08070_amd import pb

    if warm:
        o = opts
        if warm_tol is not None:
            o = pb.pb_solve_opts.from_buffer_copy(opts)
            o.tol = warm_tol
        pb.pb_ibim_solve(ctx, band, at, prm, o, q, allow_noconv=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st = pb.pb_ibim_solve(ctx, band, at, prm, opts, q)
    torch.cuda.synchronize()
    return time.perf_counter() - t1, st


def heldout_rows(ctx, net, seeds, tol):
    """Time to tol on held-out 5000-atom globules at h = 0.5 (never in training): plain FP64
    GMRES, mixed GMRES-IR, and mixed with the learned x0 and right preconditioner, also with
    the treecode far field as the inner operator. Each solve after a warm-up at 1e-2."""
    import torch

    from paper_1709_08070_amd import pb, synth

    n_atoms, _, h = WORKLOADS["heldout5000"]
    prm = pb.params(h, ls_mode=pb.PB_LS_SES)
    rows = []
    for seed in seeds:
        atoms = synth.globule(n_atoms, seed)
        grid = pb.pb_grid_for_atoms(atoms, prm)
        at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
        phi = pb.pb_build_levelset(ctx, at, prm, grid)
        band = pb.pb_narrowband_compact(ctx, grid, phi, prm)
        q = torch.zeros(2 * band.n, dtype=torch.float64, device="cuda")
        row = {"seed": seed, "atoms": n_atoms, "h": h, "band_nodes": band.n}
        for name, o in (("fp64", pb.solve_opts(tol=tol, precision=pb.PB_FP64)),
                        ("mixed", pb.solve_opts(tol=tol, precision=pb.PB_MIXED)),
                        ("learned_mixed", pb.solve_opts(tol=tol, precision=pb.PB_MIXED, x0=pb.PB_X0_LEARNED,
                                                        precond=pb.PB_PRECOND_LEARNED, nn=net.handle)),
                        ("learned_tree", pb.solve_opts(tol=tol, precision=pb.PB_TREE, x0=pb.PB_X0_LEARNED,
                                                       precond=pb.PB_PRECOND_LEARNED, nn=net.handle))):
            t, st = timed_solve(ctx, band, at, prm, o, q, warm_tol=1e-2)
            row[name + "_s"] = t
            row[name + "_iters"] = st.iters
            row[name + "_relres"] = st.true_relres
            if name.startswith("learned"):
                row[name + "_fallback"] = st.fallback_used
            if name == "learned_mixed":
                row["learned_mixed_pairs"] = st.pairs
            row[name + "_g_pol_kcal"] = pb.pb_solvation_energy(ctx, band, at, prm, q).g_pol_kcal
        for name in ("mixed", "learned_mixed", "learned_tree"):
            row[f"speedup_{name}_vs_fp64"] = row["fp64_s"] / row[name + "_s"]
            row[f"energy_rel_diff_{name}_vs_fp64"] = abs(row[name + "_g_pol_kcal"] / row["fp64_g_pol_kcal"] - 1)
        log(f"held-out {seed}: n={band.n} fp64 {row['fp64_s']:.3f}s/{row['fp64_iters']} it, mixed "
            f"{row['mixed_s']:.3f}s/{row['mixed_iters']} it, learned {row['learned_mixed_s']:.3f}s/"
            f"{row['learned_mixed_iters']} it (fallback {row['learned_mixed_fallback']}), learned tree "
            f"{row['learned_tree_s']:.3f}s/{row['learned_tree_iters']} it")
        rows.append(row)
    return rows


def bench_heldout(args):
    """Time to 1e-6 on up to 8 held-out 5000-atom globules (h = 0.5)."""
    from paper_1709_08070_amd import pb

    n_atoms, seed0, h = WORKLOADS["heldout5000"]
    ctx = pb.Context(0)
    net, rec = load_net(ctx, args)
    if net is None:
        log("heldout5000 needs a network: the weights file or --learned-train N")
        sys.exit(2)
    n_mol = max(1, min(args.steps, 8))
    rows = heldout_rows(ctx, net, [seed0 + i for i in range(n_mol)], args.tol)

    def mean(k):
        return sum(r[k] for r in rows) / len(rows)

    ttsol = {k: mean(k) for k in ("fp64_s", "mixed_s", "learned_mixed_s", "learned_tree_s", "fp64_iters",
                                  "mixed_iters", "learned_mixed_iters", "learned_tree_iters")}
    for name in ("mixed", "learned_mixed", "learned_tree"):
        ttsol[f"speedup_{name}_vs_fp64"] = ttsol["fp64_s"] / ttsol[name + "_s"]
        ttsol[f"max_energy_rel_diff_{name}_vs_fp64"] = max(r[f"energy_rel_diff_{name}_vs_fp64"] for r in rows)
    ttsol["speedup_learned_mixed_vs_mixed"] = ttsol["mixed_s"] / ttsol["learned_mixed_s"]
    ttsol["fallbacks"] = sum(r["learned_mixed_fallback"] + r["learned_tree_fallback"] for r in rows)
    ttsol["per_molecule"] = rows
    ttsol["network"] = rec
    pairs = sum(r["learned_mixed_pairs"] for r in rows)
    t_learned = sum(r["learned_mixed_s"] for r in rows)
    out = {
        "metric": METRIC, "value": pairs / t_learned, "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": n_mol, "warmup": 1, "ms_per_step": 1e3 * t_learned / n_mol, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "accumulate": "f64", "data": "synthetic",
        "config": {"workload": f"heldout5000: {n_mol} held-out synthetic globules of {n_atoms} atoms (seeds "
                               f"{seed0}+i), h={h} A, SES; time to {args.tol:g} of FP64 GMRES, mixed GMRES-IR and "
                               "learned-preconditioned mixed GMRES-IR, dense and treecode inner operator "
                               "(value: pair rate of the learned dense solves)",
                   "parallelism": "single GPU"},
        "time_to_tol": ttsol, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def batch_setup(ctx, prm):
    """The 64 molecules of the batched workload: atoms, grids, level sets and bands."""
    import torch

    from paper_1709_08070_amd import pb, synth

    _, seed0, _ = WORKLOADS["batch64"]
    sizes = synth.batch_sizes(64, seed0)
    mols = [synth.globule(n, seed0 + m) for m, n in enumerate(sizes)]
    grids, ats, phis, bands = [], [], [], []
    for atoms in mols:
        g = pb.pb_grid_for_atoms(atoms, prm)
        at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
        phi = pb.pb_build_levelset(ctx, at, prm, g)
        grids.append(g)
        ats.append(at)
        phis.append(phi)
        bands.append(pb.pb_narrowband_compact(ctx, g, phi, prm))
    ns = [b.n for b in bands]
    log(f"batch64: atoms {min(sizes)}-{max(sizes)}, band nodes {min(ns)}-{max(ns)}, total {sum(ns)}, "
        f"sum n^2 {sum(float(n) * n for n in ns):.3e}")
    return sizes, grids, ats, phis, bands


def batch_learned(ctx, net, rec, prm, bands, ats, ps, tol, t_plain):
    """One batched solve with the learned x0 and preconditioner (after a warm-up at 1e-2)."""
    import torch

    from paper_1709_08070_amd import pb

    lopts = pb.solve_opts(tol=tol, precision=pb.PB_MIXED, x0=pb.PB_X0_LEARNED, precond=pb.PB_PRECOND_LEARNED,
                          nn=net.handle)
    lps = [torch.zeros_like(p) for p in ps]
    warm = pb.pb_solve_opts.from_buffer_copy(lopts)
    warm.tol = 1e-2
    pb.pb_ibim_solve_batched(ctx, bands, ats, prm, warm, lps, allow_noconv=True)
    torch.cuda.synchronize()
    _, lstats, lbst = pb.pb_ibim_solve_batched(ctx, bands, ats, prm, lopts, lps)
    rel = max(abs(pb.pb_solvation_energy(ctx, b, at, prm, q).g_pol / pb.pb_solvation_energy(ctx, b, at, prm, p).g_pol
                  - 1) for b, at, q, p in zip(bands, ats, lps, ps))
    learned = {"solve_s": lbst.t_total_s, "p50_solve_s": lbst.t_p50_s, "p99_solve_s": lbst.t_p99_s,
               "graph_replays": lbst.graph_replays, "outer": lbst.outer,
               "fallbacks": sum(st.fallback_used for st in lstats),
               "max_relres": max(st.true_relres for st in lstats),
               "max_energy_rel_diff_vs_plain": rel,
               "speedup_vs_plain_batched": t_plain / lbst.t_total_s, "network": rec}
    log(f"learned batch: replays={lbst.graph_replays} solve={lbst.t_total_s:.3f}s p50={lbst.t_p50_s:.3f}s "
        f"p99={lbst.t_p99_s:.3f}s fallbacks={learned['fallbacks']} energy diff {rel:.2e}")
    return learned, lps


def batch_leg(net, rec, tol):
    """The batched workload as a leg of the default run: one plain and one learned batched
    solve of the 64 molecules (each after a warm-up at 1e-2), on a context of its own."""
    import torch

    from paper_1709_08070_amd import pb

    _, _, h = WORKLOADS["batch64"]
    ctx = pb.Context(0)
    prm = pb.params(h, ls_mode=pb.PB_LS_SES)
    sizes, grids, ats, phis, bands = batch_setup(ctx, prm)
    ns = [b.n for b in bands]
    ps = [torch.zeros(2 * n, dtype=torch.float64, device="cuda") for n in ns]
    opts = pb.solve_opts(tol=tol, precision=pb.PB_MIXED)
    warm = pb.pb_solve_opts.from_buffer_copy(opts)
    warm.tol = 1e-2
    pb.pb_ibim_solve_batched(ctx, bands, ats, prm, warm, ps, allow_noconv=True)
    torch.cuda.synchronize()
    _, stats, bst = pb.pb_ibim_solve_batched(ctx, bands, ats, prm, opts, ps)
    log(f"batch64 leg: replays={bst.graph_replays} solve={bst.t_total_s:.3f}s p50={bst.t_p50_s:.3f}s "
        f"p99={bst.t_p99_s:.3f}s max relres={max(st.true_relres for st in stats):.2e}")
    out = {"molecules": len(ns), "atoms_range": [min(sizes), max(sizes)], "h": h,
           "band_nodes_total": sum(ns), "band_nodes_range": [min(ns), max(ns)],
           "sum_n2": sum(float(n) * n for n in ns), "solve_s": bst.t_total_s, "p50_solve_s": bst.t_p50_s,
           "p99_solve_s": bst.t_p99_s, "graph_replays": bst.graph_replays, "pairs": bst.pairs,
           "pairs_per_s": bst.pairs / bst.t_total_s, "far_symmetric": bst.far_symmetric,
           "work_items": bst.n_items, "max_relres": max(st.true_relres for st in stats), "learned": None}
    if net is not None:
        # the network belongs to another context: load the same weights into this one
        lnet = pb.Net(ctx, seed=1)
        lnet.set_params(net.params())
        out["learned"], _ = batch_learned(ctx, lnet, rec, prm, bands, ats, ps, tol, bst.t_total_s)
        lnet.close()
    ctx.close()
    return out


def bench_batch(args):
    """64 molecules of uneven size: per step, every level set and band, then one batched
    mixed-precision solve (persistent far-field launch, captured Arnoldi-step graph) and
    every energy."""
    import torch

    from paper_1709_08070_amd import pb

    _, seed0, h = WORKLOADS["batch64"]
    ctx = pb.Context(0)
    prm = pb.params(h, ls_mode=pb.PB_LS_SES)
    sizes, grids, ats, phis, bands = batch_setup(ctx, prm)
    ns = [b.n for b in bands]
    ps = [torch.zeros(2 * n, dtype=torch.float64, device="cuda") for n in ns]
    opts = pb.solve_opts(tol=args.tol, precision=pb.PB_MIXED)

    def step():
        for g, at, phi, b in zip(grids, ats, phis, bands):
            pb.pb_build_levelset(ctx, at, prm, g, phi)
            pb.pb_narrowband_compact(ctx, g, phi, prm, b)
        _, stats, bst = pb.pb_ibim_solve_batched(ctx, bands, ats, prm, opts, ps)
        for at, b, p in zip(ats, bands, ps):
            pb.pb_solvation_energy(ctx, b, at, prm, p)
        return stats, bst

    for w in range(args.warmup):
        stats, bst = step()
        log(f"warmup {w}: replays={bst.graph_replays} outer={bst.outer} p50={bst.t_p50_s:.3f}s p99={bst.t_p99_s:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs, p50, p99, tsolve = 0.0, [], [], []
    for s in range(args.steps):
        stats, bst = step()
        pairs += bst.pairs
        p50.append(bst.t_p50_s)
        p99.append(bst.t_p99_s)
        tsolve.append(bst.t_total_s)
        log(f"step {s}: replays={bst.graph_replays} outer={bst.outer} tile={bst.far_tile}x{bst.far_tpl} "
            f"items={bst.n_items} solve={bst.t_total_s:.3f}s p50={bst.t_p50_s:.3f}s p99={bst.t_p99_s:.3f}s "
            f"max relres={max(st.true_relres for st in stats):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    learned, lps = None, None
    net, rec = load_net(ctx, args)
    if net is not None:
        learned, lps = batch_learned(ctx, net, rec, prm, bands, ats, ps, args.tol, sum(tsolve) / len(tsolve))
    fp64 = None
    if "fp64" in [x for x in args.legs.split(",") if x] and not args.no_compare:
        # plain FP64 GMRES on the same 64 molecules, one after the other (x0 = Λ⁻¹g)
        o64 = pb.solve_opts(tol=args.tol, precision=pb.PB_FP64)
        pb.pb_ibim_solve(ctx, bands[0], ats[0], prm, o64)  # warm the FP64 kernel choice
        torch.cuda.synchronize()
        t64, e64, iters64 = 0.0, [], []
        for b, at in zip(bands, ats):
            t1 = time.perf_counter()
            q64, st64 = pb.pb_ibim_solve(ctx, b, at, prm, o64)
            torch.cuda.synchronize()
            t64 += time.perf_counter() - t1
            iters64.append(st64.iters)
            e64.append(pb.pb_solvation_energy(ctx, b, at, prm, q64).g_pol)
        e_plain = [pb.pb_solvation_energy(ctx, b, at, prm, p).g_pol for b, at, p in zip(bands, ats, ps)]
        fp64 = {"solve_s_total": t64, "iters_range": [min(iters64), max(iters64)],
                "max_energy_rel_diff_batched_vs_fp64": max(abs(a / c - 1) for a, c in zip(e_plain, e64))}
        if learned is not None:
            e_l = [pb.pb_solvation_energy(ctx, b, at, prm, q).g_pol for b, at, q in zip(bands, ats, lps)]
            fp64["max_energy_rel_diff_learned_batched_vs_fp64"] = max(abs(a / c - 1) for a, c in zip(e_l, e64))
            fp64["speedup_learned_batched_vs_fp64"] = t64 / learned["solve_s"]
        fp64["speedup_batched_vs_fp64"] = t64 / (sum(tsolve) / len(tsolve))
        log(f"FP64 GMRES, one molecule after the other: {t64:.3f} s, energies within "
            f"{fp64['max_energy_rel_diff_batched_vs_fp64']:.2e} of the batched solve")
    out = {
        "metric": METRIC, "value": pairs / elapsed, "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "accumulate": "f64",
        "data": "synthetic",
        "config": {"workload": f"batch64: 64 synthetic globules, atom counts log-uniform 50-2000 (seeds {seed0}+m), "
                               f"h={h} A, SES; level sets + bands + one batched mixed solve to {args.tol:g} + energies",
                   "band_nodes_total": sum(ns), "band_nodes_range": [min(ns), max(ns)],
                   "parallelism": "single GPU"},
        "batch": {"solve_s_mean": sum(tsolve) / len(tsolve), "p50_solve_s": sum(p50) / len(p50),
                  "p99_solve_s": sum(p99) / len(p99), "graph_replays": bst.graph_replays,
                  "far_tile": bst.far_tile, "far_targets_per_lane": bst.far_tpl, "work_items": bst.n_items,
                  "learned": learned, "fp64_sequential": fp64},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def issue_rates():
    """Measured issue rates of single-instruction streams (wave instructions per second) from the
    committed summary of probes/issue_rates.hip, or None when the probe has changed since."""
    path = os.path.join(ROOT, "profiles", "valu_issue_rates_mi355x.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.split("#")[0].strip()
    try:
        if kernel_source_hash(os.path.join(ROOT, kv["probe"])) != kv.get("source_sha256_16"):
            return None
        return {k: float(v) for k, v in kv.items() if k.endswith("_wave_insts_per_s")}
    except (KeyError, OSError, ValueError):
        return None


def executed_counts(kernel: str, workload: str, pairs_per_launch: float, launch_s: float):
    """Executed VALU work of the kernel from the committed rocprofv3 counter summary (only while
    the kernel's source is unchanged), against the measured launch time."""
    path = os.path.join(ROOT, "profiles", f"{kernel.replace('k_', '')}_{workload}_valu.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.split("#")[0].strip()
    try:
        if kernel_source_hash(os.path.join(ROOT, kv["source"])) != kv.get("source_sha256_16"):
            return None
        valu = float(kv["SQ_INSTS_VALU"])
        fma, mul, add = (float(kv[f"SQ_INSTS_VALU_{x}_F32"]) for x in ("FMA", "MUL", "ADD"))
        trans = float(kv["SQ_INSTS_VALU_TRANS_F32"])
    except (KeyError, OSError, ValueError):
        return None
    flops = 64.0 * (2.0 * fma + mul + add)  # wave instructions × 64 lanes, FMA = 2
    out = {"source": os.path.relpath(path, ROOT), "valu_insts_per_pair": valu * 64.0 / pairs_per_launch,
           "executed_fp32_tflops": flops / launch_s / 1e12, "frac_of_peak": flops / launch_s / PEAK_FP32,
           "wave_insts_per_s": valu / launch_s, "transcendentals_per_s": 64.0 * trans / launch_s}
    rates = issue_rates()
    if rates and "fp32_fma_stream_wave_insts_per_s" in rates:
        # the kernel's VALU issue rate against a stream of FP32 FMAs on vector registers
        out["frac_of_fp32_fma_stream"] = valu / launch_s / rates["fp32_fma_stream_wave_insts_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="globule5000", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--step-solve", default="learned", choices=("learned", "mixed"),
                    help="solve of each timed step: mixed GMRES-IR with the learned x0 and preconditioner "
                         "(default), or without the network")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip every time-to-solution leg")
    ap.add_argument("--no-tree", action="store_true", help="skip the treecode time-to-solution legs")
    ap.add_argument("--no-heldout", action="store_true", help="skip the held-out learned-preconditioner leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-molecule leg")
    ap.add_argument("--legs", default="fp64,mixed,learned,tree,learned_tree",
                    help="time-to-solution legs, comma separated: fp64, mixed, learned, tree, learned_tree")
    ap.add_argument("--learned-train", type=int, default=0, metavar="N",
                    help="train the learned preconditioner on N generated molecules (200-1500 atoms, h=0.5) and "
                         "add its time-to-tolerance on the (held-out) workload molecule")
    ap.add_argument("--learned-epochs", type=int, default=2)
    ap.add_argument("--learned-weights", default=WEIGHTS,
                    help="weights file of the learned preconditioner (default: the committed one, if present)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of this many MiB (a reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_08070_amd import pb, synth

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "heldout5000":
        return bench_heldout(args)

    n_atoms, seed, h = WORKLOADS[args.workload]
    atoms = synth.globule(n_atoms, seed)
    dev = torch.device("cuda", 0)
    ctx = pb.Context(0)
    prm = pb.params(h, ls_mode=pb.PB_LS_SES)
    grid = pb.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device=dev)
    phi = pb.pb_build_levelset(ctx, at, prm, grid)
    band = pb.pb_narrowband_compact(ctx, grid, phi, prm)
    n = band.n
    p = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    net, rec = load_net(ctx, args)
    if args.step_solve == "learned" and net is None:
        log("--step-solve learned needs the network: the weights file or --learned-train N")
        sys.exit(2)
    learned_kw = dict(x0=pb.PB_X0_LEARNED, precond=pb.PB_PRECOND_LEARNED, nn=net.handle) if net else {}
    opts = pb.solve_opts(tol=args.tol, precision=pb.PB_MIXED, **(learned_kw if args.step_solve == "learned" else {}))
    log(f"workload {args.workload}: atoms={n_atoms} grid={grid.nx}x{grid.ny}x{grid.nz} band nodes={n}; "
        f"step solve {args.step_solve}")

    def step():
        pb.pb_build_levelset(ctx, at, prm, grid, phi)
        pb.pb_narrowband_compact(ctx, grid, phi, prm, band)
        _, st = pb.pb_ibim_solve(ctx, band, at, prm, opts, p)
        en = pb.pb_solvation_energy(ctx, band, at, prm, p)
        return st, en

    for w in range(args.warmup):
        st, en = step()
        log(f"warmup {w}: iters={st.iters} outer={st.outer} relres={st.true_relres:.2e} fallback={st.fallback_used}")
    torch.cuda.synchronize()
    ctx.set_timing(2)  # events around the far-field launches only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs, fallbacks = 0.0, 0
    for s in range(args.steps):
        st, en = step()
        pairs += st.pairs
        fallbacks += st.fallback_used
        log(f"step {s}: iters={st.iters} outer={st.outer} fp64_mv={st.matvecs_fp64} mixed_mv={st.matvecs_mixed} "
            f"relres={st.true_relres:.2e} fallback={st.fallback_used} G_pol={en.g_pol_kcal:.3f} kcal/mol")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    f32_ms, f32_n = ctx.kernel_time("p2p_f32")
    f64_ms, f64_n = ctx.kernel_time("p2p_f64")
    ctx.set_timing(1)  # the near-field product, timed outside the timed region
    for _ in range(3):
        pb.pb_ibim_matvec(ctx, band, prm, p, pb.PB_MIXED)
    near_ms, near_n = ctx.kernel_time("near_f64")
    ctx.set_timing(0)
    value = pairs / elapsed
    step_stats = {"iters": st.iters, "outer": st.outer, "matvecs_mixed": st.matvecs_mixed,
                  "matvecs_fp64": st.matvecs_fp64, "true_relres": st.true_relres, "fallbacks": fallbacks,
                  "g_pol_kcal": en.g_pol_kcal, "area": en.area, "pairs_per_step": pairs / max(args.steps, 1)}

    per_launch_s = f32_ms * 1e-3 / max(f32_n, 1)
    pairs_launch = float(n) * float(n)
    achieved = FLOP_PER_PAIR * pairs_launch / per_launch_s if f32_n else 0.0
    cfg = ctx.far_kernel(n)
    kname = "k_p2p_f32_sym" if cfg == 4 else "k_p2p_f32<%d, %d>" % ((256, 1), (512, 1), (256, 2), (512, 2))[cfg]
    kfile = "k_p2p_f32_sym" if cfg == 4 else "k_p2p_f32"
    roofline = {"kernel": kname, "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                "traffic": measured_traffic(kfile, args.workload),
                "basis": f"algorithmic: {FLOP_PER_PAIR} FP32 FLOP (FMA = 2) per ordered pair-interaction of the "
                         "dense definition x n^2 per launch / HIP-event launch time; the kernel executes fewer "
                         "(see executed)",
                "executed": executed_counts(kfile, args.workload, pairs_launch, per_launch_s) if f32_n else None,
                "avg_launch_ms": per_launch_s * 1e3, "launches": f32_n,
                "pairs_per_s": pairs_launch / per_launch_s if f32_n else 0.0,
                "p2p_f64_avg_ms": f64_ms / max(f64_n, 1), "near_f64_avg_ms": near_ms / max(near_n, 1)}

    ttsol = None
    legs = [] if args.no_compare else [x for x in args.legs.split(",") if x]
    if args.no_tree:
        legs = [x for x in legs if "tree" not in x]
    if legs:
        ttsol = {}
        # (name in the record, precision, learned?): FP64 GMRES, mixed GMRES-IR, and the treecode
        # far field as the inner operator of the refinement (the exact FP64 residual stays outside).
        # The FP64, mixed and learned solves run warm from the timed steps (same operator kernels
        # and workspace); the treecode legs first build their plan in a solve to 1e-2.
        table = {"fp64": ("fp64", pb.PB_FP64, False), "mixed": ("mixed", pb.PB_MIXED, False),
                 "learned": ("learned_mixed", pb.PB_MIXED, True), "tree": ("tree", pb.PB_TREE, False),
                 "learned_tree": ("learned_tree", pb.PB_TREE, True)}
        for leg in legs:
            name, prec, learned = table[leg]
            if learned and net is None:
                ttsol[name + "_s"] = None
                continue
            o = pb.solve_opts(tol=args.tol, precision=prec, **(learned_kw if learned else {}))
            q = torch.zeros_like(p)
            warm = prec == pb.PB_TREE
            log(f"time to {args.tol:g}: {name} solve" + (" (after a warm-up to 1e-2)" if warm else ""))
            t, st = timed_solve(ctx, band, at, prm, o, q, warm=warm, warm_tol=1e-2)
            ttsol[name + "_s"] = t
            ttsol[name + "_iters"] = st.iters
            ttsol[name + "_outer"] = st.outer
            ttsol[name + "_relres"] = st.true_relres
            ttsol[name + "_g_pol_kcal"] = pb.pb_solvation_energy(ctx, band, at, prm, q).g_pol_kcal
            if learned:
                ttsol[name + "_fallback"] = st.fallback_used
            log(f"time to {args.tol:g}: {name} {t:.3f} s, {st.iters} iterations, {st.outer} outer steps")
        if net is not None:
            ttsol["network"] = rec
        if ttsol.get("fp64_s"):
            for name in ("mixed", "learned_mixed", "tree", "learned_tree"):
                if ttsol.get(name + "_s"):
                    ttsol[f"speedup_{name}_vs_fp64"] = ttsol["fp64_s"] / ttsol[name + "_s"]
                    ttsol[f"energy_rel_diff_{name}_vs_fp64"] = abs(ttsol[name + "_g_pol_kcal"] /
                                                                  ttsol["fp64_g_pol_kcal"] - 1)
        if ttsol.get("mixed_s") and ttsol.get("learned_mixed_s"):
            ttsol["speedup_learned_mixed_vs_mixed"] = ttsol["mixed_s"] / ttsol["learned_mixed_s"]
        if any("tree" in x for x in legs):
            # the treecode far field as it runs inside a solve (one more plain treecode solve,
            # events around the far-field launches only); isolated applications would each
            # rebuild the plan and start on an idle, clocked-down GPU
            ctx.set_timing(2)
            q = torch.zeros_like(p)
            pb.pb_ibim_solve(ctx, band, at, prm, pb.solve_opts(tol=args.tol, precision=pb.PB_TREE), q)
            ms1, c1 = ctx.kernel_time("tree_f32")
            msf, cf = ctx.kernel_time("tree_fine_f32")
            ctx.set_timing(0)
            info = ctx.tree_info()
            far_ms = ms1 / max(c1, 1)
            # algorithmic work: 61 FLOP per direct pair (the dense definition), 36 per
            # target-proxy interaction; the far-field kernels are bound by the FP32 VALUs
            flops = 61.0 * info["direct_pairs"] + 36.0 * info["proxy_interactions"]
            ttsol["tree_operator"] = dict(
                degree=prm.tree_degree, theta=prm.tree_theta, far_ms=far_ms, applications=c1,
                fine_far_ms=msf / cf if cf else None, fine_applications=cf,
                algorithmic_tflops=flops / (far_ms * 1e-3) / 1e12 if far_ms > 0 else None,
                dense_equivalent_pairs_per_s=float(n) * n / (far_ms * 1e-3) if far_ms > 0 else None,
                mean_batch=n / max(info["batches"], 1), **info)

    heldout = None
    if not args.no_compare and not args.no_heldout and net is not None:
        # the learned-preconditioner configuration: a held-out 5000-atom molecule at h = 0.5
        log("held-out 5000-atom globule (h = 0.5): fp64, mixed, learned mixed, learned treecode")
        heldout = heldout_rows(ctx, net, [WORKLOADS["heldout5000"][1]], args.tol)[0]
        heldout["network"] = rec

    batch = None
    if not args.no_compare and not args.no_batch:
        log("batch of 64 molecules (h = 0.5): one plain and one learned batched solve")
        batch = batch_leg(net, rec, args.tol)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        nodes = band.table()
        oprm = oracle.params(h)
        x = np.random.default_rng(0).normal(size=2 * n)
        t1 = time.perf_counter()
        oracle.matvec_rows(nodes, oprm, x, np.arange(min(n, 256)))  # load, warm, and size the sample
        per_row = (time.perf_counter() - t1) / min(n, 256)
        if per_row * n <= 10.0:  # whole operator applications, about 10 s of them
            reps, t_cpu = 0, 0.0
            while t_cpu < 10.0 and reps < 8:
                t1 = time.perf_counter()
                oracle.matvec(nodes, oprm, x)
                t_cpu += time.perf_counter() - t1
                reps += 1
            pairs_cpu = reps * float(n) * float(n)
            sample = f"{reps} full FP64 operator applications (matvec) on the same {n}-node band, {t_cpu:.1f} s"
        else:  # large bands: random operator rows against every source, about 10 s
            rows = np.sort(np.random.default_rng(1).choice(n, max(64, int(10.0 / per_row)), replace=False))
            t1 = time.perf_counter()
            oracle.matvec_rows(nodes, oprm, x, rows)
            t_cpu = time.perf_counter() - t1
            pairs_cpu = len(rows) * float(n)
            sample = (f"{len(rows)} random operator rows x {n} sources of the same band (FP64 oracle), "
                      f"{t_cpu:.1f} s")
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": pairs_cpu / t_cpu, "unit": "pair-interactions/s", "cores": cores,
               "kind": "oracle", "sample": sample,
               "cpu_model": cpu_model(), "one_thread": one_thread_rate(oracle, nodes, oprm, x, cores)}

    solve_desc = ("mixed GMRES-IR with the learned x0 and right preconditioner" if args.step_solve == "learned"
                  else "mixed GMRES-IR")
    out = {
        "metric": METRIC, "value": value, "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "accumulate": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n_atoms}-atom synthetic globule (seed {seed}), SES probe 1.4 A, "
                               f"h={h} A, eps=2h, tau=h; level set + band + {solve_desc} to {args.tol:g} + energy",
                   "band_nodes": n, "grid": [grid.nx, grid.ny, grid.nz], "parallelism": "single GPU"},
        "roofline": roofline, "step": step_stats, "time_to_tol": ttsol, "heldout_c5": heldout, "batch_c4": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
