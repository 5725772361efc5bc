"""Training driver of the learned initial guess / right preconditioner.

Orchestration only: molecules come from synth, every level set, band, solve, operator
application, forward and backward pass and Adam step runs in the library's HIP kernels
through the C-ABI. A training example is a pair (v, u = A⁻¹v) on one band:
  * (g, p*) — the right-hand side of a molecule and its solution (mixed solve to 1e-8);
  * (A·e, e) — a smooth random field e on the band and its image under the operator
    (one mixed operator application), so the network also sees residual-like inputs.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import pb, synth


def smooth_field(band: pb.Band, rng: np.random.Generator, n_bumps: int = 8) -> torch.Tensor:
    """Sum of Gaussian bumps of random sign over the band's projections, for ψ and for ψ_n."""
    x = torch.stack([band.px[: band.n], band.py[: band.n], band.pz[: band.n]], 1)
    out = []
    for scale in (1.0, 0.02):
        f = torch.zeros(band.n, dtype=torch.float64, device=x.device)
        idx = rng.integers(0, band.n, n_bumps)
        for i in idx:
            c = x[int(i)]
            w = float(rng.uniform(2.0, 8.0))
            f += float(rng.normal()) * torch.exp(-((x - c) ** 2).sum(1) / (w * w))
        out.append(scale * f)
    return torch.cat(out)


def make_example(ctx: pb.Context, n_atoms: int, seed: int, h: float, n_random: int, rng: np.random.Generator,
                 tol: float = 1e-8):
    """One molecule: (prm, band, list of (v, u) pairs)."""
    atoms = synth.globule(n_atoms, seed)
    prm = pb.params(h, ls_mode=pb.PB_LS_SES)
    grid = pb.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pb.pb_build_levelset(ctx, at, prm, grid)
    band = pb.pb_narrowband_compact(ctx, grid, phi, prm)
    g = pb.pb_ibim_rhs(ctx, band, at, prm)
    u, st = pb.pb_ibim_solve(ctx, band, at, prm, pb.solve_opts(tol=tol, precision=pb.PB_MIXED))
    pairs = [(g, u)]
    for _ in range(n_random):
        e = smooth_field(band, rng)
        pairs.append((pb.pb_ibim_matvec(ctx, band, prm, e, pb.PB_MIXED), e))
    return prm, band, pairs


def train(ctx: pb.Context, net: pb.Net, n_mol: int = 2000, lo: int = 200, hi: int = 1500, h: float = 0.5,
          seed0: int = 100000, epochs: int = 2, lr: float = 1e-3, n_random: int = 1, log=None,
          tol: float = 1e-8, h_choices=None) -> dict:
    """Builds the training set (n_mol molecules, atom counts uniform in [lo, hi], seeds
    seed0 + i, grid spacing h or, with h_choices, one of those drawn per molecule) and trains."""
    rng = np.random.default_rng(seed0)
    t0 = time.perf_counter()
    data = []
    for i in range(n_mol):
        na = int(rng.integers(lo, hi + 1))
        hm = float(h_choices[int(rng.integers(len(h_choices)))]) if h_choices else h
        data.append(make_example(ctx, na, seed0 + i, hm, n_random, rng, tol))
        if log and (i + 1) % max(1, n_mol // 10) == 0:
            log(f"training set: {i + 1}/{n_mol} molecules")
    t_data = time.perf_counter() - t0
    t1 = time.perf_counter()
    history = []
    total = epochs * sum(len(pairs) for _, _, pairs in data)
    done = 0
    for ep in range(epochs):
        order = rng.permutation(len(data))
        tot, cnt = 0.0, 0
        for k in order:
            prm, band, pairs = data[k]
            pb.pb_nn_prepare(ctx, band, prm)
            for v, u in pairs:
                step_lr = lr * 0.5 * (1 + math.cos(math.pi * done / max(1, total)))  # cosine decay over all steps
                done += 1
                tot += pb.pb_nn_train_step(ctx, net, band, prm, v, u, step_lr)
                cnt += 1
                if log and cnt % 1000 == 0:
                    log(f"epoch {ep}: {cnt} steps, mean loss so far {tot / cnt:.4f}")
        history.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.4f}")
    return {"molecules": n_mol, "epochs": epochs, "t_data_s": t_data, "t_train_s": time.perf_counter() - t1,
            "loss": history}


def main(argv=None):
    """Trains the network on generated molecules and saves its weights (and a JSON record of
    the run beside them)."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--molecules", type=int, default=2000)
    ap.add_argument("--lo", type=int, default=200)
    ap.add_argument("--hi", type=int, default=1500)
    ap.add_argument("--h", type=float, default=0.5)
    ap.add_argument("--seed0", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-7, help="tolerance of the solves that give the targets")
    ap.add_argument("--net-seed", type=int, default=1)
    ap.add_argument("--n-random", type=int, default=1, help="random-field pairs per molecule besides (g, p*)")
    ap.add_argument("--h-choices", default="", help="comma-separated grid spacings, one drawn per molecule")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    ctx = pb.Context(0)
    net = pb.Net(ctx, seed=args.net_seed)
    info = train(ctx, net, n_mol=args.molecules, lo=args.lo, hi=args.hi, h=args.h, seed0=args.seed0,
                 epochs=args.epochs, lr=args.lr, n_random=args.n_random, log=log, tol=args.tol,
                 h_choices=[float(x) for x in args.h_choices.split(",") if x] or None)
    net.save(args.out)
    info.update({k: getattr(args, k) for k in ("lo", "hi", "h", "seed0", "lr", "tol", "net_seed", "n_random",
                                                 "h_choices")})
    with open(args.out.rsplit(".", 1)[0] + ".json", "w") as f:
        json.dump(info, f, indent=1)
    log(f"saved {args.out}: loss per epoch {info['loss']}, data {info['t_data_s']:.0f} s, "
        f"training {info['t_train_s']:.0f} s")


if __name__ == "__main__":
    main()
