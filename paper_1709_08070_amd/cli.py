"""Solvation energy of a molecule from a PQR file on the GPU:

    python -m paper_1709_08070_amd.cli molecule.pqr [--h 0.5] [--precision mixed|fp64|tree]
        [--learned WEIGHTS] [--tol 1e-6] [--vdw] [--jacobian] [--central] [--curved]

Runs the whole method (level set, band, right-hand side, GMRES, energy) through the C-ABI
and prints one JSON object: band size, iterations, the true relative residual, the
polarization energy (paper units and kcal/mol), the surface area and the wall times.
"""
from __future__ import annotations

import argparse
import json
import time


def run(path: str, h: float = 0.5, precision: str = "mixed", tol: float = 1e-6, learned: str | None = None,
        vdw: bool = False, jacobian: bool = False, central: bool = False, curved: bool = False) -> dict:
    import torch

    from . import pb, pqr

    atoms = pqr.read_pqr(path)
    ctx = pb.Context(0)
    prm = pb.params(h, ls_mode=pb.PB_LS_VDW if vdw else pb.PB_LS_SES,
                    jacobian=pb.PB_JAC_FULL if jacobian else pb.PB_JAC_ONE,
                    grad_scheme=pb.PB_GRAD_CENTRAL if central else pb.PB_GRAD_WENO,
                    reg_avg=pb.PB_AVG_CURVED if curved else pb.PB_AVG_FLAT)
    t0 = time.perf_counter()
    grid = pb.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pb.pb_build_levelset(ctx, at, prm, grid)
    band = pb.pb_narrowband_compact(ctx, grid, phi, prm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prec = {"fp64": pb.PB_FP64, "mixed": pb.PB_MIXED, "tree": pb.PB_TREE}[precision]
    kw = {}
    net = None
    if learned:
        net = pb.Net(ctx, seed=1)
        net.load(learned)
        kw = dict(x0=pb.PB_X0_LEARNED, precond=pb.PB_PRECOND_LEARNED, nn=net.handle)
    q, st = pb.pb_ibim_solve(ctx, band, at, prm, pb.solve_opts(tol=tol, precision=prec, **kw))
    en = pb.pb_solvation_energy(ctx, band, at, prm, q)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"file": path, "atoms": len(atoms), "h": h, "grid": [grid.nx, grid.ny, grid.nz], "band_nodes": band.n,
           "precision": precision, "learned": bool(learned), "iterations": st.iters, "outer_steps": st.outer,
           "converged": bool(st.converged), "true_relres": st.true_relres, "fallback": bool(st.fallback_used),
           "g_pol": en.g_pol, "g_pol_kcal": en.g_pol_kcal, "area": en.area,
           "t_geometry_s": t1 - t0, "t_solve_s": t2 - t1}
    ctx.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("pqr")
    ap.add_argument("--h", type=float, default=0.5)
    ap.add_argument("--precision", choices=("mixed", "fp64", "tree"), default="mixed")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--learned", metavar="WEIGHTS", default=None, help="network weights (.npz) for x0 and preconditioner")
    ap.add_argument("--vdw", action="store_true", help="van der Waals surface instead of the SES")
    ap.add_argument("--jacobian", action="store_true", help="explicit Jacobian in the band weights")
    ap.add_argument("--central", action="store_true", help="central-difference normals instead of the WENO average")
    ap.add_argument("--curved", action="store_true", help="curvature-corrected disc averages")
    a = ap.parse_args(argv)
    print(json.dumps(run(a.pqr, a.h, a.precision, a.tol, a.learned, a.vdw, a.jacobian, a.central, a.curved)))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
