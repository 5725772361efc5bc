"""Seeded synthetic molecules, the inputs for both the GPU library and the oracle.

This module holds none of the method's arithmetic: it only draws atoms (centre,
radius, charge). They stand in for the PDB/PQR protein files of the paper's
experiments, which are not available here.

Recipe (globule):
  * centres by random sequential addition, uniform in an ellipsoid with semi-axes
    (14, 12, 10)·(n/500)^{1/3} Å, minimum centre distance 2.0 Å (cell-list check);
    after 1000·n rejected draws the distance is scaled by 0.95;
  * radii uniform from {1.2, 1.5, 1.7, 1.8} Å;
  * charges q ~ N(0, 0.35²) e, then shifted by (Q − Σq)/n so the net charge is an
    integer Q drawn uniformly from {−3, …, 3}.
Random numbers come from numpy's PCG64 generator seeded with the given seed.
"""
from __future__ import annotations

import math

import numpy as np

RADII = (1.2, 1.5, 1.7, 1.8)


def globule(n: int, seed: int, axes=(14.0, 12.0, 10.0), d_min: float = 2.0) -> np.ndarray:
    """n atoms as an (n, 5) float64 array of (x, y, z, r, q)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = (n / 500.0) ** (1.0 / 3.0)
    ax = np.array(axes, dtype=np.float64) * s
    cell = d_min
    grid: dict[tuple[int, int, int], list[int]] = {}
    pts = np.zeros((n, 3))
    count, rejects = 0, 0
    while count < n:
        p = (rng.random(3) * 2.0 - 1.0) * ax
        if float(np.sum((p / ax) ** 2)) > 1.0:
            continue
        key = tuple(int(math.floor(c / cell)) for c in p)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for q in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if float(np.sum((pts[q] - p) ** 2)) < d_min * d_min:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            rejects += 1
            if rejects > 1000 * n:
                d_min *= 0.95
                rejects = 0
            continue
        pts[count] = p
        grid.setdefault(key, []).append(count)
        count += 1
    radii = rng.choice(np.array(RADII), size=n)
    q = rng.normal(0.0, 0.35, size=n)
    Q = int(rng.integers(-3, 4))
    q = q + (Q - q.sum()) / n
    return np.column_stack([pts, radii, q])


def born_ion(radius: float = 2.0, charge: float = 1.0, centre=(0.0123, 0.0456, 0.0789)) -> np.ndarray:
    """One charged sphere; the default centre is off the lattice to avoid symmetric ties."""
    return np.array([[centre[0], centre[1], centre[2], radius, charge]], dtype=np.float64)


def batch_sizes(n_mol: int = 64, seed0: int = 64000, lo: int = 50, hi: int = 2000) -> list[int]:
    """Atom counts log-uniform over [lo, hi], one seeded draw per molecule."""
    out = []
    for m in range(n_mol):
        rng = np.random.Generator(np.random.PCG64(seed0 + m))
        out.append(int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))))
    return out


def batch(n_mol: int = 64, seed0: int = 64000, lo: int = 50, hi: int = 2000) -> list[np.ndarray]:
    """Molecules of the batched workload: globule(n_m, seed0 + m)."""
    return [globule(n, seed0 + m) for m, n in enumerate(batch_sizes(n_mol, seed0, lo, hi))]


def shell(r_shell: float = 6.0, r_atom: float = 1.6, spacing: float = 2.2, seed: int = 7) -> np.ndarray:
    """Atoms tiling a closed spherical shell around an empty void (a cavity test case)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = max(12, int(4.0 * math.pi * r_shell * r_shell / (spacing * spacing)))
    k = np.arange(n) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / n)
    theta = math.pi * (1.0 + 5.0 ** 0.5) * k
    pts = r_shell * np.column_stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)])
    q = rng.normal(0.0, 0.35, size=n)
    return np.column_stack([pts, np.full(n, r_atom), q])
