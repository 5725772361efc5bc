"""PQR files: atoms with charges and radii, the input the paper's experiments start from
(section "Numerical experiments": proteins converted with their CHARMM charges and radii).

A PQR record is a PDB ATOM/HETATM line whose last five whitespace-separated fields are
x, y, z (Å), charge (e) and radius (Å); the chain identifier may be absent, so the fields
are counted from the end of the line. Other records (REMARK, TER, END, …) are skipped.
Atoms come back as an (n, 5) float64 array of (x, y, z, radius, charge), the layout every
entry point of the library takes.
"""
from __future__ import annotations

import numpy as np


def read_pqr(path: str) -> np.ndarray:
    rows = []
    with open(path) as f:
        for lineno, line in enumerate(f, 1):
            if not (line.startswith("ATOM") or line.startswith("HETATM")):
                continue
            fields = line.split()
            if len(fields) < 8:
                raise ValueError(f"{path}:{lineno}: a PQR atom record needs x y z charge radius")
            try:
                x, y, z, q, r = (float(v) for v in fields[-5:])
            except ValueError as e:
                raise ValueError(f"{path}:{lineno}: {e}") from None
            if not (r > 0.0) or not np.isfinite([x, y, z, q, r]).all():
                raise ValueError(f"{path}:{lineno}: radius must be positive and every value finite")
            rows.append((x, y, z, r, q))
    if not rows:
        raise ValueError(f"{path}: no ATOM/HETATM records")
    return np.array(rows, dtype=np.float64)


def write_pqr(path: str, atoms: np.ndarray, name: str = "X", residue: str = "MOL") -> None:
    """Writes (x, y, z, radius, charge) rows as PQR ATOM records (one residue per atom)."""
    atoms = np.asarray(atoms, dtype=np.float64)
    with open(path, "w") as f:
        for i, (x, y, z, r, q) in enumerate(atoms, 1):
            f.write(f"ATOM  {i:5d} {name:<4s} {residue:>3s} A{i % 10000:4d}    "
                    f"{x:8.3f}{y:8.3f}{z:8.3f} {q:7.4f} {r:6.4f}\n")
        f.write("END\n")
