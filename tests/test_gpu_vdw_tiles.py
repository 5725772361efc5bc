"""GPU: the van der Waals distance F(x) = min_k |x − z_k| − r_k (eq. vdW-levelset-fn) of the
tiled kernel against the FP64 oracle, which scans every atom at every node.

The kernel keeps, per tile of 4 × 8 × 8 nodes, only the atoms that can attain the minimum at
one of its nodes (a bound from the tile centre), and scans all atoms when more than 512 would
be kept. A filter that dropped the minimizing atom anywhere would show up as an error of the
order of the atoms' spacing, so the bar is 1e-13 absolute over the whole grid (the same
arithmetic on both sides). Cases: a dense 2000-atom globule on its own grid (h = 0.4), and a
5000-atom globule on a grid padded by 60 Å (h = 1.5), whose far tiles keep about 1000 atoms and
take the full scan.
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


def _vdw_gpu(pbm, atoms, prm, grid):
    import torch

    ctx = pbm.Context(0)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid).cpu().numpy()
    ctx.close()
    return phi


def _kept_per_tile(atoms, origin, h, tiles):
    """Atoms kept by the tile filter (|c − z| ≤ U + 2R + r, U = min |c − z| − r at the tile
    centre c, R the tile's radius) for the given (bi, bj, bk) tiles of 4 × 8 × 8 nodes."""
    R = 0.5 * h * np.sqrt(3.0 ** 2 + 7.0 ** 2 + 7.0 ** 2)
    z, r = atoms[:, :3], atoms[:, 3]
    out = []
    for bi, bj, bk in tiles:
        c = np.asarray(origin) + h * np.array([4 * bi + 1.5, 8 * bj + 3.5, 8 * bk + 3.5])
        d = np.linalg.norm(z - c, axis=1)
        out.append(int(np.sum(d <= (d - r).min() + 2 * R + r)))
    return out


def test_vdw_dense_globule(pbm):
    atoms = synth.globule(2000, 2024)
    h = 0.4
    say(f"case: vdW distance, globule 2000 atoms seed 2024 h={h}, library grid")
    prm = pbm.params(h, ls_mode=pbm.PB_LS_VDW)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    phi = _vdw_gpu(pbm, atoms, prm, grid)
    dims, origin = (grid.nx, grid.ny, grid.nz), tuple(grid.origin)
    ophi = oracle.vdw(dims, origin, h, atoms)
    d = np.max(np.abs(phi - ophi))
    say(f"  grid {dims}: max |Δφ| {d:.3e}, bitwise equal nodes {np.mean(phi == ophi):.6f}")
    assert d <= 1e-13


def test_vdw_far_tiles_scan_every_atom(pbm):
    atoms = synth.globule(5000, 5000)
    h = 1.5
    prm = pbm.params(h, ls_mode=pbm.PB_LS_VDW)
    lo = atoms[:, :3].min(axis=0) - 60.0
    hi = atoms[:, :3].max(axis=0) + 60.0
    grid = pbm.pb_grid()
    grid.nx, grid.ny, grid.nz = (int(np.ceil((hi[c] - lo[c]) / h)) + 1 for c in range(3))
    for c in range(3):
        grid.origin[c] = float(lo[c])
    grid.h = h
    dims, origin = (grid.nx, grid.ny, grid.nz), tuple(grid.origin)
    nt = ((dims[0] + 3) // 4, (dims[1] + 7) // 8, (dims[2] + 7) // 8)
    corners = [(i, j, k) for i in (0, nt[0] - 1) for j in (0, nt[1] - 1) for k in (0, nt[2] - 1)]
    faces = [(nt[0] // 2, nt[1] // 2, 0), (0, nt[1] // 2, nt[2] // 2), (nt[0] // 2, 0, nt[2] // 2)]
    kept = _kept_per_tile(atoms, origin, h, corners + faces)
    say(f"case: vdW distance, globule 5000 atoms seed 5000 h={h}, grid {dims} padded by 60 A; atoms kept "
        f"by the corner and face tiles {kept}")
    assert max(kept) > 512  # the full scan runs for some tiles
    phi = _vdw_gpu(pbm, atoms, prm, grid)
    ophi = oracle.vdw(dims, origin, h, atoms)
    d = np.max(np.abs(phi - ophi))
    say(f"  max |Δφ| {d:.3e}, bitwise equal nodes {np.mean(phi == ophi):.6f}")
    assert d <= 1e-13
