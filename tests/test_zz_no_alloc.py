"""GPU: pb_solvation_energy_noalloc (include/pb.h), the entry point for callers that cannot
allocate device memory, against pb_solvation_energy through the C-ABI.

Two calls in a row on one context, the second with a smaller molecule (fewer atoms, a
smaller band), each with the scratch array (psi_rxn = NULL) and with a caller's ψ_rxn array:
G_pol, G_pol in kcal/mol and the area equal pb_solvation_energy's bit for bit, and so does
ψ_rxn. A fresh context's calls leave the device's free memory unchanged; more atoms than the
scratch array holds are refused with PB_EINVAL unless the caller passes ψ_rxn.
"""
import ctypes as C
import sys

import numpy as np
import pytest

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


def _molecule(pbm, ctx, atoms, h):
    import torch

    prm = pbm.params(h, ls_mode=pbm.PB_LS_SES)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    phi = pbm.pb_build_levelset(ctx, at, prm, grid)
    band = pbm.pb_narrowband_compact(ctx, grid, phi, prm)
    p, st = pbm.pb_ibim_solve(ctx, band, at, prm, pbm.solve_opts(tol=1e-8, precision=pbm.PB_MIXED))
    assert st.converged
    return prm, at, band, p


def test_noalloc_energy_matches_and_allocates_nothing(pbm):
    import torch

    ctx = pbm.Context(0)
    mols = []
    for na, seed, h in ((60, 31, 0.5), (14, 32, 0.5)):
        say(f"case: noalloc energy, globule {na} atoms seed {seed} h={h}")
        mols.append(_molecule(pbm, ctx, synth.globule(na, seed), h))
    assert mols[1][2].n < mols[0][2].n and mols[1][1].shape[0] < mols[0][1].shape[0]
    # the allocating entry point on the same inputs (this also loads the kernels)
    refs = []
    for prm, at, band, p in mols:
        psi_ref = torch.zeros(at.shape[0], dtype=torch.float64, device="cuda")
        ref = pbm.pb_solvation_energy(ctx, band, at, prm, p, psi_ref)
        refs.append((np.array([ref.g_pol, ref.g_pol_kcal, ref.area]), psi_ref.cpu().numpy()))
    # a fresh context whose calls must not change the device's free memory
    ctx2 = pbm.Context(0)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    psi_mine = torch.zeros(60, dtype=torch.float64, device="cuda")
    out.fill_(np.nan)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (prm, at, band, p), (want, psi_ref) in zip(mols, refs):
        for use_psi in (False, True):
            out.fill_(np.nan)
            psi = psi_mine[: at.shape[0]] if use_psi else None
            pbm.pb_solvation_energy_noalloc(ctx2, band, at, prm, p, out, psi)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            say(f"  n={band.n} atoms={at.shape[0]} psi={'caller' if use_psi else 'scratch'}: {got} vs {want}")
            assert np.array_equal(got, want)
            if use_psi:
                assert np.array_equal(psi.cpu().numpy(), psi_ref)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"  free device memory before {free0} after {free1}")
    assert free1 == free0
    # beyond the scratch array: refused unless the caller passes ψ_rxn
    prm, at, band, p = mols[1]
    big = torch.zeros((131073, 5), dtype=torch.float64, device="cuda")
    st = pbm.lib.pb_solvation_energy_noalloc(ctx2.handle, C.byref(band.struct()), C.c_void_p(big.data_ptr()), 131073,
                                             C.byref(prm), C.c_void_p(p.data_ptr()), C.c_void_p(out.data_ptr()), None)
    assert st == pbm.PB_EINVAL
    assert "scratch" in pbm.lib.pb_last_error(ctx2.handle).decode()
    ctx2.close()
    ctx.close()
