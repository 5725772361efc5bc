"""GPU: the size protocol of pb_build_levelset (include/pb.h), called through the C-ABI.

  * phi = NULL is a size query: *needed = nx·ny·nz and no device work.
  * A buffer shorter than the grid is refused with PB_ECAPACITY before any launch: *needed
    is set and every entry of the buffer keeps its sentinel value.
  * A buffer of exactly the grid's size, or larger, is filled with the same φ; entries past
    the grid are left untouched.
  * Grids the level set cannot take (an axis over 4096 nodes) are refused with PB_EINVAL.
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


def _call(pbm, ctx, at, prm, grid, phi, cap, needed):
    ptr = C.c_void_p(phi.data_ptr()) if phi is not None else None
    return pbm.lib.pb_build_levelset(ctx.handle, C.c_void_p(at.data_ptr()) if at is not None else None,
                                     at.shape[0] if at is not None else 0, C.byref(prm), C.byref(grid), ptr, cap,
                                     C.byref(needed) if needed is not None else None)


def test_levelset_size_query_and_short_buffer(pbm):
    import torch

    say("case: pb_build_levelset size protocol, globule 40 atoms seed 9 h=0.5 SES")
    ctx = pbm.Context(0)
    atoms = synth.globule(40, 9)
    prm = pbm.params(0.5, ls_mode=pbm.PB_LS_SES)
    grid = pbm.pb_grid_for_atoms(atoms, prm)
    count = grid.nx * grid.ny * grid.nz
    at = torch.tensor(atoms, dtype=torch.float64, device="cuda")
    need = C.c_size_t(0)
    assert _call(pbm, ctx, None, prm, grid, None, 0, need) == pbm.PB_OK
    assert need.value == count
    # one element short: refused, nothing written
    short = torch.full((count - 1,), 7.25, dtype=torch.float64, device="cuda")
    need = C.c_size_t(0)
    assert _call(pbm, ctx, at, prm, grid, short, short.numel(), need) == pbm.PB_ECAPACITY
    assert need.value == count
    assert "needs" in pbm.lib.pb_last_error(ctx.handle).decode()
    torch.cuda.synchronize()
    assert bool((short == 7.25).all())
    # exact and oversize buffers: the same φ, the tail untouched
    exact = pbm.pb_build_levelset(ctx, at, prm, grid)
    assert exact.numel() == count
    big = torch.full((count + 100,), -3.5, dtype=torch.float64, device="cuda")
    assert _call(pbm, ctx, at, prm, grid, big, big.numel(), None) == pbm.PB_OK
    torch.cuda.synchronize()
    assert torch.equal(big[:count], exact)
    assert bool((big[count:] == -3.5).all())
    # the binding passes the tensor's own size
    with pytest.raises(pbm.PBError) as e:
        pbm.pb_build_levelset(ctx, at, prm, grid, short)
    assert e.value.status == pbm.PB_ECAPACITY
    # an axis the level set cannot take
    g2 = pbm.pb_grid()
    g2.nx, g2.ny, g2.nz, g2.h = 4097, 8, 8, prm.h
    assert _call(pbm, ctx, None, prm, g2, None, 0, C.c_size_t(0)) == pbm.PB_EINVAL
    ctx.close()
