"""lbm_nn_fields_noalloc, the allocation-free variant of lbm_nn_fields (scratch in the library's fixed
device array): through the C ABI it returns exactly what the allocating entry point returns, on two
calls in a row (the second smaller, so that it runs over the scratch the first one left), and it
rejects lattices beyond its scratch before any device work."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(nx, ny, seed, nan_sites=0):
    import torch
    rng = np.random.default_rng(seed)
    pred = rng.standard_normal((ny * nx, 8)).astype(np.float32)
    if nan_sites:
        pred[rng.choice(ny * nx, nan_sites, replace=False), 1] = np.nan
    solid = (rng.random((ny, nx)) < 0.3).astype(np.uint8)
    return torch.from_numpy(pred).cuda(), torch.from_numpy(solid.reshape(-1)).cuda()


def test_noalloc_fields_equal_the_allocating_entry_point():
    import torch
    from paper_2012_14707_amd import lbm
    torch.cuda.set_device(0)
    cases = [(256, 256, 4, True, 0, 11), (96, 64, 2, False, 5, 12)]  # second call smaller than the first
    for nx, ny, smooth, periodic, nans, seed in cases:
        _say(f"[no-alloc] {nx}x{ny}, {smooth} smoothing passes, periodic {periodic}, {nans} non-finite sites")
        pred, solid = _inputs(nx, ny, seed, nans)
        outs = {}
        for noalloc in (False, True):
            rho, ux, uy = (torch.full((ny * nx,), -7.0, dtype=torch.float64, device="cuda") for _ in range(3))
            bad = lbm.nn_fields(pred, solid, nx, ny, 2e-3, 5e-4, 1.0, rho, ux, uy, smooth_iters=smooth,
                                periodic=periodic, noalloc=noalloc)
            torch.cuda.synchronize()
            outs[noalloc] = (bad, rho.cpu().numpy(), ux.cpu().numpy(), uy.cpu().numpy())
        a, b = outs[False], outs[True]
        assert a[0] == b[0]
        assert (a[0] > 0) == (nans > 0)
        for x, y in zip(a[1:], b[1:]):
            assert np.array_equal(x, y, equal_nan=True)
        fluid = solid.cpu().numpy() == 0
        assert np.all(b[1][~fluid] == 1.0) and np.all(b[2][~fluid] == 0.0)


def test_noalloc_fields_reject_lattices_beyond_the_scratch():
    import torch
    from paper_2012_14707_amd import lbm
    nx, ny = 1024, 512
    pred = torch.zeros((ny * nx, 8), dtype=torch.float32, device="cuda")
    solid = torch.zeros(ny * nx, dtype=torch.uint8, device="cuda")
    rho, ux, uy = (torch.zeros(ny * nx, dtype=torch.float64, device="cuda") for _ in range(3))
    with pytest.raises(lbm.LbmError) as e:
        lbm.nn_fields(pred, solid, nx, ny, 1.0, 1.0, 1.0, rho, ux, uy, noalloc=True)
    assert e.value.status == -1 and "scratch" in str(e.value)
