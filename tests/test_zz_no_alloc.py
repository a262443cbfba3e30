"""The allocation-free scan (cox_warp_scan_noalloc, on the library's fixed
device scratch) against cox_warp_scan with a caller workspace and against
the oracle, through the C ABI: bit-exact int32 results on consecutive calls
that reuse the scratch, the second smaller than the first, at the default
schedule and at the smallest one up to the scratch's capacity."""

import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu

CAP = 1 << 20


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def _check_pair(torch, cox, x, cfg, err):
    xg = torch.from_numpy(x).cuda()
    got = cox.warp_scan_noalloc(xg, cfg=cfg, err=err)
    want = cox.warp_scan(xg, cfg=cfg)
    torch.cuda.synchronize()
    assert int(err.cpu()[0]) == 0
    g = got.cpu().numpy()
    assert np.array_equal(g, want.cpu().numpy())
    return g


@pytest.mark.parametrize("sizes", [(3 * 32768 * 9 + 1001, 70001), (1 << 24, (1 << 20) + 5)])
def test_noalloc_scan_matches_workspace_scan_twice(dev, oracle_mod, sizes):
    torch, cox = dev
    k, W = cox.default_cfg(cox.OP_SCAN)[:2]
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for i, n in enumerate(sizes):
        print(f"noalloc scan: call {i}, n={n}, sigma=({k},{W})", flush=True)
        x = inputs.primitive_inputs(n, seed=20 + i)[0]
        g = _check_pair(torch, cox, x, None, err)
        if n <= (1 << 21):
            assert np.array_equal(g, oracle_mod.scan_i32(x, k, W))
        else:
            # wrapping prefix sums: the last element is the sum mod 2^32
            assert int(g[-1]) == int(np.int64(x.astype(np.int64).sum()).astype(np.int32))


def test_noalloc_scan_at_the_scratch_limit(dev, oracle_mod):
    torch, cox = dev
    small = cox.make_cfg(1, 1)
    n_max = ((CAP - 256) // 8 - 1) * 32  # the largest n whose packed look-back words fit
    assert 256 + 8 * (n_max // 32 + 1) <= CAP < 256 + 8 * (n_max // 32 + 2)
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for i, n in enumerate((n_max, 1000)):
        print(f"noalloc scan at the limit: call {i}, n={n}, sigma=(1,1)", flush=True)
        x = inputs.primitive_inputs(n, seed=40 + i)[0]
        g = _check_pair(torch, cox, x, small, err)
        assert np.array_equal(g, oracle_mod.scan_i32(x, 1, 1))
    x = torch.zeros(n_max + 32, dtype=torch.int32, device="cuda")
    with pytest.raises(cox.CoxError) as e:
        cox.warp_scan_noalloc(x, cfg=small)
    assert e.value.code == 5


def test_noalloc_scan_empty_and_tiny(dev):
    torch, cox = dev
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    assert cox.warp_scan_noalloc(e, err=err).numel() == 0
    torch.cuda.synchronize()
    assert int(err.cpu()[0]) == 0
    x = torch.tensor([5, -2, 7], dtype=torch.int32, device="cuda")
    assert cox.warp_scan_noalloc(x).cpu().tolist() == [5, 3, 10]
