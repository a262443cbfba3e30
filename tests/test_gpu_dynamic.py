"""GPU parity of the dynamic-group kernel (coalesced_threads, match_any /
match_all, the six reduce_*_sync, warp-aggregated append) against the
oracle on the same seeded inputs: per-element outputs and per-warp records
bit for bit; the appended members checked for what is unique (the set,
the count, each warp's run in rank order), since the order of the warps'
runs is the order their appends happen to take."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs
from runs_check import runs_partition

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def runs_valid(filt, x, D):
    """The appended members of every 32-lane warp form one run in rank
    order, the runs disjoint and together covering filt."""
    members = (x.view(np.uint32) & 1023) < D
    assert filt.size == int(members.sum())
    assert np.array_equal(np.sort(filt), np.sort(x[members]))
    cnt = members.reshape(-1, 32).sum(1)
    ok, why = runs_partition(filt, x[members], cnt)
    assert ok, why


@pytest.mark.parametrize("D", (0, 1, 102, 512, 922, 1024))
@pytest.mark.parametrize("n", (32, 32 * 513, 32 * 16384 + 32 * 77))
def test_dynamic_matches_oracle(dev, oracle_mod, D, n):
    torch, cox = dev
    print("dynamic D", D, "n", n, flush=True)
    x = inputs.masked_input(n)
    mm, rk, rec, filt, cnt = cox.warp_dynamic(torch.from_numpy(x).cuda(), D)
    omm, ork, orec, ofilt, ocnt = oracle_mod.warp_dynamic(x, D)
    assert np.array_equal(mm.cpu().numpy().view(np.uint32), omm)
    assert np.array_equal(rk.cpu().numpy().view(np.uint32), ork)
    assert np.array_equal(rec.cpu().numpy().view(np.uint32), orec)
    c = int(cnt.cpu()[0])
    assert c == ocnt
    runs_valid(filt.cpu().numpy()[:c], x, D)


def test_dynamic_all_keys_equal_and_repeat(dev, oracle_mod):
    """Every member holding the same key (match_all returns the mask);
    two calls in a row on the same outputs (the counter restarts)."""
    torch, cox = dev
    x = (np.arange(32 * 4096, dtype=np.int64) % 1024 | (5 << 10)).astype(np.int32)
    outs = cox.warp_dynamic(torch.from_numpy(x).cuda(), 512)
    for _ in range(2):
        mm, rk, rec, filt, cnt = cox.warp_dynamic(torch.from_numpy(x).cuda(), 512, *outs)
        omm, ork, orec, ofilt, ocnt = oracle_mod.warp_dynamic(x, 512)
        assert np.array_equal(rec.cpu().numpy().view(np.uint32), orec)
        assert np.array_equal(mm.cpu().numpy().view(np.uint32), omm)
        assert int(cnt.cpu()[0]) == ocnt
        runs_valid(filt.cpu().numpy()[:ocnt], x, 512)
