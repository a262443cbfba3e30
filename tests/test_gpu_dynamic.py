"""GPU parity of the dynamic-group kernel (coalesced_threads, match_any /
match_all, the six reduce_*_sync, warp-aggregated append) against the
oracle on the same seeded inputs: per-element outputs and per-warp records
bit for bit; the appended members checked for what is unique (the set,
the count, each warp's run in rank order), since the order of the warps'
runs is the order their appends happen to take."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def runs_valid(filt, x, D):
    """filt holds every warp's members as one run in rank order, the runs
    disjoint and together covering filt: walking filt from the start, each
    position begins the run of a warp not yet used whose first member has
    that value and whose whole run matches there; the walk must use every
    warp with members exactly once and end at the end of filt."""
    members = (x.view(np.uint32) & 1023) < D
    assert filt.size == int(members.sum())
    assert np.array_equal(np.sort(filt), np.sort(x[members]))
    ps = members.reshape(-1, 32)
    cnt = ps.sum(1)
    allv = x[members]  # the runs, concatenated in warp order
    start = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    warps = np.nonzero(cnt)[0]
    cand = {}
    for w, v in zip(warps.tolist(), allv[start[warps]].tolist()):
        cand.setdefault(v, []).append(w)
    total, p = filt.size, 0
    while p < total:
        lst = cand.get(int(filt[p]))
        assert lst, f"position {p} starts no warp's run"
        for i, w in enumerate(lst):
            c = int(cnt[w])
            if p + c <= total and np.array_equal(filt[p:p + c], allv[start[w]:start[w] + c]):
                lst.pop(i)
                p += c
                break
        else:
            raise AssertionError(f"no unused warp's run matches at position {p}")
    assert p == total
    assert not any(cand.values()), "some warps' runs are missing"


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
