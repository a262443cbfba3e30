"""CPU checks of the run-partition helper used by the append tests."""
import numpy as np

from runs_check import runs_partition


def _case():
    # warp 0: [5], warp 1: [5, 7], warp 2: [], warp 3: [7, 9, 9]
    allv = np.array([5, 5, 7, 7, 9, 9], np.int32)
    cnt = np.array([1, 2, 0, 3])
    return allv, cnt


def test_accepts_every_order_of_runs_including_alike_starts():
    allv, cnt = _case()
    runs = {0: [5], 1: [5, 7], 3: [7, 9, 9]}
    import itertools

    for order in itertools.permutations([0, 1, 3]):
        filt = np.array(sum((runs[w] for w in order), []), np.int32)
        ok, why = runs_partition(filt, allv, cnt)
        assert ok, (order, why)


def test_rejects_split_or_reordered_runs():
    allv, cnt = _case()
    for bad in ([5, 5, 7, 9, 7, 9], [7, 5, 5, 7, 9, 9], [5, 7, 5, 9, 9, 7], [5, 5, 7, 7, 9]):
        ok, _ = runs_partition(np.array(bad, np.int32), allv, cnt)
        assert not ok, bad


def test_appends_of_short_runs_with_repeated_values():
    """Sixteen thousand short runs with values drawn as the append tests'
    members are (about 2e5 distinct values, so hundreds of warps share a
    first member, and one-member runs are prefixes of longer ones), in a
    random order: accepted; the same output with one member moved out of
    its run: rejected."""
    rng = np.random.default_rng(3)
    cnt = rng.binomial(32, 0.1, size=16384)
    allv = rng.integers(0, 200_000, size=int(cnt.sum())).astype(np.int32)
    start = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    order = rng.permutation(np.nonzero(cnt)[0])
    filt = np.concatenate([allv[start[w]:start[w] + cnt[w]] for w in order])
    assert runs_partition(filt, allv, cnt)[0]
    # move one member of a three-member run to the end of the output
    w3 = next(w for w in order if cnt[w] == 3)
    pos = sum(int(cnt[w]) for w in order[:list(order).index(w3)])
    bad = np.concatenate([filt[:pos + 1], filt[pos + 2:], filt[pos + 1:pos + 2]])
    assert not runs_partition(bad, allv, cnt)[0]
