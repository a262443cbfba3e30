"""Checks that an append output is a concatenation of per-warp runs.

A warp-aggregated append writes each warp's members as one run (in rank
order) at a place its atomic reservation picks, so only the partition is
unique: the output must split into consecutive runs, each equal to a
different warp's run, using every warp with members.  Two warps' runs can
start alike (a one-member run can be the first member of a longer run), so
the split is searched with backtracking instead of taken greedily.
"""
import numpy as np


def runs_partition(filt, allv, cnt, max_steps=None):
    """filt: the output; allv: every warp's members concatenated in warp
    order; cnt: members per warp.  Returns (ok, reason); a search longer
    than max_steps (default: four steps per warp plus a million) counts as
    a failure."""
    filt = np.asarray(filt)
    cnt = np.asarray(cnt, np.int64)
    total = int(filt.size)
    if total != int(cnt.sum()):
        return False, f"{total} outputs for {int(cnt.sum())} members"
    start = np.concatenate(([0], np.cumsum(cnt)[:-1])).astype(np.int64)
    warps = np.nonzero(cnt)[0]
    cand = {}
    for w, v in zip(warps.tolist(), allv[start[warps]].tolist()):
        cand.setdefault(v, []).append(w)
    used = np.zeros(cnt.size, bool)
    if max_steps is None:
        max_steps = 4 * int(cnt.size) + 1_000_000

    def options(p):
        # unused warps whose run matches at p, one per distinct run (warps
        # with equal runs are interchangeable)
        out, seen = [], set()
        for w in cand.get(int(filt[p]), ()):
            c = int(cnt[w])
            if not used[w] and p + c <= total and np.array_equal(filt[p:p + c], allv[start[w]:start[w] + c]):
                key = allv[start[w]:start[w] + c].tobytes()
                if key not in seen:
                    seen.add(key)
                    out.append(w)
        return out

    if total == 0:
        return True, ""
    stack = [[0, options(0), 0]]  # position, its candidate warps, next candidate
    deepest, steps = 0, 0
    while stack:
        steps += 1
        if steps > max_steps:
            return False, f"search gave up after {max_steps} steps (furthest position {deepest})"
        top = stack[-1]
        p, opts, i = top
        if i > 0:
            used[opts[i - 1]] = False  # the previous choice led nowhere
        if i == len(opts):
            stack.pop()
            continue
        w = opts[i]
        used[w] = True
        top[2] = i + 1
        q = p + int(cnt[w])
        if q == total:
            return True, ""
        deepest = max(deepest, q)
        stack.append([q, options(q), 0])
    return False, f"no split into warp runs (furthest position reached {deepest})"
