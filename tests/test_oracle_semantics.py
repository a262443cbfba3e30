"""Pins of the oracle's warp-function semantics (CPU only).

Each test checks the oracle's builtins against something other than their
own definition: the paper's worked examples (Code 1, Code 4, Code 5), a
textbook algorithm composed from the builtin (Kogge-Stone scan, reduction
tree, butterfly all-reduce) compared with numpy, algebraic properties
(involution, permutation), or the documented out-of-range rules.
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


WIDTHS = (1, 2, 4, 8, 16, 32)


def _rng(seed=1):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- paper examples
def test_code1_all_ones_tree(oracle_mod):
    o = oracle_mod
    g = gold("code1_shfl_down_allones.json")
    val = np.full(32, g["initial_value"], np.int32)
    for off in g["offsets"]:
        val = val + o.warp_shfl(val, o.SHFL_DOWN, off)
    assert val[0] == g["lane0_result"]
    # CUDA's out-of-range rule (own value) makes every lane 32, not 32 - l
    assert np.all(val == 32)
    assert not np.array_equal(val, 32 - np.arange(32))


def test_code4_vote_all(oracle_mod):
    o = oracle_mod
    g = gold("code4_vote_all.json")
    pred = np.arange(256, dtype=np.int32) % 2
    bal, aa = o.warp_vote(pred)
    assert np.all((aa >> 1) & 1 == g["all_result_every_lane"])
    assert np.all(aa & 1 == g["companions"]["any"])
    assert np.all(bal == int(g["companions"]["ballot"], 16))


def test_code5_back_to_back_votes(oracle_mod):
    o = oracle_mod
    g = gold("code5_back_to_back_votes.json")
    a = np.full(32, g["first_operand"], np.int32)
    b = np.full(32, g["second_operand"], np.int32)
    r1, r2 = o.code5(a, b)
    assert np.all(r1 == g["first_all"]) and np.all(r2 == g["second_all"])
    # independent operands: the second vote sees only its own operands
    a2 = np.ones(32, np.int32)
    b2 = np.ones(32, np.int32)
    b2[7] = 0
    r1, r2 = o.code5(a2, b2)
    assert np.all(r1 == 1) and np.all(r2 == 0)
    r1, r2 = o.code5(b2, a2)
    assert np.all(r1 == 0) and np.all(r2 == 1)
    # without the RAW/WAR barriers the checks must refuse to produce values
    with pytest.raises(o.OracleError) as e:
        o.code5(a2, b2, barriers=False)
    assert e.value.code == o.ERR_UB


# ---------------------------------------------------------------- shuffles
@pytest.mark.parametrize("w", WIDTHS)
def test_shfl_up_kogge_stone_is_segmented_cumsum(oracle_mod, w):
    """A Kogge-Stone scan built from shfl_up(., d, w) with the guard
    (l mod w) >= d equals numpy's cumsum restarted every w lanes."""
    o = oracle_mod
    x = _rng(w).integers(-1000, 1000, size=32 * 64, dtype=np.int32)
    r = x.copy()
    lane = np.arange(x.size) % 32
    d = 1
    while d < w:
        t = o.warp_shfl(r, o.SHFL_UP, d, w)
        r = np.where(lane % w >= d, r + t, r).astype(np.int32)
        d *= 2
    ref = np.cumsum(x.reshape(-1, w), axis=1).reshape(-1).astype(np.int32)
    assert np.array_equal(r, ref)


@pytest.mark.parametrize("w", WIDTHS)
def test_shfl_up_down_out_of_range_keep_own(oracle_mod, w):
    """Lanes whose source would leave the width-segment keep their value."""
    o = oracle_mod
    v = np.arange(1000, 1000 + 32 * 4, dtype=np.int32)
    lane = np.arange(v.size) % 32
    for d in range(32):
        up = o.warp_shfl(v, o.SHFL_UP, d, w)
        dn = o.warp_shfl(v, o.SHFL_DOWN, d, w)
        in_up = (lane % w) >= d
        in_dn = (lane % w) + d < w
        assert np.array_equal(up[~in_up], v[~in_up])
        assert np.array_equal(dn[~in_dn], v[~in_dn])
        # in range they move the data by exactly d lanes
        assert np.array_equal(up[in_up], v[np.nonzero(in_up)[0] - d])
        assert np.array_equal(dn[in_dn], v[np.nonzero(in_dn)[0] + d])


@pytest.mark.parametrize("w", WIDTHS[1:])
def test_shfl_down_tree_gives_segment_sum(oracle_mod, w):
    o = oracle_mod
    x = _rng(10 + w).integers(-10**6, 10**6, size=32 * 32, dtype=np.int32)
    r = x.copy()
    off = w // 2
    while off >= 1:
        r = (r + o.warp_shfl(r, o.SHFL_DOWN, off, w)).astype(np.int32)
        off //= 2
    seg = x.reshape(-1, w).sum(axis=1)
    assert np.array_equal(r[::w], seg.astype(np.int32))


@pytest.mark.parametrize("w", WIDTHS[1:])
def test_shfl_xor_butterfly_allreduce(oracle_mod, w):
    o = oracle_mod
    x = _rng(20 + w).integers(-10**6, 10**6, size=32 * 32, dtype=np.int32)
    r = x.copy()
    m = 1
    while m < w:
        r = (r + o.warp_shfl(r, o.SHFL_XOR, m, w)).astype(np.int32)
        m *= 2
    seg = np.repeat(x.reshape(-1, w).sum(axis=1), w).astype(np.int32)
    assert np.array_equal(r, seg)


@pytest.mark.parametrize("w", WIDTHS)
def test_shfl_xor_involution_and_asymmetry(oracle_mod, w):
    o = oracle_mod
    v = np.arange(7, 7 + 32 * 2, dtype=np.int32)
    lane = np.arange(v.size) % 32
    for m in range(32):
        once = o.warp_shfl(v, o.SHFL_XOR, m, w)
        j = lane ^ m
        base = lane & ~(w - 1)
        readable = j < base + w
        # readable partners (own segment or an earlier one) are read,
        # partners in a later segment give the caller's own value
        src = np.where(readable, (np.arange(v.size) & ~31) + j, np.arange(v.size))
        assert np.array_equal(once, v[src])
        if m < w:
            assert np.array_equal(o.warp_shfl(once, o.SHFL_XOR, m, w), v)


def test_shfl_xor_reads_earlier_segment_only():
    """Width 8, mask 8 (PTX ISA shfl.sync bfly rule): segment 0 (lanes 0-7)
    would read lanes 8-15 of a later segment and keeps its values; segment 1
    (lanes 8-15) reads lanes 0-7 of the earlier segment."""
    import oracle as o

    v = np.arange(100, 132, dtype=np.int32)
    r = o.warp_shfl(v, o.SHFL_XOR, 8, 8)
    assert np.array_equal(r[0:8], v[0:8])
    assert np.array_equal(r[8:16], v[0:8])
    assert np.array_equal(r[16:24], v[16:24])
    assert np.array_equal(r[24:32], v[16:24])


@pytest.mark.parametrize("w", WIDTHS)
def test_shfl_idx_permutation_and_broadcast(oracle_mod, w):
    o = oracle_mod
    rng = _rng(30 + w)
    v = rng.integers(-10**9, 10**9, size=32 * 16, dtype=np.int32)
    lane = np.arange(v.size) % 32
    base = (np.arange(v.size) & ~31) + (lane & ~(w - 1))
    # per-lane sources, including out-of-range and negative ones (mod width)
    src = rng.integers(-64, 64, size=v.size, dtype=np.int32)
    r = o.warp_shfl(v, o.SHFL_IDX, argv=src, width=w)
    assert np.array_equal(r, v[base + (src & (w - 1))])
    # a permutation within each segment is undone by its inverse
    perm = np.concatenate([rng.permutation(w) for _ in range(v.size // w)]).astype(np.int32)
    inv = np.empty_like(perm)
    for s in range(v.size // w):
        inv[s * w + perm[s * w:(s + 1) * w]] = np.arange(w)
    back = o.warp_shfl(o.warp_shfl(v, o.SHFL_IDX, argv=perm, width=w), o.SHFL_IDX, argv=inv, width=w)
    assert np.array_equal(back, v)
    # broadcast of the segment's lane 0
    b0 = o.warp_shfl(v, o.SHFL_IDX, 0, w)
    assert np.array_equal(b0, v[base])


def test_masked_shuffle_source_outside_mask_is_undefined(oracle_mod):
    o = oracle_mod
    v = np.arange(32, dtype=np.int32)
    mask = np.array([0x0000FFFF], np.uint32)
    # lanes 0-15 read lane 20, which is not in the mask
    with pytest.raises(o.OracleError) as e:
        o.warp_shfl(v, o.SHFL_IDX, 20, 32, mask=mask)
    assert e.value.code == o.ERR_UB
    # reading a lane inside the mask is fine; lanes outside keep their input
    r = o.warp_shfl(v, o.SHFL_IDX, 3, 32, mask=mask)
    assert np.all(r[:16] == 3) and np.array_equal(r[16:], v[16:])


def test_invalid_shuffle_arguments_rejected(oracle_mod):
    o = oracle_mod
    v = np.zeros(32, np.int32)
    with pytest.raises(o.OracleError):
        o.warp_shfl(v, o.SHFL_DOWN, 32, 32)
    with pytest.raises(o.OracleError):
        o.warp_shfl(v, o.SHFL_XOR, 1, 3)
    with pytest.raises(o.OracleError):
        o.warp_shfl(np.zeros(33, np.int32), o.SHFL_XOR, 1, 32)


# ---------------------------------------------------------------- votes
def test_ballot_popcount_equals_predicate_count(oracle_mod):
    o = oracle_mod
    rng = _rng(40)
    pred = (rng.random(32 * 4096) < rng.random()).astype(np.int32)
    bal, aa = o.warp_vote(pred)
    pc = np.array([bin(int(b)).count("1") for b in bal])
    assert np.array_equal(pc, pred.reshape(-1, 32).sum(axis=1))
    # bit i of the ballot is lane i's predicate
    bits = ((bal[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.int32)
    assert np.array_equal(bits.reshape(-1), pred)
    assert np.array_equal(aa & 1, pred.reshape(-1, 32).any(axis=1).astype(np.int32))
    assert np.array_equal((aa >> 1) & 1, pred.reshape(-1, 32).all(axis=1).astype(np.int32))


def test_masked_votes_exhaustive_on_low_lanes(oracle_mod):
    """Every mask and predicate pattern of lanes 0-3 (lanes 4-31 outside the
    mask hold garbage predicates that must not matter)."""
    o = oracle_mod
    masks, preds = [], []
    rng = _rng(41)
    for m in range(1, 16):
        for p in range(16):
            masks.append(m)
            lanes = np.array([(p >> i) & 1 for i in range(4)] + list(rng.integers(0, 2, 28)))
            preds.append(lanes)
    mask = np.array(masks, np.uint32)
    pred = np.array(preds, np.int32).reshape(-1)
    bal, aa = o.warp_vote(pred, mask)
    for g, (m, p) in enumerate(zip(masks, preds)):
        want = sum(1 << i for i in range(4) if (m >> i) & 1 and p[i])
        assert bal[g] == want
        assert (aa[g] & 1) == int(want != 0)
        assert ((aa[g] >> 1) & 1) == int(want == m)


def test_empty_mask_vote_records_zero(oracle_mod):
    o = oracle_mod
    bal, aa = o.warp_vote(np.ones(32, np.int32), np.zeros(1, np.uint32))
    assert bal[0] == 0 and aa[0] == 0


# ---------------------------------------------------------------- tile-scoped votes
@pytest.mark.parametrize("T", [1, 2, 4, 8, 16, 32])
def test_tile_votes_reassemble_the_warp_vote(oracle_mod, T):
    """Pinned to the warp vote (itself pinned by Code 4): the T-bit ballots
    of a warp's 32/T tiles, each shifted to its tile's first lane, OR to the
    warp's full-mask ballot; any is the tile ballot being nonzero and all
    the tile ballot being every one of its T bits.  At T = 32 the records
    are the warp vote's."""
    o = oracle_mod
    rng = _rng(50 + T)
    pred = (rng.random(32 * 500) < rng.random()).astype(np.int32) * rng.integers(-3, 4, 32 * 500).astype(np.int32)
    pred[: 32 * 4] = np.repeat([0, 1, 0, 1], 32)  # all-false and all-true warps
    tb, ta = o.tile_vote(pred, T)
    wb, wa = o.warp_vote(pred)
    per = 32 // T
    shifted = tb.astype(np.uint64).reshape(-1, per) << (T * np.arange(per, dtype=np.uint64))
    assert np.array_equal(np.bitwise_or.reduce(shifted, axis=1).astype(np.uint32), wb)
    full = (1 << T) - 1
    assert np.all(tb <= full)
    assert np.array_equal(ta & 1, (tb != 0).astype(np.int32))
    assert np.array_equal((ta >> 1) & 1, (tb == full).astype(np.int32))
    if T == 32:
        assert np.array_equal(tb, wb) and np.array_equal(ta, wa)


def test_tile_votes_on_the_code4_predicate(oracle_mod):
    """Code 4's predicate tx % 2 (odd lanes true): every tile of T >= 2
    lanes has ballot 0b1010.. over its T bits, any true and all false;
    tiles of one lane vote their own predicate."""
    o = oracle_mod
    pred = np.arange(256, dtype=np.int32) % 2
    for T in (2, 4, 8, 16, 32):
        tb, ta = o.tile_vote(pred, T)
        assert np.all(tb == 0xAAAAAAAA & ((1 << T) - 1)), T
        assert np.all(ta == 1), T
    tb, ta = o.tile_vote(pred, 1)
    assert np.array_equal(tb, pred.astype(np.uint32)) and np.array_equal(ta, pred * 3)


def test_tile_vote_rejects_bad_tiles(oracle_mod):
    for T in (0, 3, 64):
        with pytest.raises(oracle_mod.OracleError, match="tile_vote"):
            oracle_mod.tile_vote(np.zeros(64, np.int32), T)
    with pytest.raises(oracle_mod.OracleError, match="tile_vote"):
        oracle_mod.tile_vote(np.zeros(33, np.int32), 1)
