"""Pins of the oracle's collapsed kernels (CPU only).

Every kernel is checked against something other than itself: a plain
definition computed another way (numpy reshape/cumsum/sort/boolean mask), a
closed form (sum 1..n, scan of ones), an invariant (ballot popcount equals
the predicate count, sorted permutation, 0-1 principle, the appendix's
execution-count theorem), an independent array-halving formulation of the
fixed FP tree, or the exact sum within an a-priori error bound.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2112_10034_amd import inputs

SIGMAS = [(1, 1), (1, 8), (2, 4), (4, 8), (8, 2), (16, 8), (32, 4), (4, 32)]


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- K-R0
@pytest.mark.parametrize("n", [256, 1000, 4096 + 37, 1 << 16])
def test_block_reduce_matches_reshape_sums(oracle_mod, n):
    x = inputs.block_reduce_input(n)
    bs, wc = oracle_mod.reduce_blocks_i32(x)
    pad = np.zeros(-(-n // 256) * 256, np.int64)
    pad[:n] = x
    assert np.array_equal(bs, pad.reshape(-1, 256).sum(1).astype(np.int32))
    padp = np.zeros(-(-n // 32) * 32, np.int64)
    padp[:n] = x > 0
    assert np.array_equal(wc, padp.reshape(-1, 32).sum(1))


def test_block_reduce_all_ones(oracle_mod):
    bs, wc = oracle_mod.reduce_blocks_i32(np.ones(1 << 12, np.int32))
    assert np.all(bs == 256) and np.all(wc == 32)


def test_appendix_invariant_execution_counts(oracle_mod):
    """Every statement of the input kernel runs once per thread of the block
    (b_size = 256 times), the peeled branch condition is evaluated by every
    thread, and the statements inside the branch run for warp 0 only."""
    o = oracle_mod
    nb = 5
    o.set_threads(1)
    try:
        o.counts_reset()
        o.reduce_blocks_i32(inputs.block_reduce_input(256 * nb))
        c = o.counts()
    finally:
        o.set_threads(8)
    assert c[o.ST_LOAD] == 256 * nb
    assert c[o.ST_SHFL] == 5 * 256 * nb
    assert c[o.ST_VOTE] == 256 * nb
    assert c[o.ST_PEEL] == 256 * nb
    assert c[o.ST_BODY] == 5 * 32 * nb


def test_peeled_branch_must_be_uniform(oracle_mod):
    o = oracle_mod
    x = rng(1).integers(-100, 100, size=32 * 4, dtype=np.int32)
    cond = np.repeat(np.array([1, 0, 1, 0], np.int32), 32)
    out = o.uniform_branch(cond, x)
    sums = x.reshape(-1, 32).sum(1)
    assert out[0] == sums[0] and out[64] == sums[2]
    assert np.array_equal(out[32:64], x[32:64])
    cond[5] = 0  # warp 0 now diverges around its barriers
    with pytest.raises(o.OracleError) as e:
        o.uniform_branch(cond, x)
    assert e.value.code == o.ERR_DIVERGENT


# ---------------------------------------------------------------- K-R int
@pytest.mark.parametrize("k,W", SIGMAS)
def test_int_reduce_plain_definition(oracle_mod, k, W):
    x, _, _ = inputs.primitive_inputs(50_000 + 123)
    part, tot = oracle_mod.reduce(x, k, W)
    S = 32 * W * k
    pad = np.zeros(len(part) * S, np.int64)
    pad[: x.size] = x
    assert np.array_equal(part, pad.reshape(-1, S).sum(1).astype(np.int32))
    assert tot == int(x.astype(np.int64).sum())


def test_int_reduce_closed_form(oracle_mod):
    n = 1 << 18
    x = np.arange(1, n + 1, dtype=np.int32)
    _, tot = oracle_mod.reduce(x, 16, 8)
    assert tot == n * (n + 1) // 2


@pytest.mark.slow
def test_int_reduce_closed_form_full_size_wraps(oracle_mod):
    n = 1 << 28
    x = np.arange(1, n + 1, dtype=np.int32)  # wraps at 2^31 - 1; sum mod 2^32 is 2^27
    _, tot = oracle_mod.reduce(x, 16, 8)
    assert tot % (1 << 32) == 1 << 27


def test_empty_inputs(oracle_mod):
    o = oracle_mod
    e32 = np.zeros(0, np.int32)
    assert o.reduce(e32, 16, 8)[1] == 0
    t = o.reduce(np.zeros(0, np.float32), 16, 8)[1]
    assert t == 0.0 and math.copysign(1.0, t) == -1.0
    assert o.scan_i32(e32, 16, 8).size == 0
    assert o.compact_i32(e32, 16, 8)[1] == 0
    assert o.tile_sort_u32(np.zeros(0, np.uint32)).size == 0


# ---------------------------------------------------------------- K-S
@pytest.mark.parametrize("k,W", SIGMAS)
def test_scan_is_cumsum_mod_2_32(oracle_mod, k, W):
    x, _, _ = inputs.primitive_inputs(70_000 + 77)
    y = oracle_mod.scan_i32(x, k, W)
    assert np.array_equal(y, np.cumsum(x.astype(np.int64)).astype(np.int32))


def test_scan_of_ones_is_index(oracle_mod):
    n = 3 * 4096 + 5
    y = oracle_mod.scan_i32(np.ones(n, np.int32), 16, 8)
    assert np.array_equal(y, np.arange(1, n + 1, dtype=np.int32))


def test_scan_wraps(oracle_mod):
    x = np.full(1 << 14, 1 << 30, np.int32)
    y = oracle_mod.scan_i32(x, 4, 8)
    ref = ((np.arange(1, x.size + 1, dtype=np.int64) << 30) % (1 << 32)).astype(np.uint32).view(np.int32)
    assert np.array_equal(y, ref)


# ---------------------------------------------------------------- K-C
@pytest.mark.parametrize("k,W", SIGMAS)
def test_compaction_plain_definition(oracle_mod, k, W):
    x, _, _ = inputs.primitive_inputs(60_000 + 11)
    out, cnt = oracle_mod.compact_i32(x, k, W)
    ref = x[x > 0]
    assert cnt == ref.size and np.array_equal(out, ref)


@pytest.mark.parametrize("frac", [0.0, 0.01, 0.5, 0.99, 1.0])
def test_compaction_densities(oracle_mod, frac):
    r = rng(int(frac * 100))
    x = np.where(r.random(20_000) < frac, r.integers(1, 100, 20_000), -r.integers(0, 100, 20_000)).astype(np.int32)
    out, cnt = oracle_mod.compact_i32(x, 8, 4)
    assert cnt == int((x > 0).sum()) and np.array_equal(out, x[x > 0])


# ---------------------------------------------------------------- K-T
@pytest.mark.parametrize("n", [32, 32 * 1000, 32 * 1000 + 17])
def test_tile_sort_matches_numpy(oracle_mod, n):
    _, keys, _ = inputs.primitive_inputs(n)
    out = oracle_mod.tile_sort_u32(keys)
    full = n // 32 * 32
    assert np.array_equal(out[:full], np.sort(keys[:full].reshape(-1, 32), axis=1).reshape(-1))
    assert np.array_equal(out[full:], np.sort(keys[full:]))


@pytest.mark.parametrize("G", [2, 4, 8, 16])
def test_tile_sort_zero_one_principle_exhaustive(oracle_mod, G):
    """0-1 principle: a comparator network sorts every input iff it sorts
    every 0/1 input.  All 2^G patterns for groups of G keys."""
    pats = np.array(list(itertools.product([0, 1], repeat=G)), np.uint32)
    keys = pats.reshape(-1)
    if keys.size % 32:
        keys = np.concatenate([keys, np.zeros(32 - keys.size % 32, np.uint32)])
    out = oracle_mod.tile_sort_u32(keys, G)
    got = out[: pats.size].reshape(-1, G)
    assert np.array_equal(got, np.sort(pats, axis=1))


def test_tile_sort_adversarial(oracle_mod):
    o = oracle_mod
    cases = [np.full(32, 7, np.uint32), np.arange(32, dtype=np.uint32)[::-1].copy(),
             np.array([0, 0xFFFFFFFF] * 16, np.uint32), np.array([0x80000000, 0x7FFFFFFF] * 16, np.uint32)]
    for c in cases:
        assert np.array_equal(o.tile_sort_u32(c), np.sort(c))


@pytest.mark.parametrize("G", [2, 32, 64, 256, 1024, 4096])
@pytest.mark.parametrize("n", [1, 63, 5000, 3 * 4096 + 1001])
def test_group_sort_matches_numpy(oracle_mod, G, n):
    g = np.random.default_rng(G + n)
    keys = g.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    keys[::7] = keys[0]  # ties
    out = oracle_mod.group_sort_u32(keys, G)
    for s in range(0, n, G):
        assert np.array_equal(out[s:s + G], np.sort(keys[s:s + G]))
    if G == 32:
        assert np.array_equal(out, oracle_mod.tile_sort_u32(keys))


def test_group_sort_rejects_bad_sizes(oracle_mod):
    for G in (0, 3, 8192):
        with pytest.raises(oracle_mod.OracleError):
            oracle_mod.group_sort_u32(np.zeros(8, np.uint32), G)


@pytest.mark.parametrize("n,kmax", [(32, 4), (32 * 1000, 8), (32 * 1000 + 17, 1 << 32), (31, 2), (1, 5)])
def test_tile_sort_kv_is_the_stable_sort(oracle_mod, n, kmax):
    g = np.random.default_rng(n)
    keys = g.integers(0, kmax, n, dtype=np.uint64).astype(np.uint32)
    vals = g.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    ok, ov = oracle_mod.tile_sort_kv_u32(keys, vals)
    for s in range(0, n, 32):
        order = np.argsort(keys[s:s + 32], kind="stable")
        assert np.array_equal(ok[s:s + 32], keys[s:s + 32][order])
        assert np.array_equal(ov[s:s + 32], vals[s:s + 32][order])
    # the keys agree with the bitonic key-only sort (a different algorithm)
    assert np.array_equal(ok, oracle_mod.tile_sort_u32(keys))


def test_tile_sort_kv_stability_and_edges(oracle_mod):
    o = oracle_mod
    idx = np.arange(64, dtype=np.uint32)
    # all keys equal: the identity permutation
    ok, ov = o.tile_sort_kv_u32(np.full(64, 9, np.uint32), idx)
    assert np.array_equal(ov, idx)
    # reversed keys with values = positions: values reverse within each group
    keys = np.tile(np.arange(32, dtype=np.uint32)[::-1], 2)
    ok, ov = o.tile_sort_kv_u32(keys, idx)
    assert np.array_equal(ov, np.concatenate([idx[:32][::-1], idx[32:][::-1]]))
    # maximal keys in a partial group keep their order; ties at 0 and 2^32-1
    keys = np.array([0xFFFFFFFF, 0, 0xFFFFFFFF, 0, 5], np.uint32)
    ok, ov = o.tile_sort_kv_u32(keys, np.arange(5, dtype=np.uint32))
    assert ok.tolist() == [0, 0, 5, 0xFFFFFFFF, 0xFFFFFFFF] and ov.tolist() == [1, 3, 4, 0, 2]
    assert o.tile_sort_kv_u32(np.zeros(0, np.uint32), np.zeros(0, np.uint32))[0].size == 0


# ---------------------------------------------------------------- K-TR
@pytest.mark.parametrize("T", inputs.TILE_SIZES)
def test_tile_reduce_plain_definition(oracle_mod, T):
    x = inputs.masked_input(32 * 999 + 5)
    out = oracle_mod.tile_reduce_i32(x, T)
    pad = np.zeros(-(-x.size // T) * T, np.int64)
    pad[: x.size] = x
    assert np.array_equal(out, pad.reshape(-1, T).sum(1).astype(np.int32))


# ---------------------------------------------------------------- K-M
def _masked_reference(x, D):
    """The masked workload written directly from its definition, warp by
    warp, with plain Python lists (no exchange arrays, no ballots)."""
    out = np.empty_like(x)
    rec = np.zeros((x.size // 32, 4), np.uint32)
    for g in range(x.size // 32):
        xs = [int(v) for v in x[32 * g:32 * g + 32]]
        act = [l for l in range(32) if (xs[l] & 1023) < D]
        if not act:
            out[32 * g:32 * g + 32] = np.iinfo(np.int32).min
            continue
        m = sum(1 << l for l in act)
        b = sum(1 << l for l in act if xs[l] > 0)
        A = int(any(((xs[l] >> 10) & 31) == 0 for l in act))
        L = int(all(((xs[l] >> 15) & 31) != 0 for l in act))
        for l in range(32):
            out[32 * g + l] = np.iinfo(np.int32).min
        for idx, l in enumerate(act):
            out[32 * g + l] = xs[act[(idx + 1) % len(act)]]
        rec[g] = [m, b, A | (L << 1), xs[act[0]] & 0xFFFFFFFF]
    return out, rec


@pytest.mark.parametrize("D", inputs.MASK_DENSITIES + (0, 1, 1024))
def test_masked_ops_definition(oracle_mod, D):
    x = inputs.masked_input(32 * 300)
    out, rec = oracle_mod.warp_masked(x, D)
    ref_out, ref_rec = _masked_reference(x, D)
    assert np.array_equal(out, ref_out)
    assert np.array_equal(rec, ref_rec)
    pc = np.array([bin(int(m)).count("1") for m in rec[:, 0]])
    assert np.array_equal(pc, (((x.view(np.uint32) & 1023) < D).reshape(-1, 32)).sum(1))
    assert np.all(rec[:, 1] & ~rec[:, 0] == 0)


# ---------------------------------------------------------------- FP trees
def _fmaf_np(a, b, c):
    """Correctly rounded binary32 fused multiply-add, from its definition:
    the product of two binary32 values is exact in binary64; (p + c) is
    formed as s + e exactly (TwoSum in binary64); s is rounded to binary32,
    except where s lies exactly halfway between two binary32 values and
    e != 0, where the exact value is on e's side of the midpoint (s is
    first moved one binary64 ulp towards it)."""
    a, b, c = (np.asarray(v, np.float32).astype(np.float64) for v in (a, b, c))
    p = a * b
    s = p + c
    bb = s - p
    e = (p - (s - bb)) + (c - bb)
    t = s.astype(np.float32)
    tt = t.astype(np.float64)
    lo = np.where(tt > s, np.nextafter(t, np.float32(-np.inf)), t).astype(np.float64)
    hi = np.where(tt > s, t, np.nextafter(t, np.float32(np.inf))).astype(np.float64)
    tie = (s == (lo + hi) / 2) & (e != 0) & (tt != s)
    s2 = np.where(tie, np.nextafter(s, np.where(e > 0, np.inf, -np.inf)), s)
    return s2.astype(np.float32)


def _sigma_tree_np(x, k, W, compensated=False, y=None, V=4):
    """Independent array-halving form of the fixed reduction schedule:
    lane-serial accumulation in (row, vector-slot) order, then the shfl_down
    tree at lane 0 written as recursive halving (lanes l and l + h).
    x (and y for a dot) are binary32 values (bfloat16 inputs widened
    exactly); V is the vector width of the element mapping (4 for 4-byte
    elements, 8 for bfloat16), capped at k.  Sum: s + x, or TwoSum
    compensation; dot: s = fmaf(x, y, s), or Dot2 (TwoProduct, TwoSum,
    c = c + (pe + q)); tails pad x with -0.0 and y with +0.0."""
    T, V = 32 * W, min(k, V)
    R, S = k // V, 32 * W * k
    nch = -(-x.size // S)
    xp = np.full(nch * S, -0.0, np.float32)
    xp[: x.size] = x
    a = xp.reshape(nch, W, R, 32, V)
    if y is not None:
        yp = np.zeros(nch * S, np.float32)
        yp[: y.size] = y
        b = yp.reshape(nch, W, R, 32, V)
    s = np.full((nch, W, 32), -0.0, np.float32)
    c = np.full((nch, W, 32), -0.0, np.float32)

    def two_sum(p, q):
        t = p + q
        bb = t - p
        return t, (p - (t - bb)) + (q - bb)

    for i in range(R):
        for v in range(V):
            xv = a[:, :, i, :, v]
            if y is None:
                if compensated:
                    s, e = two_sum(s, xv)
                    c = c + e
                else:
                    s = s + xv
            else:
                yv = b[:, :, i, :, v]
                if compensated:
                    p = xv * yv
                    pe = (xv.astype(np.float64) * yv.astype(np.float64) - p.astype(np.float64)).astype(np.float32)
                    s, q = two_sum(s, p)
                    c = c + (pe + q)
                else:
                    s = _fmaf_np(xv, yv, s)

    def halve(s, c):
        while s.shape[-1] > 1:
            h = s.shape[-1] // 2
            if compensated:
                t, e = two_sum(s[..., :h], s[..., h:])
                c = (c[..., :h] + c[..., h:]) + e
                s = t
            else:
                s = s[..., :h] + s[..., h:]
        return s[..., 0], c[..., 0]

    ws, wc = halve(s, c)
    ss = np.full((nch, 32), -0.0, np.float32)
    cc = np.full((nch, 32), -0.0, np.float32)
    ss[:, :W] = ws
    cc[:, :W] = wc
    return halve(ss, cc)


def _final_np(vals):
    """Independent form of the FP64 final tree: 256 strided serial sums,
    then recursive halving within each group of 32, then over the 8."""
    m = -(-vals.size // 256) * 256
    p = np.full(m, -0.0)
    p[: vals.size] = vals
    t = np.full(256, -0.0)
    for row in p.reshape(-1, 256):
        t = t + row
    t = t.reshape(8, 32)
    while t.shape[-1] > 1:
        h = t.shape[-1] // 2
        t = t[:, :h] + t[:, h:]
    top = np.full(32, -0.0)
    top[:8] = t[:, 0]
    while top.size > 1:
        top = top[: top.size // 2] + top[top.size // 2:]
    return top[0]


@pytest.mark.parametrize("k,W", SIGMAS)
def test_fp32_reduce_tree_matches_halving_form(oracle_mod, k, W):
    _, _, f = inputs.primitive_inputs(40_000 + 3)
    part, tot = oracle_mod.reduce(f, k, W)
    want, _ = _sigma_tree_np(f, k, W)
    assert np.array_equal(part.view(np.uint32), want.view(np.uint32))
    assert np.float64(tot).view(np.uint64) == np.float64(_final_np(part.astype(np.float64))).view(np.uint64)


@pytest.mark.parametrize("k,W", SIGMAS[:5])
def test_fp32_twosum_tree_matches_halving_form(oracle_mod, k, W):
    f, _ = inputs.precision_inputs(1 << 14, target=1e4)[0], None
    part, tot = oracle_mod.reduce(f, k, W, oracle_mod.TWOSUM)
    ws, wc = _sigma_tree_np(f, k, W, compensated=True)
    assert np.array_equal(part[:, 0].view(np.uint32), ws.view(np.uint32))
    assert np.array_equal(part[:, 1].view(np.uint32), wc.view(np.uint32))
    vals = part[:, 0].astype(np.float64) + part[:, 1].astype(np.float64)
    assert np.float64(tot) == _final_np(vals)


def test_fmaf_np_is_the_correctly_rounded_fma():
    """The halving form's FMA against exact rational arithmetic, rounded
    to binary32 by hand (nearest, ties to even), on random operands and on
    constructed ties where rounding p + c in binary64 first would be wrong."""
    r = rng(11)
    a = (r.standard_normal(3000) * 10.0 ** r.uniform(-3, 3, 3000)).astype(np.float32)
    b = (r.standard_normal(3000) * 10.0 ** r.uniform(-3, 3, 3000)).astype(np.float32)
    c = (r.standard_normal(3000) * 10.0 ** r.uniform(-6, 6, 3000)).astype(np.float32)
    # ties: a*b = 1 + 2^-24 + 2^-47 (just above a binary32 midpoint), c = 0,
    # and products whose low part decides the direction next to a midpoint
    a = np.concatenate([a, np.float32([1 + 2.0 ** -23, 1 + 2.0 ** -12, 3.0])])
    b = np.concatenate([b, np.float32([1 + 2.0 ** -23, 1 + 2.0 ** -12 - 2.0 ** -23, 1 + 2.0 ** -22])])
    c = np.concatenate([c, np.float32([-1.0, 2.0 ** -30, -2.0 ** -40])])
    got = _fmaf_np(a, b, c)

    def rn32(q):
        if q == 0:
            return 0.0
        m, ex = math.frexp(float(q))  # only for the scale; the rounding below is exact
        e = ex - 24
        while Fraction(2) ** (e + 24) <= abs(q):
            e += 1
        while Fraction(2) ** (e + 23) > abs(q):
            e -= 1
        unit = Fraction(2) ** e
        t = q / unit
        fl = math.floor(t)
        rem = t - fl
        if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
            fl += 1
        return float(fl * unit)

    for x, yv, z, g in zip(a.tolist(), b.tolist(), c.tolist(), got.tolist()):
        want = rn32(Fraction(x) * Fraction(yv) + Fraction(z))
        assert np.float32(want).view(np.uint32) == np.float32(g).view(np.uint32) or (want == 0 and g == 0), (x, yv, z)


def _bf16_case(n, seed):
    r = rng(seed)
    bits = inputs._to_bf16_bits((r.standard_normal(n) * 10.0 ** r.uniform(-2, 2, n)).astype(np.float32))
    return bits, inputs.bf16_to_f32(bits)


@pytest.mark.parametrize("k,W", SIGMAS)
@pytest.mark.parametrize("acc", [0, 1])
def test_bf16_reduce_tree_matches_halving_form(oracle_mod, k, W, acc):
    """bfloat16 inputs: eight elements per 16-byte vector (V = min(k, 8))."""
    bits, f = _bf16_case(40_000 + 5, 12)
    part, tot = oracle_mod.reduce(bits, k, W, acc)
    ws, wc = _sigma_tree_np(f, k, W, compensated=bool(acc), V=8)
    if acc:
        assert np.array_equal(part[:, 0].view(np.uint32), ws.view(np.uint32))
        assert np.array_equal(part[:, 1].view(np.uint32), wc.view(np.uint32))
        vals = part[:, 0].astype(np.float64) + part[:, 1].astype(np.float64)
    else:
        assert np.array_equal(part.view(np.uint32), ws.view(np.uint32))
        vals = part.astype(np.float64)
    assert np.float64(tot).view(np.uint64) == np.float64(_final_np(vals)).view(np.uint64)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("k,W", SIGMAS)
@pytest.mark.parametrize("acc", [0, 1])
def test_dot_tree_matches_halving_form(oracle_mod, dtype, k, W, acc):
    """Plain dot: s = fmaf(x, y, s) per element (one rounding, not two);
    Dot2: TwoProduct by the exact binary64 product, TwoSum, and the
    correction c + (pe + q).  Tails pad x with -0.0 and y with +0.0."""
    n = 30_000 + 7
    if dtype == "f32":
        r = rng(13)
        x = (r.standard_normal(n) * 10.0 ** r.uniform(-2, 2, n)).astype(np.float32)
        y = (r.standard_normal(n) * 10.0 ** r.uniform(-2, 2, n)).astype(np.float32)
        xa, ya, V = x, y, 4
    else:
        xa, x = _bf16_case(n, 14)
        ya, y = _bf16_case(n, 15)
        V = 8
    part, tot = oracle_mod.dot(xa, ya, k, W, acc)
    ws, wc = _sigma_tree_np(x, k, W, compensated=bool(acc), y=y, V=V)
    if acc:
        assert np.array_equal(part[:, 0].view(np.uint32), ws.view(np.uint32))
        assert np.array_equal(part[:, 1].view(np.uint32), wc.view(np.uint32))
        vals = part[:, 0].astype(np.float64) + part[:, 1].astype(np.float64)
    else:
        assert np.array_equal(part.view(np.uint32), ws.view(np.uint32))
        vals = part.astype(np.float64)
    assert np.float64(tot).view(np.uint64) == np.float64(_final_np(vals)).view(np.uint64)


@pytest.mark.parametrize("acc", [0, 1])
def test_signed_zero_dot_and_sum(oracle_mod, acc):
    """-0.0 times +1.0 is -0.0 and a sum of -0.0 is -0.0 in round to
    nearest, so every plain partial and total is -0.0 -- including the
    ragged last chunk, whose padding (x = -0.0, y = +0.0) must leave a
    -0.0 accumulator unchanged.  Compensated: the sums s stay -0.0, and
    TwoSum's error of (-0.0) + (-0.0) is (-0.0 - (-0.0)) + (-0.0 - (+0.0))
    = +0.0, so every compensation c and the total s + c are +0.0."""
    n = 32 * 8 * 4 * 3 + 77
    x = np.full(n, -0.0, np.float32)
    y = np.ones(n, np.float32)
    want_tot = np.float64(-0.0 if acc == 0 else 0.0).view(np.uint64)

    def check(part):
        if acc == 0:
            assert np.all(part.view(np.uint32) == 0x80000000)
        else:
            assert np.all(part[:, 0].view(np.uint32) == 0x80000000)
            assert np.all(part[:, 1].view(np.uint32) == 0)

    for k, W in ((4, 8), (1, 1), (8, 2)):
        part, tot = oracle_mod.dot(x, y, k, W, acc)
        check(part)
        assert np.float64(tot).view(np.uint64) == want_tot, (k, W)
        part, tot = oracle_mod.reduce(x, k, W, acc)
        check(part)
        assert np.float64(tot).view(np.uint64) == want_tot, (k, W)
    bits = np.full(n, 0x8000, np.uint16)  # bfloat16 -0.0 times +1.0
    part, tot = oracle_mod.dot(bits, np.full(n, 0x3F80, np.uint16), 16, 8, acc)
    check(part)
    assert np.float64(tot).view(np.uint64) == want_tot


def test_integer_valued_dot_and_bf16_are_exact_for_any_schedule(oracle_mod):
    """Small integers make every product and every partial sum exact in
    binary32 (|partials| < 2^24), so every tree gives the exact result."""
    r = rng(16)
    n = 200_000 + 3
    a = r.integers(-16, 17, size=n).astype(np.float32)
    b = r.integers(-16, 17, size=n).astype(np.float32)
    exact = float((a.astype(np.int64) * b.astype(np.int64)).sum())
    ai = r.integers(-128, 129, size=n).astype(np.float32)
    ab = inputs._to_bf16_bits(ai)
    assert np.array_equal(inputs.bf16_to_f32(ab), ai)
    exact_b = float(ai.astype(np.int64).sum())
    a16, b16 = inputs._to_bf16_bits(a), inputs._to_bf16_bits(b)
    for k, W in SIGMAS:
        for acc in (0, 1):
            assert oracle_mod.dot(a, b, k, W, acc)[1] == exact, (k, W, acc)
            assert oracle_mod.dot(a16, b16, k, W, acc)[1] == exact, (k, W, acc)
            assert oracle_mod.reduce(ab, k, W, acc)[1] == exact_b, (k, W, acc)


def test_fp_tree_order_matters_pin(oracle_mod):
    """A case where the fixed tree and a serial sum differ: the tree pairs
    lane l with lane l + 16 first, so 1e8 + (-1e8) cancels before the ones
    are absorbed."""
    x = np.zeros(32, np.float32)
    x[0], x[16] = 1e8, -1e8
    x[1:16] = 1.0
    part, tot = oracle_mod.reduce(x, 1, 1)
    assert part[0] == 15.0 and tot == 15.0
    serial = np.float32(0)
    for v in x:
        serial = np.float32(serial + v)
    assert serial != 15.0


def test_integer_valued_fp_is_exact_for_any_schedule(oracle_mod):
    r = rng(5)
    f = r.integers(-1024, 1024, size=300_000).astype(np.float32)
    exact = float(f.astype(np.int64).sum())
    for k, W in SIGMAS:
        assert oracle_mod.reduce(f, k, W)[1] == exact
        assert oracle_mod.reduce(f, k, W, oracle_mod.TWOSUM)[1] == exact


def test_two_sum_two_prod_error_free(oracle_mod):
    r = rng(6)
    a = (r.standard_normal(2000) * 10.0 ** r.uniform(-6, 6, 2000)).astype(np.float32)
    b = (r.standard_normal(2000) * 10.0 ** r.uniform(-6, 6, 2000)).astype(np.float32)
    for x, y in zip(a.tolist(), b.tolist()):
        s, e = oracle_mod.two_sum(x, y)
        assert Fraction(s) + Fraction(e) == Fraction(x) + Fraction(y)
        p, pe = oracle_mod.two_prod(x, y)
        assert Fraction(p) + Fraction(pe) == Fraction(x) * Fraction(y)


def test_exact_accumulator_vs_fsum(oracle_mod):
    r = rng(7)
    for _ in range(20):
        v = r.standard_normal(5000) * 10.0 ** r.uniform(-60, 60, 5000)  # within the 2^-384..2^320 range
        v = np.concatenate([v, -v[:2500] * (1 + 1e-15)])
        assert oracle_mod.exact_sum_f64(v) == math.fsum(v.tolist())
    f = inputs.precision_inputs(1 << 16)[0]
    assert oracle_mod.exact_sum(f) == math.fsum(f.astype(np.float64).tolist())
    a, b, _ = inputs.precision_inputs(1 << 16, kind="dot")
    prods = (a.astype(np.float64) * b.astype(np.float64)).tolist()  # exact products
    assert oracle_mod.exact_sum(a, b) == math.fsum(prods)


def _gamma(h, u=2.0 ** -24):
    return h * u / (1 - h * u)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["sum", "dot"])
def test_precision_errors_within_bounds(oracle_mod, dtype, kind):
    """Plain: |err| <= gamma_h * sum|terms|; compensated:
    |err| <= u|S| + gamma_h^2 * sum|terms| (+ the FP64 final's own error),
    with tree height h = k + 10 for a 32-lane warp tree, 32-warp block and
    serial chunk accumulation bounded by the chunk count."""
    o = oracle_mod
    n = 1 << 18
    arrs = inputs.precision_inputs(n, target=1e6, kind=kind, dtype=dtype)
    data, info = arrs[:-1], arrs[-1]
    conv = (lambda a: inputs.bf16_to_f32(a)) if dtype == "bf16" else (lambda a: a)
    k, W = 16, 8
    if kind == "sum":
        exact = o.exact_sum(data[0])
        absum = float(np.abs(conv(data[0]).astype(np.float64)).sum())
        plain = o.reduce(data[0], k, W)[1]
        comp = o.reduce(data[0], k, W, o.TWOSUM)[1]
    else:
        exact = o.exact_sum(data[0], data[1])
        absum = float(np.abs(conv(data[0]).astype(np.float64) * conv(data[1]).astype(np.float64)).sum())
        plain = o.dot(data[0], data[1], k, W)[1]
        comp = o.dot(data[0], data[1], k, W, o.TWOSUM)[1]
    nch = n // (32 * W * k)
    h = k + 5 + 5 + nch
    assert abs(plain - exact) <= _gamma(h) * absum
    fp64_final = 2 * nch * 2.0 ** -53 * absum
    assert abs(comp - exact) <= 2.0 ** -24 * abs(exact) + _gamma(h) ** 2 * absum * 4 + fp64_final
    assert abs(comp - exact) < abs(plain - exact) or plain == exact


def test_precision_generator_hits_condition_target():
    for dtype in ("f32", "bf16"):
        for kind in ("sum", "dot"):
            info = inputs.precision_inputs(1 << 20, target=1e7, kind=kind, dtype=dtype)[-1]
            assert 5e6 <= info["cond"] <= 2e7, info


# ---------------------------------------------------------------- K-G
def _seg_small():
    off = np.array([0, 0, 1, 5000, 5000, 9000, 20000, 20001, 31000], np.int64)
    x, f = inputs.segment_values(int(off[-1]))
    return off, x, f


@pytest.mark.parametrize("k,W", [(1, 1), (4, 8), (16, 8), (8, 32)])
def test_segmented_int_plain_definitions(oracle_mod, k, W):
    off, x, _ = _seg_small()
    tot, y, oc, cnt = oracle_mod.segmented(x, off, k, W)
    for s in range(off.size - 1):
        a, b = off[s], off[s + 1]
        seg = x[a:b].astype(np.int64)
        assert tot[s] == seg.sum()
        assert np.array_equal(y[a:b], np.cumsum(seg).astype(np.int32))
        kept = x[a:b][x[a:b] > 0]
        assert cnt[s] == kept.size and np.array_equal(oc[a:a + kept.size], kept)
    assert tot.sum() == x.astype(np.int64).sum()


def test_segmented_fp_exact_on_integer_values(oracle_mod):
    off, x, _ = _seg_small()
    f = (x % 2048).astype(np.float32) - 1024
    tot, y, oc, cnt = oracle_mod.segmented(f, off, 4, 8)
    for s in range(off.size - 1):
        a, b = off[s], off[s + 1]
        seg = f[a:b].astype(np.float64)
        assert tot[s] == seg.sum()
        assert np.array_equal(y[a:b], np.cumsum(seg).astype(np.float32))
        kept = f[a:b][f[a:b] > 0]
        assert cnt[s] == kept.size and np.array_equal(oc[a:a + kept.size], kept)
    assert tot[0] == 0.0 and math.copysign(1, tot[0]) == -1  # empty segment: -0.0


def test_segmented_fp_within_bounds(oracle_mod):
    off, _, f = _seg_small()
    tot, y, _, _ = oracle_mod.segmented(f, off, 16, 8)
    for s in range(off.size - 1):
        a, b = off[s], off[s + 1]
        if a == b:
            continue
        seg = f[a:b].astype(np.float64)
        exact = math.fsum(seg.tolist())
        absum = np.abs(seg).sum()
        assert abs(tot[s] - exact) <= _gamma(40 + (b - a) // 4096) * absum
        pref = np.cumsum(seg)
        abspref = np.cumsum(np.abs(seg))
        assert np.all(np.abs(y[a:b] - pref) <= _gamma(64) * abspref + 2.0 ** -24 * np.abs(pref))


def test_segment_generator_shape():
    off = inputs.segment_offsets()
    lens = np.diff(off)
    assert off.size == inputs.NSEG + 1 and lens.max() <= inputs.SEG_CAP
    assert 0.9e8 < off[-1] < 2.0e8
    assert 1500 < np.median(lens) < 2600


def test_segmented_fp_scan_worked_example(oracle_mod):
    """A hand-derived worked example of the FP32 chunk scan tree and the
    FP64 chunk carry at sigma = (1, 1) (one 32-lane warp per chunk):
    x = 2^24 in lane 0 and 1.0 in lanes 1..31, where every rounding is a
    tie, so the result depends on the exact order of the additions.

    Row 0 (lanes 0..15), Kogge-Stone shfl_up by 1, 2, 4, 8 (identity below
    the row start): 2^24 + 1 rounds to 2^24, so r = 2^24 + [0, 0, 2, 2, 4,
    4, 6, 6, 8, 8, 10, 10, 12, 12, 14, 14].  Row 1 (lanes 16..31) holds
    1..16 after its own steps, then adds lane 15 (2^24 + 14): 2^24 + 15 + j
    rounds an odd offset to the multiple of 4 next to it, r = 2^24 + [16,
    16, 16, 18, 20, 20, 20, 22, 24, 24, 24, 26, 28, 28, 28, 30].  The output
    q_l = ((E + C) + ex_l) + z_l with E = C = -0.0, ex_l = r_{l-1} (the
    identity at lane 0) and z_l = x_l: 2^24 + r_{l-1} + 1 again rounds odd
    offsets to a multiple of 4, giving 2^24 + [0, 0, 0, 4, 4, 4, 4, 8, 8, 8,
    8, 12, 12, 12, 12, 16, 16, 16, 16, 16, 20, 20, 20, 20, 24, 24, 24, 24,
    28, 28, 28, 28] (the exact prefix is 2^24 + l, a serial FP32 scan gives
    2^24 everywhere).  The reduce tree for lane 0 (xor 16, 8, 4, 2, 1):
    2^24 + 1 -> 2^24, + 2, + 4, + 8, + 16 = 2^24 + 30 (exact sum 2^24 + 31).

    Segments [0, 32) and [32, 96): the second has two chunks; the second
    chunk's carry is the FP64 sum of the first chunk's total T = q_31 =
    2^24 + 28, so its outputs are (float)(2^24 + 28 + q_l) = 2^25 + 28 +
    offset_l (multiples of 4 are exact at 2^25); its total is the FP64 sum
    of the two partials, 2^25 + 60."""
    pat = np.ones(32, np.float32)
    pat[0] = 2.0 ** 24
    f = np.tile(pat, 3)
    off = np.array([0, 32, 96], np.int64)
    tot, y, oc, cnt = oracle_mod.segmented(f, off, 1, 1)
    offs = np.array([0, 0, 0, 4, 4, 4, 4, 8, 8, 8, 8, 12, 12, 12, 12, 16,
                     16, 16, 16, 16, 20, 20, 20, 20, 24, 24, 24, 24, 28, 28, 28, 28], np.float64)
    want = np.concatenate([2.0 ** 24 + offs, 2.0 ** 24 + offs, 2.0 ** 25 + 28 + offs]).astype(np.float32)
    assert np.array_equal(y.view(np.uint32), want.view(np.uint32))
    assert tot[0] == 2.0 ** 24 + 30 and tot[1] == 2.0 ** 25 + 60
    assert np.array_equal(cnt, [32, 64]) and np.array_equal(oc, f)


@pytest.mark.parametrize("k,W", [(1, 1), (32, 16)])
def test_segmented_fp_carry_and_total_kept_in_fp64(oracle_mod, k, W):
    """A hand-derived case where the running chunk carry leaves FP32's
    grid, with S = 32kW elements per chunk (32 at sigma = (1, 1), 16384 at
    (32, 16)): one segment of three chunks holding 2^24, 1 and 1 in their
    first elements and zeros elsewhere.
    Each chunk's scan is exact (it adds only zeros), so chunk 0 outputs
    2^24; chunk 1 outputs (float)(2^24 + 1), a tie that rounds to the even
    2^24; chunk 2's carry is the FP64 sum 2^24 + 1, so it outputs
    (float)(2^24 + 2) = 2^24 + 2.  A carry kept in FP32 would hold 2^24
    there and give 2^24 again.  The segment total is the FP64 sum of the
    chunk partials, 2^24 + 2; rounding it to FP32 per chunk gives 2^24."""
    S = 32 * k * W
    f = np.zeros(3 * S, np.float32)
    f[0], f[S], f[2 * S] = 2.0 ** 24, 1.0, 1.0
    off = np.array([0, 3 * S], np.int64)
    tot, y, oc, cnt = oracle_mod.segmented(f, off, k, W)
    want = np.repeat(np.array([2.0 ** 24, 2.0 ** 24, 2.0 ** 24 + 2], np.float32), S)
    assert np.array_equal(y.view(np.uint32), want.view(np.uint32))
    assert tot[0] == 2.0 ** 24 + 2
    assert cnt[0] == 3 and np.array_equal(oc[:3], [2.0 ** 24, 1.0, 1.0])


# ---------------------------------------------------------------- dynamic groups
def _dyn_plain(x, D):
    """Plain definitions of the dynamic-group workload per warp: members
    p = (x & 1023) < D, their mask, ranks, match sets and reductions."""
    u = x.view(np.uint32).reshape(-1, 32)
    p = (u & 1023) < D
    bit = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    m = (p.astype(np.uint64) * bit).sum(1).astype(np.uint32)
    rank = np.where(p, np.cumsum(p, axis=1) - 1, 0xFFFFFFFF).astype(np.uint32)
    keys = (u >> 10) & 7
    same = (keys[:, :, None] == keys[:, None, :]) & p[:, None, :]
    mm = np.where(p, (same.astype(np.uint64) * bit).sum(2), 0).astype(np.uint32)
    rec = np.zeros((u.shape[0], 8), np.uint32)
    for g in range(u.shape[0]):
        if not p[g].any():
            continue
        v = u[g][p[g]]
        k = keys[g][p[g]]
        rec[g] = [m[g], m[g] if (k == k[0]).all() else 0, int((v & 0xFFFF).astype(np.uint64).sum()) & 0xFFFFFFFF,
                  np.uint32(v.view(np.int32).min()), np.uint32(v.view(np.int32).max()),
                  np.bitwise_and.reduce(v), np.bitwise_or.reduce(v), np.bitwise_xor.reduce(v)]
    return m, rank.reshape(-1), mm.reshape(-1), rec


@pytest.mark.parametrize("D", (0, 1, 102, 512, 922, 1024))
def test_dynamic_groups_plain_definitions(oracle_mod, D):
    x = inputs.masked_input(32 * 997)
    mm, rank, rec, filt, cnt = oracle_mod.warp_dynamic(x, D)
    m, wrank, wmm, wrec = _dyn_plain(x, D)
    assert np.array_equal(rank, wrank) and np.array_equal(mm, wmm) and np.array_equal(rec, wrec)
    members = (x.view(np.uint32) & 1023) < D
    assert cnt == int(members.sum()) == sum(bin(int(v)).count("1") for v in m)
    # the append: every warp's members, contiguous and in rank order
    assert np.array_equal(np.sort(filt), np.sort(x[members]))
    xs, ps = x.reshape(-1, 32), members.reshape(-1, 32)
    pos = {}
    for g in range(xs.shape[0]):
        run = xs[g][ps[g]]
        if run.size:
            hits = np.flatnonzero(filt == run[0])
            assert any(np.array_equal(filt[h:h + run.size], run) for h in hits)


def test_dynamic_groups_special_cases(oracle_mod):
    # every key equal inside a warp: match_all returns the mask, match_any
    # the whole mask for every member
    x = (np.arange(32 * 32, dtype=np.int64) | (5 << 10)).astype(np.int32)
    mm, rank, rec, filt, cnt = oracle_mod.warp_dynamic(x, 512)
    p = (x.view(np.uint32) & 1023) < 512
    m = rec[:, 0]
    # low bits 32g + l: warps 0..15 are all members, warps 16..31 have none
    assert np.array_equal(rec[:, 1], m) and np.all(m[:16] == 0xFFFFFFFF) and np.all(rec[16:] == 0)
    assert np.array_equal(mm[p], np.repeat(m, 32)[p])
    assert cnt == p.sum()
    # one member: reductions are its own value, rank 0, match set itself
    x = np.full(32, 1023, np.int32)
    x[7] = 5 | (3 << 10)
    mm, rank, rec, filt, cnt = oracle_mod.warp_dynamic(x, 512)
    assert rec[0].tolist() == [1 << 7, 1 << 7, int(x[7]) & 0xFFFF, x[7], x[7], x[7], x[7], x[7]]
    assert rank[7] == 0 and mm[7] == 1 << 7 and cnt == 1 and filt[0] == x[7]
