"""The SIMD-collapsed CPU executor against the plain collapsed oracle, bit
for bit, on every kernel it runs, for every build this host can run
(AVX-512, AVX2, and the scalar build without SIMD), at several schedules,
ragged sizes and edge cases, on one and on eight threads."""
import numpy as np
import pytest

import simd_collapsed as sc
from paper_2112_10034_amd import inputs

ISAS = sc.host_isas()
SIGMAS = [(1, 1), (1, 8), (2, 4), (4, 8), (8, 2), (16, 8), (32, 4), (4, 32), (32, 32)]


@pytest.fixture(params=ISAS)
def isa(request):
    sc.set_threads(4, request.param)
    return request.param


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64) if a.dtype.itemsize == 8 else a.view(np.uint32)


def same(a, b):
    return np.array_equal(bits(a), bits(b))


def test_builds_report_their_isa():
    want = {"avx512": 512, "avx2": 256, "scalar": 0}
    for isa in ISAS:
        assert sc.lib(isa).coxs_isa() == want[isa]


def test_shfl_every_op_width_arg(oracle_mod, isa):
    r = np.random.default_rng(1)
    v = r.integers(-2**31, 2**31, size=32 * 4, dtype=np.int64).astype(np.int32)
    for op in range(4):
        for w in (1, 2, 4, 8, 16, 32):
            for arg in range(32):
                assert np.array_equal(sc.warp_shfl(v, op, arg, w, isa=isa), oracle_mod.warp_shfl(v, op, arg, w)), \
                    (op, w, arg)


def test_shfl_per_lane_args_masks_and_undefined(oracle_mod, isa):
    r = np.random.default_rng(2)
    n = 32 * 300
    v = r.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)
    for op in range(4):
        for w in (4, 32):
            argv = (r.integers(-100, 100, n) if op == 0 else r.integers(0, 32, n)).astype(np.int32)
            assert np.array_equal(sc.warp_shfl(v, op, 0, w, argv=argv, isa=isa),
                                  oracle_mod.warp_shfl(v, op, 0, w, argv=argv))
    masks = r.integers(1, 2**32, size=n // 32, dtype=np.uint64).astype(np.uint32)
    lead = np.repeat(np.array([int(m & -m).bit_length() - 1 for m in masks.tolist()], np.int32), 32)
    assert np.array_equal(sc.warp_shfl(v, 0, 0, 32, mask=masks, argv=lead, isa=isa),
                          oracle_mod.warp_shfl(v, 0, 0, 32, mask=masks, argv=lead))
    # a lane of the mask reading a lane outside it: undefined, reported
    m = np.full(n // 32, 0x0000FFFF, np.uint32)
    with pytest.raises(sc.CoxsError, match="status 8"):
        sc.warp_shfl(v, 2, 16, 32, mask=m, isa=isa)
    with pytest.raises(sc.CoxsError, match="status 1"):
        sc.warp_shfl(v, 1, 32, 32, isa=isa)


def test_votes(oracle_mod, isa):
    r = np.random.default_rng(3)
    n = 32 * 2000
    pred = (r.random(n) < 0.5).astype(np.int32) * r.integers(1, 9, n).astype(np.int32)
    masks = r.integers(0, 2**32, size=n // 32, dtype=np.uint64).astype(np.uint32)
    masks[:5] = [0, 1, 0x80000000, 0xFFFFFFFF, 0xAAAAAAAA]
    for m in (masks, None):
        gb, ga = sc.warp_vote(pred, m, isa=isa)
        wb, wa = oracle_mod.warp_vote(pred, m)
        assert np.array_equal(gb, wb) and np.array_equal(ga, wa)


@pytest.mark.parametrize("n", [0, 1, 255, 256, 1000, (1 << 16) + 37])
def test_block_reduce(oracle_mod, isa, n):
    x = inputs.block_reduce_input(n) if n else np.zeros(0, np.int32)
    a, b = sc.reduce_blocks_i32(x, isa=isa), oracle_mod.reduce_blocks_i32(x)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("k,W", SIGMAS)
def test_reduce_all_dtypes_and_accumulations(oracle_mod, isa, k, W):
    n = 32 * W * k * 3 + 77
    x, _, f = inputs.primitive_inputs(n)
    r = np.random.default_rng(k * 100 + W)
    h = inputs._to_bf16_bits((r.standard_normal(n) * 10.0 ** r.uniform(-2, 2, n)).astype(np.float32))
    a, b = sc.reduce(x, k, W, isa=isa), oracle_mod.reduce(x, k, W)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    for arr in (f, h):
        for acc in (0, 1):
            a, b = sc.reduce(arr, k, W, acc, isa=isa), oracle_mod.reduce(arr, k, W, acc)
            assert same(a[0], b[0]), (arr.dtype, acc)
            assert np.float64(a[1]).view(np.uint64) == np.float64(b[1]).view(np.uint64), (arr.dtype, acc)


@pytest.mark.parametrize("k,W", SIGMAS[:7])
def test_dot_and_dot2(oracle_mod, isa, k, W):
    n = 32 * W * k * 2 + 45
    r = np.random.default_rng(7 + k + W)
    x = (r.standard_normal(n) * 10.0 ** r.uniform(-2, 2, n)).astype(np.float32)
    y = (r.standard_normal(n) * 10.0 ** r.uniform(-2, 2, n)).astype(np.float32)
    for a_, b_ in ((x, y), (inputs._to_bf16_bits(x), inputs._to_bf16_bits(y))):
        for acc in (0, 1):
            a, b = sc.dot(a_, b_, k, W, acc, isa=isa), oracle_mod.dot(a_, b_, k, W, acc)
            assert same(a[0], b[0]) and np.float64(a[1]).view(np.uint64) == np.float64(b[1]).view(np.uint64)


def test_precision_workload_sample(oracle_mod, isa):
    f, _ = inputs.precision_inputs(1 << 16)
    a, b, _ = inputs.precision_inputs(1 << 16, kind="dot")
    for acc in (0, 1):
        for k, W in ((32, 32), (16, 16)):
            p, q = sc.reduce(f, k, W, acc, isa=isa), oracle_mod.reduce(f, k, W, acc)
            assert same(p[0], q[0]) and p[1] == q[1]
            p, q = sc.dot(a, b, k, W, acc, isa=isa), oracle_mod.dot(a, b, k, W, acc)
            assert same(p[0], q[0]) and p[1] == q[1]


@pytest.mark.parametrize("k,W", SIGMAS)
def test_scan_and_compaction(oracle_mod, isa, k, W):
    for n in (0, 5, 32 * W * k, 32 * W * k * 3 + 101):
        x, _, _ = inputs.primitive_inputs(n) if n else (np.zeros(0, np.int32), None, None)
        assert np.array_equal(sc.scan_i32(x, k, W, isa=isa), oracle_mod.scan_i32(x, k, W)), n
        oc, c = sc.compact_i32(x, k, W, isa=isa)
        ro, rc = oracle_mod.compact_i32(x, k, W)
        assert c == rc and np.array_equal(oc, ro), n


@pytest.mark.parametrize("G", [2, 4, 8, 16, 32])
def test_tile_sort(oracle_mod, isa, G):
    r = np.random.default_rng(G)
    for n in (32 * 50, 32 * 50 + 13, 7):
        keys = r.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        keys[:64] = np.array([0, 0xFFFFFFFF] * 32, np.uint32)[: min(64, n)]
        assert np.array_equal(sc.tile_sort_u32(keys, G, isa=isa), oracle_mod.tile_sort_u32(keys, G))


@pytest.mark.parametrize("T", [2, 4, 8, 16, 32])
def test_tile_reduce(oracle_mod, isa, T):
    for n in (1, 7, 32 * 100 + 19, 4096 * 3):
        x = inputs.masked_input(n)
        assert np.array_equal(sc.tile_reduce_i32(x, T, isa=isa), oracle_mod.tile_reduce_i32(x, T))


@pytest.mark.parametrize("D", [0, 1, 102, 512, 922, 1024])
def test_masked(oracle_mod, isa, D):
    x = inputs.masked_input(32 * 3001)
    a, b = sc.warp_masked(x, D, isa=isa), oracle_mod.warp_masked(x, D)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("k,W", [(1, 1), (4, 8), (8, 4), (16, 8), (32, 8), (2, 16)])
@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_segmented(oracle_mod, isa, k, W, dtype):
    off = np.array([0, 0, 1, 5000, 5000, 9000, 20000, 20001, 31000, 31003, 31003 + 4097 * 3 + 11], np.int64)
    xi, xf = inputs.segment_values(int(off[-1]))
    x = xi if dtype == "i32" else xf
    got, want = sc.segmented(x, off, k, W, isa=isa), oracle_mod.segmented(x, off, k, W)
    for g, w_ in zip(got, want):
        assert np.ascontiguousarray(g).tobytes() == np.ascontiguousarray(w_).tobytes()


def test_threads_do_not_change_results(isa):
    x, keys, f = inputs.primitive_inputs((1 << 18) + 5)
    out = []
    for t in (1, 8):
        sc.set_threads(t, isa)
        out.append([sc.reduce(f, 32, 32, 1, isa=isa)[0].tobytes(), sc.scan_i32(x, 32, 32, isa=isa).tobytes(),
                    sc.compact_i32(x, 32, 32, isa=isa)[0].tobytes(), sc.tile_sort_u32(keys, isa=isa).tobytes()])
    assert out[0] == out[1]


def test_vote_bench_runs(isa):
    for op in (0, 1):
        ns = sc.vote_bench(op, 200_000, isa=isa)
        assert 0 < ns < 1e4
