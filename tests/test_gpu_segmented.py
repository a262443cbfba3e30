"""GPU parity of the segmented batched path (fused persistent kernel, its
single-output variants, the per-segment baseline and graph-captured
plans) against the oracle, bit for bit, on the same seeded inputs."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu

SIGMAS = [(1, 1), (4, 8), (8, 4), (16, 8), (2, 16), (8, 16), (16, 4), (32, 8), (32, 2), (32, 16)]


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def small_case():
    """Empty, length-1, ragged and many-chunk segments, plus one segment
    that does not start on a 16-byte boundary."""
    off = np.array([0, 0, 1, 5000, 5000, 9000, 20000, 20001, 31000, 31003, 31003 + 4097 * 3 + 11], np.int64)
    xi, xf = inputs.segment_values(int(off[-1]))
    return off, xi, xf


def bits(a):
    a = np.asarray(a)
    return a.view(np.uint64) if a.dtype.itemsize == 8 else a.view(np.uint32)


def check(torch, got, want, nseg):
    tot, y, oc, cnt = [None if g is None else g.cpu().numpy() for g in got]
    wt, wy, woc, wcnt = want
    assert np.array_equal(bits(tot), bits(wt)), "segment totals"
    assert np.array_equal(bits(y), bits(wy)), "segmented scan"
    assert np.array_equal(cnt, wcnt), "kept counts"
    assert np.array_equal(bits(oc), bits(woc)), "compacted output"


@pytest.mark.parametrize("dtype", ["i32", "f32"])
@pytest.mark.parametrize("k,W", SIGMAS)
def test_segmented_fused_bit_exact(dev, oracle_mod, dtype, k, W):
    torch, cox = dev
    off, xi, xf = small_case()
    x = xi if dtype == "i32" else xf
    print("segmented", dtype, k, W, flush=True)
    got = cox.segmented(torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda(), 7, cfg=(k, W))
    check(torch, got, oracle_mod.segmented(x, off, k, W), off.size - 1)


def short_mix(k, W, seed):
    """Segments of one chunk or less at every round count (1 .. W parts of
    32k elements), the round boundaries (32k, 32k + 1), one element, a
    whole chunk, a chunk plus one, empty segments, and a few long ones,
    shuffled so that warps of one wave and one block get unlike lengths."""
    S, RW = 32 * W * k, 32 * k
    rng = np.random.default_rng(seed)
    lens = [1, 2, 3, RW - 1, RW, RW + 1, S - 1, S, S + 1, 2 * S + 5, 0, 0]
    lens += [int(r * RW - rng.integers(0, RW)) for r in range(1, W + 1) for _ in range(5)]
    lens += [int(v) for v in rng.integers(1, S + 1, size=150)]
    lens = np.array(lens, np.int64)
    rng.shuffle(lens)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xi, xf = inputs.segment_values(int(off[-1]), seed=seed)
    return off, xi, xf


@pytest.mark.parametrize("dtype", ["i32", "f32"])
@pytest.mark.parametrize("k,W", [(4, 8), (32, 8), (8, 4), (4, 1), (1, 2), (2, 16), (16, 32)])
def test_short_segments_by_one_warp(dev, oracle_mod, dtype, k, W):
    """Segments no longer than a chunk run on one logical warp each, their
    parts one after another; every output must still be the oracle's."""
    torch, cox = dev
    off, xi, xf = short_mix(k, W, 31 + k + W)
    x = xi if dtype == "i32" else xf
    print("short segments", dtype, k, W, "nseg", off.size - 1, "n", off[-1], flush=True)
    xg, og = torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda()
    want = oracle_mod.segmented(x, off, k, W)
    check(torch, cox.segmented(xg, og, 7, cfg=(k, W)), want, off.size - 1)
    # single outputs take the same path
    t, _, _, _ = cox.segmented(xg, og, cox.SEG_REDUCE, cfg=(k, W))
    assert np.array_equal(bits(t.cpu().numpy()), bits(want[0]))
    _, y, _, _ = cox.segmented(xg, og, cox.SEG_SCAN, cfg=(k, W))
    assert np.array_equal(bits(y.cpu().numpy()), bits(want[1]))
    _, _, oc, cnt = cox.segmented(xg, og, cox.SEG_COMPACT, cfg=(k, W))
    assert np.array_equal(cnt.cpu().numpy(), want[3]) and np.array_equal(bits(oc.cpu().numpy()), bits(want[2]))


@pytest.mark.parametrize("dtype", ["i32", "f32"])
@pytest.mark.parametrize("nseg", [16384, 16385, 40000])
def test_many_segments(dev, oracle_mod, dtype, nseg):
    """Eight and nine setup blocks (2048 segments each) and twenty, with
    empty, short and a few long segments."""
    torch, cox = dev
    rng = np.random.default_rng(nseg)
    lens = rng.integers(0, 400, size=nseg)
    lens[rng.integers(0, nseg, size=20)] = rng.integers(5000, 40000, size=20)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xi, xf = inputs.segment_values(int(off[-1]), seed=nseg)
    x = xi if dtype == "i32" else xf
    print("many segments", dtype, "nseg", nseg, "n", off[-1], flush=True)
    xg, og = torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda()
    want = oracle_mod.segmented(x, off, 4, 8)
    check(torch, cox.segmented(xg, og, 7, cfg=(4, 8)), want, nseg)


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_segmented_single_outputs_match_fused(dev, oracle_mod, dtype):
    torch, cox = dev
    off, xi, xf = small_case()
    x = xi if dtype == "i32" else xf
    xg, og = torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda()
    wt, wy, woc, wcnt = oracle_mod.segmented(x, off, 4, 8)
    t, _, _, _ = cox.segmented(xg, og, cox.SEG_REDUCE, cfg=(4, 8))
    assert np.array_equal(bits(t.cpu().numpy()), bits(wt))
    _, y, _, _ = cox.segmented(xg, og, cox.SEG_SCAN, cfg=(4, 8))
    assert np.array_equal(bits(y.cpu().numpy()), bits(wy))
    _, _, oc, cnt = cox.segmented(xg, og, cox.SEG_COMPACT, cfg=(4, 8))
    assert np.array_equal(cnt.cpu().numpy(), wcnt) and np.array_equal(bits(oc.cpu().numpy()), bits(woc))


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_per_segment_baseline_matches_oracle(dev, oracle_mod, dtype):
    torch, cox = dev
    off, xi, xf = small_case()
    x = xi if dtype == "i32" else xf
    got = cox.segmented_per_segment(torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda(),
                                    torch.from_numpy(off), cfg=(8, 8))
    check(torch, got, oracle_mod.segmented(x, off, 8, 8), off.size - 1)


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_plan_graph_replays(dev, oracle_mod, dtype):
    """An autotuned plan replayed several times, with eager work and
    synchronisations between replays; every replay is checked."""
    torch, cox = dev
    off, xi, xf = small_case()
    x = xi if dtype == "i32" else xf
    xg, og = torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda()
    plan = cox.Plan(xg, og, 7, autotune=True)
    k, W, G = plan.cfg()
    print("plan sigma", k, W, G, flush=True)
    want = oracle_mod.segmented(x, off, k, W)
    for rep in range(4):
        for t in (plan.seg_total, plan.y, plan.out, plan.seg_count):
            t.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        got = plan.execute()
        torch.cuda.synchronize()
        check(torch, got, want, off.size - 1)
        assert torch.isfinite(junk)
    plan.close()


def test_plan_fixed_schedule_and_reuse_with_other_calls(dev, oracle_mod):
    torch, cox = dev
    off, xi, _ = small_case()
    xg, og = torch.from_numpy(xi).cuda(), torch.from_numpy(off).cuda()
    plan = cox.Plan(xg, og, 7, cfg=(8, 4), autotune=False)
    assert plan.cfg()[:2] == (8, 4)
    want = oracle_mod.segmented(xi, off, 8, 4)
    for _ in range(3):
        cox.segmented(xg, og, 7, cfg=(16, 8))  # other calls on their own workspace in between
        check(torch, plan.execute(), want, off.size - 1)
    plan.close()


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_segmented_full_workload(dev, oracle_mod, dtype):
    """The full batching workload (10,000 lognormal segments) with the
    default schedule, compared element by element with the oracle."""
    torch, cox = dev
    off = inputs.segment_offsets()
    xi, xf = inputs.segment_values(int(off[-1]))
    x = xi if dtype == "i32" else xf
    k, W, _ = cox.default_cfg(cox.OP_SEGMENTED, cox.I32 if dtype == "i32" else cox.F32)
    print("full segmented", dtype, "n", off[-1], "sigma", k, W, flush=True)
    got = cox.segmented(torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda(), 7)
    want = oracle_mod.segmented(x, off, k, W)
    check(torch, got, want, off.size - 1)


def test_segmented_fp_worked_example(dev, oracle_mod):
    """The tie-rounding worked example of the oracle tests (2^24 and ones,
    sigma = (1, 1)): the GPU's FP32 scan tree, FP64 carry and totals give
    the hand-derived bits."""
    torch, cox = dev
    pat = np.ones(32, np.float32)
    pat[0] = 2.0 ** 24
    f = np.tile(pat, 3)
    off = np.array([0, 32, 96], np.int64)
    got = cox.segmented(torch.from_numpy(f).cuda(), torch.from_numpy(off).cuda(), 7, cfg=(1, 1))
    check(torch, got, oracle_mod.segmented(f, off, 1, 1), 2)
    offs = np.array([0, 0, 0, 4, 4, 4, 4, 8, 8, 8, 8, 12, 12, 12, 12, 16,
                     16, 16, 16, 16, 20, 20, 20, 20, 24, 24, 24, 24, 28, 28, 28, 28], np.float64)
    want = np.concatenate([2.0 ** 24 + offs, 2.0 ** 24 + offs, 2.0 ** 25 + 28 + offs]).astype(np.float32)
    assert np.array_equal(got[1].cpu().numpy().view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("k,W", [(1, 1), (32, 16)])
def test_segmented_fp_carry_kept_in_fp64(dev, oracle_mod, k, W):
    """The oracle's three-chunk case whose carry leaves FP32's grid (2^24,
    1, 1 at the starts of chunks of S = 32kW elements; (32, 16) is the
    10,000-segment workload's tuned schedule): the last chunk outputs
    2^24 + 2 and the total is 2^24 + 2 only if the look-back carries and
    sums the chunk partials in FP64."""
    torch, cox = dev
    S = 32 * k * W
    f = np.zeros(3 * S, np.float32)
    f[0], f[S], f[2 * S] = 2.0 ** 24, 1.0, 1.0
    off = np.array([0, 3 * S], np.int64)
    print("segmented fp64 carry, sigma", k, W, flush=True)
    got = cox.segmented(torch.from_numpy(f).cuda(), torch.from_numpy(off).cuda(), 7, cfg=(k, W))
    check(torch, got, oracle_mod.segmented(f, off, k, W), 1)
    want = np.repeat(np.array([2.0 ** 24, 2.0 ** 24, 2.0 ** 24 + 2], np.float32), S)
    assert np.array_equal(got[1].cpu().numpy().view(np.uint32), want.view(np.uint32))
    assert got[0].cpu().item() == 2.0 ** 24 + 2


def test_workspace_reuse_across_layouts(dev, oracle_mod):
    """Calls with different segment counts and schedules share the cached
    workspace, whose layout moves with them: each call must start from
    cleared counters and words, whatever the previous call left there."""
    torch, cox = dev
    off_a, xa, _ = small_case()
    rng = np.random.default_rng(7)
    lens = rng.integers(0, 300, size=400)
    off_b = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xb, _ = inputs.segment_values(int(off_b[-1]), seed=99)
    cases = [(off_a, xa, (16, 16)), (off_b, xb, (1, 1)), (off_a, xa, (2, 16)), (off_b, xb, (8, 4)),
             (off_a, xa, (1, 1))]
    for rep in range(2):
        for off, x, cfg in cases:
            print("layout case", off.size - 1, "segments, sigma", cfg, flush=True)
            got = cox.segmented(torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda(), 7, cfg=cfg)
            check(torch, got, oracle_mod.segmented(x, off, *cfg), off.size - 1)
            got = cox.segmented_per_segment(torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda(),
                                            torch.from_numpy(off), cfg=cfg)
            check(torch, got, oracle_mod.segmented(x, off, *cfg), off.size - 1)


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_overlapping_offsets_stay_inside_the_workspace(dev, oracle_mod, dtype):
    """Offsets that go down and up again ([0, n] five times) make five
    overlapping segments of 10 chunks each, 50 chunks for a workspace that
    holds n / S + nseg + 1 = 20.  The call must drop the chunks past the
    capacity, report COX_ERR_INVALID through the workspace status, write
    nothing past the workspace or the outputs, and leave the two segments
    that fit with their correct totals; the workspace then serves a valid
    call."""
    import ctypes as C

    torch, cox = dev
    k, W = 4, 8
    S = 32 * W * k
    n = 10 * S
    off = np.array([0, n] * 5, np.int64)
    nseg = off.size - 1
    xi, xf = inputs.segment_values(n)
    x = xi if dtype == "i32" else xf
    dt = cox.I32 if dtype == "i32" else cox.F32
    cfg = cox.make_cfg(k, W)
    L = cox.lib()
    need = L.cox_workspace_bytes(cox.OP_SEGMENTED, dt, n, nseg, C.byref(cfg))
    assert need > 0
    guard = 1 << 16
    ws = torch.empty(need + guard, dtype=torch.uint8, device="cuda")
    ws[need:] = 0xA5
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.cox_workspace_init(C.c_void_p(ws.data_ptr()), need, st) == 0
    xg = torch.from_numpy(x).cuda()
    og = torch.from_numpy(off).cuda()
    pad = 4096
    sentinel = np.int32(0x5A5A5A5A)
    y = torch.full((n + pad,), int(sentinel), dtype=torch.int32, device="cuda")
    oc = torch.full((n + pad,), int(sentinel), dtype=torch.int32, device="cuda")
    tot = torch.zeros(nseg, dtype=torch.int64 if dtype == "i32" else torch.float64, device="cuda")
    cnt = torch.zeros(nseg, dtype=torch.int64, device="cuda")
    print("overlapping offsets", dtype, flush=True)
    rc = L.cox_segmented(C.c_void_p(xg.data_ptr()), dt, C.c_void_p(og.data_ptr()), nseg, n,
                         C.c_void_p(tot.data_ptr()), C.c_void_p(y.data_ptr()), C.c_void_p(oc.data_ptr()),
                         C.c_void_p(cnt.data_ptr()), 7, C.byref(cfg), C.c_void_p(ws.data_ptr()), need, st)
    assert rc == 0
    assert L.cox_workspace_status(C.c_void_p(ws.data_ptr()), st) == 1  # COX_ERR_INVALID
    assert L.cox_workspace_status(C.c_void_p(ws.data_ptr()), st) == 0  # the flag was cleared
    assert bool((ws[need:] == 0xA5).all()), "bytes written past the workspace"
    assert bool((y[n:] == int(sentinel)).all()) and bool((oc[n:] == int(sentinel)).all()), \
        "bytes written past the outputs"
    # segments 0 and 2 are the first 20 chunks, which fit: their totals are
    # those of x[0, n) alone
    wt, _, _, _ = oracle_mod.segmented(x, np.array([0, n], np.int64), k, W)
    t = tot.cpu().numpy()
    assert np.array_equal(bits(t[[0, 2]]), bits(np.array([wt[0], wt[0]])))
    # the same workspace then serves a valid call
    off2 = np.array([0, 3, n // 2, n], np.int64)
    og2 = torch.from_numpy(off2).cuda()
    tot2 = torch.zeros(3, dtype=tot.dtype, device="cuda")
    y2 = torch.empty_like(xg)
    oc2 = torch.zeros_like(xg)
    cnt2 = torch.zeros(3, dtype=torch.int64, device="cuda")
    rc = L.cox_segmented(C.c_void_p(xg.data_ptr()), dt, C.c_void_p(og2.data_ptr()), 3, n,
                         C.c_void_p(tot2.data_ptr()), C.c_void_p(y2.data_ptr()), C.c_void_p(oc2.data_ptr()),
                         C.c_void_p(cnt2.data_ptr()), 7, C.byref(cfg), C.c_void_p(ws.data_ptr()), need, st)
    assert rc == 0
    assert L.cox_workspace_status(C.c_void_p(ws.data_ptr()), st) == 0
    check(torch, (tot2, y2, oc2, cnt2), oracle_mod.segmented(x, off2, k, W), 3)


def test_plan_creation_writes_the_outputs(dev, oracle_mod):
    """A plan with a given schedule (nothing tuned) leaves the call's
    results in its outputs when creation returns."""
    torch, cox = dev
    off, _, xf = small_case()
    xg, og = torch.from_numpy(xf).cuda(), torch.from_numpy(off).cuda()
    plan = cox.Plan(xg, og, 7, cfg=(4, 8), autotune=False)
    torch.cuda.synchronize()
    check(torch, (plan.seg_total, plan.y, plan.out, plan.seg_count), oracle_mod.segmented(xf, off, 4, 8),
          off.size - 1)
    plan.close()


def test_plan_forced_schedule_and_tuning_cache(dev, oracle_mod, tmp_path, monkeypatch):
    """COX_FORCE_CFG fixes a plan's schedule without tuning; COX_TUNE_CACHE
    records a tuned schedule and a later plan of the same call shape reuses
    it (so the float results repeat across processes)."""
    torch, cox = dev
    off, _, xf = small_case()
    xg, og = torch.from_numpy(xf).cuda(), torch.from_numpy(off).cuda()
    monkeypatch.setenv("COX_FORCE_CFG", "2,8")
    plan = cox.Plan(xg, og, 7, autotune=True)
    assert plan.cfg()[:2] == (2, 8)
    check(torch, plan.execute(), oracle_mod.segmented(xf, off, 2, 8), off.size - 1)
    plan.close()
    monkeypatch.delenv("COX_FORCE_CFG")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("COX_TUNE_CACHE", str(cache))
    p1 = cox.Plan(xg, og, 7, autotune=True)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("segmented/dt2/")
    k, W, G = p1.cfg()
    assert [int(v) for v in lines[0].split()[1:4]] == [k, W, G]
    p1.close()
    # a planted entry for the same key is taken as is, without tuning
    key = lines[0].split()[0]
    cache.write_text(lines[0] + "\n" + f"{key} 4 32 {G} 0.0\n")
    p2 = cox.Plan(xg, og, 7, autotune=True)
    assert p2.cfg() == (4, 32, G)
    assert len(cache.read_text().splitlines()) == 2
    check(torch, p2.execute(), oracle_mod.segmented(xf, off, 4, 32), off.size - 1)
    p2.close()


def test_per_segment_launches_captured_in_a_graph(dev, oracle_mod):
    """The per-segment baseline's launches (a workspace clear, then one
    launch per segment) captured in one graph: every replay, with eager
    work between replays, gives the oracle's results."""
    torch, cox = dev
    off, _, xf = small_case()
    xg, og, oh = torch.from_numpy(xf).cuda(), torch.from_numpy(off).cuda(), torch.from_numpy(off)
    nseg = off.size - 1
    tot = torch.zeros(nseg, dtype=torch.float64, device="cuda")
    y, oc = torch.zeros_like(xg), torch.zeros_like(xg)
    cnt = torch.zeros(nseg, dtype=torch.int64, device="cuda")

    def run():
        cox.segmented_per_segment(xg, og, oh, cfg=(8, 8), seg_total=tot, y=y, out=oc, seg_count=cnt)
    run()  # the workspace and the kernel are set up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        run()
    want = oracle_mod.segmented(xf, off, 8, 8)
    for _ in range(3):
        for t in (tot, y, oc, cnt):
            t.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(torch, (tot, y, oc, cnt), want, nseg)
        assert torch.isfinite(junk)


def test_segments_past_2p31_elements(dev):
    """2^31 + 4099 int32 elements in segments of 2^30 + 3 and 2^30 + 14
    elements, an empty one, a short one and a ragged last one, at the
    default schedule: totals against numpy's int64 sums, the scan against
    its definition (each segment's prefix sum wrapping mod 2^32) and each
    segment's kept run (at the segment's own offset) against numpy's
    selection of x > 0."""
    torch, cox = dev
    n = (1 << 31) + 4099
    off = np.array([0, (1 << 30) + 3, (1 << 31) + 17, (1 << 31) + 17, (1 << 31) + 4000, n], np.int64)
    print("segments past 2^31 elements, n =", n, flush=True)
    x = inputs.masked_input(n, seed=78)
    xg, og = torch.from_numpy(x).cuda(), torch.from_numpy(off).cuda()
    tot, y, oc, cnt = cox.segmented(xg, og, 7)
    tot, cnt = tot.cpu().numpy(), cnt.cpu().numpy()
    y = y.cpu().numpy()
    for s in range(off.size - 1):
        a, b = int(off[s]), int(off[s + 1])
        seg = x[a:b]
        assert int(tot[s]) == int(seg.sum(dtype=np.int64)), s
        assert np.array_equal(y[a:b], np.cumsum(seg.view(np.uint32), dtype=np.uint32).view(np.int32)), s
        keep = seg[seg > 0]
        assert int(cnt[s]) == keep.size, s
        assert np.array_equal(oc[a:a + keep.size].cpu().numpy(), keep), s
    cox.workspace(cox.OP_SEGMENTED, cox.I32, n, off.size - 1).status()
