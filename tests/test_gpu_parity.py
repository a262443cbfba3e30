"""GPU parity: every HIP entry point against the CPU oracle, element by
element on the same seeded inputs.  Integer results and same-schedule FP32
results must be bit-exact; the schedule (items_per_lane, warps_per_block) is
passed to both sides.  Sizes span several chunks plus a ragged tail."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu

SIGMAS = [(1, 1), (2, 4), (4, 8), (8, 2), (16, 8), (32, 4), (16, 16), (4, 32)]


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def up(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def down(t):
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------- warp builtins
def test_shfl_all_ops_widths_args(dev, oracle_mod):
    torch, cox = dev
    rng = np.random.default_rng(1)
    v = rng.integers(-2**31, 2**31, size=32 * 8, dtype=np.int64).astype(np.int32)
    vg = up(torch, v)
    for op in range(4):
        for w in (1, 2, 4, 8, 16, 32):
            for arg in range(32):
                got = down(cox.warp_shfl(vg, op, arg, w))
                want = oracle_mod.warp_shfl(v, op, arg, w)
                assert np.array_equal(got, want), (op, w, arg)


def test_shfl_per_lane_args_and_masks(dev, oracle_mod):
    torch, cox = dev
    rng = np.random.default_rng(2)
    n = 32 * 512
    v = rng.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)
    for op in range(4):
        for w in (4, 32):
            argv = (rng.integers(-100, 100, size=n) if op == 0 else rng.integers(0, 32, size=n)).astype(np.int32)
            got = down(cox.warp_shfl(up(torch, v), op, 0, w, argv=up(torch, argv)))
            want = oracle_mod.warp_shfl(v, op, 0, w, argv=argv)
            assert np.array_equal(got, want), (op, w)
    # masked broadcast from a lane inside the mask
    masks = rng.integers(1, 2**32, size=n // 32, dtype=np.uint64).astype(np.uint32)
    srcl = np.array([int(m & -m).bit_length() - 1 for m in masks.tolist()], np.int32)
    argv = np.repeat(srcl, 32)
    got = down(cox.warp_shfl(up(torch, v), 0, 0, 32, mask=up(torch, masks.view(np.int32)), argv=up(torch, argv)))
    want = oracle_mod.warp_shfl(v, 0, 0, 32, mask=masks, argv=argv)
    assert np.array_equal(got, want)


def test_votes_random_masks(dev, oracle_mod):
    torch, cox = dev
    rng = np.random.default_rng(3)
    n = 32 * 4096
    pred = (rng.random(n) < 0.5).astype(np.int32) * rng.integers(1, 100, n).astype(np.int32)
    masks = rng.integers(0, 2**32, size=n // 32, dtype=np.uint64).astype(np.uint32)
    masks[:5] = [0, 1, 0x80000000, 0xFFFFFFFF, 0xAAAAAAAA]
    gb, ga = cox.warp_vote(up(torch, pred), up(torch, masks.view(np.int32)))
    wb, wa = oracle_mod.warp_vote(pred, masks)
    assert np.array_equal(down(gb).view(np.uint32), wb)
    assert np.array_equal(down(ga), wa)


@pytest.mark.parametrize("T", [1, 2, 4, 8, 16, 32])
def test_tile_votes(dev, oracle_mod, T):
    """Tile-scoped ballot / any / all against the oracle, predicates of
    every density from all-false to all-true warps."""
    torch, cox = dev
    rng = np.random.default_rng(60 + T)
    n = 32 * 20000
    dens = np.repeat(rng.random(n // 1024), 1024)
    pred = (rng.random(n) < dens).astype(np.int32) * rng.integers(-5, 6, n).astype(np.int32)
    pred[:64] = np.repeat([0, 1], 32)
    gb, ga = cox.tile_vote(up(torch, pred), T)
    wb, wa = oracle_mod.tile_vote(pred, T)
    assert np.array_equal(down(gb).view(np.uint32), wb)
    assert np.array_equal(down(ga), wa)


def test_paper_code1_and_code4_on_gpu(dev):
    torch, cox = dev
    val = torch.ones(32 * 4, dtype=torch.int32, device="cuda")
    for off in (16, 8, 4, 2, 1):
        val = val + cox.warp_shfl(val, cox.SHFL_DOWN, off)
    assert torch.all(val == 32)
    pred = torch.arange(256, dtype=torch.int32, device="cuda") % 2
    bal, aa = cox.warp_vote(pred)
    assert torch.all(((aa >> 1) & 1) == 0) and torch.all((aa & 1) == 1)
    assert np.all(down(bal).view(np.uint32) == 0xAAAAAAAA)


# ---------------------------------------------------------------- block reduce
@pytest.mark.parametrize("n", [1, 31, 256, 1000, 4096 * 3 + 77, 1 << 20])
def test_block_reduce(dev, oracle_mod, n):
    torch, cox = dev
    say("block_reduce n", n)
    x = inputs.block_reduce_input(n)
    bs, wc = cox.warp_reduce_blocks_i32(up(torch, x))
    obs, owc = oracle_mod.reduce_blocks_i32(x)
    assert np.array_equal(down(bs), obs) and np.array_equal(down(wc), owc)


# ---------------------------------------------------------------- chunked reduce
@pytest.mark.parametrize("k,W", SIGMAS)
def test_reduce_i32_and_f32(dev, oracle_mod, k, W):
    torch, cox = dev
    n = 3 * 32 * W * k + 123
    say("reduce sigma", k, W, "n", n)
    x, _, f = inputs.primitive_inputs(n)
    t, p = cox.warp_reduce(up(torch, x), cfg=(k, W))
    op, ot = oracle_mod.reduce(x, k, W)
    assert np.array_equal(down(p), op) and int(down(t)[0]) == ot
    t, p = cox.warp_reduce(up(torch, f), cfg=(k, W))
    op, ot = oracle_mod.reduce(f, k, W)
    assert np.array_equal(down(p).view(np.uint32), op.view(np.uint32))
    assert down(t).view(np.uint64)[0] == np.float64(ot).view(np.uint64)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["sum", "dot"])
@pytest.mark.parametrize("acc", [0, 1])
@pytest.mark.parametrize("k,W", [(1, 2), (8, 8), (16, 8), (32, 4)])
def test_precision_variants_bit_exact(dev, oracle_mod, dtype, kind, acc, k, W):
    torch, cox = dev
    n = 5 * 32 * W * k + 1001
    n += n % 2
    say("precision", dtype, kind, acc, k, W, n)
    arrs = inputs.precision_inputs(n, target=1e6, kind=kind, dtype=dtype)
    data = arrs[:-1]
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    g = [up(torch, a).view(tdt) if dtype == "bf16" else up(torch, a) for a in data]
    if kind == "sum":
        t, p = cox.warp_reduce(g[0], acc=acc, cfg=(k, W))
        op, ot = oracle_mod.reduce(data[0], k, W, acc)
    else:
        t, p = cox.warp_dot(g[0], g[1], acc=acc, cfg=(k, W))
        op, ot = oracle_mod.dot(data[0], data[1], k, W, acc)
    assert np.array_equal(down(p).view(np.uint32), op.view(np.uint32))
    assert down(t).view(np.uint64)[0] == np.float64(ot).view(np.uint64)


def test_reduce_empty_and_tiny(dev, oracle_mod):
    torch, cox = dev
    for n in (0, 1, 5):
        x = np.arange(1, n + 1, dtype=np.int32)
        t, _ = cox.warp_reduce(up(torch, x), partials=False)
        assert int(down(t)[0]) == n * (n + 1) // 2
        f = np.arange(1, n + 1, dtype=np.float32)
        t, _ = cox.warp_reduce(up(torch, f), partials=False)
        want = oracle_mod.reduce(f, 16, 8)[1]
        assert down(t).view(np.uint64)[0] == np.float64(want).view(np.uint64)


# ---------------------------------------------------------------- scan / compaction
@pytest.mark.parametrize("k,W", SIGMAS)
def test_scan(dev, oracle_mod, k, W):
    torch, cox = dev
    n = 7 * 32 * W * k + 5
    say("scan sigma", k, W, "n", n)
    x, _, _ = inputs.primitive_inputs(n)
    y = down(cox.warp_scan(up(torch, x), cfg=(k, W)))
    assert np.array_equal(y, oracle_mod.scan_i32(x, k, W))


@pytest.mark.parametrize("k,W", SIGMAS)
def test_compaction(dev, oracle_mod, k, W):
    torch, cox = dev
    n = 7 * 32 * W * k + 5
    say("compact sigma", k, W, "n", n)
    x, _, _ = inputs.primitive_inputs(n)
    out, cnt = cox.ballot_compact(up(torch, x), cfg=(k, W))
    ref, rc = oracle_mod.compact_i32(x, k, W)
    c = int(down(cnt)[0])
    assert c == rc and np.array_equal(down(out)[:c], ref)


def test_scan_compaction_edge_sizes_and_reuse(dev, oracle_mod):
    """Back-to-back calls on one workspace (epoch tags), sizes around the
    chunk size, empty input, and a many-chunk case with small chunks so the
    look-back walks more than one 32-entry window."""
    torch, cox = dev
    S = 32 * 8 * 16
    for n in (0, 1, 31, S - 1, S, S + 1, 3 * S, 40 * 32 * 2 + 3):
        x, _, _ = inputs.primitive_inputs(n)
        xg = up(torch, x)
        y = down(cox.warp_scan(xg))
        assert np.array_equal(y, np.cumsum(x.astype(np.int64)).astype(np.int32)), n
        out, cnt = cox.ballot_compact(xg)
        c = int(down(cnt)[0])
        assert c == int((x > 0).sum()) and np.array_equal(down(out)[:c], x[x > 0]), n
    x, _, _ = inputs.primitive_inputs(200_000)
    y = down(cox.warp_scan(up(torch, x), cfg=(1, 1)))  # 6250 chunks of 32
    assert np.array_equal(y, np.cumsum(x.astype(np.int64)).astype(np.int32))
    for ws in cox._ws_cache.values():
        ws.status()


def test_compaction_many_chunks_and_reuse(dev):
    """Many small chunks (look-backs over several status windows), inputs
    shorter than one chunk, empty inputs, and schedules alternating on one
    workspace (every call leaves the ticket counter and the epoch ready for
    the next)."""
    torch, cox = dev
    for cfg, n in (((1, 1), 200_000), ((1, 2), 64 * 1000 + 17), ((32, 16), 16384 * 9 + 4000), ((32, 16), 5000),
                   ((32, 16), 0), ((32, 32), 3 * 32768 + 7), ((2, 16), 1024 * 300 + 1), ((32, 32), 0),
                   ((32, 16), 16384 * 40), ((4, 8), 1)):
        say("compact case", cfg, n)
        x, _, _ = inputs.primitive_inputs(n)
        out, cnt = cox.ballot_compact(up(torch, x), cfg=cfg)
        c = int(down(cnt)[0])
        assert c == int((x > 0).sum()), (cfg, n)
        assert np.array_equal(down(out)[:c], x[x > 0]), (cfg, n)
    for ws in cox._ws_cache.values():
        ws.status()


@pytest.mark.parametrize("k,W", [(32, 8), (4, 4), (8, 4), (16, 16), (32, 32), (2, 8)])
def test_scan_and_compaction_few_blocks(dev, k, W):
    """Grids of one, two and five blocks, so that every block takes many
    chunks in turn, each chunk's rows requested during the previous one."""
    torch, cox = dev
    S = 32 * W * k
    x, _, _ = inputs.primitive_inputs(S * 21 + 77)
    want_y = np.cumsum(x.astype(np.int64)).astype(np.int32)
    want_c = x[x > 0]
    for G in (1, 2, 5):
        say("scan/compaction few blocks", k, W, G)
        y = down(cox.warp_scan(up(torch, x), cfg=(k, W, G)))
        assert np.array_equal(y, want_y), G
        out, cnt = cox.ballot_compact(up(torch, x), cfg=(k, W, G))
        c = int(down(cnt)[0])
        assert c == want_c.size and np.array_equal(down(out)[:c], want_c), G
    for ws in cox._ws_cache.values():
        ws.status()


def test_compaction_grid_sizes(dev):
    """Grids of one block, of a few blocks, and of more blocks than chunks."""
    torch, cox = dev
    x, _, _ = inputs.primitive_inputs(16384 * 23 + 99)
    want = x[x > 0]
    for G in (1, 3, 8, 13, 300):
        say("compact grid", G)
        out, cnt = cox.ballot_compact(up(torch, x), cfg=(32, 16, G))
        c = int(down(cnt)[0])
        assert c == want.size and np.array_equal(down(out)[:c], want), G
    for ws in cox._ws_cache.values():
        ws.status()


def test_scan_of_ones_and_determinism(dev):
    torch, cox = dev
    n = 1_000_003
    ones = torch.ones(n, dtype=torch.int32, device="cuda")
    y = cox.warp_scan(ones)
    assert torch.equal(y, torch.arange(1, n + 1, dtype=torch.int32, device="cuda"))
    x, _, f = inputs.primitive_inputs(n)
    xg = up(torch, x)
    a = cox.warp_scan(xg)
    b = cox.warp_scan(xg)
    assert torch.equal(a, b)
    fg = up(torch, f)
    t1, p1 = cox.warp_reduce(fg)
    t2, p2 = cox.warp_reduce(fg)
    assert torch.equal(p1, p2) and torch.equal(t1, t2)


# ---------------------------------------------------------------- tile sort
@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("n", [32, 32 * 3333, 32 * 3333 + 19])
def test_tile_sort(dev, oracle_mod, k, n):
    torch, cox = dev
    say("sort k", k, "n", n)
    _, keys, _ = inputs.primitive_inputs(n)
    got = down(cox.tile_sort(up(torch, keys.view(np.int32)), cfg=(k, 0))).view(np.uint32)
    assert np.array_equal(got, oracle_mod.tile_sort_u32(keys))


def test_tile_sort_adversarial_and_zero_one(dev):
    torch, cox = dev
    rng = np.random.default_rng(9)
    cases = [np.full(32 * 64, 7, np.uint32), np.tile(np.arange(32, dtype=np.uint32)[::-1], 64),
             np.tile(np.array([0, 0xFFFFFFFF], np.uint32), 32 * 32),
             np.tile(np.array([0x80000000, 0x7FFFFFFF], np.uint32), 32 * 32),
             (rng.random(32 * 100000) < 0.5).astype(np.uint32)]
    for c in cases:
        for k in (1, 4, 8):
            got = down(cox.tile_sort(up(torch, c.view(np.int32)), cfg=(k, 0))).view(np.uint32)
            assert np.array_equal(got, np.sort(c.reshape(-1, 32), axis=1).reshape(-1))


@pytest.mark.parametrize("k", [4, 1, 8, 16])
def test_tile_sort_all_zero_one_groups(dev, k):
    """The 0-1 principle (Knuth, TAOCP vol. 3, 5.3.4): a comparator network
    sorts every input iff it sorts every 0/1 input.  All 2^32 0/1 patterns
    of a 32-key group go through the GPU network, 2^24 patterns per launch;
    a sorted 0/1 group is (32 - c) zeros then c ones, c = its popcount."""
    torch, cox = dev
    per = 1 << 24
    lanes = torch.arange(32, device="cuda", dtype=torch.int64)
    out = torch.empty(per * 32, dtype=torch.int32, device="cuda")
    for b in range((1 << 32) // per):
        pat = torch.arange(b * per, (b + 1) * per, device="cuda", dtype=torch.int64)
        keys = ((pat[:, None] >> lanes) & 1).to(torch.int32).reshape(-1)
        cox.tile_sort(keys, cfg=(k, 0), out=out)
        ones = keys.view(-1, 32).sum(1, keepdim=True)
        want = (lanes[None, :] >= 32 - ones).to(torch.int32)
        if not torch.equal(out.view(-1, 32), want):
            bad = int((out.view(-1, 32) != want).any(1).nonzero()[0, 0])
            raise AssertionError(f"pattern {b * per + bad:#010x} not sorted")
        del keys, ones, want, pat
    print("all 2^32 zero-one groups sorted, keys per lane", k, flush=True)


# ---------------------------------------------------------------- tile reduce / masked
@pytest.mark.parametrize("T", [2, 4, 8, 16, 32])
@pytest.mark.parametrize("n", [1, 7, 256 * 8 * 5 + 37, 4096 * 700 + 4093])
def test_tile_reduce(dev, oracle_mod, T, n):
    torch, cox = dev
    say("tile reduce T", T, "n", n)
    x = inputs.masked_input(n)
    got = down(cox.tile_reduce(up(torch, x), T))
    assert np.array_equal(got, oracle_mod.tile_reduce_i32(x, T))


@pytest.mark.parametrize("T", [2, 8, 32])
def test_tile_reduce_unaligned_input(dev, oracle_mod, T):
    """x starting 4 bytes past a 16-byte boundary (a tensor view)."""
    torch, cox = dev
    n = 4096 * 9 + 301
    x = inputs.masked_input(n + 1)
    g = up(torch, x)[1:]
    got = down(cox.tile_reduce(g, T))
    assert np.array_equal(got, oracle_mod.tile_reduce_i32(x[1:], T))


@pytest.mark.parametrize("T", [4, 8, 16, 32])
def test_tile_reduce_unaligned_output(dev, oracle_mod, T):
    """out starting 4 bytes past a 16-byte boundary: tiles of 8 and 16 then
    store one sum per tile instead of 16-byte vectors.  The words around
    the output stay untouched."""
    torch, cox = dev
    n = 2048 * 40 + 96
    x = inputs.masked_input(n)
    nt = (n + T - 1) // T
    buf = torch.full((nt + 8,), -7, dtype=torch.int32, device="cuda")
    got = cox.tile_reduce(up(torch, x), T, out=buf[1:1 + nt])
    assert got.data_ptr() % 16 == 4
    b = down(buf)
    assert np.array_equal(b[1:1 + nt], oracle_mod.tile_reduce_i32(x, T))
    assert b[0] == -7 and np.all(b[1 + nt:] == -7)


@pytest.mark.parametrize("D", (0, 1, 102, 512, 922, 1024))
def test_masked_ops(dev, oracle_mod, D):
    torch, cox = dev
    n = 32 * 20011
    x = inputs.masked_input(n)
    out, rec = cox.warp_masked(up(torch, x), D)
    oo, orec = oracle_mod.warp_masked(x, D)
    assert np.array_equal(down(out), oo)
    assert np.array_equal(down(rec).view(np.uint32), orec)


@pytest.mark.parametrize("D", (102, 922))
def test_masked_ops_unaligned_output(dev, oracle_mod, D):
    """out starting 4 bytes past a 16-byte boundary takes one store per
    lane instead of 16-byte vectors; the words around it stay untouched."""
    torch, cox = dev
    n = 32 * 20011
    x = inputs.masked_input(n)
    buf = torch.full((n + 8,), -7, dtype=torch.int32, device="cuda")
    out, rec = cox.warp_masked(up(torch, x), D, out=buf[1:1 + n])
    assert out.data_ptr() % 16 == 4
    oo, orec = oracle_mod.warp_masked(x, D)
    b = down(buf)
    assert np.array_equal(b[1:1 + n], oo) and b[0] == -7 and np.all(b[1 + n:] == -7)
    assert np.array_equal(down(rec).view(np.uint32), orec)
