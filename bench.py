#!/usr/bin/env python3
"""Throughput of the warp-primitive hot path on one MI355X.

One step = one pass of the whole primitive set over one batch of 2^28
synthetic elements already resident in HBM:
  int32 sum reduce, int32 inclusive scan, ballot compaction (keep x > 0),
  uint32 32-key bitonic tile sort, FP32 shuffle-tree sum.
value = elements processed per second over the five kernels (GElem/s).

The JSON line also carries per-kernel GElem/s and HBM fractions, the
roofline of the dominant kernel (algorithmic bytes over its average launch
time, timed with HIP events on the stream the kernels run on), and the
oracle's CPU throughput on a bounded sample of the same inputs.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GElem/s and % of HBM peak per warp-primitive kernel; batched vs per-launch speedup"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "reduce_i32": ["paper_2112_10034_amd/csrc/reduce.hip", "paper_2112_10034_amd/csrc/cox_warp.hpp"],
    "scan_i32": ["paper_2112_10034_amd/csrc/scan.hip", "paper_2112_10034_amd/csrc/cox_warp.hpp"],
    "compact_i32": ["paper_2112_10034_amd/csrc/scan.hip", "paper_2112_10034_amd/csrc/cox_warp.hpp"],
    "tile_sort_u32": ["paper_2112_10034_amd/csrc/sort.hip", "paper_2112_10034_amd/csrc/cox_warp.hpp"],
    "reduce_f32": ["paper_2112_10034_amd/csrc/reduce.hip", "paper_2112_10034_amd/csrc/cox_warp.hpp"],
}


def measured_traffic(name, launches_bytes):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(name)
    if not k or k.get("src_hash") != src_hash(KERNEL_SOURCES[name]):
        return None
    return k["hbm_bytes_per_launch"]


def host_info():
    """nproc, the threads this process may use, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_threads": usable, "model": model}


def _cpu_leg(mod, x, keys, f, sample, sig, threads, runs=3, isa=None):
    """Median wall time of `runs` passes of the five primitives over the
    first `sample` elements of each input, on `threads` threads."""
    kw = {} if isa is None else {"isa": isa}
    mod.set_threads(threads, **kw)
    xs, ks, fs = x[:sample].copy(), keys[:sample].copy(), f[:sample].copy()
    (kr, Wr), (kf, Wf) = sig["reduce_i32"], sig["reduce_f32"]
    (kS, WS), (kC, WC) = sig["scan"], sig["compact"]
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        mod.reduce(xs, kr, Wr, **kw)
        mod.scan_i32(xs, kS, WS, **kw)
        mod.compact_i32(xs, kC, WC, **kw)
        mod.tile_sort_u32(ks, **kw)
        mod.reduce(fs, kf, Wf, **kw)
        ts.append(time.perf_counter() - t0)
    dt = sorted(ts)[len(ts) // 2]
    return {"value": round(5 * sample / dt / 1e9, 4), "unit": "GElem/s", "cores": threads,
            "sample": f"first {sample} elements of each input, all five primitives once; median of {runs} "
                      f"passes ({dt:.2f} s wall each)"}


def cpu_baseline(x, keys, f, sample, sig, single_sample):
    """The oracle as it stands, on all usable host threads (at most 16,
    the box's share) and on one thread, plus the host it ran on."""
    import oracle

    host = host_info()
    cores = min(16, host["usable_threads"])
    allc = _cpu_leg(oracle, x, keys, f, sample, sig, cores)
    one = _cpu_leg(oracle, x, keys, f, single_sample, sig, 1)
    out = dict(allc)
    out.update({"kind": "oracle", "single_thread": one, "host": host})
    return out


def simd_baseline(x, keys, f, sample, sig, single_sample):
    """The SIMD-collapsed CPU executor (warp builtins on whole warps with
    AVX-512 / AVX2) on the same samples, and the per-call cost of its vote
    builtins with and without SIMD.  The paper's Table 2 figures (0.241 /
    0.236 us per any / all call with AVX, 2.542 / 2.992 us without, Xeon
    Silver 4210) are context: its workload sizes are not given."""
    import simd_collapsed as sc

    host = host_info()
    cores = min(16, host["usable_threads"])
    isa = sc.default_isa()
    out = _cpu_leg(sc, x, keys, f, sample, sig, cores, isa=isa)
    out.update({"kind": f"simd-collapsed executor ({isa})",
                "single_thread": _cpu_leg(sc, x, keys, f, single_sample, sig, 1, isa=isa), "host": host})
    votes = {}
    for i in sc.host_isas():
        votes[i] = {"any_ns_per_call": round(sc.vote_bench(0, isa=i), 3),
                    "all_ns_per_call": round(sc.vote_bench(1, isa=i), 3)}
    out["vote_builtins"] = {"per_isa": votes,
                            "paper_table2_context_us": {"any_avx": 0.241, "any_no_avx": 2.542,
                                                        "all_avx": 0.236, "all_no_avx": 2.992,
                                                        "host": "Xeon Silver 4210, 8 cores"}}
    return out


def _timed(fn, reps):
    """Average milliseconds of fn() over reps back-to-back launches (HIP
    events on torch's current stream, the stream the binding launches on)."""
    import torch

    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _stats(ms):
    s = sorted(ms)

    def q(p):
        return s[min(len(s) - 1, max(0, int(round(p * (len(s) - 1)))))]
    return {"median": q(0.5), "p10": q(0.1), "p90": q(0.9), "runs": len(s)}


class Scrub:
    """A 1 GiB buffer that is read and written (x += 1, plain loads and
    stores) before a timed launch, so that neither the L2 caches nor the
    256 MB memory-side cache still hold the launch's inputs."""

    def __init__(self, nbytes=1 << 30):
        import torch

        self.buf = torch.zeros(nbytes // 4, dtype=torch.int32, device="cuda")

    def __call__(self):
        self.buf.add_(1)


def _timed_each(fn, reps, scrub=None):
    """Per-launch milliseconds of fn(): reps launches, each between its own
    pair of HIP events on torch's current stream, each preceded (outside
    the events) by a cache scrub when one is given.  Median, p10, p90."""
    import torch

    fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        if scrub is not None:
            scrub()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return _stats([a.elapsed_time(b) for a, b in evs])


def _entry(n, nbytes, st, warm_ms=None):
    """Figures of a kernel from its scrubbed per-launch statistics."""
    ms = st["median"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    e = {"ms": round(ms, 4), "ms_p10": round(st["p10"], 4), "ms_p90": round(st["p90"], 4),
         "gelem_s": round(n / (ms * 1e-3) / 1e9, 2), "gb_s": round(gbs, 1),
         "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes), "scrubbed": True}
    if warm_ms is not None:
        e["warm_ms"] = round(warm_ms, 4)
        e["warm_hbm_frac"] = round(nbytes / (warm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return e


def _measure(n, nbytes, fn, scrub, reps=20, warm_reps=10):
    return _entry(n, nbytes, _timed_each(fn, reps, scrub), _timed(fn, warm_reps))


def other_kernels(fg, scrub, reps=20):
    """The kernels outside the timed step, each timed on its own: the
    block reduce (2^20 int32), the masked warp operations at three
    densities, the dynamic groups and the tile reductions (2^26 int32),
    the key-value tile sort (2^28 pairs), the 64- and 1024-key group sorts
    (2^28 keys), the integral image (8192 x 8192),
    and the precision
    variants over 2^28 elements (float32 and bfloat16, sum and dot, plain
    and TwoSum).  Their timing does not depend on the values, so the
    precision variants run on the primitive set's float32 N(0, 1) array, a
    second seeded float32 array and their bfloat16 roundings.  Every kernel
    is timed per launch after a 1 GiB cache scrub (median, p10, p90 of
    `reps` launches), and also back to back (warm_ms)."""
    import torch

    from paper_2112_10034_amd import cox, inputs

    res = {}
    xb = torch.from_numpy(inputs.block_reduce_input()).cuda()
    nb = xb.numel()
    bs, wc = cox.warp_reduce_blocks_i32(xb)
    res["block_reduce_i32_2p20"] = _measure(nb, 4 * nb + 4 * (nb // 256) + 4 * (nb // 32), lambda: cox.warp_reduce_blocks_i32(xb, bs, wc), scrub, reps)
    xm = torch.from_numpy(inputs.masked_input()).cuda()
    nm = xm.numel()
    out, rec = torch.empty_like(xm), torch.empty((nm // 32, 4), dtype=torch.int32, device="cuda")
    for D in inputs.MASK_DENSITIES:
        res[f"masked_d{D}_2p26"] = _measure(nm, 8 * nm + 16 * (nm // 32), lambda: cox.warp_masked(xm, D, out, rec), scrub, reps)
    mm_, rk_, rc_ = torch.empty_like(xm), torch.empty_like(xm), torch.empty((nm // 32, 8), dtype=torch.int32,
                                                                            device="cuda")
    fl_, fc_ = torch.empty_like(xm), torch.empty(1, dtype=torch.int64, device="cuda")
    members = int((((xm.view(torch.int32) & 1023) < 512)).sum().item())
    res["dynamic_groups_d512_2p26"] = _measure(nm, 12 * nm + 32 * (nm // 32) + 4 * members, lambda: cox.warp_dynamic(xm, 512, mm_, rk_, rc_, fl_, fc_), scrub, reps)
    del mm_, rk_, rc_, fl_, fc_
    for T in inputs.TILE_SIZES:
        to = torch.empty(nm // T, dtype=torch.int32, device="cuda")
        res[f"tile_reduce_t{T}_2p26"] = _measure(nm, 4 * nm + 4 * (nm // T), lambda: cox.tile_reduce(xm, T, to), scrub, reps)
    del xm, out, rec
    n = fg.numel()
    # key-value tile sort over 2^28 pairs (a network's time does not depend
    # on the values): uint32 keys, 4-byte values; 16 bytes per pair
    gk = torch.Generator(device="cuda")
    gk.manual_seed(2112100344)
    kk = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda", generator=gk)
    kv = torch.arange(n, dtype=torch.int32, device="cuda")
    ok_, ov_ = torch.empty_like(kk), torch.empty_like(kv)
    res["tile_sort_kv_2p28"] = _measure(n, 16 * n, lambda: cox.tile_sort_kv(kk, kv, None, ok_, ov_), scrub, reps)
    # wider groups: 64 keys over a full wave (one key per lane) and 1024 keys
    # over four waves (four keys per lane), 8 bytes per key
    for kpl, tile in ((1, 64), (4, 1024)):
        res[f"group_sort_t{tile}_k{kpl}_2p28"] = _measure(n, 8 * n, lambda: cox.tile_sort(kk, tile=tile, cfg=(kpl, 0), out=ok_), scrub, reps)
    del kk, kv, ok_, ov_
    # integral image of the 8192 x 8192 uint8 image: 1 byte read and 4
    # written per pixel
    img = torch.from_numpy(inputs.image_u8()).cuda()
    H, W = img.shape
    sat = torch.empty((H, W), dtype=torch.int32, device="cuda")
    res[f"integral_image_{H}x{W}"] = _measure(H * W, 5 * H * W, lambda: cox.integral_image(img, sat), scrub, reps)
    del img, sat
    g2 = torch.Generator(device="cuda")
    g2.manual_seed(2112100343)
    f2 = torch.randn(n, dtype=torch.float32, device="cuda", generator=g2)
    h1, h2 = fg.to(torch.bfloat16), f2.to(torch.bfloat16)
    tot = torch.empty(1, dtype=torch.float64, device="cuda")
    for name, a, b, es in (("f32", fg, f2, 4), ("bf16", h1, h2, 2)):
        for acc, an in ((cox.PLAIN, "plain"), (cox.TWOSUM, "twosum")):
            res[f"reduce_{name}_{an}_2p28"] = _measure(n, es * n, lambda: cox.warp_reduce(a, acc=acc, partials=False, total=tot), scrub, reps)
            res[f"dot_{name}_{an}_2p28"] = _measure(n, 2 * es * n, lambda: cox.warp_dot(a, b, acc=acc, partials=False, total=tot), scrub, reps)
    del f2, h1, h2
    for ws in cox._ws_cache.values():
        ws.status()
    return res


def grid_sync_bench(iters=50, reps=3, rounds=2000):
    """Grid-wide barriers.  The exchange kernel (two barriers per round) at
    one and two 1024-thread blocks per compute unit gives the barrier
    latency.  The conjugate-gradient solve of the tridiagonal system at
    2^20 and 2^24 rows (iters iterations, tol = 0) runs once as one
    cooperative launch and once as one launch per phase; every timed solve
    starts from x = 0 (the zero fill is inside the timed region).
    Algorithmic bytes per iteration: row_ptr 4 (n + 1) and the entries
    8 nnz, plus per row 16 bytes when the block's rows stay in registers
    (p and r gathered, p and r stored) or 40 bytes when they stream
    through memory (also q stored, and p, q, x, r read, x stored).  When
    the one-launch solve also keeps every block's CSR rows in shared memory
    (they fit: at most 65535 entries and the compute unit's 160 KiB less
    the static part), row_ptr and the entries are read once per solve and
    count 1 / iters of their bytes per iteration."""
    import torch

    from paper_2112_10034_amd import cox, inputs

    res = {}
    cap = cox.grid_capacity()
    for G in sorted({cap // 2, cap}):
        out = torch.empty((G, 1024), dtype=torch.int32, device="cuda")
        ms = _timed(lambda: cox.grid_exchange(G, rounds, out), reps)
        res[f"barrier_us_g{G}"] = round(ms * 1e3 / (2 * rounds), 3)
    R, W, _ = cox.default_cfg(cox.OP_CG, cox.F32)
    for n in inputs.CG_N:
        rp, ci, val, b = inputs.cg_tridiag(n)
        d = [torch.from_numpy(a).cuda() for a in (rp, ci, val, b)]
        x = torch.zeros(n, dtype=torch.float32, device="cuda")
        nnz = ci.size
        S = 32 * W * R
        nch = -(-n // S)
        resident = nch <= torch.cuda.get_device_properties(0).multi_processor_count
        row_bytes = 16 if resident else 40
        # the resident kernel's fit rule, with its static shared memory
        # (window of S + 128 floats, 2.3 KiB of reduction slots, 512 B slack)
        most = int(max(rp[min((c + 1) * S, n)] - rp[c * S] for c in range(nch)))
        staged = resident and most <= 0xFFFF and 4 * S + 8 * most <= 160 * 1024 - 4 * (S + 128) - 2368 - 512
        entry = {"rows": n, "nnz": int(nnz), "iterations": iters, "sigma": [R, W],
                 "registers_resident": bool(resident), "csr_in_shared_memory": bool(staged)}
        for name, pp, rb in (("one_launch", False, row_bytes), ("per_phase", True, 40)):
            def solve():
                x.zero_()
                return cox.cg_solve(*d, x, iters, 0.0, per_phase=pp)
            ms = _timed(solve, reps)
            k = int(solve()[0][0].item())
            assert k == iters, (name, k)
            csr = 4 * (n + 1) + 8 * nnz
            nbytes = (csr // iters if staged and not pp else csr) + rb * n
            us = ms * 1e3 / iters
            gbs = nbytes / (us * 1e-6) / 1e9
            entry[name] = {"us_per_iteration": round(us, 3), "algorithmic_bytes_per_iteration": int(nbytes),
                           "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        entry["speedup_one_launch"] = round(entry["per_phase"]["us_per_iteration"] /
                                            entry["one_launch"]["us_per_iteration"], 3)
        res[f"cg_tridiag_2p{n.bit_length() - 1}"] = entry
        del d, x
    for ws in cox._ws_cache.values():
        ws.status()
    return res


def batching(scrub, reps=20, base_reps=2, per_segment=True):
    """The segmented workload (10,000 lognormal segments): the fused
    reduce + scan + compaction as one autotuned graph-captured launch, vs
    the same kernel launched once per segment on the stream, vs those
    10,000 launches captured in one hipGraph (the intermediate point), per
    dtype.  The plan is timed per replay after a cache scrub (median, p10,
    p90) and back to back."""
    import numpy as np
    import torch

    from paper_2112_10034_amd import cox, inputs

    off = inputs.segment_offsets()
    n = int(off[-1])
    nseg = off.size - 1
    xi, xf = inputs.segment_values(n)
    og = torch.from_numpy(off).cuda()
    oh = torch.from_numpy(off)
    res = {"workload": f"{nseg} segments, lognormal lengths (median 2000, cap 2^20), {n} elements per dtype; "
                       "segmented sum + inclusive scan + compaction (x > 0) fused",
           "n": n, "nseg": nseg}

    for name, arr in (("i32", xi), ("f32", xf)):
        xg = torch.from_numpy(arr).cuda()
        plan = cox.Plan(xg, og, 7, autotune=True)
        k, W, G = plan.cfg()
        st = _timed_each(plan.execute, reps, scrub)
        warm = _timed(plan.execute, reps)
        t_plan = st["median"]
        kept = int(plan.seg_count.sum().item())
        alg = 4 * n + 4 * n + 4 * kept + 8 * (nseg + 1) + 16 * nseg
        tot, y, oc, cnt = (torch.empty_like(plan.seg_total), torch.empty_like(plan.y), torch.empty_like(plan.out),
                           torch.empty_like(plan.seg_count))
        t_seg, t_graph, same, same_graph = None, None, None, None

        def per_seg():
            cox.segmented_per_segment(xg, og, oh, cfg=(k, W), seg_total=tot, y=y, out=oc, seg_count=cnt)
        if per_segment:
            t_seg = _timed(per_seg, base_reps)
            same = bool(torch.equal(cnt, plan.seg_count))
            # the same 10,000 launches (and the workspace clear before them)
            # captured once in a graph and replayed
            g = torch.cuda.CUDAGraph()
            torch.cuda.synchronize()
            with torch.cuda.graph(g, capture_error_mode="relaxed"):
                per_seg()
            torch.cuda.synchronize()
            cnt.zero_()
            t_graph = _timed(g.replay, base_reps + 1)
            same_graph = bool(torch.equal(cnt, plan.seg_count)) and bool(torch.equal(tot, plan.seg_total))
            del g
        plan.close()
        for ws in cox._ws_cache.values():
            ws.status()
        res[name] = {"sigma": [k, W], "grid": G, "batched_ms": round(t_plan, 4),
                     "batched_ms_p10": round(st["p10"], 4), "batched_ms_p90": round(st["p90"], 4),
                     "batched_warm_ms": round(warm, 4),
                     "batched_gelem_s": round(n / (t_plan * 1e-3) / 1e9, 2),
                     "batched_gb_s": round(alg / (t_plan * 1e-3) / 1e9, 1),
                     "batched_hbm_frac": round(alg / (t_plan * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes": int(alg),
                     "per_segment_ms": None if t_seg is None else round(t_seg, 3),
                     "per_segment_graph_ms": None if t_graph is None else round(t_graph, 3),
                     "speedup": None if t_seg is None else round(t_seg / t_plan, 2),
                     "speedup_vs_per_segment_graph": None if t_graph is None else round(t_graph / t_plan, 2),
                     "counts_agree": same, "graph_results_agree": same_graph}
        log(f"batching {name}: plan {t_plan:.3f} ms, per-segment {t_seg} ms, per-segment graph {t_graph} ms")
        del xg
    return res


def device_info():
    """What the device reports about itself (compute units, clock, caches)."""
    import torch

    p = torch.cuda.get_device_properties(0)
    out = {"name": p.name, "compute_units": p.multi_processor_count,
           "total_memory_gib": round(p.total_memory / 2 ** 30, 1)}
    for a in ("gcnArchName", "L2_cache_size", "clock_rate", "max_threads_per_multi_processor"):
        v = getattr(p, a, None)
        if v is not None:
            out[a] = v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 28, help="elements (default: the full 2^28 workload)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 28,
                    help="elements of each input the oracle runs on (default: the whole batch)")
    ap.add_argument("--cpu-single-sample", type=int, default=1 << 24,
                    help="elements of each input the single-threaded oracle runs on")
    ap.add_argument("--scrub-reps", type=int, default=20,
                    help="launches per kernel timed one by one after a cache scrub")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batching", action="store_true", help="skip the segmented batching comparison")
    ap.add_argument("--no-others", action="store_true", help="skip the kernels outside the timed step")
    ap.add_argument("--no-grid", action="store_true", help="skip the grid-barrier and conjugate-gradient timings")
    ap.add_argument("--no-per-segment", action="store_true",
                    help="skip the one-launch-per-segment baseline of the batching comparison")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_10034_amd import cox, inputs

    torch.cuda.set_device(0)
    cox.lib()
    n = args.n
    log(f"generating inputs n={n}")
    x, keys, f = inputs.primitive_inputs(n)
    xg = torch.from_numpy(x).cuda()
    kg = torch.from_numpy(keys.view(np.int32)).cuda()
    fg = torch.from_numpy(f).cuda()
    y = torch.empty_like(xg)
    cout = torch.empty_like(xg)
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    srt = torch.empty_like(kg)
    ti = torch.empty(1, dtype=torch.int64, device="cuda")
    tf = torch.empty(1, dtype=torch.float64, device="cuda")
    sig = {"reduce_i32": cox.default_cfg(cox.OP_REDUCE, cox.I32)[:2],
           "reduce_f32": cox.default_cfg(cox.OP_REDUCE, cox.F32)[:2],
           "scan": cox.default_cfg(cox.OP_SCAN)[:2], "compact": cox.default_cfg(cox.OP_COMPACT)[:2]}
    sort_k = 4
    # workspaces and partial buffers are allocated once, outside the timed region
    nch_i = -(-n // (32 * sig["reduce_i32"][1] * sig["reduce_i32"][0]))
    nch_f = -(-n // (32 * sig["reduce_f32"][1] * sig["reduce_f32"][0]))
    pi = torch.empty(nch_i, dtype=torch.int32, device="cuda")
    pf = torch.empty(nch_f, dtype=torch.float32, device="cuda")
    cox.workspace(cox.OP_REDUCE, cox.I32, n)
    cox.workspace(cox.OP_REDUCE, cox.F32, n)
    cox.workspace(cox.OP_SCAN, cox.I32, n)
    cox.workspace(cox.OP_COMPACT, cox.I32, n)
    # one plain copy of the int32 input (untimed; 1 GiB read + 1 GiB write):
    # the known-size reference kernel for HBM byte counters
    cox.stream_copy(xg, y)
    torch.cuda.synchronize()

    names = ["reduce_i32", "scan_i32", "compact_i32", "tile_sort_u32", "reduce_f32"]

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        cox.warp_reduce(xg, total=ti, partials_out=pi)
        if ev is not None:
            ev[1].record()
        cox.warp_scan(xg, out=y)
        if ev is not None:
            ev[2].record()
        cox.ballot_compact(xg, out=cout, count=cnt)
        if ev is not None:
            ev[3].record()
        cox.tile_sort(kg, cfg=(sort_k, 0), out=srt)
        if ev is not None:
            ev[4].record()
        cox.warp_reduce(fg, total=tf, partials_out=pf)
        if ev is not None:
            ev[5].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for s in range(args.steps):
        step(evs[s])
    end.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(end)
    ms_per_step = total_ms / args.steps
    per_launch = {nm: [evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(args.steps)]
                  for i, nm in enumerate(names)}
    per = {nm: sum(v) / len(v) for nm, v in per_launch.items()}
    log(f"timed: {ms_per_step:.3f} ms/step (wall {t_wall:.2f} s)")
    # the same kernels once more, each launch after a 1 GiB cache scrub
    # (outside the step clock): cold-cache medians
    scrub = Scrub()
    cold = {
        "reduce_i32": _timed_each(lambda: cox.warp_reduce(xg, total=ti, partials_out=pi), args.scrub_reps, scrub),
        "scan_i32": _timed_each(lambda: cox.warp_scan(xg, out=y), args.scrub_reps, scrub),
        "compact_i32": _timed_each(lambda: cox.ballot_compact(xg, out=cout, count=cnt), args.scrub_reps, scrub),
        "tile_sort_u32": _timed_each(lambda: cox.tile_sort(kg, cfg=(sort_k, 0), out=srt), args.scrub_reps, scrub),
        "reduce_f32": _timed_each(lambda: cox.warp_reduce(fg, total=tf, partials_out=pf), args.scrub_reps, scrub),
    }

    # bandwidth references (untimed by the step clock): plain read, plain copy
    def ref_time(fn, reps=5):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    t_rd = ref_time(lambda: cox.stream_read(xg, sink))
    t_cp = ref_time(lambda: cox.stream_copy(xg, y))
    reference = {"stream_read_gb_s": round(4 * n / (t_rd * 1e-3) / 1e9, 1),
                 "stream_copy_gb_s": round(8 * n / (t_cp * 1e-3) / 1e9, 1)}

    kept = int(cnt.item())
    for ws in cox._ws_cache.values():
        ws.status()  # raises if a cross-block wait gave up
    alg_bytes = {
        "reduce_i32": 4 * n + 4 * nch_i,
        "scan_i32": 8 * n,
        "compact_i32": 4 * n + 4 * kept + 8,
        "tile_sort_u32": 8 * n,
        "reduce_f32": 4 * n + 4 * nch_f,
    }
    kernels = {}
    for nm in names:
        ms = per[nm]
        gbs = alg_bytes[nm] / (ms * 1e-3) / 1e9
        st = _stats(per_launch[nm])
        c = cold[nm]
        kernels[nm] = {"ms": round(ms, 4), "ms_median": round(st["median"], 4), "ms_p10": round(st["p10"], 4),
                       "ms_p90": round(st["p90"], 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                       "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                       "algorithmic_bytes": int(alg_bytes[nm]),
                       "scrubbed": {"ms_median": round(c["median"], 4), "ms_p10": round(c["p10"], 4),
                                    "ms_p90": round(c["p90"], 4), "runs": c["runs"],
                                    "hbm_frac": round(alg_bytes[nm] / (c["median"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                      4)}}
    dom = max(names, key=lambda k: per[k])
    achieved = alg_bytes[dom] / (per[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, alg_bytes[dom]),
            "algorithmic_bytes_per_launch": alg_bytes[dom]}

    out = {
        "metric": METRIC,
        "value": round(5 * n / (ms_per_step * 1e-3) / 1e9, 2),
        "unit": "GElem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+u32+f32",
        "data": "synthetic (seeded numpy PCG64: int32 U[-2^20, 2^20], uint32 uniform keys, float32 N(0,1))",
        "config": {"workload": "warp primitive set over 2^28 elements: int32 sum, int32 inclusive scan, "
                               "ballot compaction (x > 0), uint32 32-key tile sort, fp32 tree sum",
                   "n": n, "sigma_reduce_i32": list(sig["reduce_i32"]), "sigma_reduce_f32": list(sig["reduce_f32"]),
                   "sigma_scan": list(sig["scan"]),
                   "sigma_compact": list(sig["compact"]),
                   "sort_keys_per_lane": sort_k},
        "kernels": kernels,
        "step_scrubbed_ms": round(sum(cold[nm]["median"] for nm in names), 4),
        "roofline": roof,
        "reference": reference,
        "device": device_info(),
    }
    if not args.no_others:
        log("other kernels")
        del kg, y, cout, srt
        out["other_kernels"] = other_kernels(fg, scrub)
    if not args.no_batching:
        del xg, fg
        torch.cuda.empty_cache()
        out["batching"] = batching(scrub, per_segment=not args.no_per_segment)
    if not args.no_grid:
        log("grid barrier and conjugate gradient")
        out["grid_sync"] = grid_sync_bench()
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, n)
        log(f"cpu baseline: oracle on {sample} elements")
        single = min(args.cpu_single_sample, sample)
        out["cpu_baseline"] = cpu_baseline(x, keys, f, sample, sig, single)
        log("cpu baseline: simd-collapsed executor")
        out["cpu_baseline_simd"] = simd_baseline(x, keys, f, sample, sig, single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
