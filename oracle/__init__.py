"""CPU oracle for the warp-primitive hot path (TEST INFRASTRUCTURE ONLY).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product library never does.

This is a thin ctypes wrapper over ``libcoxo.so`` (built from ``coxo.c`` by
``oracle/build.py``), which executes every kernel by hierarchical collapsing
(COX, Sec. 3): inter-warp loops over warps, intra-warp loops over 32 lanes,
warp functions applied to per-warp exchange arrays between RAW and WAR warp
barriers (Sec. 3.2, Code 5), loop peeling for uniform branches around
barriers (Sec. 3.3.1), one CPU thread per block at a time (Sec. 4).

All functions take and return numpy arrays on the host.  A nonzero status
from the C side raises ``OracleError``; ``COXO_ERR_UB`` (8) means an
undefined warp-function use was detected, ``COXO_ERR_DIVERGENT`` (9) a
non-uniform branch around a barrier.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# COXO_LIB names another build of coxo.c (the mutation tests load
# deliberately broken copies to show that the pins catch them)
_LIB_PATH = os.environ.get("COXO_LIB") or os.path.join(_HERE, "libcoxo.so")

I32, U32, F32, BF16 = 0, 1, 2, 3
PLAIN, TWOSUM = 0, 1
SHFL_IDX, SHFL_UP, SHFL_DOWN, SHFL_XOR = 0, 1, 2, 3
ERR_UB, ERR_DIVERGENT, ERR_RANGE = 8, 9, 10

# statement counter slots (appendix invariant)
ST_LOAD, ST_SHFL, ST_VOTE, ST_PEEL, ST_BODY = range(5)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P, I64, I = C.c_void_p, C.c_int64, C.c_int
        sig = {
            "coxo_set_threads": (I, [I]),
            "coxo_get_threads": (I, []),
            "coxo_counts_reset": (None, []),
            "coxo_counts": (I, [P, I]),
            "coxo_warp_shfl": (I, [P, P, I64, I, C.c_int32, P, I, P]),
            "coxo_warp_vote": (I, [P, P, I64, P, P]),
            "coxo_tile_vote": (I, [P, I64, I, P, P]),
            "coxo_reduce_blocks_i32": (I, [P, I64, P, P]),
            "coxo_reduce": (I, [P, I, I64, I, I, I, P, P]),
            "coxo_dot": (I, [P, P, I, I64, I, I, I, P, P]),
            "coxo_scan_i32": (I, [P, P, I64, I, I]),
            "coxo_compact_i32": (I, [P, I64, P, P, I, I]),
            "coxo_tile_sort_u32": (I, [P, P, I64, I]),
            "coxo_tile_reduce_i32": (I, [P, I64, I, P]),
            "coxo_warp_masked": (I, [P, I64, I, P, P]),
            "coxo_warp_dynamic": (I, [P, I64, I, P, P, P, P, P]),
            "coxo_segmented": (I, [P, I, P, I64, I, I, P, P, P, P]),
            "coxo_exact_sum": (I, [P, P, I, I64, P]),
            "coxo_exact_sum_f64": (I, [P, I64, P]),
            "coxo_two_sum": (None, [C.c_float, C.c_float, P, P]),
            "coxo_two_prod": (None, [C.c_float, C.c_float, P, P]),
            "coxo_code5": (I, [P, P, P, P, I]),
            "coxo_uniform_branch": (I, [P, P, I64, P]),
            "coxo_grid_exchange": (I, [I, I, I, P]),
            "coxo_tile_sort_kv_u32": (I, [P, P, P, P, I64]),
            "coxo_group_sort_u32": (I, [P, P, I64, I]),
            "coxo_integral_image_u8": (I, [P, I64, I64, P]),
            "coxo_cg": (I, [P, P, P, I64, P, P, I, C.c_double, I, I, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(code, what):
    if code != 0:
        raise OracleError(code, what)


def set_threads(n=0):
    """Number of CPU threads running blocks (0 = all online cores)."""
    return lib().coxo_set_threads(int(n))


def get_threads():
    return lib().coxo_get_threads()


def counts_reset():
    lib().coxo_counts_reset()


def counts():
    out = np.zeros(8, dtype=np.uint64)
    n = lib().coxo_counts(_p(out), 8)
    return out[:n]


def _dt_code(a):
    if a.dtype == np.int32:
        return I32
    if a.dtype == np.float32:
        return F32
    if a.dtype == np.uint16:
        return BF16
    raise TypeError(f"unsupported dtype {a.dtype}")


# ---------------------------------------------------------------- probes
def warp_shfl(v, op, arg=0, width=32, mask=None, argv=None):
    """Per 32-lane warp: lanes in ``mask`` (per warp, default all) get
    shfl/shfl_up/shfl_down/shfl_xor of ``v``; other lanes keep their input."""
    v = _c(v, np.int32)
    out = np.empty_like(v)
    m = None if mask is None else _c(mask, np.uint32)
    av = None if argv is None else _c(argv, np.int32)
    _check(lib().coxo_warp_shfl(_p(v), _p(out), v.size, op, int(arg), _p(av), width, _p(m)),
           "warp_shfl")
    return out


def warp_vote(pred, mask=None):
    """Per warp: (ballot, any | all << 1) over the lanes of ``mask``."""
    pred = _c(pred, np.int32)
    g = pred.size // 32
    bal = np.zeros(g, np.uint32)
    aa = np.zeros(g, np.int32)
    m = None if mask is None else _c(mask, np.uint32)
    _check(lib().coxo_warp_vote(_p(pred), _p(m), pred.size, _p(bal), _p(aa)), "warp_vote")
    return bal, aa


def tile_vote(pred, T):
    """Per tile of T lanes: (T-bit ballot, any | all << 1)."""
    pred = _c(pred, np.int32)
    g = pred.size // T if T > 0 else 0
    bal = np.zeros(g, np.uint32)
    aa = np.zeros(g, np.int32)
    _check(lib().coxo_tile_vote(_p(pred), pred.size, int(T), _p(bal), _p(aa)), "tile_vote")
    return bal, aa


# ---------------------------------------------------------------- kernels
def reduce_blocks_i32(x):
    x = _c(x, np.int32)
    n = x.size
    bs = np.zeros((n + 255) // 256, np.int32)
    wc = np.zeros((n + 31) // 32, np.int32)
    _check(lib().coxo_reduce_blocks_i32(_p(x), n, _p(bs), _p(wc)), "reduce_blocks_i32")
    return bs, wc


def _nchunks(n, k, W):
    S = 32 * W * k
    return (n + S - 1) // S


def reduce(x, k, W, acc=PLAIN):
    """Returns (chunk_partials, total).  int32 input: int32 partials, int64
    total.  float32 / bfloat16 (uint16 bits) input: float32 partials ((s, c)
    pairs for TWOSUM), FP64 total."""
    x = np.ascontiguousarray(x)
    dt = _dt_code(x)
    nch = _nchunks(x.size, k, W)
    if dt == I32:
        part = np.zeros(nch, np.int32)
        tot = np.zeros(1, np.int64)
    else:
        part = np.zeros(nch * (2 if acc == TWOSUM else 1), np.float32)
        tot = np.zeros(1, np.float64)
    _check(lib().coxo_reduce(_p(x), dt, x.size, acc, k, W, _p(part), _p(tot)), "reduce")
    if acc == TWOSUM:
        part = part.reshape(nch, 2)
    return part, tot[0]


def dot(a, b, k, W, acc=PLAIN):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    assert a.dtype == b.dtype and a.size == b.size
    dt = _dt_code(a)
    nch = _nchunks(a.size, k, W)
    part = np.zeros(nch * (2 if acc == TWOSUM else 1), np.float32)
    tot = np.zeros(1, np.float64)
    _check(lib().coxo_dot(_p(a), _p(b), dt, a.size, acc, k, W, _p(part), _p(tot)), "dot")
    if acc == TWOSUM:
        part = part.reshape(nch, 2)
    return part, tot[0]


def scan_i32(x, k, W):
    x = _c(x, np.int32)
    y = np.empty_like(x)
    _check(lib().coxo_scan_i32(_p(x), _p(y), x.size, k, W), "scan_i32")
    return y


def compact_i32(x, k, W):
    x = _c(x, np.int32)
    out = np.zeros_like(x)
    cnt = np.zeros(1, np.int64)
    _check(lib().coxo_compact_i32(_p(x), x.size, _p(out), _p(cnt), k, W), "compact_i32")
    return out[: int(cnt[0])], int(cnt[0])


def tile_sort_u32(keys, group=32):
    keys = _c(keys, np.uint32)
    out = np.empty_like(keys)
    _check(lib().coxo_tile_sort_u32(_p(keys), _p(out), keys.size, group), "tile_sort_u32")
    return out


def group_sort_u32(keys, G):
    """Every group of G consecutive keys sorted ascending (unsigned); G a
    power of two up to 4096."""
    k = _c(keys, np.uint32)
    out = np.empty_like(k)
    _check(lib().coxo_group_sort_u32(_p(k), _p(out), k.size, int(G)), "group_sort_u32")
    return out


def tile_sort_kv_u32(keys, vals):
    """Stable sort of every 32-pair group by unsigned key; returns
    (out_keys, out_vals)."""
    k = _c(keys, np.uint32)
    v = _c(vals, np.uint32)
    ok, ov = np.empty_like(k), np.empty_like(v)
    _check(lib().coxo_tile_sort_kv_u32(_p(k), _p(v), _p(ok), _p(ov), k.size), "tile_sort_kv_u32")
    return ok, ov


def tile_reduce_i32(x, tile):
    x = _c(x, np.int32)
    out = np.zeros((x.size + tile - 1) // tile, np.int32)
    _check(lib().coxo_tile_reduce_i32(_p(x), x.size, tile, _p(out)), "tile_reduce_i32")
    return out


def warp_masked(x, D):
    x = _c(x, np.int32)
    out = np.empty_like(x)
    rec = np.zeros(4 * (x.size // 32), np.uint32)
    _check(lib().coxo_warp_masked(_p(x), x.size, D, _p(out), _p(rec)), "warp_masked")
    return out, rec.reshape(-1, 4)


def warp_dynamic(x, D):
    """Dynamic groups (coalesced_threads, match_any / match_all, the six
    reduce_*_sync, warp-aggregated append).  Returns (match_any[n],
    rank[n], rec[n/32, 8], filtered[:count], count); the order of the warps'
    runs in ``filtered`` is the order the appends happened to take."""
    x = _c(x, np.int32)
    mm = np.empty(x.size, np.uint32)
    rank = np.empty(x.size, np.uint32)
    rec = np.zeros(8 * (x.size // 32), np.uint32)
    filt = np.zeros(x.size, np.int32)
    cnt = np.zeros(1, np.int64)
    _check(lib().coxo_warp_dynamic(_p(x), x.size, D, _p(mm), _p(rank), _p(rec), _p(filt), _p(cnt)), "warp_dynamic")
    c = int(cnt[0])
    return mm, rank, rec.reshape(-1, 8), filt[:c], c


def segmented(x, offsets, k, W):
    """Returns (seg_total, y_scan, out_compact, seg_count).  Positions of
    ``y_scan`` / ``out_compact`` not written by any segment hold zeros."""
    x = np.ascontiguousarray(x)
    dt = _dt_code(x)
    off = _c(offsets, np.int64)
    nseg = off.size - 1
    tot = np.zeros(nseg, np.int64 if dt == I32 else np.float64)
    y = np.zeros_like(x)
    oc = np.zeros_like(x)
    cnt = np.zeros(nseg, np.int64)
    _check(lib().coxo_segmented(_p(x), dt, _p(off), nseg, k, W, _p(tot), _p(y), _p(oc), _p(cnt)),
           "segmented")
    return tot, y, oc, cnt


def grid_exchange(G, rounds, block=1024):
    """Exchange kernel with grid barriers: per round every block publishes
    a row of mixed values, and after a grid barrier reads the row of block
    (b + r + 1) % G.  Returns the per-thread sums, uint32[G, block]."""
    out = np.zeros(G * block, np.uint32)
    _check(lib().coxo_grid_exchange(G, block, rounds, _p(out)), "grid_exchange")
    return out.reshape(G, block)


def integral_image_u8(img):
    """Summed-area table of a uint8 image [H, W] as uint32 (mod 2^32)."""
    im = _c(img, np.uint8)
    H, W = im.shape
    sat = np.empty((H, W), np.uint32)
    _check(lib().coxo_integral_image_u8(_p(im), H, W, _p(sat)), "integral_image_u8")
    return sat


CG_CONVERGED, CG_MAX_ITER, CG_BREAKDOWN = 0, 1, 2


def cg(row_ptr, col_idx, val, b, x0, max_iter, tol, R, W):
    """Conjugate gradient on the CSR matrix (row_ptr, col_idx, val) with the
    inner-product schedule (R, W).  Returns (x, iterations, reason,
    rr_hist[: iterations + 1])."""
    rp = _c(row_ptr, np.int32)
    ci = _c(col_idx, np.int32)
    va = _c(val, np.float32)
    bb = _c(b, np.float32)
    x = np.array(x0, dtype=np.float32, copy=True)
    n = bb.size
    res = np.zeros(2, np.int32)
    hist = np.zeros(max_iter + 1, np.float64)
    _check(lib().coxo_cg(_p(rp), _p(ci), _p(va), n, _p(bb), _p(x), int(max_iter), float(tol), R, W,
                         _p(res), _p(hist)), "cg")
    k = int(res[0])
    return x, k, int(res[1]), hist[: k + 1]


def exact_sum(x, y=None):
    """Exact sum of x (or of x*y), rounded once to binary64."""
    x = np.ascontiguousarray(x)
    dt = _dt_code(x)
    out = np.zeros(1, np.float64)
    yy = None if y is None else np.ascontiguousarray(y, dtype=x.dtype)
    _check(lib().coxo_exact_sum(_p(x), _p(yy), dt, x.size, _p(out)), "exact_sum")
    return float(out[0])


def exact_sum_f64(x):
    x = _c(x, np.float64)
    out = np.zeros(1, np.float64)
    _check(lib().coxo_exact_sum_f64(_p(x), x.size, _p(out)), "exact_sum_f64")
    return float(out[0])


def code5(a, b, barriers=True):
    """Two consecutive all() votes over one warp (Code 5)."""
    a = _c(a, np.int32)
    b = _c(b, np.int32)
    r1 = np.zeros(32, np.int32)
    r2 = np.zeros(32, np.int32)
    _check(lib().coxo_code5(_p(a), _p(b), _p(r1), _p(r2), int(bool(barriers))), "code5")
    return r1, r2


def uniform_branch(cond, x):
    """Per warp: if (cond) x += shfl_down tree else x unchanged; the branch
    encloses warp barriers, so cond must be uniform across each warp."""
    cond = _c(cond, np.int32)
    x = _c(x, np.int32)
    out = np.empty_like(x)
    _check(lib().coxo_uniform_branch(_p(cond), _p(x), x.size, _p(out)), "uniform_branch")
    return out


def two_sum(a, b):
    s, e = C.c_float(), C.c_float()
    lib().coxo_two_sum(a, b, C.byref(s), C.byref(e))
    return s.value, e.value


def two_prod(a, b):
    p, e = C.c_float(), C.c_float()
    lib().coxo_two_prod(a, b, C.byref(p), C.byref(e))
    return p.value, e.value
