"""ctypes binding of the SIMD-collapsed CPU executor (a CPU executor and
baseline of the warp-level kernels; the GPU library never uses it).

The functions take and return numpy arrays, with the same arguments and
results as the plain collapsed oracle's binding.  ``isa`` picks the build:
"avx512", "avx2" or "scalar" (no SIMD); the default is the widest one the
host supports.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

I32, U32, F32, BF16 = 0, 1, 2, 3
PLAIN, TWOSUM = 0, 1

_libs = {}


def host_isas():
    """The builds this host can run, widest first."""
    flags = set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    flags = set(line.split(":", 1)[1].split())
                    break
    except OSError:
        pass
    out = []
    if {"avx512f", "avx512bw", "avx512dq", "avx512vl", "avx512cd", "fma"} <= flags:
        out.append("avx512")
    if {"avx2", "fma"} <= flags:
        out.append("avx2")
    out.append("scalar")
    return out


def default_isa():
    return host_isas()[0]


def lib(isa=None):
    isa = isa or default_isa()
    if isa not in _libs:
        path = _build.lib_path(isa)
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P, I64, I = C.c_void_p, C.c_int64, C.c_int
        sig = {
            "coxs_set_threads": (I, [I]),
            "coxs_get_threads": (I, []),
            "coxs_isa": (I, []),
            "coxs_warp_shfl": (I, [P, P, I64, I, C.c_int32, P, I, P]),
            "coxs_warp_vote": (I, [P, P, I64, P, P]),
            "coxs_reduce_blocks_i32": (I, [P, I64, P, P]),
            "coxs_reduce": (I, [P, I, I64, I, I, I, P, P]),
            "coxs_dot": (I, [P, P, I, I64, I, I, I, P, P]),
            "coxs_scan_i32": (I, [P, P, I64, I, I]),
            "coxs_compact_i32": (I, [P, I64, P, P, I, I]),
            "coxs_tile_sort_u32": (I, [P, P, I64, I]),
            "coxs_tile_reduce_i32": (I, [P, I64, I, P]),
            "coxs_warp_masked": (I, [P, I64, I, P, P]),
            "coxs_segmented": (I, [P, I, P, I64, I, I, P, P, P, P]),
            "coxs_vote_bench": (I, [I, I64, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _libs[isa] = L
    return _libs[isa]


class CoxsError(RuntimeError):
    pass


def _check(code, what):
    if code != 0:
        raise CoxsError(f"{what}: status {code}")


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _dt_code(a):
    if a.dtype == np.int32:
        return I32
    if a.dtype == np.float32:
        return F32
    if a.dtype == np.uint16:
        return BF16
    raise TypeError(f"unsupported dtype {a.dtype}")


def set_threads(n, isa=None):
    return lib(isa).coxs_set_threads(int(n))


def warp_shfl(v, op, arg=0, width=32, mask=None, argv=None, isa=None):
    v = _c(v, np.int32)
    out = np.empty_like(v)
    m = None if mask is None else _c(mask, np.uint32)
    av = None if argv is None else _c(argv, np.int32)
    _check(lib(isa).coxs_warp_shfl(_p(v), _p(out), v.size, op, int(arg), _p(av), width, _p(m)), "warp_shfl")
    return out


def warp_vote(pred, mask=None, isa=None):
    pred = _c(pred, np.int32)
    g = pred.size // 32
    bal = np.zeros(g, np.uint32)
    aa = np.zeros(g, np.int32)
    m = None if mask is None else _c(mask, np.uint32)
    _check(lib(isa).coxs_warp_vote(_p(pred), _p(m), pred.size, _p(bal), _p(aa)), "warp_vote")
    return bal, aa


def reduce_blocks_i32(x, isa=None):
    x = _c(x, np.int32)
    bs = np.zeros((x.size + 255) // 256, np.int32)
    wc = np.zeros((x.size + 31) // 32, np.int32)
    _check(lib(isa).coxs_reduce_blocks_i32(_p(x), x.size, _p(bs), _p(wc)), "reduce_blocks_i32")
    return bs, wc


def _nchunks(n, k, W):
    S = 32 * W * k
    return (n + S - 1) // S


def reduce(x, k, W, acc=PLAIN, isa=None):
    x = np.ascontiguousarray(x)
    dt = _dt_code(x)
    nch = _nchunks(x.size, k, W)
    if dt == I32:
        part, tot = np.zeros(nch, np.int32), np.zeros(1, np.int64)
    else:
        part, tot = np.zeros(nch * (2 if acc == TWOSUM else 1), np.float32), np.zeros(1, np.float64)
    _check(lib(isa).coxs_reduce(_p(x), dt, x.size, acc, k, W, _p(part), _p(tot)), "reduce")
    if acc == TWOSUM:
        part = part.reshape(nch, 2)
    return part, tot[0]


def dot(a, b, k, W, acc=PLAIN, isa=None):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    assert a.dtype == b.dtype and a.size == b.size
    nch = _nchunks(a.size, k, W)
    part, tot = np.zeros(nch * (2 if acc == TWOSUM else 1), np.float32), np.zeros(1, np.float64)
    _check(lib(isa).coxs_dot(_p(a), _p(b), _dt_code(a), a.size, acc, k, W, _p(part), _p(tot)), "dot")
    if acc == TWOSUM:
        part = part.reshape(nch, 2)
    return part, tot[0]


def scan_i32(x, k, W, isa=None):
    x = _c(x, np.int32)
    y = np.empty_like(x)
    _check(lib(isa).coxs_scan_i32(_p(x), _p(y), x.size, k, W), "scan_i32")
    return y


def compact_i32(x, k, W, isa=None):
    x = _c(x, np.int32)
    out = np.empty_like(x)
    cnt = np.zeros(1, np.int64)
    _check(lib(isa).coxs_compact_i32(_p(x), x.size, _p(out), _p(cnt), k, W), "compact_i32")
    return out[: int(cnt[0])], int(cnt[0])


def tile_sort_u32(keys, group=32, isa=None):
    keys = _c(keys, np.uint32)
    out = np.empty_like(keys)
    _check(lib(isa).coxs_tile_sort_u32(_p(keys), _p(out), keys.size, group), "tile_sort_u32")
    return out


def tile_reduce_i32(x, tile, isa=None):
    x = _c(x, np.int32)
    out = np.zeros((x.size + tile - 1) // tile, np.int32)
    _check(lib(isa).coxs_tile_reduce_i32(_p(x), x.size, tile, _p(out)), "tile_reduce_i32")
    return out


def warp_masked(x, D, isa=None):
    x = _c(x, np.int32)
    out = np.empty_like(x)
    rec = np.zeros(4 * (x.size // 32), np.uint32)
    _check(lib(isa).coxs_warp_masked(_p(x), x.size, D, _p(out), _p(rec)), "warp_masked")
    return out, rec.reshape(-1, 4)


def segmented(x, offsets, k, W, isa=None):
    x = np.ascontiguousarray(x)
    dt = _dt_code(x)
    off = _c(offsets, np.int64)
    nseg = off.size - 1
    tot = np.zeros(nseg, np.int64 if dt == I32 else np.float64)
    y, oc = np.zeros_like(x), np.zeros_like(x)
    cnt = np.zeros(nseg, np.int64)
    _check(lib(isa).coxs_segmented(_p(x), dt, _p(off), nseg, k, W, _p(tot), _p(y), _p(oc), _p(cnt)), "segmented")
    return tot, y, oc, cnt


def vote_bench(op, iters=10_000_000, isa=None):
    """Nanoseconds per call of the warp_any (op 0) / warp_all (op 1)
    builtin over a 32-entry flag array."""
    ns, chk = C.c_double(), C.c_int64()
    _check(lib(isa).coxs_vote_bench(int(op), int(iters), C.byref(ns), C.byref(chk)), "vote_bench")
    return ns.value
