"""Thin ctypes binding over libcox.so (the C ABI declared in include/cox.h).

Every function here only marshals arguments: it checks tensor dtype, device
and contiguity, allocates outputs and workspaces with torch (device memory
plumbing), passes raw device pointers and torch's current HIP stream to the
C entry point of the same name, and raises ``CoxError`` on a nonzero
status.  All computation happens in the library's HIP kernels; there is no
CPU fallback.  If libcox.so has not been built, loading raises.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcox.so")

I32, U32, F32, BF16 = 0, 1, 2, 3
PLAIN, TWOSUM = 0, 1
SHFL_IDX, SHFL_UP, SHFL_DOWN, SHFL_XOR = 0, 1, 2, 3
OP_REDUCE, OP_DOT, OP_SCAN, OP_COMPACT, OP_SEGMENTED, OP_CG, OP_GRID_EXCHANGE, OP_INTEGRAL_IMAGE = range(8)
CG_CONVERGED, CG_MAX_ITER, CG_BREAKDOWN, CG_ABORTED = 0, 1, 2, 3

ERR_TIMEOUT = 7


class CoxError(RuntimeError):
    def __init__(self, code, what, lib=None):
        msg = f"{what}: status {code}"
        if lib is not None:
            msg += f" ({lib.cox_status_string(code).decode()})"
            if code == 4:
                msg += f", hipError {lib.cox_last_hip_error()}"
        super().__init__(msg)
        self.code = code


class cox_cfg(C.Structure):
    _fields_ = [("items_per_lane", C.c_int32), ("warps_per_block", C.c_int32),
                ("grid_blocks", C.c_int32), ("reserved", C.c_int32)]


_lib = None

_P, _I64, _I, _SZ = C.c_void_p, C.c_int64, C.c_int, C.c_size_t
_SIGS = {
    "cox_status_string": (C.c_char_p, [_I]),
    "cox_last_hip_error": (_I, []),
    "cox_version": (_I, []),
    "cox_default_cfg": (_I, [_I, _I, C.POINTER(cox_cfg)]),
    "cox_workspace_bytes": (_SZ, [_I, _I, _I64, _I64, C.POINTER(cox_cfg)]),
    "cox_workspace_init": (_I, [_P, _SZ, _P]),
    "cox_workspace_status": (_I, [_P, _P]),
    "cox_warp_shfl": (_I, [_P, _P, _I64, _I, C.c_int32, _P, _I, _P, _P]),
    "cox_warp_vote": (_I, [_P, _P, _I64, _P, _P, _P]),
    "cox_tile_vote": (_I, [_P, _I64, _I, _P, _P, _P]),
    "cox_warp_reduce_blocks_i32": (_I, [_P, _I64, _P, _P, _P]),
    "cox_warp_reduce": (_I, [_P, _I, _I64, _I, C.POINTER(cox_cfg), _P, _P, _P, _SZ, _P]),
    "cox_warp_dot": (_I, [_P, _P, _I, _I64, _I, C.POINTER(cox_cfg), _P, _P, _P, _SZ, _P]),
    "cox_warp_scan": (_I, [_P, _P, _I64, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_warp_scan_noalloc": (_I, [_P, _P, _I64, C.POINTER(cox_cfg), _P, _P]),
    "cox_ballot_compact": (_I, [_P, _I64, _P, _P, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_tile_sort": (_I, [_P, _P, _I64, _I, C.POINTER(cox_cfg), _P]),
    "cox_tile_sort_kv": (_I, [_P, _P, _P, _P, _I64, _I, C.POINTER(cox_cfg), _P]),
    "cox_tile_reduce": (_I, [_P, _I64, _I, _P, _P]),
    "cox_warp_masked": (_I, [_P, _I64, _I, _P, _P, _P]),
    "cox_warp_dynamic": (_I, [_P, _I64, _I, _P, _P, _P, _P, _P, _P]),
    "cox_segmented": (_I, [_P, _I, _P, _I64, _I64, _P, _P, _P, _P, _I, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_segmented_reduce": (_I, [_P, _I, _P, _I64, _I64, _P, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_segmented_scan": (_I, [_P, _I, _P, _I64, _I64, _P, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_segmented_compact": (_I, [_P, _I, _P, _I64, _I64, _P, _P, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_segmented_fused": (_I, [_P, _I, _P, _I64, _I64, _P, _P, _P, _P, C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_segmented_per_segment": (_I, [_P, _I, _P, _P, _I64, _I64, _P, _P, _P, _P, C.POINTER(cox_cfg), _P,
                                       _SZ, _P]),
    "cox_plan_segmented": (_I, [_P, _I, _P, _I64, _I64, _P, _P, _P, _P, _I, C.POINTER(cox_cfg), _I, _P, _SZ, _P,
                                C.POINTER(C.c_void_p)]),
    "cox_plan_execute": (_I, [_P, _P]),
    "cox_plan_get_cfg": (_I, [_P, C.POINTER(cox_cfg)]),
    "cox_plan_destroy": (_I, [_P]),
    "cox_integral_image": (_I, [_P, _I64, _I64, _P, _P, _SZ, _P]),
    "cox_grid_capacity": (_I, [C.POINTER(C.c_int32)]),
    "cox_grid_exchange": (_I, [C.c_int32, C.c_int32, _P, _P, _SZ, _P]),
    "cox_grid_exchange_absent": (_I, [C.c_int32, C.c_int32, C.c_int32, C.c_uint32, _P, _P, _SZ, _P]),
    "cox_cg_solve": (_I, [_P, _P, _P, _I64, _I64, _P, _P, C.c_int32, C.c_double, _P, _P, C.POINTER(cox_cfg), _P,
                          _SZ, _P]),
    "cox_cg_solve_per_phase": (_I, [_P, _P, _P, _I64, _I64, _P, _P, C.c_int32, C.c_double, _P, _P,
                                    C.POINTER(cox_cfg), _P, _SZ, _P]),
    "cox_stream_read": (_I, [_P, _SZ, _P, C.c_int32, _P]),
    "cox_stream_copy": (_I, [_P, _P, _SZ, C.c_int32, _P]),
}


def lib():
    """Loads libcox.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _check(code, what):
    if code != 0:
        raise CoxError(code, what, lib())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _dtype_code(t):
    if t.dtype == torch.int32:
        return I32
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


def make_cfg(items_per_lane=0, warps_per_block=0, grid_blocks=0):
    return cox_cfg(int(items_per_lane), int(warps_per_block), int(grid_blocks), 0)


def _cfgp(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, (tuple, list)):
        cfg = make_cfg(*cfg)
    return C.byref(cfg)


def default_cfg(op, dtype=I32):
    c = cox_cfg()
    _check(lib().cox_default_cfg(op, dtype, C.byref(c)), "cox_default_cfg")
    return (c.items_per_lane, c.warps_per_block, c.grid_blocks)


# ---------------------------------------------------------------- workspaces
class Workspace:
    """A zero-initialised device workspace owned by the caller."""

    def __init__(self, nbytes, device=None):
        nbytes = max(256, (int(nbytes) + 255) // 256 * 256)
        self.tensor = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
        self.nbytes = nbytes
        _check(lib().cox_workspace_init(_ptr(self.tensor), nbytes, _stream()), "cox_workspace_init")

    def status(self):
        """Synchronises the stream; raises CoxError(COX_ERR_TIMEOUT) if a
        bounded cross-block wait gave up since the last check."""
        _check(lib().cox_workspace_status(_ptr(self.tensor), _stream()), "cox_workspace_status")


_ws_cache = {}


def workspace(op, dtype, n, nseg=0, cfg=None, device=None):
    """Per-(op, device) cached workspace large enough for this call."""
    need = lib().cox_workspace_bytes(op, dtype, int(n), int(nseg), _cfgp(cfg))
    if need == 0:
        raise CoxError(1, "cox_workspace_bytes", lib())
    dev = torch.device(device or "cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = (op, dev.index)
    ws = _ws_cache.get(key)
    if ws is None or ws.nbytes < need:
        ws = Workspace(need, dev)
        _ws_cache[key] = ws
    return ws


# ---------------------------------------------------------------- entry points
def warp_shfl(v, op, arg=0, width=32, mask=None, argv=None, out=None):
    _need(v, torch.int32, "v")
    n = v.numel()
    out = torch.empty_like(v) if out is None else out
    if mask is not None:
        _need(mask, torch.int32, "mask")  # uint32 bits carried in int32
    if argv is not None:
        _need(argv, torch.int32, "argv")
    _check(lib().cox_warp_shfl(_ptr(v), _ptr(out), n, int(op), int(arg), _ptr(argv), int(width),
                               _ptr(mask), _stream()), "cox_warp_shfl")
    return out


def warp_vote(pred, mask=None):
    _need(pred, torch.int32, "pred")
    g = pred.numel() // 32
    bal = torch.zeros(g, dtype=torch.int32, device=pred.device)
    aa = torch.zeros(g, dtype=torch.int32, device=pred.device)
    if mask is not None:
        _need(mask, torch.int32, "mask")
    _check(lib().cox_warp_vote(_ptr(pred), _ptr(mask), pred.numel(), _ptr(bal), _ptr(aa), _stream()),
           "cox_warp_vote")
    return bal, aa


def tile_vote(pred, tile):
    """Per tile of `tile` lanes: (T-bit ballot, any | all << 1) as int32
    device tensors of n / tile entries."""
    _need(pred, torch.int32, "pred")
    g = pred.numel() // tile if tile > 0 else 0
    bal = torch.zeros(g, dtype=torch.int32, device=pred.device)
    aa = torch.zeros(g, dtype=torch.int32, device=pred.device)
    _check(lib().cox_tile_vote(_ptr(pred), pred.numel(), int(tile), _ptr(bal), _ptr(aa), _stream()),
           "cox_tile_vote")
    return bal, aa


def warp_reduce_blocks_i32(x, block_sums=None, warp_pos_count=None):
    _need(x, torch.int32, "x")
    n = x.numel()
    if block_sums is None:
        block_sums = torch.empty((n + 255) // 256, dtype=torch.int32, device=x.device)
    if warp_pos_count is None:
        warp_pos_count = torch.empty((n + 31) // 32, dtype=torch.int32, device=x.device)
    _check(lib().cox_warp_reduce_blocks_i32(_ptr(x), n, _ptr(block_sums), _ptr(warp_pos_count), _stream()),
           "cox_warp_reduce_blocks_i32")
    return block_sums, warp_pos_count


def _kw(cfg):
    if cfg is None:
        return 0, 0
    if isinstance(cfg, (tuple, list)):
        return (tuple(cfg) + (0, 0))[:2]
    return cfg.items_per_lane, cfg.warps_per_block


def _nchunks(n, cfg, op, dt):
    k, W = _kw(cfg)
    dk, dW, _ = default_cfg(op, dt)
    k, W = k or dk, W or dW
    S = 32 * W * k
    return (n + S - 1) // S


def warp_reduce(x, acc=PLAIN, cfg=None, partials=True, total=None, partials_out=None):
    """Returns (total, chunk_partials or None) as device tensors: total is
    int64 for int32 input, float64 otherwise."""
    dt = _dtype_code(x)
    _need(x, x.dtype, "x")
    n = x.numel()
    if total is None:
        total = torch.empty(1, dtype=torch.int64 if dt == I32 else torch.float64, device=x.device)
    part = partials_out
    if part is None and partials:
        nch = _nchunks(n, cfg, OP_REDUCE, dt)
        shape = (nch, 2) if acc == TWOSUM else (nch,)
        part = torch.empty(shape, dtype=torch.int32 if dt == I32 else torch.float32, device=x.device)
    ws = workspace(OP_REDUCE, dt, n, cfg=cfg, device=x.device)
    _check(lib().cox_warp_reduce(_ptr(x), dt, n, int(acc), _cfgp(cfg), _ptr(part), _ptr(total),
                                 _ptr(ws.tensor), ws.nbytes, _stream()), "cox_warp_reduce")
    return total, part


def warp_dot(a, b, acc=PLAIN, cfg=None, partials=True, total=None, partials_out=None):
    dt = _dtype_code(a)
    _need(a, a.dtype, "a")
    _need(b, a.dtype, "b")
    if a.numel() != b.numel():
        raise ValueError("a and b differ in size")
    n = a.numel()
    if total is None:
        total = torch.empty(1, dtype=torch.float64, device=a.device)
    part = partials_out
    if part is None and partials:
        nch = _nchunks(n, cfg, OP_DOT, dt)
        shape = (nch, 2) if acc == TWOSUM else (nch,)
        part = torch.empty(shape, dtype=torch.float32, device=a.device)
    ws = workspace(OP_DOT, dt, n, cfg=cfg, device=a.device)
    _check(lib().cox_warp_dot(_ptr(a), _ptr(b), dt, n, int(acc), _cfgp(cfg), _ptr(part), _ptr(total),
                              _ptr(ws.tensor), ws.nbytes, _stream()), "cox_warp_dot")
    return total, part


def warp_scan(x, cfg=None, out=None):
    _need(x, torch.int32, "x")
    n = x.numel()
    y = torch.empty_like(x) if out is None else out
    ws = workspace(OP_SCAN, I32, n, cfg=cfg, device=x.device)
    _check(lib().cox_warp_scan(_ptr(x), _ptr(y), n, _cfgp(cfg), _ptr(ws.tensor), ws.nbytes, _stream()),
           "cox_warp_scan")
    return y


def warp_scan_noalloc(x, cfg=None, out=None, err=None):
    """cox_warp_scan on the library's fixed device scratch (no workspace).
    err: optional 1-element int32 device tensor receiving the wait status."""
    _need(x, torch.int32, "x")
    y = torch.empty_like(x) if out is None else out
    if err is not None:
        _need(err, torch.int32, "err")
    _check(lib().cox_warp_scan_noalloc(_ptr(x), _ptr(y), x.numel(), _cfgp(cfg), _ptr(err), _stream()),
           "cox_warp_scan_noalloc")
    return y


def ballot_compact(x, cfg=None, out=None, count=None):
    """Returns (out buffer of capacity n, count as a 1-element int64 device
    tensor); the kept elements are out[:count]."""
    _need(x, torch.int32, "x")
    n = x.numel()
    out = torch.empty_like(x) if out is None else out
    count = torch.empty(1, dtype=torch.int64, device=x.device) if count is None else count
    ws = workspace(OP_COMPACT, I32, n, cfg=cfg, device=x.device)
    _check(lib().cox_ballot_compact(_ptr(x), n, _ptr(out), _ptr(count), _cfgp(cfg), _ptr(ws.tensor),
                                    ws.nbytes, _stream()), "cox_ballot_compact")
    return out, count


def tile_sort(keys, tile=32, cfg=None, out=None):
    """keys: int32 tensor holding uint32 bit patterns (sorted as unsigned)."""
    _need(keys, torch.int32, "keys")
    out = torch.empty_like(keys) if out is None else out
    _check(lib().cox_tile_sort(_ptr(keys), _ptr(out), keys.numel(), int(tile), _cfgp(cfg), _stream()),
           "cox_tile_sort")
    return out


def tile_sort_kv(keys, vals, cfg=None, out_keys=None, out_vals=None):
    """Stable sort of every 32-pair group by unsigned key (keys: int32 view
    of uint32 keys; vals: any 4-byte int32 / float32 tensor).  Returns
    (out_keys, out_vals)."""
    _need(keys, torch.int32, "keys")
    if vals.dtype not in (torch.int32, torch.float32):
        raise TypeError("vals must be a 4-byte tensor (int32 or float32)")
    _need(vals, vals.dtype, "vals")
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and vals differ in size")
    out_keys = torch.empty_like(keys) if out_keys is None else out_keys
    out_vals = torch.empty_like(vals) if out_vals is None else out_vals
    _check(lib().cox_tile_sort_kv(_ptr(keys), _ptr(vals), _ptr(out_keys), _ptr(out_vals), n, 32, _cfgp(cfg),
                                  _stream()), "cox_tile_sort_kv")
    return out_keys, out_vals


def tile_reduce(x, tile, out=None):
    _need(x, torch.int32, "x")
    n = x.numel()
    out = torch.empty((n + tile - 1) // tile, dtype=torch.int32, device=x.device) if out is None else out
    _check(lib().cox_tile_reduce(_ptr(x), n, int(tile), _ptr(out), _stream()), "cox_tile_reduce")
    return out


def warp_masked(x, density, out=None, rec=None):
    _need(x, torch.int32, "x")
    n = x.numel()
    out = torch.empty_like(x) if out is None else out
    rec = torch.empty((n // 32, 4), dtype=torch.int32, device=x.device) if rec is None else rec
    _check(lib().cox_warp_masked(_ptr(x), n, int(density), _ptr(out), _ptr(rec), _stream()),
           "cox_warp_masked")
    return out, rec


def warp_dynamic(x, density, match_any=None, rank=None, rec=None, filtered=None, count=None):
    """Dynamic groups (coalesced_threads, match_any / match_all, the six
    reduce_*_sync, warp-aggregated append).  Returns (match_any, rank,
    rec[n/32, 8], filtered (capacity n), count as a 1-element int64 device
    tensor); the members are filtered[:count]."""
    _need(x, torch.int32, "x")
    n = x.numel()
    dev = x.device
    match_any = torch.empty(n, dtype=torch.int32, device=dev) if match_any is None else match_any
    rank = torch.empty(n, dtype=torch.int32, device=dev) if rank is None else rank
    rec = torch.empty((n // 32, 8), dtype=torch.int32, device=dev) if rec is None else rec
    filtered = torch.empty_like(x) if filtered is None else filtered
    count = torch.empty(1, dtype=torch.int64, device=dev) if count is None else count
    _check(lib().cox_warp_dynamic(_ptr(x), n, int(density), _ptr(match_any), _ptr(rank), _ptr(rec), _ptr(filtered),
                                  _ptr(count), _stream()), "cox_warp_dynamic")
    return match_any, rank, rec, filtered, count


def integral_image(img, out=None):
    """Summed-area table (mod 2^32) of a uint8 device image [H, W]; returns
    an int32 tensor holding the uint32 sums."""
    _need(img, torch.uint8, "img")
    if img.dim() != 2:
        raise ValueError("img must be 2-D [height, width]")
    H, W = img.shape
    out = torch.empty((H, W), dtype=torch.int32, device=img.device) if out is None else out
    ws = workspace(OP_INTEGRAL_IMAGE, U32, H, W)
    _check(lib().cox_integral_image(_ptr(img), H, W, _ptr(out), _ptr(ws.tensor), ws.nbytes, _stream()),
           "cox_integral_image")
    return out


def grid_capacity():
    """Largest grid of 1024-thread blocks a cooperative launch can hold."""
    v = C.c_int32()
    _check(lib().cox_grid_capacity(C.byref(v)), "cox_grid_capacity")
    return v.value


def grid_exchange(grid_blocks, rounds, out=None):
    """Exchange kernel over a grid barrier; returns uint32 sums as an int32
    device tensor [grid_blocks, 1024].  The workspace's timeout flag is
    checked (synchronising)."""
    out = torch.empty((grid_blocks, 1024), dtype=torch.int32, device="cuda") if out is None else out
    ws = workspace(OP_GRID_EXCHANGE, U32, grid_blocks)
    _check(lib().cox_grid_exchange(int(grid_blocks), int(rounds), _ptr(out), _ptr(ws.tensor), ws.nbytes, _stream()),
           "cox_grid_exchange")
    ws.status()
    return out


def grid_exchange_absent(grid_blocks, rounds, absent_block, spin_limit):
    """The exchange kernel with one block absent from the first barrier and
    a small spin bound: returns the workspace status afterwards (expected
    COX_ERR_TIMEOUT); synchronises."""
    out = torch.empty((grid_blocks, 1024), dtype=torch.int32, device="cuda")
    ws = workspace(OP_GRID_EXCHANGE, U32, grid_blocks)
    _check(lib().cox_grid_exchange_absent(int(grid_blocks), int(rounds), int(absent_block), int(spin_limit),
                                          _ptr(out), _ptr(ws.tensor), ws.nbytes, _stream()),
           "cox_grid_exchange_absent")
    return lib().cox_workspace_status(_ptr(ws.tensor), _stream())


def cg_solve(row_ptr, col_idx, val, b, x, max_iter, tol=0.0, cfg=None, rr_hist=None, result=None,
             per_phase=False):
    """Conjugate gradient on the CSR system (row_ptr, col_idx, val) x = b,
    updating the float32 device tensor x in place (it holds x_0 on entry).
    One cooperative launch, or one launch per phase with per_phase=True.
    Returns (result, rr_hist): result = int32 device tensor {iterations,
    reason}, rr_hist = float64 device tensor [max_iter + 1]."""
    _need(row_ptr, torch.int32, "row_ptr")
    _need(col_idx, torch.int32, "col_idx")
    _need(val, torch.float32, "val")
    _need(b, torch.float32, "b")
    _need(x, torch.float32, "x")
    n, nnz = b.numel(), col_idx.numel()
    if row_ptr.numel() != n + 1 or val.numel() != nnz or x.numel() != n:
        raise CoxError(1, "cg_solve: inconsistent CSR / vector sizes")
    dev = b.device
    result = torch.zeros(2, dtype=torch.int32, device=dev) if result is None else result
    rr_hist = torch.zeros(max_iter + 1, dtype=torch.float64, device=dev) if rr_hist is None else rr_hist
    ws = workspace(OP_CG, F32, n, cfg=cfg)
    fn = lib().cox_cg_solve_per_phase if per_phase else lib().cox_cg_solve
    _check(fn(_ptr(row_ptr), _ptr(col_idx), _ptr(val), n, nnz, _ptr(b), _ptr(x), int(max_iter), float(tol),
              _ptr(result), _ptr(rr_hist), _cfgp(cfg), _ptr(ws.tensor), ws.nbytes, _stream()),
           "cox_cg_solve_per_phase" if per_phase else "cox_cg_solve")
    return result, rr_hist


def stream_read(x, sink=None, grid_blocks=0):
    """Bandwidth reference: reads every byte of tensor x once."""
    sink = torch.zeros(1, dtype=torch.int32, device=x.device) if sink is None else sink
    _check(lib().cox_stream_read(_ptr(x), x.numel() * x.element_size(), _ptr(sink), int(grid_blocks),
                                 _stream()), "cox_stream_read")
    return sink


def stream_copy(src, dst, grid_blocks=0):
    """Bandwidth reference: copies src into dst (same byte size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("size mismatch")
    _check(lib().cox_stream_copy(_ptr(src), _ptr(dst), nb, int(grid_blocks), _stream()), "cox_stream_copy")
    return dst


# ---------------------------------------------------------------- segmented
SEG_REDUCE, SEG_SCAN, SEG_COMPACT = 1, 2, 4

# the plan autotuner's candidates all use chunks of at least 4096 elements
_SEG_MIN_CHUNK_CFG = (8, 16)


def _seg_outputs(x, offsets, which, seg_total, y, out, seg_count):
    dt = _dtype_code(x)
    nseg = offsets.numel() - 1
    dev = x.device
    if which & SEG_REDUCE and seg_total is None:
        seg_total = torch.empty(nseg, dtype=torch.int64 if dt == I32 else torch.float64, device=dev)
    if which & SEG_SCAN and y is None:
        y = torch.empty_like(x)
    if which & SEG_COMPACT:
        if out is None:
            out = torch.zeros_like(x)
        if seg_count is None:
            seg_count = torch.empty(nseg, dtype=torch.int64, device=dev)
    return dt, nseg, seg_total, y, out, seg_count


def segmented(x, offsets, which=7, cfg=None, seg_total=None, y=None, out=None, seg_count=None):
    """Segmented totals / scan / compaction over CSR offsets (device int64,
    nseg + 1 entries) in one fused launch.  Returns (seg_total, y, out,
    seg_count) with None for outputs not selected by `which`."""
    _need(offsets, torch.int64, "offsets")
    if x.dtype not in (torch.int32, torch.float32):
        raise TypeError("x must be int32 or float32")
    _need(x, x.dtype, "x")
    dt, nseg, seg_total, y, out, seg_count = _seg_outputs(x, offsets, which, seg_total, y, out, seg_count)
    ws = workspace(OP_SEGMENTED, dt, x.numel(), nseg, cfg=cfg, device=x.device)
    _check(lib().cox_segmented(_ptr(x), dt, _ptr(offsets), nseg, x.numel(), _ptr(seg_total), _ptr(y), _ptr(out),
                               _ptr(seg_count), int(which), _cfgp(cfg), _ptr(ws.tensor), ws.nbytes, _stream()),
           "cox_segmented")
    return seg_total, y, out, seg_count


def segmented_per_segment(x, offsets, offsets_host, cfg=None, seg_total=None, y=None, out=None, seg_count=None):
    """Baseline: the fused kernel launched once per segment."""
    _need(offsets, torch.int64, "offsets")
    _need(x, x.dtype, "x")
    oh = offsets_host.contiguous()
    dt, nseg, seg_total, y, out, seg_count = _seg_outputs(x, offsets, 7, seg_total, y, out, seg_count)
    ws = workspace(OP_SEGMENTED, dt, x.numel(), nseg, cfg=cfg, device=x.device)
    _check(lib().cox_segmented_per_segment(_ptr(x), dt, _ptr(offsets), C.c_void_p(oh.data_ptr()), nseg, x.numel(),
                                           _ptr(seg_total), _ptr(y), _ptr(out), _ptr(seg_count), _cfgp(cfg),
                                           _ptr(ws.tensor), ws.nbytes, _stream()), "cox_segmented_per_segment")
    return seg_total, y, out, seg_count


class Plan:
    """A segmented call bound to its buffers and captured in a hipGraph;
    execute() replays it on torch's current stream."""

    def __init__(self, x, offsets, which=7, cfg=None, autotune=True, seg_total=None, y=None, out=None,
                 seg_count=None):
        _need(offsets, torch.int64, "offsets")
        _need(x, x.dtype, "x")
        dt, nseg, self.seg_total, self.y, self.out, self.seg_count = _seg_outputs(
            x, offsets, which, seg_total, y, out, seg_count)
        self.x, self.offsets = x, offsets
        wcfg = cfg if cfg is not None and any(_kw(cfg)) else _SEG_MIN_CHUNK_CFG
        nbytes = lib().cox_workspace_bytes(OP_SEGMENTED, dt, x.numel(), nseg, _cfgp(wcfg))
        forced = os.environ.get("COX_FORCE_CFG", "")
        if forced and (cfg is None or not any(_kw(cfg)[:2])):
            # the library takes this schedule when the caller gives none
            try:
                fk = [int(v) for v in forced.split(",")][:3]
                nbytes = max(nbytes, lib().cox_workspace_bytes(OP_SEGMENTED, dt, x.numel(), nseg,
                                                               _cfgp(tuple(fk[:2]))))
            except ValueError:
                pass
        self.ws = Workspace(nbytes, x.device)  # a plan owns its workspace
        h = C.c_void_p()
        _check(lib().cox_plan_segmented(_ptr(x), dt, _ptr(offsets), nseg, x.numel(), _ptr(self.seg_total),
                                        _ptr(self.y), _ptr(self.out), _ptr(self.seg_count), int(which), _cfgp(cfg),
                                        int(bool(autotune)), _ptr(self.ws.tensor), self.ws.nbytes, _stream(),
                                        C.byref(h)), "cox_plan_segmented")
        self.handle = h

    def execute(self):
        _check(lib().cox_plan_execute(self.handle, _stream()), "cox_plan_execute")
        return self.seg_total, self.y, self.out, self.seg_count

    def cfg(self):
        c = cox_cfg()
        _check(lib().cox_plan_get_cfg(self.handle, C.byref(c)), "cox_plan_get_cfg")
        return (c.items_per_lane, c.warps_per_block, c.grid_blocks)

    def close(self):
        if getattr(self, "handle", None):
            lib().cox_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
