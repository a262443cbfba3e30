"""Seeded synthetic inputs for the five warp-primitive workloads.

This module holds only random-number recipes (numpy PCG64 streams); it does
none of the kernels' arithmetic.  Both the GPU tests and the CPU oracle's
tests draw their inputs from here, so the two sides see the same bits.

Each workload gets its own seed (``BASE_SEED + index``) and each array of a
workload its own child stream of ``SeedSequence(seed).spawn(...)``, in the
order the arrays are listed below.

Workloads (element counts are the full sizes; every generator takes ``n``
so tests can draw smaller instances from the same recipe):

0. block reduce: int32 uniform in [-1000, 1000], n = 2^20.
1. primitive set: int32 uniform in [-2^20, 2^20]; uint32 uniform keys;
   float32 N(0, 1); n = 2^28.
2. masked / tile: int32 uniform in [-2^20, 2^20], n = 2^26.
3. precision: float32 / bfloat16 with magnitudes 10^U(-3, 3), random signs,
   built from cancelling pairs so that the condition number
   sum|x| / |sum x| is about 1e8; n = 2^28.
4. segments: 10,000 segment lengths min(round(lognormal(ln 2000, 1.97)),
   2^20); int32 uniform in [-2^20, 2^20] and float32 N(0, 1) values.
5. conjugate gradient systems (CSR, float32 values, columns ascending in
   each row):
   - tridiagonal: off-diagonal pairs a(i, i+1) = a(i+1, i) = -U[0, 1),
     diagonal 3 + U[0, 1) (strictly diagonally dominant, hence positive
     definite, eigenvalues in (1, 6)); right-hand side U[-1, 1); n = 2^20
     rows and 2^24;
   - irregular: about n * deg / 2 off-diagonal pairs (i, j), i != j, with i
     drawn as floor(n * U^2) (so low rows are long) and j uniform, value
     -U[0, 1) mirrored to (j, i) (duplicate pairs stay as separate
     entries); diagonal 1 + U[0, 1) + the row's sum of |off-diagonal|;
     right-hand side U[-1, 1).
6. integral image: uint8 pixels uniform in [0, 255], row-major [H, W];
   8192 x 8192 for the benchmark, ragged shapes for the tests.
"""
import numpy as np

BASE_SEED = 2112100340

FULL_N = {0: 1 << 20, 1: 1 << 28, 2: 1 << 26, 3: 1 << 28}
CG_N = (1 << 20, 1 << 24)
IMAGE_HW = (8192, 8192)
NSEG = 10_000
SEG_MEDIAN = 2000
SEG_SIGMA = 1.97
SEG_CAP = 1 << 20


def _streams(index, count, seed=None):
    s = BASE_SEED + index if seed is None else seed
    return [np.random.Generator(np.random.PCG64(c)) for c in np.random.SeedSequence(s).spawn(count)]


def block_reduce_input(n=FULL_N[0], seed=None):
    (g,) = _streams(0, 1, seed)
    return g.integers(-1000, 1001, size=n, dtype=np.int32)


def primitive_inputs(n=FULL_N[1], seed=None):
    """(x_i32, keys_u32, x_f32) of workload 1."""
    g_i, g_k, g_f = _streams(1, 3, seed)
    x = g_i.integers(-(1 << 20), (1 << 20) + 1, size=n, dtype=np.int32)
    keys = g_k.integers(0, 1 << 32, size=n, dtype=np.uint32)
    f = g_f.standard_normal(size=n, dtype=np.float32)
    return x, keys, f


def masked_input(n=FULL_N[2], seed=None):
    (g,) = _streams(2, 1, seed)
    return g.integers(-(1 << 20), (1 << 20) + 1, size=n, dtype=np.int32)


# densities of the masked workload: predicate ((uint32)x & 1023) < D
MASK_DENSITIES = (102, 512, 922)
TILE_SIZES = (4, 8, 16, 32)


def _to_bf16_bits(a32):
    """Round float32 to bfloat16 (nearest even) and return the uint16 bits."""
    u = a32.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_to_f32(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32)


def _loguniform(g, m):
    return np.power(10.0, g.uniform(-3.0, 3.0, size=m))


_BLK = 1 << 20  # elements per block of the precision generator's passes


def _slices(m):
    for a in range(0, m, _BLK):
        yield slice(a, min(a + _BLK, m))


def _scatter(parts, perm):
    """The concatenation of ``parts``, element j placed at position perm[j]."""
    out = np.empty(perm.size, parts[0].dtype)
    o = 0
    for p in parts:
        out[perm[o:o + p.size]] = p
        o += p.size
    return out


def precision_inputs(n=FULL_N[3], seed=None, target=1e8, kind="sum", dtype="f32"):
    """Cancelling data of workload 3.

    kind="sum": returns (x, info); kind="dot": returns (a, b, info).
    float32: half the values x_i are drawn, each is paired with
    -fl32(x_i (1 + eps u_i)), u_i ~ U(-1, 1), and eps is rescaled until the
    measured condition number is within a factor 2 of ``target``.
    bfloat16: the partner is -x_i, with its magnitude moved by one bfloat16
    ulp (random direction) on the first j pairs (pairs are i.i.d., so these
    are a random subset); j is the prefix whose condition number is closest
    to the target.  Dots pair (a, b) with (-a, b') where b' is b perturbed
    the same way.  The pairs' elements are scattered to the positions of one
    seeded shuffle of 0..n-1.  ``info`` records eps or j / (n/2) and the
    achieved condition number sum|t| / |sum t| over the terms t, summed in
    float64 pair by pair (the exact reference comes from the oracle's exact
    accumulator, not from here).  The passes run over blocks of 2^20 pairs
    so that full-size inputs need few large temporaries.
    """
    assert n % 2 == 0
    h = n // 2
    g_mag, g_sgn, g_del, g_perm, g_b, g_dir = _streams(3, 6, seed)
    mag = g_mag.uniform(-3.0, 3.0, size=h)
    np.power(10.0, mag, out=mag)
    np.negative(mag, out=mag, where=g_sgn.integers(0, 2, size=h, dtype=np.uint8) == 0)
    u = g_del.uniform(-1.0, 1.0, size=h)
    perm = np.arange(n, dtype=np.int32 if n < (1 << 31) else np.int64)
    g_perm.shuffle(perm)
    bmag = None
    if kind == "dot":
        bmag = g_b.uniform(-3.0, 3.0, size=h)
        np.power(10.0, bmag, out=bmag)
    ddir = (g_dir.integers(0, 2, size=h, dtype=np.int8) * 2 - 1).astype(np.int8)

    if dtype == "f32":
        xa = mag.astype(np.float32)
        bb = bmag.astype(np.float32) if kind == "dot" else None
        del mag, bmag

        def build(eps, keep):
            # float32 x float32 products and sums of two float32 are exact in float64
            part = np.empty(h, np.float32) if keep else None
            tot = absum = 0.0
            for sl in _slices(h):
                x64 = xa[sl].astype(np.float64)
                f = 1.0 + eps * u[sl]
                if kind == "sum":
                    q = (-(x64 * f)).astype(np.float32)
                    q64 = q.astype(np.float64)
                    tot += float(np.sum(x64 + q64))
                    absum += float(np.abs(x64).sum() + np.abs(q64).sum())
                else:
                    b64 = bb[sl].astype(np.float64)
                    q = (b64 * f).astype(np.float32)
                    q64 = q.astype(np.float64)
                    tot += float(np.sum(x64 * b64 - x64 * q64))
                    absum += float((np.abs(x64) * (b64 + q64)).sum())
                if keep:
                    part[sl] = q
            return part, absum / max(abs(tot), 1e-300)

        # cond ~ 1/eps: rescale until within a factor 2 of the target
        p = 1e-4
        for it in range(6):
            _, c = build(p, False)
            if target / 2 <= c <= target * 2 or it == 5:
                break
            p = p * c / target
        part, c = build(p, True)
        info = {"param": p, "cond": c, "kind": kind, "dtype": dtype}
        if kind == "sum":
            return _scatter([xa, part], perm), info
        return _scatter([xa, -xa], perm), _scatter([bb, part], perm), info

    # bfloat16: pair i is nudged (its partner's magnitude moved by one
    # bfloat16 ulp in direction ddir_i) iff i < j.  Each pair contributes c_i
    # to the sum (0 when not nudged), so the sum over the first j pairs is a
    # prefix sum; j is the prefix whose condition number is closest to the
    # target.
    xa = _to_bf16_bits(mag.astype(np.float32))
    bb = _to_bf16_bits(bmag.astype(np.float32)) if kind == "dot" else None
    del mag, bmag

    def terms(sl, step):
        """float64 pair terms (first, partner) of pairs sl with the given nudges."""
        x64 = bf16_to_f32(xa[sl]).astype(np.float64)
        if kind == "sum":
            q = ((xa[sl] ^ 0x8000).astype(np.int32) + step).astype(np.uint16)  # -(x_i +/- 1 ulp)
            return x64, bf16_to_f32(q).astype(np.float64)
        b64 = bf16_to_f32(bb[sl]).astype(np.float64)
        q = (bb[sl].astype(np.int32) + step).astype(np.uint16)
        return x64 * b64, -x64 * bf16_to_f32(q).astype(np.float64)

    absum = 0.0
    for sl in _slices(h):
        t0, _ = terms(sl, 0)
        absum += 2.0 * float(np.abs(t0).sum())
    best, j, run = np.inf, 1, 0.0
    for sl in _slices(h):
        t0, t1 = terms(sl, ddir[sl])
        _, z1 = terms(sl, 0)
        pref = np.abs(run + np.cumsum((t0 + t1) - (t0 + z1)))
        run = run + float(np.sum((t0 + t1) - (t0 + z1)))
        with np.errstate(divide="ignore"):
            score = np.abs(np.log(np.maximum(pref, 1e-300) * target / absum))
        i = int(np.argmin(score))
        if score[i] < best:
            best, j = float(score[i]), sl.start + i + 1
    step = np.zeros(h, np.int8)
    step[:j] = ddir[:j]
    part = np.empty(h, np.uint16)
    tot = absum = 0.0
    for sl in _slices(h):
        t0, t1 = terms(sl, step[sl])
        tot += float(np.sum(t0 + t1))
        absum += float(np.abs(t0).sum() + np.abs(t1).sum())
        part[sl] = ((xa[sl] ^ 0x8000).astype(np.int32) + step[sl]).astype(np.uint16) if kind == "sum" else \
            (bb[sl].astype(np.int32) + step[sl]).astype(np.uint16)
    info = {"param": j / h, "cond": absum / max(abs(tot), 1e-300), "kind": kind, "dtype": dtype}
    if kind == "sum":
        return _scatter([xa, part], perm), info
    return _scatter([xa, xa ^ 0x8000], perm), _scatter([bb, part], perm), info


def segment_offsets(nseg=NSEG, seed=None, median=SEG_MEDIAN, sigma=SEG_SIGMA, cap=SEG_CAP):
    """CSR offsets (int64, nseg + 1 entries) of workload 4."""
    g_len, _, _ = _streams(4, 3, seed)
    lens = np.minimum(np.rint(g_len.lognormal(np.log(median), sigma, size=nseg)), cap)
    off = np.zeros(nseg + 1, np.int64)
    np.cumsum(lens.astype(np.int64), out=off[1:])
    return off


def segment_values(total, seed=None):
    """(x_i32, x_f32) of workload 4 for ``total`` elements."""
    _, g_i, g_f = _streams(4, 3, seed)
    x = g_i.integers(-(1 << 20), (1 << 20) + 1, size=total, dtype=np.int32)
    f = g_f.standard_normal(size=total, dtype=np.float32)
    return x, f


def _csr(rows, cols, vals, n):
    order = np.lexsort((cols, rows))
    rp = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return rp, cols[order].astype(np.int32), vals[order].astype(np.float32)


def cg_tridiag(n, seed=None):
    """(row_ptr, col_idx, val, b) of the tridiagonal system of workload 5."""
    g_off, g_diag, g_b = _streams(5, 3, seed)
    u = g_off.random(size=max(n - 1, 0), dtype=np.float32)
    d = np.float32(3) + g_diag.random(size=n, dtype=np.float32)
    b = g_b.random(size=n, dtype=np.float32) * np.float32(2) - np.float32(1)
    i = np.arange(n, dtype=np.int64)
    cols = np.stack([i - 1, i, i + 1], axis=1)
    vals = np.zeros((n, 3), np.float32)
    vals[1:, 0] = -u
    vals[:, 1] = d
    vals[:-1, 2] = -u
    valid = (cols >= 0) & (cols < n)
    rp = np.zeros(n + 1, np.int32)
    np.cumsum(valid.sum(axis=1), out=rp[1:])
    return rp, cols[valid].astype(np.int32), vals[valid], b


def cg_irregular(n, deg=6, seed=None):
    """(row_ptr, col_idx, val, b) of the irregular system of workload 5."""
    g_i, g_j, g_v, g_d, g_b = _streams(5, 5, None if seed is None else seed + 1)
    m = n * deg // 2
    i = np.floor(n * g_i.random(size=m) ** 2).astype(np.int64)
    j = g_j.integers(0, n, size=m, dtype=np.int64)
    keep = i != j
    i, j = i[keep], j[keep]
    v = -g_v.random(size=i.size, dtype=np.float32)
    rows = np.concatenate([i, j, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([j, i, np.arange(n, dtype=np.int64)])
    absrow = np.bincount(np.concatenate([i, j]), weights=np.abs(np.concatenate([v, v])).astype(np.float64),
                         minlength=n)
    diag = (1.0 + g_d.random(size=n) + absrow).astype(np.float32)
    vals = np.concatenate([v, v, diag])
    b = g_b.random(size=n, dtype=np.float32) * np.float32(2) - np.float32(1)
    rp, ci, va = _csr(rows, cols, vals, n)
    return rp, ci, va, b


def image_u8(H=IMAGE_HW[0], W=IMAGE_HW[1], seed=None):
    """uint8 image [H, W] of workload 6."""
    (g,) = _streams(6, 1, seed)
    return g.integers(0, 256, size=(H, W), dtype=np.uint8)
