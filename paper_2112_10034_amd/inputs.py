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
"""
import numpy as np

BASE_SEED = 2112100340

FULL_N = {0: 1 << 20, 1: 1 << 28, 2: 1 << 26, 3: 1 << 28}
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


def _cond(terms64):
    s = float(np.sum(terms64, dtype=np.float64))
    return float(np.sum(np.abs(terms64), dtype=np.float64)) / max(abs(s), 1e-300)


def precision_inputs(n=FULL_N[3], seed=None, target=1e8, kind="sum", dtype="f32"):
    """Cancelling data of workload 3.

    kind="sum": returns (x, info); kind="dot": returns (a, b, info).
    float32: half the values x_i are drawn, each is paired with
    -fl32(x_i (1 + eps u_i)), u_i ~ U(-1, 1), and eps is rescaled until the
    measured condition number is within a factor 2 of ``target``.
    bfloat16: the partner is -x_i, with its magnitude moved by one bfloat16
    ulp (random direction) on the fraction f of the pairs with the smallest
    u_i; f is chosen so that the condition number is closest to the target.
    Dots pair (a, b) with (-a, b') where b' is b perturbed the same way.  The arrays are
    shuffled with a seeded permutation.  ``info`` records eps or f and the
    achieved condition number, measured in float64 (the exact reference
    comes from the oracle's exact accumulator, not from here).
    """
    assert n % 2 == 0
    h = n // 2
    g_mag, g_sgn, g_del, g_perm, g_b, g_dir = _streams(3, 6, seed)
    mag = _loguniform(g_mag, h)
    sgn = np.where(g_sgn.integers(0, 2, size=h) == 1, 1.0, -1.0)
    u = g_del.uniform(-1.0, 1.0, size=h)
    perm = g_perm.permutation(n)
    bmag = _loguniform(g_b, h) if kind == "dot" else None
    ddir = np.where(g_dir.integers(0, 2, size=h) == 1, 1, -1).astype(np.int32)

    if dtype == "f32":
        xa = (sgn * mag).astype(np.float32)
        bb = bmag.astype(np.float32) if kind == "dot" else None

        def build(eps):
            if kind == "sum":
                xp = (-(xa.astype(np.float64) * (1.0 + eps * u))).astype(np.float32)
                v = np.concatenate([xa, xp])[perm]
                return (v,), v.astype(np.float64)
            a = np.concatenate([xa, -xa])[perm]
            bp = (bb.astype(np.float64) * (1.0 + eps * u)).astype(np.float32)
            b = np.concatenate([bb, bp])[perm]
            return (a, b), a.astype(np.float64) * b.astype(np.float64)

        # cond ~ 1/eps: rescale until within a factor 2 of the target
        p = 1e-4
        for _ in range(6):
            arrs, t = build(p)
            c = _cond(t)
            if target / 2 <= c <= target * 2:
                break
            p = p * c / target
        info = {"param": p, "cond": c, "kind": kind, "dtype": dtype}
        return (*arrs, info)

    # bfloat16: pair i is nudged (its partner's magnitude moved by one
    # bfloat16 ulp in direction ddir_i) iff u_i is below a threshold.  Each
    # pair contributes c_i to the sum (0 when not nudged), so ordering the
    # pairs by u turns the sum into a prefix sum; the threshold is the
    # prefix whose condition number is closest to the target.
    xa = _to_bf16_bits((sgn * mag).astype(np.float32))
    bb = _to_bf16_bits(bmag.astype(np.float32)) if kind == "dot" else None
    if kind == "sum":
        xa64 = bf16_to_f32(xa).astype(np.float64)
        moved = (xa.astype(np.int32) + ddir).astype(np.uint16)
        contrib = xa64 - bf16_to_f32(moved).astype(np.float64)
        absum = 2.0 * np.abs(xa64).sum()
    else:
        a64 = bf16_to_f32(xa).astype(np.float64)
        b64 = bf16_to_f32(bb).astype(np.float64)
        moved = (bb.astype(np.int32) + ddir).astype(np.uint16)
        contrib = a64 * b64 - a64 * bf16_to_f32(moved).astype(np.float64)
        absum = 2.0 * np.abs(a64 * b64).sum()
    order = np.argsort(u, kind="stable")
    pref = np.abs(np.cumsum(contrib[order]))
    with np.errstate(divide="ignore"):
        score = np.abs(np.log(np.maximum(pref, 1e-300) * target / absum))
    j = int(np.argmin(score)) + 1
    nudged = np.zeros(h, bool)
    nudged[order[:j]] = True
    step = np.where(nudged, ddir, 0).astype(np.int32)
    if kind == "sum":
        xp = ((xa ^ 0x8000).astype(np.int32) + step).astype(np.uint16)  # -(x_i +/- 1 ulp)
        v = np.concatenate([xa, xp])[perm]
        t = bf16_to_f32(v).astype(np.float64)
        arrs = (v,)
    else:
        a = np.concatenate([xa, xa ^ 0x8000])[perm]
        bp = (bb.astype(np.int32) + step).astype(np.uint16)
        b = np.concatenate([bb, bp])[perm]
        t = bf16_to_f32(a).astype(np.float64) * bf16_to_f32(b).astype(np.float64)
        arrs = (a, b)
    info = {"param": j / h, "cond": _cond(t), "kind": kind, "dtype": dtype}
    return (*arrs, info)


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
