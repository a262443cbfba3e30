"""Pins of the oracle's conjugate-gradient solver and grid-barrier exchange.

The CG oracle follows Hestenes and Stiefel's method (the solver of the CG
sample that Table 1 lists as needing grid synchronisation); these tests tie
it to facts that do not come from the oracle itself:
  - the solution agrees with numpy's dense solver;
  - with k distinct eigenvalues CG converges in k iterations (exact
    arithmetic gives a zero residual; a wrong alpha, beta or sign does not);
  - the A-norm of the error decreases monotonically (CG minimises it);
  - the recurrence residual rr_k equals the true residual |b - A x_k|^2;
  - the inner products equal the exact sums (bit-exact when every partial
    sum is exact, within n * 2^-53 * sum|terms| otherwise);
  - the degenerate cases: empty system, zero iterations, exact start,
    breakdown on an indefinite matrix.
"""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore")


def dense(rp, ci, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        for jj in range(rp[i], rp[i + 1]):
            A[i, ci[jj]] += float(val[jj])
    return A


def diag_csr(d):
    n = d.size
    return np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d.astype(np.float32)


def test_cg_solves_tridiagonal_system(oracle_mod):
    n = 300
    rp, ci, val, b = inputs.cg_tridiag(n, seed=7)
    x, k, reason, hist = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), 200, 1e-5, 4, 8)
    assert reason == oracle_mod.CG_CONVERGED and 0 < k < 60
    want = np.linalg.solve(dense(rp, ci, val, n), b.astype(np.float64))
    assert np.max(np.abs(x - want)) <= 1e-5 * np.max(np.abs(want)) + 1e-6
    assert hist[-1] <= 1e-10 and hist.size == k + 1


def test_cg_irregular_system(oracle_mod):
    n = 1500
    rp, ci, val, b = inputs.cg_irregular(n, seed=3)
    assert np.diff(rp).max() > 20 and np.diff(rp).min() >= 1
    x, k, reason, _ = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), 500, 1e-5, 2, 16)
    assert reason == oracle_mod.CG_CONVERGED
    want = np.linalg.solve(dense(rp, ci, val, n), b.astype(np.float64))
    assert np.max(np.abs(x - want)) <= 1e-4 * np.max(np.abs(want))


@pytest.mark.parametrize("levels", [(1.0, 2.0, 5.0), (0.5, 3.0, 4.0, 7.0)])
def test_cg_converges_in_as_many_steps_as_distinct_eigenvalues(oracle_mod, levels):
    g = np.random.default_rng(11)
    n = 4000
    d = np.array(levels, np.float32)[g.integers(0, len(levels), n)]
    rp, ci, val = diag_csr(d)
    b = g.uniform(-1, 1, n).astype(np.float32)
    m = len(levels)
    _, k, reason, hist = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), m, 0.0, 4, 32)
    assert k == m and reason == oracle_mod.CG_MAX_ITER
    assert hist[m] <= 1e-9 * hist[0]
    assert hist[m - 1] >= 1e-4 * hist[0]


def test_cg_error_decreases_in_a_norm(oracle_mod):
    n = 500
    rp, ci, val, b = inputs.cg_tridiag(n, seed=21)
    A = dense(rp, ci, val, n)
    xs = np.linalg.solve(A, b.astype(np.float64))
    errs = []
    for k in range(0, 9):
        x, kk, _, _ = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), k, 0.0, 1, 8)
        assert kk == k
        e = x.astype(np.float64) - xs
        errs.append(float(e @ A @ e))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


@pytest.mark.parametrize("k", [1, 3, 8])
def test_cg_recurrence_residual_is_true_residual(oracle_mod, k):
    n = 2000
    rp, ci, val, b = inputs.cg_irregular(n, seed=5)
    A = dense(rp, ci, val, n)
    x, kk, _, hist = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), k, 0.0, 4, 8)
    assert kk == k
    res = b.astype(np.float64) - A @ x.astype(np.float64)
    true_rr = float(res @ res)
    assert abs(hist[k] - true_rr) <= 1e-3 * true_rr + 1e-6 * hist[0]


@pytest.mark.parametrize("n,R,W", [(1, 1, 8), (255, 1, 8), (5000, 2, 8), (3 * 4096 + 17, 4, 32), (70001, 8, 16)])
def test_cg_inner_product_is_the_exact_sum(oracle_mod, n, R, W):
    g = np.random.default_rng(n)
    rp, ci, val = diag_csr(np.ones(n, np.float32))
    # integer values: every partial sum is exact, so the schedule's result is
    # the exact sum whatever its order
    b = g.integers(-100, 101, n).astype(np.float32)
    _, _, _, hist = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), 0, 0.0, R, W)
    assert hist[0] == float(np.sum(b.astype(np.int64) ** 2))
    b = g.standard_normal(n).astype(np.float32)
    _, _, _, hist = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), 0, 0.0, R, W)
    terms = b.astype(np.float64) ** 2
    exact = oracle_mod.exact_sum_f64(terms)
    assert abs(hist[0] - exact) <= n * 2.0 ** -53 * terms.sum()


def test_cg_degenerate_cases(oracle_mod):
    # empty system: rr_0 is the empty sum -0.0 and the solver stops at once
    x, k, reason, hist = oracle_mod.cg(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32),
                                       np.zeros(0, np.float32), np.zeros(0, np.float32), 10, 0.0, 4, 32)
    assert (k, reason, x.size) == (0, oracle_mod.CG_CONVERGED, 0) and np.signbit(hist[0])
    # zero iterations: x unchanged
    n = 100
    rp, ci, val, b = inputs.cg_tridiag(n, seed=1)
    x0 = np.linspace(-1, 1, n).astype(np.float32)
    x, k, reason, hist = oracle_mod.cg(rp, ci, val, b, x0, 0, 0.0, 1, 8)
    assert (k, reason) == (0, oracle_mod.CG_MAX_ITER) and np.array_equal(x, x0) and hist.size == 1
    # exact start: A = I, x0 = b gives r_0 = 0
    rp, ci, val = diag_csr(np.ones(n, np.float32))
    x, k, reason, hist = oracle_mod.cg(rp, ci, val, b, b, 10, 0.0, 1, 8)
    assert (k, reason) == (0, oracle_mod.CG_CONVERGED) and hist[0] == 0.0 and np.array_equal(x, b)
    # indefinite A = diag(1, -1) and b = (1, 1): p = r = b, <p, A p> = 0
    rp, ci, val = diag_csr(np.array([1.0, -1.0], np.float32))
    x, k, reason, hist = oracle_mod.cg(rp, ci, val, np.ones(2, np.float32), np.zeros(2, np.float32), 10, 0.0, 1, 8)
    assert (k, reason) == (0, oracle_mod.CG_BREAKDOWN) and np.array_equal(x, np.zeros(2, np.float32))


def test_cg_schedules_agree_to_rounding(oracle_mod):
    n = 20000
    rp, ci, val, b = inputs.cg_tridiag(n, seed=9)
    xa, ka, _, _ = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), 30, 0.0, 4, 32)
    xb, kb, _, _ = oracle_mod.cg(rp, ci, val, b, np.zeros(n, np.float32), 30, 0.0, 1, 8)
    assert ka == kb == 30
    assert np.max(np.abs(xa - xb)) <= 1e-5 * np.max(np.abs(xa))


def test_cg_rejects_bad_csr(oracle_mod):
    rp = np.array([0, 2, 1], np.int32)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.cg(rp, np.zeros(2, np.int32), np.ones(2, np.float32), np.ones(2, np.float32),
                      np.zeros(2, np.float32), 1, 0.0, 1, 8)
    rp = np.array([0, 1, 2], np.int32)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.cg(rp, np.array([0, 2], np.int32), np.ones(2, np.float32), np.ones(2, np.float32),
                      np.zeros(2, np.float32), 1, 0.0, 1, 8)


def _fmix32(h):
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    return h


def test_fmix32_known_values():
    # MurmurHash3's finaliser: 0 is a fixed point and it is a bijection
    assert _fmix32(0) == 0
    vals = {_fmix32(v) for v in range(1 << 16)}
    assert len(vals) == 1 << 16


@pytest.mark.parametrize("G,rounds", [(1, 3), (5, 7), (9, 20)])
def test_grid_exchange_closed_form(oracle_mod, G, rounds):
    out = oracle_mod.grid_exchange(G, rounds, block=64)
    for b in range(G):
        for t in (0, 1, 37, 63):
            want = 0
            for r in range(rounds):
                want = (want + _fmix32((r << 20) ^ (((b + r + 1) % G) << 10) ^ t)) & 0xFFFFFFFF
            assert int(out[b, t]) == want
