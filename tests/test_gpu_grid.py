"""GPU parity of the grid-wide barrier and the conjugate-gradient solver.

1. Exchange kernel: every block publishes a row per round and reads another
   block's row of the same round after a grid barrier; the per-thread sums
   must equal the oracle's (a stale or early read changes them).
2. CG in one cooperative launch, and as one launch per phase: x, the
   iteration count, the stop reason and every rr_k bit-exact against the
   oracle on the same inner-product schedule, for sizes that span one
   chunk, several chunks with a ragged tail, and the full workload sizes;
   results identical for every grid size, and whether a block of the
   resident kernel keeps its CSR rows in shared memory or streams them.
"""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10034_amd import cox

    cox.lib()
    return torch, cox


def up(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("G,rounds", [(1, 3), (3, 5), (8, 17), (9, 40), (0, 64)])
def test_grid_exchange(dev, oracle_mod, G, rounds):
    torch, cox = dev
    cap = cox.grid_capacity()
    assert cap >= 256
    G = cap if G == 0 else G
    print("grid exchange", G, rounds, flush=True)
    got = cox.grid_exchange(G, rounds).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.grid_exchange(G, rounds, block=1024))


def test_grid_exchange_rejects_oversized_grid(dev):
    torch, cox = dev
    with pytest.raises(cox.CoxError) as e:
        cox.grid_exchange(cox.grid_capacity() + 1, 1)
    assert e.value.code == 1


@pytest.mark.parametrize("G,absent", [(8, 3), (64, 0), (0, 511)])
def test_grid_barrier_gives_up_when_a_block_is_absent(dev, oracle_mod, G, absent):
    """Failure handling forced from the host: one block never arrives and the
    waits are bounded by 2000 polls, so every block finishes, the workspace
    reports COX_ERR_TIMEOUT, and the next call on it is correct."""
    torch, cox = dev
    G = cox.grid_capacity() if G == 0 else G
    absent = min(absent, G - 1)
    print("grid exchange with block", absent, "of", G, "absent", flush=True)
    assert cox.grid_exchange_absent(G, 4, absent, 2000) == cox.ERR_TIMEOUT
    got = cox.grid_exchange(G, 5).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.grid_exchange(G, 5, block=1024))


def test_grid_exchange_absent_rejects_bad_arguments(dev):
    torch, cox = dev
    for G, absent, spins in ((8, 8, 10), (8, -1, 10), (8, 0, 0), (8, 0, (1 << 20) + 1)):
        with pytest.raises(cox.CoxError) as e:
            cox.grid_exchange_absent(G, 1, absent, spins)
        assert e.value.code == 1


def _system(kind, n, seed):
    return inputs.cg_tridiag(n, seed=seed) if kind == "tri" else inputs.cg_irregular(n, seed=seed)


def _solve(torch, cox, sysm, x0, max_iter, tol, cfg, per_phase, grid=0):
    rp, ci, val, b = sysm
    x = up(torch, x0.astype(np.float32))
    c = None if cfg is None else cox.make_cfg(cfg[0], cfg[1], grid)
    res, hist = cox.cg_solve(up(torch, rp), up(torch, ci), up(torch, val), up(torch, b), x, max_iter, tol, cfg=c,
                             per_phase=per_phase)
    cox.workspace(cox.OP_CG, cox.F32, b.size, cfg=c).status()
    res = res.cpu().numpy()
    k = int(res[0])
    return x.cpu().numpy(), k, int(res[1]), hist.cpu().numpy()[: k + 1]


def _check(got, want):
    x, k, reason, hist = got
    wx, wk, wreason, whist = want
    assert (k, reason) == (wk, wreason)
    assert np.array_equal(hist.view(np.uint64), whist.view(np.uint64))
    assert np.array_equal(x.view(np.uint32), wx.view(np.uint32))


CASES = [
    ("tri", 1, (1, 8), 5, 0.0),
    ("tri", 37, (4, 32), 12, 0.0),
    ("tri", 3 * 4096 + 17, (4, 32), 25, 0.0),
    ("irr", 3 * 2048 + 333, (2, 32), 25, 0.0),
    ("irr", 70001, (8, 16), 30, 0.0),
    ("irr", 20000, (1, 8), 400, 1e-4),
    ("tri", 100000, (4, 32), 400, 1e-5),
]


@pytest.mark.parametrize("per_phase", [False, True])
@pytest.mark.parametrize("kind,n,sigma,max_iter,tol", CASES)
def test_cg_matches_oracle(dev, oracle_mod, kind, n, sigma, max_iter, tol, per_phase):
    torch, cox = dev
    sysm = _system(kind, n, seed=n)
    x0 = np.zeros(n, np.float32)
    print("cg", kind, n, sigma, max_iter, tol, "per_phase" if per_phase else "coop", flush=True)
    want = oracle_mod.cg(*sysm, x0, max_iter, tol, *sigma)
    _check(_solve(torch, cox, sysm, x0, max_iter, tol, sigma, per_phase), want)
    if tol > 0:
        assert want[2] == oracle_mod.CG_CONVERGED


@pytest.mark.parametrize("kind", ["irr", "tri"])
@pytest.mark.parametrize("grid", [1, 3, 7, 0])
def test_cg_result_is_independent_of_the_grid(dev, oracle_mod, grid, kind):
    """Grids below the chunk count run the streaming kernel, the others the
    resident one; the tridiagonal rows fit in shared memory there, the
    irregular ones (seven entries a row) do not."""
    torch, cox = dev
    n = 5 * 4096 + 99
    sysm = _system(kind, n, seed=4)
    x0 = np.linspace(-1, 1, n).astype(np.float32)
    print("cg grid", kind, grid, flush=True)
    want = oracle_mod.cg(*sysm, x0, 20, 0.0, 4, 32)
    _check(_solve(torch, cox, sysm, x0, 20, 0.0, (4, 32), False, grid), want)


def _block_diagonal(S, tail, seed):
    """SPD block-diagonal system: a tridiagonal block over the first two
    chunks of S rows, then a band of half-width 8 (17 entries a row) over
    S + tail rows.  In the resident kernel the first two chunks and the
    short last chunk keep their rows in shared memory, the third (about
    17 S entries) cannot."""
    sp = pytest.importorskip("scipy.sparse")
    rng = np.random.default_rng(seed)
    n1, n2 = 2 * S, S + tail
    off1 = -rng.random(n1 - 1)
    T = sp.diags([off1, 3.0 + rng.random(n1), off1], [-1, 0, 1])
    bands = [20.0 + rng.random(n2)]
    offs = [0]
    for d in range(1, 9):
        v = -rng.random(n2 - d)
        bands += [v, v]
        offs += [d, -d]
    B = sp.diags(bands, offs)
    A = sp.block_diag((T, B)).astype(np.float32).tocsr()
    A.sort_indices()
    b = rng.uniform(-1, 1, n1 + n2).astype(np.float32)
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float32), b


def test_cg_with_staged_and_streamed_blocks(dev, oracle_mod):
    torch, cox = dev
    sysm = _block_diagonal(4096, 17, seed=11)
    n = sysm[3].size
    x0 = np.zeros(n, np.float32)
    print("cg staged and streamed blocks", n, flush=True)
    want = oracle_mod.cg(*sysm, x0, 30, 0.0, 4, 32)
    for pp in (False, True):
        _check(_solve(torch, cox, sysm, x0, 30, 0.0, (4, 32), pp), want)


def test_cg_degenerate_cases(dev, oracle_mod):
    torch, cox = dev
    # empty system
    e = (np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    print("cg empty", flush=True)
    for pp in (False, True):
        _check(_solve(torch, cox, e, np.zeros(0, np.float32), 10, 0.0, None, pp),
               oracle_mod.cg(*e, np.zeros(0, np.float32), 10, 0.0, 4, 32))
    n = 1000
    sysm = _system("tri", n, seed=2)
    x0 = np.linspace(-1, 1, n).astype(np.float32)
    print("cg zero iterations", flush=True)
    for pp in (False, True):
        _check(_solve(torch, cox, sysm, x0, 0, 0.0, None, pp), oracle_mod.cg(*sysm, x0, 0, 0.0, 4, 32))
    # exact start (A = I, x0 = b) and breakdown (A = diag(1, -1), b = (1, 1))
    ident = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32), sysm[3])
    indef = (np.arange(3, dtype=np.int32), np.arange(2, dtype=np.int32), np.array([1, -1], np.float32),
             np.ones(2, np.float32))
    print("cg exact start and breakdown", flush=True)
    for pp in (False, True):
        got = _solve(torch, cox, ident, sysm[3], 10, 0.0, None, pp)
        _check(got, oracle_mod.cg(*ident, sysm[3], 10, 0.0, 4, 32))
        assert got[1:3] == (0, cox.CG_CONVERGED)
        got = _solve(torch, cox, indef, np.zeros(2, np.float32), 10, 0.0, None, pp)
        _check(got, oracle_mod.cg(*indef, np.zeros(2, np.float32), 10, 0.0, 4, 32))
        assert got[1:3] == (0, cox.CG_BREAKDOWN)


def test_cg_rejects_unsupported_schedule_and_grid(dev):
    torch, cox = dev
    sysm = _system("tri", 64, seed=1)
    x = np.zeros(64, np.float32)
    # R = 3 is no schedule at all (rejected when the workspace is sized);
    # W = 4 and R = 16 are schedules the solver does not compile
    for cfg, code in (((3, 32), 1), ((4, 4), 6), ((16, 32), 6)):
        with pytest.raises(cox.CoxError) as e:
            _solve(torch, cox, sysm, x, 3, 0.0, cfg, False)
        assert e.value.code == code
    with pytest.raises(cox.CoxError) as e:
        _solve(torch, cox, _system("tri", 1 << 20, seed=1), np.zeros(1 << 20, np.float32), 1, 0.0, (4, 32), False,
               grid=10 ** 6)
    assert e.value.code == 1


@pytest.mark.parametrize("n,max_iter", [(inputs.CG_N[0], 60), (inputs.CG_N[1], 4)])
def test_cg_full_size(dev, oracle_mod, n, max_iter):
    torch, cox = dev
    print("generating the CG system", n, flush=True)
    sysm = _system("tri", n, seed=None)
    x0 = np.zeros(n, np.float32)
    k, W, _ = cox.default_cfg(cox.OP_CG, cox.F32)
    print("cg full size", n, (k, W), max_iter, flush=True)
    want = oracle_mod.cg(*sysm, x0, max_iter, 0.0, k, W)
    for pp in (False, True):
        _check(_solve(torch, cox, sysm, x0, max_iter, 0.0, None, pp), want)
