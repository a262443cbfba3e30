"""The seeded input recipes: reproducible bit for bit, and with the
properties the workloads rely on (the CG systems symmetric, strictly
diagonally dominant and therefore positive definite; images uint8 of the
requested shape)."""
import numpy as np
import pytest

from paper_2112_10034_amd import inputs


def _dense(rp, ci, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        for jj in range(rp[i], rp[i + 1]):
            A[i, ci[jj]] += float(val[jj])
    return A


@pytest.mark.parametrize("make", [inputs.cg_tridiag, inputs.cg_irregular])
def test_cg_systems_are_reproducible_and_well_formed(make):
    n = 700
    a = make(n, seed=3)
    b = make(n, seed=3)
    for x, y in zip(a, b):
        assert x.dtype == y.dtype and np.array_equal(x, y)
    rp, ci, val, rhs = a
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and val.dtype == np.float32 and rhs.dtype == np.float32
    assert rp[0] == 0 and rp[-1] == ci.size == val.size and np.all(np.diff(rp) >= 1)
    assert ci.min() >= 0 and ci.max() < n
    for i in range(n):  # columns ascending inside every row
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) >= 0)
    A = _dense(rp, ci, val, n)
    assert np.array_equal(A, A.T)
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) > off)  # strictly diagonally dominant, positive diagonal
    assert np.linalg.eigvalsh(A).min() > 0
    assert np.all(np.abs(rhs) <= 1)
    assert not np.array_equal(make(n, seed=4)[3], rhs)


def test_tridiagonal_eigenvalues_in_the_stated_interval():
    rp, ci, val, _ = inputs.cg_tridiag(400, seed=8)
    ev = np.linalg.eigvalsh(_dense(rp, ci, val, 400))
    assert ev.min() > 1 and ev.max() < 6


def test_tridiagonal_shape_of_the_full_workloads():
    assert inputs.CG_N == (1 << 20, 1 << 24)
    rp, ci, val, b = inputs.cg_tridiag(1 << 12)
    assert ci.size == 3 * (1 << 12) - 2 and b.size == 1 << 12


def test_images_are_reproducible_uint8():
    a = inputs.image_u8(37, 1001, seed=2)
    assert a.dtype == np.uint8 and a.shape == (37, 1001)
    assert np.array_equal(a, inputs.image_u8(37, 1001, seed=2))
    assert a.min() == 0 and a.max() == 255
    assert inputs.IMAGE_HW == (8192, 8192)
