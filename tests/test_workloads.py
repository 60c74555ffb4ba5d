"""The seeded input generators (CPU): the starting factorization built
from a rating matrix, including rank-deficient inputs that break the
Golub-Kahan recurrence down."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W


def _check(A, Q, d, e, P, tol):
    m, n = A.shape
    Bd = np.zeros((m, n))
    Bd[np.arange(n), np.arange(n)] = d
    Bd[np.arange(n - 1), np.arange(1, n)] = e
    assert np.linalg.norm(Q @ Bd @ P.T - A) <= tol * max(np.linalg.norm(A), 1.0)
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= tol * m
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= tol * n
    assert np.all(d >= 0) and np.all(e >= 0)
    # the singular values survive the construction
    sa = np.linalg.svd(A, compute_uv=False)
    sb = np.linalg.svd(Bd[:n], compute_uv=False)
    assert np.max(np.abs(sa - sb)) <= tol * max(sa[0], 1.0)


@pytest.mark.parametrize("users,items", [(120, 40), (300, 97), (64, 64)])
def test_bidiagonal_factors_of_ratings(users, items):
    A = W.ratings(users, items, density=0.05, seed=users + items)
    _check(A, *W.bidiagonal_factors(A, seed=1), tol=1e-13)


def test_bidiagonal_factors_rank_deficient():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((80, 6)) @ rng.standard_normal((6, 30))  # rank 6
    Q, d, e, P = W.bidiagonal_factors(A, seed=2)
    _check(A, Q, d, e, P, tol=1e-12)
    assert np.count_nonzero(d == 0.0) + np.count_nonzero(e == 0.0) >= 1


def test_bidiagonal_factors_zero_columns():
    A = np.zeros((20, 8))
    A[3, 2] = 4.0
    _check(A, *W.bidiagonal_factors(A, seed=3), tol=1e-14)


def test_bidiagonal_factors_rejects_wide():
    with pytest.raises(ValueError):
        W.bidiagonal_factors(np.ones((3, 5)))
