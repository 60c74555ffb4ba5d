"""Pins of the oracle's truncated bidiagonal approximation (Section 1.3,
eqs. (trBD) and (errtrBD)) against dense products and the SVD."""
import itertools

import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W


def _A(f):
    return f.dense()


@pytest.mark.parametrize("m,n,r", [(30, 20, 5), (12, 12, 1), (40, 25, 25), (50, 30, 12)])
def test_error_formula_is_exact(oracle, m, n, r):
    f = W.factorization(m, n, 200 + r)
    idx, err2, Qr, Pr = oracle.truncated_bd(f.Q, f.d, f.e, f.P, r)
    dense = np.linalg.norm(_A(f) - Qr @ Pr.T) ** 2
    assert abs(dense - err2) <= 1e-12 * max(np.linalg.norm(_A(f)) ** 2, 1.0)
    assert len(set(idx.tolist())) == r


def test_diagonal_case_is_the_truncated_svd(oracle):
    """With e = 0 the bidiagonal factorization is an SVD (up to signs and
    order) and the error is the sum of the smallest squared values."""
    m, n, r = 20, 15, 6
    f = W.factorization(m, n, 9)
    e = np.zeros(n - 1)
    _, err2, Qr, Pr = oracle.truncated_bd(f.Q, f.d, e, f.P, r)
    s = np.sort(np.abs(f.d))
    assert abs(err2 - np.sum(s[: n - r] ** 2)) <= 1e-12 * np.sum(s ** 2)


def test_selection_is_optimal_among_column_subsets(oracle):
    m, n, r = 10, 7, 3
    f = W.factorization(m, n, 17)
    A = _A(f)
    _, err2, _, _ = oracle.truncated_bd(f.Q, f.d, f.e, f.P, r)
    for S in itertools.combinations(range(n), r):
        Qs = np.column_stack([f.d[i] * f.Q[:, i] + (f.e[i - 1] * f.Q[:, i - 1] if i else 0) for i in S])
        Ps = f.P[:, list(S)]
        assert np.linalg.norm(A - Qs @ Ps.T) ** 2 >= err2 - 1e-12


def test_ties_keep_the_lower_index(oracle):
    n = 6
    Q, P = np.eye(8), np.eye(n)
    d = np.array([1.0, 2.0, 2.0, 1.0, 2.0, 0.5])
    e = np.zeros(n - 1)
    idx, err2, _, _ = oracle.truncated_bd(Q, d, e, P, 2)
    assert idx.tolist() == [1, 2]
    assert err2 == 1.0 + 1.0 + 4.0 + 0.25
