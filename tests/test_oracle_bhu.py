"""Pins of the oracle's Householder bidiagonal update (BHU; Section 3.3,
Theorem 1, Algorithm 1, eqs. (house), (TR), (QP)).

- Theorem 1 (with eq. (QP) inside it): the representation B - U M^{-1} V^T
  equals Q_i^T (B + b c^T) P_j formed densely as the product of the explicit
  reflectors I - 2 y y^T, for numbers of left and right reflectors i = j and
  i = j + 1 (the two forms Algorithm 1 uses).
- Algorithm 1 reaches what a textbook dense Householder bidiagonalization of
  the formed matrix B + b c^T reaches with the same reflector conventions
  (written out below, applying each reflector to the dense matrix).
- The update reconstructs A + b c^T with orthogonal factors, its singular
  values are those of the dense matrix (LAPACK), and a zero update changes
  nothing, bit for bit.
- |d|, |e| agree with the oracle's dense C Householder bidiagonalization
  (which uses reflectors also when there is nothing left to annihilate, so
  signs may differ).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_02840_amd import workloads as W


def _bd(d, e, m):
    n = len(d)
    B = np.zeros((m, n))
    B[np.arange(n), np.arange(n)] = d
    B[np.arange(n - 1), np.arange(1, n)] = e
    return B


def _reflectors(rng, size, count, shift):
    """count unit vectors of length size, vector q zero above entry q + shift."""
    Y = np.zeros((size, count))
    for q in range(count):
        v = rng.standard_normal(size - q - shift)
        Y[q + shift:, q] = v / np.linalg.norm(v)
    return Y


def _product(Y):
    M = np.eye(Y.shape[0])
    for q in range(Y.shape[1]):
        M = M @ (np.eye(Y.shape[0]) - 2.0 * np.outer(Y[:, q], Y[:, q]))
    return M


@pytest.mark.parametrize("m,n,i,j", [(7, 7, 3, 3), (7, 7, 4, 3), (9, 6, 5, 4), (9, 6, 1, 0), (5, 5, 0, 0),
                                     (12, 10, 7, 7), (12, 10, 8, 7)])
def test_theorem1_representation(m, n, i, j):
    rng = np.random.default_rng(100 + 7 * m + i)
    d, e = rng.standard_normal(n), rng.standard_normal(n - 1)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    Y = _reflectors(rng, m, i, 0)
    Wr = _reflectors(rng, n, j, 1)
    U, M, V = O.bhu_repr(d, e, b, c, Y, Wr)
    got = _bd(d, e, m) - U @ np.linalg.solve(M, V.T)
    want = _product(Y).T @ (_bd(d, e, m) + np.outer(b, c)) @ _product(Wr)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def _dense_bhu(A):
    """Textbook Householder bidiagonalization of the dense A, reflectors
    applied to A itself: left ones on columns 0..kl-1, right ones on rows
    0..n-3; the identity where the entries to annihilate are already zero."""
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    kl = n - 1 if m == n else n
    kr = n - 2
    Y = np.zeros((m, kl))
    Wr = np.zeros((n, max(kr, 0)))
    for k in range(kl):
        x = A[k:, k].copy()
        if np.any(x[1:] != 0.0):
            nrm = np.linalg.norm(x)
            alpha = -nrm if x[0] >= 0.0 else nrm
            x[0] -= alpha
            v = x / np.linalg.norm(x)
            A[k:, :] -= 2.0 * np.outer(v, v @ A[k:, :])
            Y[k:, k] = v
        if k < kr:
            x = A[k, k + 1:].copy()
            if np.any(x[1:] != 0.0):
                nrm = np.linalg.norm(x)
                alpha = -nrm if x[0] >= 0.0 else nrm
                x[0] -= alpha
                v = x / np.linalg.norm(x)
                A[:, k + 1:] -= 2.0 * np.outer(A[:, k + 1:] @ v, v)
                Wr[k + 1:, k] = v
    return np.diag(A)[:n].copy(), np.diag(A, 1)[:n - 1].copy(), Y, Wr, A


@pytest.mark.parametrize("m,n", [(2, 2), (3, 2), (5, 2), (3, 3), (6, 6), (9, 6), (20, 20), (41, 30), (60, 60),
                                 (80, 7), (120, 3)])
def test_algorithm1_matches_dense_householder(m, n):
    rng = np.random.default_rng(200 + m + n)
    d, e = rng.standard_normal(n), rng.standard_normal(n - 1)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    A = _bd(d, e, m) + np.outer(b, c)
    dp, ep, Y, Wr = O.bhu_bidiag(d, e, b, c, m)
    dd, ed, Yd, Wd, R = _dense_bhu(A)
    scale = np.linalg.norm(A)
    # the dense sweep leaves a bidiagonal matrix
    assert np.abs(R - _bd(dd, ed, m)).max() < 1e-13 * scale * n
    assert np.abs(dp - dd).max() < 1e-12 * scale
    assert np.abs(ep - ed).max() < 1e-12 * scale
    assert Y.shape == Yd.shape and Wr.shape == Wd.shape
    assert np.abs(Y - Yd).max() < 1e-10
    if Wr.size:
        assert np.abs(Wr - Wd).max() < 1e-10


@pytest.mark.parametrize("m,n", [(2, 2), (5, 4), (16, 16), (40, 33)])
def test_update_reconstructs_with_orthogonal_factors(m, n):
    f = W.factorization(m, n, 300 + m)
    rng = np.random.default_rng(301 + n)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    Q2, d2, e2, P2 = O.bhu_update(f.Q, f.d, f.e, f.P, b, c)
    A2 = f.dense() + np.outer(b, c)
    scale = np.linalg.norm(A2)
    assert np.abs(Q2 @ _bd(d2, e2, m) @ P2.T - A2).max() < 1e-13 * scale * n
    assert np.abs(Q2.T @ Q2 - np.eye(m)).max() < 1e-13 * n
    assert np.abs(P2.T @ P2 - np.eye(n)).max() < 1e-13 * n
    sv = np.sort(np.linalg.svd(_bd(d2, e2, m), compute_uv=False))
    assert np.abs(sv - np.sort(np.linalg.svd(A2, compute_uv=False))).max() < 1e-13 * scale * n


def test_zero_update_changes_nothing():
    m, n = 12, 9
    f = W.factorization(m, n, 310)
    Q2, d2, e2, P2 = O.bhu_update(f.Q, f.d, f.e, f.P, np.zeros(m), np.ones(n))
    assert np.array_equal(d2, f.d) and np.array_equal(e2, f.e)
    assert np.array_equal(Q2, f.Q) and np.array_equal(P2, f.P)


@pytest.mark.parametrize("m,n", [(8, 8), (11, 7), (30, 30)])
def test_magnitudes_agree_with_dense_c_bidiagonalization(m, n):
    rng = np.random.default_rng(320 + m)
    d, e = rng.standard_normal(n), rng.standard_normal(n - 1)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    A = _bd(d, e, m) + np.outer(b, c)
    dp, ep, _, _ = O.bhu_bidiag(d, e, b, c, m)
    _, dc, ec, _ = O.bidiag_householder(A)
    scale = np.linalg.norm(A)
    assert np.abs(np.abs(dp) - np.abs(dc)).max() < 1e-12 * scale
    assert np.abs(np.abs(ep) - np.abs(ec)).max() < 1e-12 * scale
