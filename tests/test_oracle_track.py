"""Pins of the oracle's subspace-tracking update (Section 4, eqs. (lrup) to
(bdlrup)): each check compares against something the oracle does not
compute the same way (dense products, dense singular values, numpy norms),
and planted mistakes in the oracle are caught."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

SHAPES = [(30, 20, 4), (12, 9, 1), (40, 40, 7), (64, 33, 16), (9, 25, 5)]


def _case(m, n, r, seed):
    return W.tracking_state(m, n, r, seed), W.tracking_update(m, n, seed + 1)


def _bd(d, e):
    return np.diag(d) + np.diag(e, 1)


@pytest.mark.parametrize("m,n,r", SHAPES)
def test_exact_rank_r_plus_1_factorization(oracle, m, n, r):
    (U, d, e, V), (b, c) = _case(m, n, r, 11 + r)
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    U2, d2, e2, V2, info = oracle.track_update(U, d, e, V, b, c, keep_all=True)
    assert U2.shape == (m, r + 1) and V2.shape == (n, r + 1)
    assert np.linalg.norm(A - U2 @ _bd(d2, e2) @ V2.T) <= 1e-13 * np.linalg.norm(A)
    assert np.linalg.norm(U2.T @ U2 - np.eye(r + 1)) <= 1e-13
    assert np.linalg.norm(V2.T @ V2 - np.eye(r + 1)) <= 1e-13
    # delta, gamma: norms of the parts of b, c outside span(U), span(V)
    bperp = b - U @ (U.T @ b)
    cperp = c - V @ (V.T @ c)
    assert abs(info[0] - np.linalg.norm(bperp)) <= 1e-13 * np.linalg.norm(b)
    assert abs(info[1] - np.linalg.norm(cperp)) <= 1e-13 * np.linalg.norm(c)


@pytest.mark.parametrize("m,n,r", SHAPES)
def test_middle_matrix_singular_values(oracle, m, n, r):
    """Bbar carries the singular values of the dense middle matrix
    [B 0; 0 0] + [U^T b; delta][V^T c; gamma]^T of eq. (equivlrup)."""
    (U, d, e, V), (b, c) = _case(m, n, r, 21 + r)
    _, d2, e2, _, (delta, gamma, _) = oracle.track_update(U, d, e, V, b, c, keep_all=True)
    M = np.zeros((r + 1, r + 1))
    M[:r, :r] = _bd(d, e)
    M += np.outer(np.append(U.T @ b, np.linalg.norm(b - U @ (U.T @ b))),
                  np.append(V.T @ c, np.linalg.norm(c - V @ (V.T @ c))))
    s_dense = oracle.jacobi_sv(M)
    s_bgu = oracle.jacobi_sv(_bd(d2, e2))
    assert np.allclose(s_bgu, s_dense, rtol=1e-13, atol=1e-13 * s_dense[0])


@pytest.mark.parametrize("m,n,r", SHAPES)
def test_truncation_drops_the_smallest_column(oracle, m, n, r):
    """The rank-r result is the rank-(r+1) one without the row and column of
    smallest column norm: its error is exactly the norm of what was dropped,
    and it keeps orthonormal columns."""
    (U, d, e, V), (b, c) = _case(m, n, r, 31 + r)
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    Uf, df, ef, Vf, _ = oracle.track_update(U, d, e, V, b, c, keep_all=True)
    Ut, dt, et, Vt, (_, _, k) = oracle.track_update(U, d, e, V, b, c)
    Bf = _bd(df, ef)
    norms = np.linalg.norm(Bf, axis=0)
    assert norms[k] == norms.min()
    assert k == max(np.flatnonzero(norms == norms.min()))
    keep = [j for j in range(r + 1) if j != k]
    assert np.array_equal(dt, df[keep])
    assert np.array_equal(_bd(dt, et), Bf[np.ix_(keep, keep)])
    dropped = np.sqrt(np.sum(Bf[k, :] ** 2) + np.sum(Bf[:, k] ** 2) - Bf[k, k] ** 2)
    err = np.linalg.norm(A - Ut @ _bd(dt, et) @ Vt.T)
    assert abs(err - dropped) <= 1e-12 * np.linalg.norm(A)
    assert np.array_equal(Ut, Uf[:, keep]) and np.array_equal(Vt, Vf[:, keep])
    assert np.linalg.norm(Ut.T @ Ut - np.eye(r)) <= 1e-13


def test_vectors_in_the_span_are_rejected(oracle):
    """delta = 0 exactly (b in span(U)): the paper does not augment; the
    oracle reports it instead of dividing by zero."""
    m, n, r = 10, 8, 3
    U = np.eye(m)[:, :r]
    V = np.eye(n)[:, :r]
    b = np.zeros(m)
    b[:r] = [1.0, -2.0, 0.5]
    c = np.arange(1.0, n + 1)
    with pytest.raises(ValueError, match="-11"):
        oracle.track_update(U, np.ones(r), np.ones(r - 1), V, b, c)


def test_stream_stays_a_factorization(oracle):
    """A short tracking stream: after each update the factors are
    orthonormal and the truncation error never exceeds that of the best
    rank-r approximation of the exact rank-(r+1) matrix by more than the
    dropped part's norm (both small here)."""
    m, n, r = 50, 30, 5
    (U, d, e, V), _ = _case(m, n, r, 41)
    rng = np.random.default_rng(42)
    for step in range(8):
        b = rng.standard_normal(m) * 0.3
        c = rng.standard_normal(n) * 0.3
        U, d, e, V, _ = oracle.track_update(U, d, e, V, b, c)
        assert np.linalg.norm(U.T @ U - np.eye(r)) <= 1e-12
        assert np.linalg.norm(V.T @ V - np.eye(r)) <= 1e-12


@pytest.mark.parametrize("mutation", [8, 9, 10])
def test_planted_tracking_mistakes_are_caught(oracle, mutation):
    """Residual sign, the missing delta and the wrong truncation index each
    break one of the pins above."""
    m, n, r = 30, 20, 4
    (U, d, e, V), (b, c) = _case(m, n, r, 15)
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    oracle.set_mutation(mutation)
    try:
        Uf, df, ef, Vf, _ = oracle.track_update(U, d, e, V, b, c, keep_all=True)
        Ut, dt, et, Vt, (_, _, k) = oracle.track_update(U, d, e, V, b, c)
    finally:
        oracle.set_mutation(0)
    exact = np.linalg.norm(A - Uf @ _bd(df, ef) @ Vf.T) <= 1e-13 * np.linalg.norm(A)
    orth = np.linalg.norm(Uf.T @ Uf - np.eye(r + 1)) <= 1e-13
    norms = np.linalg.norm(_bd(df, ef), axis=0)
    smallest = norms[k] == norms.min()
    assert not (exact and orth and smallest)
