"""Pins of the oracle's subspace-tracking update (Section 4, eqs. (lrup) to
(bdlrup), including the unaugmented case that follows eq. (bdlrup)): each
check compares against something the oracle does not compute the same way
(dense products, dense singular values, numpy norms, closed forms of the
zero-start stream), and planted mistakes in the oracle are caught."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

SHAPES = [(30, 20, 4), (12, 9, 1), (40, 40, 7), (64, 33, 16), (9, 25, 5)]


def _case(m, n, r, seed):
    return W.tracking_state(m, n, r, seed), W.tracking_update(m, n, seed + 1)


def _bd(d, e):
    return np.diag(d) + np.diag(e, 1)


def _sv(oracle, A):
    """Singular values by the oracle's one-sided Jacobi (which wants rows >= columns)."""
    return oracle.jacobi_sv(A if A.shape[0] >= A.shape[1] else A.T)


def _orth(X):
    return np.linalg.norm(X.T @ X - np.eye(X.shape[1]))


@pytest.mark.parametrize("m,n,r", SHAPES)
def test_exact_rank_r_plus_1_factorization(oracle, m, n, r):
    (U, d, e, V), (b, c) = _case(m, n, r, 11 + r)
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    U2, d2, e2, V2, info = oracle.track_update(U, d, e, V, b, c, keep_all=True)
    assert U2.shape == (m, r + 1) and V2.shape == (n, r + 1) and info[3] == r + 1
    assert np.linalg.norm(A - U2 @ _bd(d2, e2) @ V2.T) <= 1e-13 * np.linalg.norm(A)
    assert _orth(U2) <= 1e-13 and _orth(V2) <= 1e-13
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
    _, d2, e2, _, (delta, gamma, _, _) = oracle.track_update(U, d, e, V, b, c, keep_all=True)
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
    Ut, dt, et, Vt, (_, _, k, rank) = oracle.track_update(U, d, e, V, b, c)
    assert rank == r
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
    assert _orth(Ut) <= 1e-13


def _in_span(rng, X):
    """A vector in span(X), rounded."""
    return X @ rng.standard_normal(X.shape[1])


@pytest.mark.parametrize("side", ["left", "right", "both"])
@pytest.mark.parametrize("m,n,r", [(30, 20, 4), (40, 40, 7), (9, 25, 5), (64, 33, 16)])
def test_unaugmented_sides_give_an_exact_rank_r_factorization(oracle, side, m, n, r):
    """b in span(U) and/or c in span(V): that side is not augmented and the
    result is the rank-r factorization of A + b c^T itself, with nothing
    dropped (the case after eq. (bdlrup)); the wide middle matrix (only c
    augmented) runs through the reversed transpose."""
    (U, d, e, V), (b, c) = _case(m, n, r, 51 + r)
    rng = np.random.default_rng(7 + r)
    if side in ("left", "both"):
        b = _in_span(rng, U)
    if side in ("right", "both"):
        c = _in_span(rng, V)
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    U2, d2, e2, V2, (delta, gamma, k, rank) = oracle.track_update(U, d, e, V, b, c)
    assert (delta == 0) == (side in ("left", "both")) and (gamma == 0) == (side in ("right", "both"))
    assert k == -1 and rank == r and U2.shape == (m, r) and V2.shape == (n, r)
    assert np.linalg.norm(A - U2 @ _bd(d2, e2) @ V2.T) <= 1e-13 * np.linalg.norm(A)
    assert _orth(U2) <= 1e-13 and _orth(V2) <= 1e-13
    s_dense = _sv(oracle, A)[:r]
    s_bgu = oracle.jacobi_sv(_bd(d2, e2))
    assert np.allclose(s_bgu, s_dense, rtol=1e-12, atol=1e-13 * s_dense[0])


def test_wide_middle_matches_its_direct_factorization(oracle):
    """Only c augmented: the reversed-transpose pass gives the same
    bidiagonal, up to signs, as any bidiagonalization of the middle matrix
    with the same first right vector is not fixed, so compare what is
    unique: singular values of B2 against the dense r x (r+1) middle."""
    m, n, r = 30, 20, 6
    (U, d, e, V), (_, c) = _case(m, n, r, 71)
    b = _in_span(np.random.default_rng(3), U)
    _, d2, e2, _, (delta, gamma, _, _) = oracle.track_update(U, d, e, V, b, c)
    assert delta == 0 and gamma > 0
    M = np.hstack([_bd(d, e), np.zeros((r, 1))])
    M += np.outer(U.T @ b, np.append(V.T @ c, gamma))
    s_dense = oracle.jacobi_sv(M.T)
    assert np.allclose(oracle.jacobi_sv(_bd(d2, e2)), s_dense, rtol=1e-13, atol=1e-13 * s_dense[0])


def test_near_span_vector_is_reorthogonalized(oracle):
    """b = U x + 1e-14 noise: one Gram-Schmidt pass leaves b_perp mostly
    rounding noise, not orthogonal to U; the second pass makes the appended
    column orthogonal to working precision, so the factors stay orthonormal."""
    m, n, r = 60, 30, 6
    (U, d, e, V), (_, c) = _case(m, n, r, 81)
    rng = np.random.default_rng(5)
    b = U @ rng.standard_normal(r) + 1e-14 * rng.standard_normal(m)
    xhat, xperp, norm, (s0, s1, s2) = oracle.track_complement(U, b)
    assert 2 * s1 < s0 and s2 >= 0 and norm > 0
    assert np.linalg.norm(U.T @ (xperp / norm)) <= 1e-14
    U2, d2, e2, V2, (delta, _, _, rank) = oracle.track_update(U, d, e, V, b, c, keep_all=True)
    assert delta == norm and rank == r + 1
    assert _orth(U2) <= 1e-13
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    assert np.linalg.norm(A - U2 @ _bd(d2, e2) @ V2.T) <= 1e-13 * np.linalg.norm(A)


def test_complement_against_numpy(oracle):
    """x_hat = A^T x and x_perp = x - A x_hat to rounding; exact zero for a
    vector built from columns of the identity."""
    rng = np.random.default_rng(9)
    A, _ = np.linalg.qr(rng.standard_normal((50, 7)))
    x = rng.standard_normal(50)
    xhat, xperp, norm, _ = oracle.track_complement(A, x)
    assert np.allclose(xhat, A.T @ x, rtol=0, atol=50 * 2.3e-16 * np.linalg.norm(x))
    assert np.allclose(xperp, x - A @ (A.T @ x), rtol=0, atol=1e-14 * np.linalg.norm(x))
    assert abs(norm - np.linalg.norm(x - A @ (A.T @ x))) <= 1e-14 * np.linalg.norm(x)
    E = np.eye(20)[:, :5]
    y = np.zeros(20)
    y[[1, 3]] = [2.0, -1.0]
    xhat, xperp, norm, _ = oracle.track_complement(E, y)
    assert norm == 0.0 and np.array_equal(xhat, y[:5]) and not xperp.any()


@pytest.mark.parametrize("m,n,r", [(40, 30, 4), (25, 12, 3)])
def test_zero_start_link_stream_is_exact_until_rank_r(oracle, m, n, r):
    """The paper's zero start (A0 = 0, U0 = I(:,1:r), V0 = I(:,1:r)) with a
    link-prediction stream c_h = e_h: for h < r every c_h lies in span(V)
    (gamma = 0), so nothing is truncated and after h updates the factors
    reproduce A_h = sum b_k e_k^T exactly, with the dense singular values;
    past h = r the right side is augmented and truncation starts."""
    U, d, e, V = W.zero_start_tracking(m, n, r)
    A = np.zeros((m, n))
    for h, (b, c) in enumerate(W.link_stream(m, n, 2 * r, seed=31, density=0.3)):
        A += np.outer(b, c)
        U, d, e, V, (delta, gamma, k, rank) = oracle.track_update(U, d, e, V, b, c)
        assert rank == r
        if h < r:
            assert gamma == 0.0 and k == -1
            assert np.linalg.norm(A - U @ _bd(d, e) @ V.T) <= 1e-13 * max(np.linalg.norm(A), 1.0)
            s = _sv(oracle, A)[:r]
            assert np.allclose(oracle.jacobi_sv(_bd(d, e)), s, rtol=1e-12, atol=1e-13 * max(s[0], 1.0))
        else:
            assert gamma == 1.0
        assert _orth(U) <= 1e-12 and _orth(V) <= 1e-12


def test_rank_one_span_case_is_refused(oracle):
    """r = 1 with an unaugmented side would need a BGU pass on a 2 x 1 or
    1 x 1 matrix; the oracle refuses it (ORC_ESPAN)."""
    m, n = 10, 8
    U = np.eye(m)[:, :1]
    V = np.eye(n)[:, :1]
    b = np.zeros(m)
    b[0] = 2.0
    with pytest.raises(ValueError, match="-11"):
        oracle.track_update(U, np.ones(1), np.zeros(0), V, b, np.arange(1.0, n + 1))


def test_stream_stays_a_factorization(oracle):
    """A short tracking stream: after each update the factors are
    orthonormal."""
    m, n, r = 50, 30, 5
    (U, d, e, V), _ = _case(m, n, r, 41)
    rng = np.random.default_rng(42)
    for step in range(8):
        b = rng.standard_normal(m) * 0.3
        c = rng.standard_normal(n) * 0.3
        U, d, e, V, _ = oracle.track_update(U, d, e, V, b, c)
        assert _orth(U) <= 1e-12 and _orth(V) <= 1e-12


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
        Ut, dt, et, Vt, (_, _, k, _) = oracle.track_update(U, d, e, V, b, c)
    finally:
        oracle.set_mutation(0)
    exact = np.linalg.norm(A - Uf @ _bd(df, ef) @ Vf.T) <= 1e-13 * np.linalg.norm(A)
    orth = _orth(Uf) <= 1e-13
    norms = np.linalg.norm(_bd(df, ef), axis=0)
    smallest = norms[k] == norms.min()
    assert not (exact and orth and smallest)


def test_planted_single_pass_is_caught(oracle):
    """Without the second orthogonalization pass the near-span case loses
    orthogonality."""
    m, n, r = 60, 30, 6
    (U, d, e, V), (_, c) = _case(m, n, r, 81)
    rng = np.random.default_rng(5)
    b = U @ rng.standard_normal(r) + 1e-14 * rng.standard_normal(m)
    oracle.set_mutation(11)
    try:
        U2, *_ = oracle.track_update(U, d, e, V, b, c, keep_all=True)
    finally:
        oracle.set_mutation(0)
    assert _orth(U2) > 1e-6


def test_planted_unreversed_superdiagonal_is_caught(oracle):
    """The wide case with e not reversed breaks the reconstruction."""
    m, n, r = 30, 20, 5
    (U, d, e, V), (_, c) = _case(m, n, r, 91)
    b = _in_span(np.random.default_rng(4), U)
    A = U @ _bd(d, e) @ V.T + np.outer(b, c)
    oracle.set_mutation(12)
    try:
        U2, d2, e2, V2, _ = oracle.track_update(U, d, e, V, b, c)
    finally:
        oracle.set_mutation(0)
    assert np.linalg.norm(A - U2 @ _bd(d2, e2) @ V2.T) > 1e-6 * np.linalg.norm(A)
