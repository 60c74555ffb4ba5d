"""GPU parity of the Householder bidiagonal update (BHU; Section 3.3,
Algorithm 1, Theorem 1) through the C ABI against the oracle.

The GPU reaches each column and row of the partially reduced matrix through
products with the stored reflectors and the explicit inverses of T and R;
the oracle solves with the middle matrix of Theorem 1.  Same mathematics,
different summation orders, so agreement is within a tolerance: both are
backward stable (backward error c n u ||A||), and for these workloads (well
separated singular values, gaps about ||A|| / n) a backward error moves the
bidiagonal entries and the factors by at most about n times that, so
d, e agree to 32 u n^2 ||A+||_F and the entries of Q+, P+ to 32 u n^2.
At the full n = 2048 size: the closed form of ||Bd+||_F, orthogonality,
sampled entries of Q+ Bd+ P+^T = A + b c^T, and the singular values of the
Givens update of the same matrix.
"""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def bdu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_02840_amd import bdu as B
    B.lib()
    return B


def _bd(d, e, m):
    n = len(d)
    B = np.zeros((m, n))
    B[np.arange(n), np.arange(n)] = d
    B[np.arange(n - 1), np.arange(1, n)] = e
    return B


@pytest.mark.parametrize("m,n", [(2, 2), (3, 2), (5, 2), (3, 3), (5, 5), (14, 12), (65, 64), (66, 64), (130, 97),
                                 (200, 200), (257, 191), (300, 17), (500, 3)])
def test_householder_update_matches_oracle(bdu, oracle, m, n):
    f = W.factorization(m, n, 500 + m)
    rng = np.random.default_rng(501 + n)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update_householder(b, c)
    Q, d, e, P = h.read()
    h.close()
    Qo, do, eo, Po = oracle.bhu_update(f.Q, f.d, f.e, f.P, b, c)
    A2 = f.dense() + np.outer(b, c)
    tol = 32 * U * n * n
    scale = np.linalg.norm(A2)
    assert np.abs(d - do).max() <= tol * scale
    assert np.abs(e - eo).max() <= tol * scale
    assert np.abs(Q - Qo).max() <= tol
    assert np.abs(P - Po).max() <= tol


def test_zero_update_is_the_identity(bdu, oracle):
    m, n = 70, 64
    f = W.factorization(m, n, 520)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update_householder(np.zeros(m), np.ones(n))
    Q, d, e, P = h.read()
    h.close()
    assert np.array_equal(d, f.d) and np.array_equal(e, f.e)
    assert np.array_equal(Q, f.Q) and np.array_equal(P, f.P)


def test_repeated_updates_and_mixed_methods(bdu, oracle):
    """Three Householder updates then a Givens one on the same handle: the
    scratch is reused, and the state stays a factorization of the sum.  After
    several updates the large singular values separate from a cluster of
    small ones, whose bidiagonal entries are then ill conditioned, so the
    comparison with the oracle is on the singular values (perturbed by at
    most the backward error) and on the reconstruction, not entry by entry."""
    m, n = 90, 80
    f = W.factorization(m, n, 530)
    rng = np.random.default_rng(531)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    A = f.dense()
    ref = (f.Q, f.d, f.e, f.P)
    for _ in range(3):
        b, c = rng.standard_normal(m), rng.standard_normal(n)
        h.update_householder(b, c)
        A = A + np.outer(b, c)
        ref = oracle.bhu_update(*ref, b, c)
    Q, d, e, P = h.read()
    scale = np.linalg.norm(A)
    assert np.abs(Q @ _bd(d, e, m) @ P.T - A).max() <= 1e-12 * scale
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 1e-13 * n
    s_gpu = np.linalg.svd(_bd(d, e, m), compute_uv=False)
    s_ref = np.linalg.svd(_bd(ref[1], ref[2], m), compute_uv=False)
    assert np.abs(s_gpu - s_ref).max() <= 1e-13 * n * scale
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    h.update(b.reshape(m, 1), c.reshape(n, 1))
    A = A + np.outer(b, c)
    Q, d, e, P = h.read()
    h.close()
    assert np.abs(Q @ _bd(d, e, m) @ P.T - A).max() <= 1e-12 * np.linalg.norm(A)


def test_full_size_properties(bdu, oracle):
    n = 2048
    f = W.factorization(n, n, 540)
    rng = np.random.default_rng(541)
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update_householder(b, c)
    Q, d, e, P = h.read()
    eq, ep = h.orth_error()
    h.close()
    # ||Bd+||_F^2 = ||A||_F^2 + 2 b^T A c + ||b||^2 ||c||^2, A = Q Bd P^T
    Bd = f.d @ f.d + f.e @ f.e
    Ac = f.Q @ (_bd(f.d, f.e, n) @ (f.P.T @ c))
    want = Bd + 2 * (b @ Ac) + (b @ b) * (c @ c)
    got = d @ d + e @ e
    assert abs(got - want) <= 1e-10 * want
    assert eq <= 1e-11 and ep <= 1e-11
    rows = rng.choice(n, 8, replace=False)
    A_rows = f.Q[rows] @ _bd(f.d, f.e, n) @ f.P.T + np.outer(b[rows], c)
    got_rows = Q[rows] @ _bd(d, e, n) @ P.T
    assert np.abs(got_rows - A_rows).max() <= 1e-11 * np.sqrt(want)
    # the Givens update of the same matrix has the same singular values
    g = bdu.Handle(f.Q, f.d, f.e, f.P)
    g.update(b.reshape(n, 1), c.reshape(n, 1))
    _, dg, eg, _ = g.read()
    g.close()
    s1 = np.linalg.svd(_bd(d, e, n), compute_uv=False)
    s2 = np.linalg.svd(_bd(dg, eg, n), compute_uv=False)
    assert np.abs(s1 - s2).max() <= 1e-10 * np.sqrt(want)

