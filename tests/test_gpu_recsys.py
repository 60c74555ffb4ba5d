"""A recommendation-shaped stream (the shape of the paper's rating
experiments, Section 4, on synthetic data).

Users x items integer ratings 1..5 (sparse, Zipf item popularity); the
initial factorization is the oracle's Householder bidiagonalization of the
rating matrix; updates replace users' rows (b = e_i, c = new row - old row)
r at a time (rank r = 1, 4, 8) and now and then subtract the row means
(b = -A e / n, c = e).  Every call is compared bit for bit with the oracle,
and the final factors reproduce the dense rating matrix.
"""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bdu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_02840_amd import bdu as B
    B.lib()
    return B


def _eq(name, x, y):
    x, y = np.asarray(x), np.asarray(y)
    assert x.shape == y.shape, name
    bad = np.flatnonzero(~(x == y).ravel())
    assert bad.size == 0, f"{name}: {bad.size} of {x.size} differ, first at {bad[0]}"


@pytest.mark.parametrize("r", [1, 4, 8])
def test_rating_stream_bit_exact(bdu, oracle, r):
    users, items = 420, 150
    A = W.ratings(users, items, density=0.05, seed=700 + r)
    Q, d, e, P = oracle.bidiag_householder(A)
    h = bdu.Handle(Q, d, e, P)
    ref = oracle.State(Q, d, e, P)
    rng = np.random.default_rng(701 + r)
    for call in range(6):
        if call == 3:  # subtract the row means: A <- A - (A e / n) e^T
            B = -(A @ np.ones(items)) / items
            C = np.ones(items)
            B, C = np.asfortranarray(B[:, None]), np.asfortranarray(C[:, None])
        else:  # replace r users' rows
            who = rng.choice(users, r, replace=False)
            B = np.zeros((users, r), order="F")
            C = np.zeros((items, r), order="F")
            for k, i in enumerate(who):
                B[i, k] = 1.0
                C[:, k] = W.rating_row(rng, items, nnz=12) - A[i]
        A = A + B @ C.T
        h.update(B, C)
        oracle.bgu_update(ref, B, C)
        got = h.read()
        for nm, x, y in zip("QdeP", got, (ref.Q, ref.d, ref.e, ref.P)):
            _eq(f"call {call} {nm}", x, y)
    Qg, dg, eg, Pg = got
    h.close()
    Bd = np.zeros((users, items))
    Bd[np.arange(items), np.arange(items)] = dg
    Bd[np.arange(items - 1), np.arange(1, items)] = eg
    assert np.linalg.norm(A - Qg @ Bd @ Pg.T) <= 1e-12 * np.linalg.norm(A)
