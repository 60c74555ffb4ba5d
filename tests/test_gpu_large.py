"""Generation with the working band in device memory (large n).

The band (offsets -2..3) and u, v of the rotation generator live in LDS up
to n = 2449 (square) and in device memory beyond.  The device-memory variant
is checked bit-exactly on small shapes (forced), then on shapes that need it
(n = 3000, 4096 and the largest served size, 8192) against the oracle on
sampled rows of Q and P and on all of d and e.
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


@pytest.mark.parametrize("m,n,r", [(2, 2, 1), (5, 5, 1), (14, 12, 2), (65, 64, 1), (200, 200, 3), (257, 191, 2)])
def test_global_band_generation_bit_exact(bdu, oracle, m, n, r):
    f = W.factorization(m, n, 600 + m)
    (B, C), = W.gaussian_updates(m, n, 1, 601 + n, r=r)
    bdu.set_generation_in_lds(False)
    try:
        h = bdu.Handle(f.Q, f.d, f.e, f.P)
    finally:
        bdu.set_generation_in_lds(True)
    h.update(B, C)
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_update(ref, B, C)
    for nm, x, y in zip("QdeP", h.read(), (ref.Q, ref.d, ref.e, ref.P)):
        _eq(nm, x, y)
    h.close()


@pytest.mark.parametrize("m,n", [(3000, 3000), (4096, 4096), (4200, 4096)])
def test_large_n_sampled_rows(bdu, oracle, m, n):
    f = W.factorization(m, n, 620 + n)
    (B, C), = W.gaussian_updates(m, n, 1, 621)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update(B, C)
    Q1, d1, e1, P1 = h.read()
    h.close()
    u = oracle.project(f.Q, B[:, 0])
    v = oracle.project(f.P, C[:, 0])
    rng = np.random.default_rng(622)
    qr = np.sort(rng.choice(m, 48, replace=False))
    pr = np.sort(rng.choice(n, 48, replace=False))
    Qr, d, e, Pr = oracle.bgu_pass_rows(m, n, f.Q[qr], f.d, f.e, f.P[pr], u, v)
    _eq("d", d1, d)
    _eq("e", e1, e)
    _eq("Q rows", Q1[qr], Qr)
    _eq("P rows", P1[pr], Pr)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("in_lds", [True, False])
@pytest.mark.parametrize("m,n,r", [(2, 2, 1), (14, 12, 2), (65, 64, 1), (257, 191, 2)])
def test_unsplit_pass_bit_exact(bdu, oracle, m, n, r, in_lds, mode):
    """Passes generated in one launch and applied after it (mode 0), or
    split after phase 1 only (mode 1), give the oracle's result too; the
    other tests run the default (phase 2 in segments)."""
    f = W.factorization(m, n, 610 + m)
    (B, C), = W.gaussian_updates(m, n, 1, 611 + n, r=r)
    bdu.set_split_pass(mode)
    bdu.set_generation_in_lds(in_lds)
    try:
        h = bdu.Handle(f.Q, f.d, f.e, f.P)
    finally:
        bdu.set_split_pass(True)
        bdu.set_generation_in_lds(True)
    h.update(B, C)
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_update(ref, B, C)
    for nm, x, y in zip("QdeP", h.read(), (ref.Q, ref.d, ref.e, ref.P)):
        _eq(nm, x, y)
    h.close()


def test_largest_served_size(bdu, oracle):
    """n = 8192, the largest size of the serving workload: one update with
    the band in device memory and the pass in segments; d, e and 16 sampled
    rows of Q and P bit for bit.  The factors are single Householder
    reflections (orthogonal and cheap to form at this size)."""
    n = 8192
    rng = np.random.default_rng(720)
    q = rng.standard_normal(n)
    q /= np.linalg.norm(q)
    p = rng.standard_normal(n)
    p /= np.linalg.norm(p)
    Q = np.asfortranarray(np.eye(n) - 2.0 * np.outer(q, q))
    P = np.asfortranarray(np.eye(n) - 2.0 * np.outer(p, p))
    d = rng.uniform(1.0, 10.0, n)
    e = rng.uniform(0.0, 1.0, n - 1)
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    h = bdu.Handle(Q, d, e, P)
    h.update(b.reshape(n, 1), c.reshape(n, 1))
    Q1, d1, e1, P1 = h.read()
    h.close()
    u = oracle.project(Q, b)
    v = oracle.project(P, c)
    qr = np.sort(rng.choice(n, 16, replace=False))
    pr = np.sort(rng.choice(n, 16, replace=False))
    Qr, dr, er, Pr = oracle.bgu_pass_rows(n, n, Q[qr], d, e, P[pr], u, v)
    _eq("d", d1, dr)
    _eq("e", e1, er)
    _eq("Q rows", Q1[qr], Qr)
    _eq("P rows", P1[pr], Pr)
