"""Truncated bidiagonal approximation (Section 1.3, eqs. (trBD), (errtrBD)) on
the GPU, bit for bit against the oracle."""
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


def _same(bdu, oracle, h, Q, d, e, P, r):
    idx, err2, Qr, Pr = h.truncated_bd(r)
    widx, werr2, wQr, wPr = oracle.truncated_bd(Q, d, e, P, r)
    assert np.array_equal(idx, widx)
    assert err2 == werr2
    assert np.array_equal(Qr, wQr) and np.array_equal(Pr, wPr)


@pytest.mark.parametrize("m,n,r", [(30, 20, 5), (12, 12, 1), (40, 25, 25), (300, 257, 64), (700, 5, 3)])
def test_matches_the_oracle(bdu, oracle, m, n, r):
    f = W.factorization(m, n, 300 + r)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    _same(bdu, oracle, h, f.Q, f.d, f.e, f.P, r)
    h.close()


def test_ties_and_after_updates(bdu, oracle):
    m, n = 40, 30
    f = W.factorization(m, n, 5)
    d = f.d.copy()
    d[3] = d[7] = d[11] = 4.0
    e = f.e.copy()
    e[2] = e[6] = e[10] = 0.0
    h = bdu.Handle(f.Q, d, e, f.P)
    _same(bdu, oracle, h, f.Q, d, e, f.P, 10)
    for B, C in W.gaussian_updates(m, n, 3, 6):
        h.update(B, C)
    Q, d2, e2, P = h.read()
    for r in (1, 7, n):
        _same(bdu, oracle, h, Q, d2, e2, P, r)
    h.close()
