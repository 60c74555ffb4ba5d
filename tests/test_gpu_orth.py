"""Orthogonality monitor and Newton-Schulz correction on the GPU (FP64
matrix cores) against the oracle's plain fp64 products.

Tolerances (u = 2^-53, gamma_m = m u / (1 - m u)): an entry of X^T X is a
length-m dot product of columns of norm ~1, so each side's rounding is at
most gamma_m and the two evaluations of E = X^T X - I differ by at most
2 gamma_m per entry, hence the drifts by at most 2 gamma_m k.  The corrected
factor X - X E / 2 then differs by at most |X| |dE| / 2 <= gamma_m sqrt(m)
per entry (rows of norm ~1), plus the final subtraction's rounding on each
side (2 u |X|)."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def gamma(m):
    return m * U / (1 - m * U)


@pytest.fixture(scope="module")
def bdu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_02840_amd import bdu as B
    B.lib()
    return B


def _perturbed(m, n, seed, eps):
    f = W.factorization(m, n, seed)
    rng = np.random.default_rng(seed + 1)
    Q = np.asfortranarray(f.Q + eps * rng.standard_normal((m, m)) / np.sqrt(m))
    P = np.asfortranarray(f.P + eps * rng.standard_normal((n, n)) / np.sqrt(n))
    return Q, f.d, f.e, P


@pytest.mark.parametrize("m,n,eps", [(200, 150, 1e-9), (300, 300, 1e-7), (513, 257, 1e-10), (130, 64, 0.0)])
def test_drift_and_step_match_the_oracle(bdu, oracle, m, n, eps):
    Q, d, e, P = _perturbed(m, n, 40 + m, eps)
    h = bdu.Handle(Q, d, e, P)
    eq, ep = h.orth_error()
    for got, X, k in ((eq, Q, m), (ep, P, n)):
        want = oracle.orth_error(X)
        assert abs(got - want) <= 2 * gamma(k) * k + 1e-12 * want, (got, want)
    before = h.reorthogonalize(0.0)
    assert before == (eq, ep)
    Q2, d2, e2, P2 = h.read()
    assert np.array_equal(d2, d) and np.array_equal(e2, e)
    for got, X, k in ((Q2, Q, m), (P2, P, n)):
        want = oracle.reorth_step(X)
        bound = gamma(k) * np.sqrt(k) + 4 * U * np.abs(X)
        assert np.all(np.abs(got - want) <= bound)
        # from drift e0 the step leaves O(e0^2) above the rounding floor
        e0 = oracle.orth_error(X)
        floor = oracle.orth_error(oracle.reorth_step(oracle.reorth_step(X)))
        assert oracle.orth_error(got) <= 4 * e0 * e0 + 4 * floor + 2 * gamma(k) * k
    h.close()


def test_tolerance_above_the_drift_changes_nothing(bdu):
    Q, d, e, P = _perturbed(120, 90, 7, 1e-12)
    h = bdu.Handle(Q, d, e, P)
    eq, ep = h.reorthogonalize(1.0)
    assert eq < 1.0 and ep < 1.0
    Q2, _, _, P2 = h.read()
    assert np.array_equal(Q2, Q) and np.array_equal(P2, P)
    h.close()


def test_stream_continues_bit_exact_after_a_correction(bdu, oracle):
    """Drift after updates matches the oracle's measure of the same factors;
    after a correction the handle keeps updating exactly like the oracle
    started from the corrected factors."""
    m, n = 160, 120
    f = W.factorization(m, n, 71)
    ups = W.gaussian_updates(m, n, 12, 72)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    for B, C in ups[:6]:
        h.update(B, C)
    Q, d, e, P = h.read()
    eq, ep = h.reorthogonalize(0.0)
    assert abs(eq - oracle.orth_error(Q)) <= 2 * gamma(m) * m
    assert abs(ep - oracle.orth_error(P)) <= 2 * gamma(n) * n
    Qc, dc, ec, Pc = h.read()
    ref = oracle.State(Qc, dc, ec, Pc)
    for B, C in ups[6:]:
        h.update(B, C)
        oracle.bgu_update(ref, B, C)
    got = h.read()
    for nm, x, y in zip("QdeP", got, (ref.Q, ref.d, ref.e, ref.P)):
        assert np.array_equal(x, y), nm
    h.close()
