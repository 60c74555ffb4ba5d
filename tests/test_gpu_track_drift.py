"""The tracker's orthogonality monitor (Section 4.2: the thin factors are
checked for loss of orthogonality periodically and reorthogonalized now
and then) against the oracle's plain fp64 products.

Tolerances as for the full factors (u = 2^-53, gamma_m = m u / (1 - m u)):
an entry of X^T X is a length-m dot product of columns of norm ~1, so the
drifts of the GPU (matrix cores) and the oracle differ by at most
2 gamma_m r, and the corrected factor X - X E / 2 by at most
gamma_m sqrt(r) + 4 u |X| per entry."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

pytestmark = pytest.mark.gpu
U_ROUND = 2.0 ** -53


def gamma(m):
    return m * U_ROUND / (1 - m * U_ROUND)


@pytest.fixture(scope="module")
def bdu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_02840_amd import bdu as B
    B.lib()
    return B


def _perturbed(m, n, r, seed, eps):
    U, d, e, V = W.tracking_state(m, n, r, seed)
    rng = np.random.default_rng(seed + 1)
    U = np.asfortranarray(U + eps * rng.standard_normal(U.shape) / np.sqrt(m))
    V = np.asfortranarray(V + eps * rng.standard_normal(V.shape) / np.sqrt(n))
    return U, d, e, V


def _check_step(oracle, got, X):
    rows, r = X.shape
    want = oracle.reorth_step(X)
    assert np.all(np.abs(got - want) <= gamma(rows) * np.sqrt(r) + 4 * U_ROUND * np.abs(X))


@pytest.mark.parametrize("m,n,r,eps", [(300, 200, 7, 1e-9), (1000, 700, 100, 1e-8), (130, 300, 64, 1e-10),
                                       (40, 40, 40, 1e-7), (500, 90, 1, 1e-9)])
def test_drift_and_step_match_the_oracle(bdu, oracle, m, n, r, eps):
    U, d, e, V = _perturbed(m, n, r, 60 + r, eps)
    t = bdu.Tracker(U, d, e, V)
    eu, ev = t.orth_error()
    for got, X, k in ((eu, U, m), (ev, V, n)):
        want = oracle.orth_error(X)
        assert abs(got - want) <= 2 * gamma(k) * r + 1e-12 * want, (got, want)
    assert t.reorthogonalize(0.0) == (eu, ev)
    U2, d2, e2, V2 = t.read()
    assert np.array_equal(d2, d) and np.array_equal(e2, e)
    _check_step(oracle, U2, U)
    _check_step(oracle, V2, V)
    for X2, X in ((U2, U), (V2, V)):
        e0 = oracle.orth_error(X)
        assert oracle.orth_error(X2) <= 4 * e0 * e0 + 64 * gamma(X.shape[0]) * X.shape[1]
    t.close()


def test_tolerance_above_the_drift_changes_nothing(bdu):
    U, d, e, V = _perturbed(200, 150, 12, 5, 1e-12)
    t = bdu.Tracker(U, d, e, V)
    eu, ev = t.reorthogonalize(1.0)
    assert eu < 1.0 and ev < 1.0
    U2, _, _, V2 = t.read()
    assert np.array_equal(U2, U) and np.array_equal(V2, V)
    t.close()


def test_periodic_check_corrects_and_the_stream_continues(bdu, oracle):
    """Every third update checks the drift; a drifted start is corrected at
    the first check, and the updates around the check follow the oracle in
    lockstep from the GPU's own factors (projections from the GPU, the rest
    bit for bit)."""
    m, n, r = 400, 300, 16
    U, d, e, V = _perturbed(m, n, r, 21, 1e-9)
    t = bdu.Tracker(U, d, e, V)
    t.set_drift_check(3, 1e-11)
    for step in range(7):
        state = t.read()
        b, c = W.tracking_update(m, n, 300 + step)
        t.update(b, c)
        if (step + 1) % 3 == 0:
            st = t.drift_stats()
            assert st["checks"] == (step + 1) // 3
            continue  # the check has changed the factors after the update
        bh, ch, qb, qc = t.last_projection()
        dl, gm, _ = t.last()
        want = oracle.track_finish(*state, bh, ch, dl, gm, qb, qc)[:4]
        for nm, x, y in zip("UdeV", t.read(), want):
            assert np.array_equal(x, y), f"step {step} {nm}"
    st = t.drift_stats()
    assert st["checks"] == 2
    assert st["corrections"] >= 2  # both sides at the first check
    eu, ev = t.orth_error()
    assert eu <= 1e-12 and ev <= 1e-12
    t.set_drift_check(0, 0.0)
    t.update(*W.tracking_update(m, n, 400))
    assert t.drift_stats()["checks"] == 2
    t.close()


def test_drift_check_at_full_rank_shape(bdu, oracle):
    """r = n = 2000 on 10000 x 2000 (the tracking shape the paper's
    recommendation runs use): the drift of the tracked factors against the
    oracle's, after a few updates."""
    m, n, r = 10000, 2000, 2000
    U, d, e, V = W.tracking_state(m, n, r, 8)
    t = bdu.Tracker(U, d, e, V)
    for step in range(3):
        t.update(*W.tracking_update(m, n, 90 + step))
    U2, _, _, V2 = t.read()
    eu, ev = t.orth_error()
    for got, X in ((eu, U2), (ev, V2)):
        want = oracle.orth_error(X)
        assert abs(got - want) <= 2 * gamma(X.shape[0]) * r + 1e-12 * want
        assert got <= 1e-11
    t.close()
