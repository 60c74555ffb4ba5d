"""Pins of the orthogonality monitor and its Newton-Schulz correction
(oracle side): closed forms for a known perturbation, the polar factor from
an SVD, quadratic convergence, and a planted sign mistake."""
import numpy as np
import pytest


def _orth(rng, k):
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return Q


@pytest.mark.parametrize("k", [5, 40, 130])
def test_orthogonal_matrix_has_no_drift(oracle, k):
    Q = _orth(np.random.default_rng(k), k)
    assert oracle.orth_error(Q) <= 10 * k * np.finfo(float).eps


@pytest.mark.parametrize("k,eps", [(8, 1e-6), (60, 1e-9), (200, 1e-11)])
def test_known_perturbation(oracle, k, eps):
    """Q = Q0 (I + eps S), S symmetric: Q^T Q - I = 2 eps S + eps^2 S^2."""
    rng = np.random.default_rng(k)
    Q0 = _orth(rng, k)
    S = rng.standard_normal((k, k))
    S = (S + S.T) / 2
    Q = Q0 @ (np.eye(k) + eps * S)
    want = np.linalg.norm(2 * eps * S + eps * eps * S @ S)
    assert abs(oracle.orth_error(Q) - want) <= 1e-6 * want + 50 * k * np.finfo(float).eps


@pytest.mark.parametrize("k,eps", [(8, 1e-6), (60, 1e-8), (200, 1e-9)])
def test_step_reaches_the_polar_factor(oracle, k, eps):
    """One step from drift e lands within O(e^2) of the polar factor U V^T
    (SVD) and leaves a drift of order e^2."""
    rng = np.random.default_rng(10 + k)
    Q0 = _orth(rng, k)
    S = rng.standard_normal((k, k))
    Q = Q0 @ (np.eye(k) + eps * (S + S.T) / 2) + eps * rng.standard_normal((k, k)) / np.sqrt(k)
    e0 = oracle.orth_error(Q)
    U, _, Vt = np.linalg.svd(Q)
    polar = U @ Vt
    Q1 = oracle.reorth_step(Q)
    tiny = 100 * k * np.finfo(float).eps
    assert np.linalg.norm(Q1 - polar) <= 2 * e0 * e0 + tiny
    assert oracle.orth_error(Q1) <= 2 * e0 * e0 + tiny
    assert oracle.orth_error(Q1) < e0


def test_planted_sign_mistake_is_caught(oracle):
    rng = np.random.default_rng(3)
    k = 30
    Q = _orth(rng, k) + 1e-8 * rng.standard_normal((k, k))
    wrong = Q + (Q @ oracle.orth_gram(Q)) / 2.0
    assert oracle.orth_error(wrong) > oracle.orth_error(Q)
    assert oracle.orth_error(oracle.reorth_step(Q)) < oracle.orth_error(Q)
