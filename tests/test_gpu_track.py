"""Subspace tracking (Section 4) on the GPU against the oracle, in lockstep.

The GPU sums its projections in another order than the oracle (chunks of
256 rows), so the two are compared in two parts:
  * the projections b_hat, c_hat, the norms delta, gamma and the unit
    complements, within the rounding bounds of the sums (below);
  * everything that follows from them (the middle BGU pass, the
    truncation, the thin products), bit for bit: the oracle's
    orc_track_finish is fed the GPU's projections and must give the same
    U, d, e, V.

Bounds (u = 2^-53).  Each b_hat_j is an inner product of length m, and
any two summation orders of it lie within 2 gamma_m sum_i |U_ij b_i| <=
2 m u ||b|| of each other (Cauchy-Schwarz, unit columns); a second pass
adds at most as much again.  The complement b - U b_hat then differs by
at most ||U db_hat|| <= sqrt(r) * 4 m u ||b|| plus the rounding of its own
r-term sums and subtraction, (r + 1) u ||b|| per entry, so its norm
delta by at most that, and the unit complement by twice that over delta."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

pytestmark = pytest.mark.gpu
U_ROUND = 2.0 ** -53


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


def _check_side(oracle, name, A, x, xhat_g, q_g, norm_g):
    rows, r = A.shape
    xhat, xperp, norm, _ = oracle.track_complement(A, x)
    nx = np.linalg.norm(x)
    t_hat = 4 * rows * U_ROUND * nx
    t_perp = (np.sqrt(r) * 4 * rows + r + 1) * U_ROUND * nx + t_hat
    assert np.max(np.abs(xhat_g - xhat), initial=0.0) <= t_hat, f"{name}: projection"
    assert (norm_g > 0) == (norm > 0), f"{name}: augmented on one side only ({norm_g} vs {norm})"
    assert abs(norm_g - norm) <= t_perp + rows * U_ROUND * norm, f"{name}: norm"
    if norm > 0:
        assert np.linalg.norm(q_g - xperp / norm) <= 2 * t_perp / norm + 4 * rows * U_ROUND, f"{name}: complement"


def _lockstep(bdu, oracle, t, state, b, c, tag):
    """One update on the GPU and the oracle's continuation from the GPU's
    projections; returns the new oracle state after comparing."""
    U, d, e, V = state
    t.update(b, c)
    dl, gm, k = t.last()
    bh, ch, qb, qc = t.last_projection()
    _check_side(oracle, f"{tag} b", U, b, bh, qb, dl)
    _check_side(oracle, f"{tag} c", V, c, ch, qc, gm)
    U2, d2, e2, V2, info = oracle.track_finish(U, d, e, V, bh, ch, dl, gm, qb if dl > 0 else None,
                                               qc if gm > 0 else None)
    for nm, x, y in zip("UdeV", t.read(), (U2, d2, e2, V2)):
        _eq(f"{tag} {nm}", x, y)
    assert k == info[2], tag
    return (U2, d2, e2, V2), (dl, gm, k)


# ragged sizes, r across the 64-column projection tile, m < n and m > n
SHAPES = [(30, 20, 4), (12, 9, 1), (9, 25, 5), (40, 40, 7), (130, 70, 64), (300, 200, 63), (257, 300, 65),
          (1000, 700, 100)]


@pytest.mark.parametrize("m,n,r", SHAPES)
def test_tracking_stream_lockstep(bdu, oracle, m, n, r):
    state = W.tracking_state(m, n, r, 500 + r)
    t = bdu.Tracker(*state)
    for step in range(4):
        b, c = W.tracking_update(m, n, 600 + 7 * step + r, scale=0.5 + step)
        state, (dl, gm, k) = _lockstep(bdu, oracle, t, state, b, c, f"step {step}")
        assert dl > 0 and gm > 0 and k >= 0
    t.close()


@pytest.mark.parametrize("m,n,r,steps", [(300, 200, 16, 34), (1000, 700, 64, 140), (40, 30, 2, 6)])
def test_zero_start_link_stream(bdu, oracle, m, n, r, steps):
    """The paper's zero start (U0 = I(:,1:r), V0 = I(:,1:r), B0 = 0) with
    c_h = e_h: the first r updates leave the right side unaugmented (gamma =
    0, nothing truncated), later ones augment both sides."""
    state = W.zero_start_tracking(m, n, r)
    t = bdu.Tracker(*state)
    A = np.zeros((m, n))
    for h, (b, c) in enumerate(W.link_stream(m, n, steps, seed=900 + r, density=0.05)):
        A += np.outer(b, c)
        state, (dl, gm, k) = _lockstep(bdu, oracle, t, state, b, c, f"h {h}")
        if h < r:
            assert gm == 0.0 and k == -1
        else:
            assert gm == 1.0
    U, d, e, V = state
    assert np.linalg.norm(U.T @ U - np.eye(r)) <= 1e-12 and np.linalg.norm(V.T @ V - np.eye(r)) <= 1e-12
    t.close()


@pytest.mark.parametrize("side", ["left", "right", "both"])
@pytest.mark.parametrize("m,n,r", [(130, 70, 9), (60, 90, 12), (400, 300, 33)])
def test_unaugmented_sides(bdu, oracle, side, m, n, r):
    """b in span(U) and/or c in span(V): exact rank-r updates, including the
    reversed transpose when only c is augmented."""
    state = W.tracking_state(m, n, r, 40 + r)
    t = bdu.Tracker(*state)
    rng = np.random.default_rng(r)
    for step in range(3):
        b, c = W.tracking_update(m, n, 70 + step)
        if side in ("left", "both"):
            b = state[0] @ rng.standard_normal(r)
        if side in ("right", "both"):
            c = state[3] @ rng.standard_normal(r)
        state, (dl, gm, k) = _lockstep(bdu, oracle, t, state, b, c, f"{side} {step}")
        assert (dl == 0) == (side in ("left", "both")) and (gm == 0) == (side in ("right", "both"))
        assert k == -1
    t.close()


def test_square_right_basis_is_never_augmented(bdu, oracle):
    """r = n: V spans everything, so gamma = 0 on every update."""
    m, n = 150, 40
    state = W.tracking_state(m, n, n, 3)
    t = bdu.Tracker(*state)
    for step in range(3):
        b, c = W.tracking_update(m, n, 10 + step)
        state, (dl, gm, k) = _lockstep(bdu, oracle, t, state, b, c, f"step {step}")
        assert gm == 0.0 and dl > 0
    t.close()


def test_near_span_vector_keeps_orthogonality(bdu, oracle):
    """b = U x + 1e-13 noise: the second orthogonalization pass keeps the
    appended column orthogonal, so U stays orthonormal."""
    m, n, r = 500, 300, 20
    state = W.tracking_state(m, n, r, 8)
    t = bdu.Tracker(*state)
    rng = np.random.default_rng(9)
    b = state[0] @ rng.standard_normal(r) + 1e-13 * rng.standard_normal(m)
    c = rng.standard_normal(n)
    state, (dl, gm, k) = _lockstep(bdu, oracle, t, state, b, c, "near span")
    assert dl > 0
    U = t.read()[0]
    assert np.linalg.norm(U.T @ U - np.eye(r)) <= 1e-13
    t.close()


def test_rank_one_span_case_is_refused_without_change(bdu, oracle):
    m, n, r = 20, 16, 1
    U = np.asfortranarray(np.eye(m)[:, :r])
    V = np.asfortranarray(np.eye(n)[:, :r])
    d, e = np.array([3.0]), np.zeros(0)
    t = bdu.Tracker(U, d, e, V)
    b = np.zeros(m)
    b[0] = 1.5
    c = np.arange(1.0, n + 1)
    with pytest.raises(bdu.BduError) as ei:
        t.update(b, c)
    assert ei.value.status == bdu.BDU_ESPAN
    for nm, x, y in zip("UdeV", t.read(), (U, d, e, V)):
        _eq(f"unchanged {nm}", x, y)
    b2 = np.linspace(-1.0, 1.0, m)
    _lockstep(bdu, oracle, t, (U, d, e, V), b2, c, "after")
    t.close()


def test_device_inputs(bdu, oracle):
    import torch
    m, n, r = 90, 60, 12
    U, d, e, V = W.tracking_state(m, n, r, 77)
    dev = lambda a: torch.from_numpy(a).to("cuda:0")
    Ut = torch.from_numpy(U.T.copy()).to("cuda:0").T  # column-major on the device
    Vt = torch.from_numpy(V.T.copy()).to("cuda:0").T
    t = bdu.Tracker(Ut, dev(d), dev(e), Vt)
    b, c = W.tracking_update(m, n, 78)
    t.update(dev(b), dev(c))
    bh, ch, qb, qc = t.last_projection()
    dl, gm, _ = t.last()
    want = oracle.track_finish(U, d, e, V, bh, ch, dl, gm, qb, qc)[:4]
    for nm, x, y in zip("UdeV", t.read(), want):
        _eq(nm, x, y)
    t.close()
