"""Pins for the CPU oracle, independent of the oracle itself.

Every check here compares the oracle with something the paper or the
mathematics fixes: closed forms (the already-bidiagonal case of Section 3.4,
zero-start streams of Section 4, 2x2 problems), invariants of the
factorization (A+ = Q+ B+ P+^T, orthogonality, the Frobenius norm the paper
reports as its error measure), dense recomputation (Jacobi singular values,
Householder and Golub-Kahan bidiagonalization of Section 2 with the
implicit-Q start vector), exact rational arithmetic, and the counts the
paper states (2n-3 phase-2 bulge chases; at most n rotations per chase).
The last test plants mistakes in the oracle and shows the pins catch them.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

EPS = np.finfo(np.float64).eps


def dense_B(d, e, m):
    n = len(d)
    Bd = np.zeros((m, n))
    Bd[np.arange(n), np.arange(n)] = d
    Bd[np.arange(n - 1), np.arange(1, n)] = e
    return Bd


def invariants(st, Aplus):
    """(reconstruction, ||Q^T Q - I||_F, ||P^T P - I||_F, Frobenius gap)"""
    rec = np.linalg.norm(Aplus - st.Q @ dense_B(st.d, st.e, st.m) @ st.P.T) / np.linalg.norm(Aplus)
    oq = np.linalg.norm(st.Q.T @ st.Q - np.eye(st.m))
    op = np.linalg.norm(st.P.T @ st.P - np.eye(st.n))
    fb = abs(np.sqrt(st.d @ st.d + st.e @ st.e) - np.linalg.norm(Aplus)) / np.linalg.norm(Aplus)
    return rec, oq, op, fb


# ---- rotation primitive (eq. giv, giv1) -------------------------------------

def test_givens_closed_forms(oracle):
    c, s, r = oracle.givens(3.0, 4.0, 1)
    assert (c, s, r) == (0.8, 0.6, 5.0)
    assert abs(c * 3.0 - s * 4.0) < 1e-15  # [c -s; s c][a; b] = [0; r]
    c, s, r = oracle.givens(3.0, 4.0, 2)
    assert (c, s, r) == (0.6, -0.8, 5.0)
    assert abs(s * 3.0 + c * 4.0) < 1e-15  # second entry annihilated
    # already-zero targets give the identity, survivors keep their sign
    assert oracle.givens(0.0, -2.5, 1) == (1.0, 0.0, -2.5)
    assert oracle.givens(-2.5, 0.0, 2) == (1.0, 0.0, -2.5)
    # gamma_k != 0, gamma_{k+1} = 0 ("permute"): c = 0, a signed swap
    c, s, r = oracle.givens(-2.0, 0.0, 1)
    assert (c, s, r) == (0.0, -1.0, 2.0)
    # extreme magnitudes do not overflow or underflow
    c, s, r = oracle.givens(3e300, 4e300, 1)
    assert abs(r / 5e300 - 1) < 4 * EPS and abs(c - 0.8) < 4 * EPS
    c, s, r = oracle.givens(3e-300, 4e-300, 2)
    assert abs(r / 5e-300 - 1) < 4 * EPS and abs(s + 0.8) < 4 * EPS


def test_givens_random_is_rotation(oracle):
    rng = np.random.default_rng(7)
    for _ in range(2000):
        a, b = rng.standard_normal(2) * 10.0 ** rng.integers(-5, 5, 2)
        for mode in (1, 2):
            c, s, r = oracle.givens(a, b, mode)
            assert abs(c * c + s * s - 1) < 4 * EPS
            G = np.array([[c, -s], [s, c]])
            out = G @ np.array([a, b])
            tgt = 0 if mode == 1 else 1
            assert abs(out[tgt]) <= 4 * EPS * abs(r)
            assert abs(out[1 - tgt] - r) <= 4 * EPS * abs(r)
            assert r >= 0


def test_rot2_matches_matrix_and_identity(oracle):
    rng = np.random.default_rng(8)
    for _ in range(500):
        t = rng.uniform(0, 2 * np.pi)
        c, s = np.cos(t), np.sin(t)
        x, y = rng.standard_normal(2)
        xo, yo = oracle.rot2(c, s, x, y)
        ref = np.array([[c, -s], [s, c]]) @ np.array([x, y])
        assert abs(xo - ref[0]) < 4 * EPS and abs(yo - ref[1]) < 4 * EPS
        assert oracle.rot2(1.0, 0.0, x, y) == (x, y)


# ---- projection (eq. bidiagsubproblem) ---------------------------------------

def _fma_exact(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_project_is_sequential_fma_exactly(oracle):
    rng = np.random.default_rng(9)
    for rows, cols in [(1, 1), (7, 5), (23, 23)]:
        A = np.asfortranarray(rng.standard_normal((rows, cols)))
        x = rng.standard_normal(rows)
        got = oracle.project(A, x)
        for i in range(cols):
            acc = 0.0
            for j in range(rows):
                acc = _fma_exact(A[j, i], x[j], acc)
            assert got[i] == acc


def test_project_normwise_bound(oracle):
    rng = np.random.default_rng(10)
    m = 300
    Q = W.orthogonal(rng, m)
    b = rng.standard_normal(m)
    u = oracle.project(Q, b)
    exact = np.array([float(sum(Fraction(Q[j, i]) * Fraction(b[j]) for j in range(m)))
                      for i in range(0, m, 37)])
    bound = m * EPS * np.linalg.norm(b)
    assert np.max(np.abs(u[::37] - exact)) <= bound


# ---- structure and counts (Section 3.4) ----------------------------------------

SHAPES = [(2, 2), (3, 2), (3, 3), (4, 4), (5, 3), (6, 6), (9, 6), (12, 12), (14, 12), (20, 20), (30, 20), (31, 31)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_one_bulge_at_a_time_and_bidiagonal(oracle, m, n):
    f = W.factorization(m, n, 11)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    rng = np.random.default_rng(12)
    u, v = rng.standard_normal(m), rng.standard_normal(n)
    counts, trace, status = oracle.bgu_pass(
        st, u, v, flags=oracle.CHECK_PHASES | oracle.CHECK_EVERY, trace_cap=10 ** 6, check_status=False)
    assert status == oracle.ORC_OK


WINDOW_SHAPES = SHAPES + [(45, 40), (64, 64), (65, 64), (100, 37), (130, 97), (200, 200)]


@pytest.mark.parametrize("m,n", WINDOW_SHAPES)
def test_rotation_windows_hold_every_nonzero(oracle, m, n):
    """Before each rotation the rotated rows (left, rows i and i+1) are zero
    outside columns i-1..i+3 and the rotated columns (right, j and j+1) zero
    outside rows j-2..j+2: a rotation changes at most these five pairs, which
    is all the generator and its dependency model touch.  Random dense
    projections, a zero start and a rank-3 stream."""
    f = W.factorization(m, n, 15)
    rng = np.random.default_rng(16)
    flags = oracle.CHECK_WINDOW | oracle.NO_QP
    st = oracle.State(f.Q, f.d, f.e, f.P)
    for _ in range(3):
        _, _, status = oracle.bgu_pass(st, rng.standard_normal(m), rng.standard_normal(n), flags=flags,
                                       check_status=False)
        assert status == oracle.ORC_OK
    z = W.zero_start(m, n)
    st = oracle.State(z.Q, z.d, z.e, z.P)
    for _ in range(3):
        _, _, status = oracle.bgu_pass(st, rng.standard_normal(m), rng.standard_normal(n), flags=flags,
                                       check_status=False)
        assert status == oracle.ORC_OK


def test_window_check_catches_a_wrong_chase(oracle):
    """A chase stepping by 2 instead of 3 leaves nonzeros outside the windows."""
    f = W.factorization(30, 30, 17)
    rng = np.random.default_rng(18)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.set_mutation(3)
    try:
        _, _, status = oracle.bgu_pass(st, rng.standard_normal(30), rng.standard_normal(30),
                                       flags=oracle.CHECK_WINDOW | oracle.NO_QP, check_status=False)
    finally:
        oracle.set_mutation(0)
    assert status == oracle.ORC_ESTRUCT


@pytest.mark.parametrize("n", [4, 5, 12, 20, 31, 60])
def test_phase2_chase_count_is_2n_minus_3(oracle, n):
    f = W.factorization(n, n, 13)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    rng = np.random.default_rng(14)
    counts, trace, _ = oracle.bgu_pass(st, rng.standard_normal(n), rng.standard_normal(n),
                                       flags=oracle.NO_QP, trace_cap=10 ** 6)
    assert counts[5] == 2 * n - 3          # bulges chased in phase 2
    assert counts[2] == 0                  # no spike when m = n
    # up to n-1 eliminations in each of u and v; each bulge leaves in < n rotations
    tr1 = trace[trace["phase"] == 1]
    assert counts[0] + counts[1] <= 4 * n * n
    # each of the <= 2(n-1) phase-1 eliminations and 2n-3 phase-2 bulges is
    # chased off in at most n rotations
    assert counts[3] <= 2 * (n - 1) * n
    assert counts[4] <= (2 * n - 3) * n
    # the first two phase-1 rotations eliminate v_1 (right), then u_1 (left)
    assert (tr1["side"][0], tr1["i"][0]) == (1, 1) and (tr1["side"][1], tr1["i"][1]) == (0, 1)


@pytest.mark.parametrize("n", [20, 30, 60, 120])
def test_rotation_count_is_quadratic(oracle, n):
    """Phase 1 and phase 2 each take about (2/3) n^2 rotations: inside the
    paper's O(2n^2) per phase."""
    f = W.factorization(n, n, 15)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    rng = np.random.default_rng(16)
    counts, _, _ = oracle.bgu_pass(st, rng.standard_normal(n), rng.standard_normal(n), flags=oracle.NO_QP)
    for ph in (3, 4):
        assert abs(counts[ph] - (2 * n * n / 3 - n)) <= 2
        assert counts[ph] <= 2 * n * n
    assert counts[0] == counts[1]


# ---- closed forms -------------------------------------------------------------

def test_already_bidiagonal_update_is_exact(oracle):
    """b+ = g_{n-1} e_{n-1} + g_n e_n and c+ = h e_n leave B + b+ c+^T
    bidiagonal (Section 3.4): no rotation does anything, only d_n and e_{n-1}
    change, by exactly g_n h and g_{n-1} h."""
    n = 9
    rng = np.random.default_rng(17)
    f = W.factorization(n, n, 18)
    d = rng.integers(1, 9, n).astype(float)
    e = rng.integers(1, 9, n - 1).astype(float)
    st = oracle.State(f.Q, d, e, f.P)
    u = np.zeros(n); u[n - 2], u[n - 1] = 3.0, -5.0
    v = np.zeros(n); v[n - 1] = 0.5
    Q0, P0 = st.Q.copy(), st.P.copy()
    counts, trace, _ = oracle.bgu_pass(st, u, v, flags=oracle.CHECK_PHASES, trace_cap=10 ** 5)
    assert np.all(trace["c"] == 1.0) and np.all(trace["s"] == 0.0)
    assert np.array_equal(st.Q, Q0) and np.array_equal(st.P, P0)
    d_ref, e_ref = d.copy(), e.copy()
    d_ref[n - 1] += -5.0 * 0.5
    e_ref[n - 2] += 3.0 * 0.5
    assert np.array_equal(st.d, d_ref) and np.array_equal(st.e, e_ref)


@pytest.mark.parametrize("m,n", [(6, 6), (40, 40), (9, 6), (30, 20)])
def test_zero_start_closed_form(oracle, m, n):
    """A0 = 0, Q0 = I, P0 = I (Section 4 streams): one update b c^T."""
    f = W.zero_start(m, n)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    rng = np.random.default_rng(19)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    oracle.bgu_update(st, b, c, flags=oracle.CHECK_PHASES)
    nc = np.linalg.norm(c)
    d_ref, e_ref = np.zeros(n), np.zeros(n - 1)
    if m == n:
        d_ref[n - 1] = b[n - 1] * nc
        e_ref[n - 2] = np.linalg.norm(b[: n - 1]) * nc
    else:
        d_ref[n - 1] = np.linalg.norm(b) * nc
    tol = 64 * EPS * np.linalg.norm(b) * nc
    assert np.max(np.abs(st.d - d_ref)) <= tol and np.max(np.abs(st.e - e_ref)) <= tol
    assert np.linalg.norm(st.Q @ dense_B(st.d, st.e, m) @ st.P.T - np.outer(b, c)) <= tol


def test_two_by_two(oracle):
    rng = np.random.default_rng(20)
    for trial in range(50):
        f = W.factorization(2, 2, 100 + trial)
        st = oracle.State(f.Q, f.d, f.e, f.P)
        b, c = rng.standard_normal(2), rng.standard_normal(2)
        A1 = f.dense() + np.outer(b, c)
        counts, trace, _ = oracle.bgu_pass(st, oracle.project(st.Q, b), oracle.project(st.P, c),
                                           flags=oracle.CHECK_PHASES, trace_cap=10)
        assert [(t["side"], t["i"]) for t in trace] == [(1, 1), (0, 1)]
        assert np.allclose(np.linalg.svd(A1, compute_uv=False),
                           np.linalg.svd(dense_B(st.d, st.e, 2), compute_uv=False), rtol=0, atol=8 * EPS * np.linalg.norm(A1))
        assert np.linalg.norm(A1 - st.Q @ dense_B(st.d, st.e, 2) @ st.P.T) <= 8 * EPS * np.linalg.norm(A1)


# ---- invariants on streams -------------------------------------------------------

def test_tiny_stream_invariants(oracle):
    """m = n = 200, 10 rank-1 updates: reconstruction 1e-12, orthogonality
    1e-12 sqrt(n), singular values of Bd vs Jacobi on dense A+ to 1e-11 sigma_1."""
    f, ups = W.tiny()
    st = oracle.State(f.Q, f.d, f.e, f.P)
    Aplus = f.dense()
    for B, C in ups:
        oracle.bgu_update(st, B, C, flags=oracle.CHECK_PHASES)
        Aplus = Aplus + B @ C.T
    rec, oq, op, fb = invariants(st, Aplus)
    assert rec <= 1e-12 and oq <= 1e-12 * np.sqrt(st.m) and op <= 1e-12 * np.sqrt(st.n)
    assert fb <= 1e-14
    sa = oracle.jacobi_sv(Aplus)
    sb = oracle.bidiag_sv(st.d, st.e)
    assert np.max(np.abs(sa - sb)) <= 1e-11 * sa[0]


def test_rectangular_stream_invariants(oracle):
    m, n = 60, 40
    f = W.factorization(m, n, 21, d_dist="loguniform")
    st = oracle.State(f.Q, f.d, f.e, f.P)
    Aplus = f.dense()
    for B, C in W.gaussian_updates(m, n, 30, 22):
        oracle.bgu_update(st, B, C, flags=oracle.CHECK_PHASES)
        Aplus = Aplus + B @ C.T
    rec, oq, op, fb = invariants(st, Aplus)
    assert rec <= 1e-12 and oq <= 1e-12 * np.sqrt(m) and op <= 1e-12 * np.sqrt(n) and fb <= 1e-13
    sa = oracle.jacobi_sv(Aplus)
    sb = oracle.bidiag_sv(st.d, st.e)
    assert np.max(np.abs(sa - sb)) <= 1e-11 * sa[0]


@pytest.mark.parametrize("m,n", [(12, 12), (14, 12), (40, 25)])
def test_windowed_rotation_equals_whole_rows(oracle, m, n):
    """Rotating only the columns i-2..i+4 (rows j-3..j+3) of the working
    matrix gives the same numbers as rotating whole rows (columns)."""
    f = W.factorization(m, n, 23)
    a, b = oracle.State(f.Q, f.d, f.e, f.P), oracle.State(f.Q, f.d, f.e, f.P)
    for B, C in W.gaussian_updates(m, n, 3, 24):
        oracle.bgu_update(a, B, C, flags=0)
        oracle.bgu_update(b, B, C, flags=oracle.FULL_ROT)
    for x, y in [(a.d, b.d), (a.e, b.e), (a.Q, b.Q), (a.P, b.P)]:
        assert np.array_equal(x, y)


def test_rank_r_is_r_rank_one_passes(oracle):
    m, n = 30, 20
    f = W.factorization(m, n, 25)
    a, b = oracle.State(f.Q, f.d, f.e, f.P), oracle.State(f.Q, f.d, f.e, f.P)
    (B, C), = W.gaussian_updates(m, n, 1, 26, r=4)
    oracle.bgu_update(a, B, C)
    for i in range(4):
        oracle.bgu_update(b, B[:, i], C[:, i])
    assert np.array_equal(a.d, b.d) and np.array_equal(a.Q, b.Q) and np.array_equal(a.P, b.P)


# ---- dense references (Section 2) ----------------------------------------------

def test_jacobi_matches_library_svd(oracle):
    rng = np.random.default_rng(27)
    for m, n in [(5, 5), (30, 17), (80, 80)]:
        A = rng.standard_normal((m, n))
        s = oracle.jacobi_sv(A)
        ref = np.linalg.svd(A, compute_uv=False)
        assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
    D = np.diag([3.0, -7.0, 0.5, 2.0])
    assert np.array_equal(oracle.jacobi_sv(D), np.array([7.0, 3.0, 2.0, 0.5]))


def test_householder_bidiagonalization(oracle):
    rng = np.random.default_rng(28)
    for m, n in [(7, 7), (40, 25), (60, 60)]:
        A = rng.standard_normal((m, n))
        Q, d, e, P = oracle.bidiag_householder(A)
        assert np.linalg.norm(A - Q @ dense_B(d, e, m) @ P.T) <= 1e-13 * np.linalg.norm(A)
        assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-13 * m
        assert np.linalg.norm(P.T @ P - np.eye(n)) <= 1e-13 * n
        assert np.array_equal(P[:, 0], np.eye(n)[:, 0])
        assert np.max(np.abs(np.linalg.svd(A, compute_uv=False) - oracle.bidiag_sv(d, e))) <= 1e-12 * np.linalg.norm(A)


def test_golub_kahan_matches_householder(oracle):
    rng = np.random.default_rng(29)
    A = rng.standard_normal((18, 14))
    Q, d, e, P = oracle.bidiag_householder(A)
    dg, eg = oracle.bidiag_gk(A, np.eye(14)[:, 0])
    assert np.max(np.abs(np.abs(dg) - np.abs(d))) <= 1e-12 * np.linalg.norm(A)
    assert np.max(np.abs(np.abs(eg) - np.abs(e))) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("m,n", [(12, 12), (16, 12), (20, 20)])
def test_implicit_q_pin(oracle, m, n):
    """The updated bidiagonal is the one any bidiagonalization of A+ reaches
    from the start vector P+ e1 (implicit-Q uniqueness for the Golub-Kahan
    recurrences of Section 2): compare with Householder bidiagonalization of
    A+ H (H a reflector with H e1 = P+ e1) and with Golub-Kahan from P+ e1."""
    f = W.factorization(m, n, 30)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    (B, C), = W.gaussian_updates(m, n, 1, 31)
    Aplus = f.dense() + B @ C.T
    oracle.bgu_update(st, B, C, flags=oracle.CHECK_PHASES)
    p1 = st.P[:, 0]
    w = np.eye(n)[:, 0] - p1
    H = np.eye(n) - 2.0 * np.outer(w, w) / (w @ w)
    _, dh, eh, _ = oracle.bidiag_householder(Aplus @ H)
    dg, eg = oracle.bidiag_gk(Aplus, p1)
    scale = np.linalg.norm(Aplus)
    # Tolerance: the BGU result and both bidiagonalizations are backward
    # stable, each the exact bidiagonal (for this start vector) of a matrix
    # within about n u ||A+|| of A+.  How far such a perturbation moves the
    # bidiagonal is measured here on the Golub-Kahan map itself (the largest
    # change over four random perturbations of norm n u ||A+||); two
    # computations, with a factor 2 of margin, give 4x that.
    rng = np.random.default_rng(1)
    sens = 0.0
    for _ in range(4):
        E = rng.standard_normal(Aplus.shape)
        E *= n * 2.0 ** -53 * scale / np.linalg.norm(E)
        d2, e2 = oracle.bidiag_gk(Aplus + E, p1)
        sens = max(sens, np.max(np.abs(np.abs(d2) - np.abs(dg))), np.max(np.abs(np.abs(e2) - np.abs(eg))))
    tol = 4.0 * sens
    assert tol <= 1e-10 * scale  # the map is well enough conditioned at these sizes to be a pin
    for dd, ee in [(dh, eh), (dg, eg)]:
        assert np.max(np.abs(np.abs(dd) - np.abs(st.d))) <= tol
        assert np.max(np.abs(np.abs(ee) - np.abs(st.e))) <= tol


# ---- golden schedule (tests/golden/schedule_12x12.txt) ------------------------------

def _golden():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "schedule_12x12.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, val = line.split(":", 1)
        out[key.strip()] = val.strip()
    return out


def _trace(oracle, m, n):
    f = W.factorization(m, n, 1)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    rng = np.random.default_rng(3)
    cnt, tr, _ = oracle.bgu_pass(st, rng.standard_normal(m), rng.standard_normal(n),
                                 flags=oracle.NO_QP, trace_cap=10 ** 6)
    return cnt, tr


def test_golden_rotation_order_12x12(oracle):
    """The oracle's rotation order at n = 12 is the hand-worked order of the
    phase rules, rotation for rotation, with 2n - 3 = 21 phase-2 chains."""
    g = _golden()
    cnt, tr = _trace(oracle, 12, 12)
    got = {ph: [("L" if s == 0 else "R") + str(i - 1) for s, p, i in zip(tr["side"], tr["phase"], tr["i"]) if p == ph]
           for ph in (1, 2)}
    assert got[1] == g["phase1"].split()
    chains = [c.split() for c in g["phase2"].split("|")]
    assert got[2] == [x for c in chains for x in c]
    assert len(chains) == 21 == cnt[5] == 2 * 12 - 3


def test_golden_counts_14x12(oracle):
    g = _golden()["counts_14x12"].split()
    want = dict(zip(g[0::2], map(int, g[1::2])))
    cnt, tr = _trace(oracle, 14, 12)
    assert (cnt[2], cnt[3], cnt[4]) == (want["spike"], want["phase1"], want["phase2"])
    assert (tr["side"][0], tr["phase"][0], tr["i"][0] - 1) == (0, 0, 12)  # L12 first


# ---- row-subset passes (the checker of the full-size GPU tests) -------------------

@pytest.mark.parametrize("m,n", [(30, 30), (45, 31), (64, 64), (700, 5), (513, 2), (260, 3), (130, 97)])
def test_pass_rows_equals_full_pass(oracle, m, n):
    """orc_bgu_pass_rows on arbitrary row subsets of Q and P gives exactly
    the rows (and d, e) of the full pass: rotations act on columns."""
    f = W.factorization(m, n, 40)
    rng = np.random.default_rng(41)
    u, v = rng.standard_normal(m), rng.standard_normal(n)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_pass(st, u, v, flags=oracle.CHECK_PHASES)
    for trial in range(3):
        qi = np.sort(rng.choice(m, size=min(m, 1 + trial * 7), replace=False))
        pi = np.sort(rng.choice(n, size=min(n, 1 + trial * 5), replace=False))
        Qr, d2, e2, Pr = oracle.bgu_pass_rows(m, n, f.Q[qi, :], f.d, f.e, f.P[pi, :], u, v)
        assert np.array_equal(Qr, st.Q[qi, :]) and np.array_equal(Pr, st.P[pi, :])
        assert np.array_equal(d2, st.d) and np.array_equal(e2, st.e)


# ---- planted mistakes are caught --------------------------------------------------

def _pins_hold(oracle, m, n):
    f = W.factorization(m, n, 32)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    Aplus = f.dense()
    try:
        for B, C in W.gaussian_updates(m, n, 2, 33):
            oracle.bgu_update(st, B, C, flags=oracle.CHECK_PHASES)
            Aplus = Aplus + B @ C.T
    except RuntimeError:
        return False
    rec, oq, op, fb = invariants(st, Aplus)
    if not (rec <= 1e-12 and oq <= 1e-12 * np.sqrt(m) and op <= 1e-12 * np.sqrt(n)):
        return False
    sa = oracle.jacobi_sv(Aplus)
    sb = oracle.bidiag_sv(st.d, st.e)
    return bool(np.max(np.abs(sa - sb)) <= 1e-11 * sa[0])


def test_planted_mistakes_are_caught(oracle):
    assert _pins_hold(oracle, 12, 12) and _pins_hold(oracle, 15, 11)
    try:
        for mut in range(1, 8):
            oracle.set_mutation(mut)
            assert not (_pins_hold(oracle, 12, 12) and _pins_hold(oracle, 15, 11)), f"mutation {mut} not caught"
    finally:
        oracle.set_mutation(0)
    assert _pins_hold(oracle, 12, 12)
