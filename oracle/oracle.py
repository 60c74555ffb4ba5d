"""TEST INFRASTRUCTURE ONLY: ctypes front end of the FP64 CPU oracle.

The oracle (``bgu_oracle.c``) is a plain, slow reference of the Givens
bidiagonal update of Brust & Saunders (Section 3.4, Algorithm 2) plus the
dense factorizations that check it (Section 2); the Householder bidiagonal
update (Section 3.3, Algorithm 1) and the other read-side utilities are
plain numpy in this module.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import this module.
It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bgu_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_bgu.so")

CHECK_PHASES = 1
CHECK_EVERY = 2
FULL_ROT = 4
NO_QP = 8
CHECK_WINDOW = 16

ORC_OK = 0
ORC_ESTRUCT = -10


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add beyond the explicit
    fma calls; IEEE sqrt and division)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-mfma",
               "-fPIC", "-shared", "-Wall", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class RotRec(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("phase", ctypes.c_int32),
                ("i", ctypes.c_int64), ("c", ctypes.c_double),
                ("s", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.orc_project.argtypes = [i64, i64, dp, i64, dp, dp]
        L.orc_project.restype = None
        L.orc_givens.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        L.orc_givens.restype = None
        L.orc_rot2.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_rot2.restype = None
        L.orc_bgu_pass.argtypes = [i64, i64, dp, i64, dp, dp, dp, i64, dp, dp,
                                   ctypes.c_int, ctypes.POINTER(RotRec), i64,
                                   ctypes.POINTER(ctypes.c_int64)]
        L.orc_bgu_pass.restype = ctypes.c_int
        L.orc_bgu_pass_rows.argtypes = [i64, i64, dp, i64, i64, dp, dp, dp, i64, i64, dp, dp,
                                        ctypes.c_int, ctypes.POINTER(RotRec), i64,
                                        ctypes.POINTER(ctypes.c_int64)]
        L.orc_bgu_pass_rows.restype = ctypes.c_int
        L.orc_bgu_update.argtypes = [i64, i64, dp, i64, dp, dp, dp, i64, dp, i64,
                                     dp, i64, ctypes.c_int, ctypes.c_int]
        L.orc_bgu_update.restype = ctypes.c_int
        L.orc_bidiag_householder.argtypes = [i64, i64, dp, i64, dp, dp, dp, dp]
        L.orc_bidiag_householder.restype = ctypes.c_int
        L.orc_bidiag_gk.argtypes = [i64, i64, dp, i64, dp, dp, dp]
        L.orc_bidiag_gk.restype = ctypes.c_int
        L.orc_jacobi_sv.argtypes = [i64, i64, dp, i64, dp]
        L.orc_jacobi_sv.restype = ctypes.c_int
        L.orc_set_mutation.argtypes = [ctypes.c_int]
        L.orc_track_update.argtypes = [i64, i64, i64, dp, i64, dp, dp, dp, i64, dp, dp, ctypes.c_int,
                                       dp, i64, dp, dp, dp, i64, dp]
        L.orc_track_complement.argtypes = [i64, i64, dp, i64, dp, dp, dp, dp, dp]
        L.orc_track_finish.argtypes = [i64, i64, i64, dp, i64, dp, dp, dp, i64, dp, dp, ctypes.c_double,
                                       ctypes.c_double, dp, dp, ctypes.c_int, dp, i64, dp, dp, dp, i64, dp]
        L.orc_set_mutation.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, order="F"):
    return np.require(np.asarray(a, dtype=np.float64), requirements=[order, "W", "A"])


def project(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """out = A^T x with sequential fma accumulation (column-major A)."""
    A = np.asfortranarray(A, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows, cols = A.shape
    out = np.empty(cols)
    lib().orc_project(rows, cols, _p(A), rows, _p(x), _p(out))
    return out


def givens(a: float, b: float, mode: int):
    c, s, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_givens(a, b, mode, ctypes.byref(c), ctypes.byref(s), ctypes.byref(r))
    return c.value, s.value, r.value


def rot2(c: float, s: float, x: float, y: float):
    xx, yy = ctypes.c_double(x), ctypes.c_double(y)
    lib().orc_rot2(c, s, ctypes.byref(xx), ctypes.byref(yy))
    return xx.value, yy.value


class State:
    """A factorization A = Q diag-bidiag(d, e) P^T held on the host."""

    def __init__(self, Q, d, e, P):
        self.Q = _f64(Q).copy(order="F")
        self.P = _f64(P).copy(order="F")
        self.d = np.array(d, dtype=np.float64)
        self.e = np.array(e, dtype=np.float64)
        self.m, self.n = self.Q.shape[0], self.P.shape[0]

    def copy(self) -> "State":
        return State(self.Q, self.d, self.e, self.P)

    def B(self) -> np.ndarray:
        Bd = np.zeros((self.m, self.n))
        Bd[np.arange(self.n), np.arange(self.n)] = self.d
        Bd[np.arange(self.n - 1), np.arange(1, self.n)] = self.e
        return Bd

    def A(self) -> np.ndarray:
        return self.Q @ self.B() @ self.P.T


def bgu_pass(st: State, u, v, flags: int = CHECK_PHASES, trace_cap: int = 0,
             check_status: bool = True):
    """One rank-1 pass from projected u (m), v (n); updates st in place.
    Returns (counts[6], trace or None, status)."""
    u = np.array(u, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    counts = (ctypes.c_int64 * 6)()
    tr = (RotRec * trace_cap)() if trace_cap else None
    Q = st.Q if not (flags & NO_QP) else np.zeros((1, 1), order="F")
    P = st.P if not (flags & NO_QP) else np.zeros((1, 1), order="F")
    ldq = st.m
    ldp = st.n
    status = lib().orc_bgu_pass(st.m, st.n, _p(Q), ldq, _p(st.d), _p(st.e), _p(P), ldp,
                                _p(u), _p(v), flags, tr, trace_cap, counts)
    if check_status and status != ORC_OK:
        raise RuntimeError(f"orc_bgu_pass failed with status {status}")
    trace = None
    if tr is not None:
        nrec = min(trace_cap, counts[0] + counts[1])
        trace = np.array([(tr[k].side, tr[k].phase, tr[k].i, tr[k].c, tr[k].s)
                          for k in range(nrec)],
                         dtype=[("side", "i4"), ("phase", "i4"), ("i", "i8"),
                                ("c", "f8"), ("s", "f8")])
    return list(counts), trace, status


def bgu_pass_rows(m: int, n: int, Qrows, d, e, Prows, u, v, flags: int = 0):
    """One pass on row subsets Qrows (k x m) and Prows (l x n); returns
    (Qrows', d', e', Prows') without touching the inputs."""
    Qr = np.array(Qrows, dtype=np.float64, order="F")
    Pr = np.array(Prows, dtype=np.float64, order="F")
    d = np.array(d, dtype=np.float64)
    e = np.array(e, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    kq, kp = Qr.shape[0], Pr.shape[0]
    status = lib().orc_bgu_pass_rows(m, n, _p(Qr), kq, max(kq, 1), _p(d), _p(e), _p(Pr), kp, max(kp, 1),
                                     _p(u), _p(v), flags, None, 0, None)
    if status != ORC_OK:
        raise RuntimeError(f"orc_bgu_pass_rows failed with status {status}")
    return Qr, d, e, Pr


def bgu_update(st: State, B, C, flags: int = 0) -> int:
    """Rank-r update A + B C^T as r rank-1 passes; updates st in place."""
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if B.ndim == 1:
        B, C = B[:, None], C[:, None]
    B, C = np.asfortranarray(B), np.asfortranarray(C)
    r = B.shape[1]
    status = lib().orc_bgu_update(st.m, st.n, _p(st.Q), st.m, _p(st.d), _p(st.e),
                                  _p(st.P), st.n, _p(B), st.m, _p(C), st.n, r, flags)
    if status != ORC_OK:
        raise RuntimeError(f"orc_bgu_update failed with status {status}")
    return status


def bidiag_householder(A):
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    Q = np.empty((m, m), order="F")
    P = np.empty((n, n), order="F")
    d = np.empty(n)
    e = np.empty(max(n - 1, 0) or 1)
    st = lib().orc_bidiag_householder(m, n, _p(A), m, _p(Q), _p(d), _p(e), _p(P))
    assert st == ORC_OK
    return Q, d, e[: n - 1], P


def bidiag_gk(A, p1):
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    p1 = np.ascontiguousarray(p1, dtype=np.float64)
    d = np.empty(n)
    e = np.empty(max(n - 1, 1))
    st = lib().orc_bidiag_gk(m, n, _p(A), m, _p(p1), _p(d), _p(e))
    assert st == ORC_OK
    return d, e[: n - 1]


def jacobi_sv(A):
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    sig = np.empty(n)
    st = lib().orc_jacobi_sv(m, n, _p(A), m, _p(sig))
    assert st == ORC_OK
    return sig


def bidiag_sv(d, e):
    """Singular values of the upper bidiagonal (d, e) by the oracle's Jacobi."""
    n = len(d)
    Bd = np.zeros((n, n))
    Bd[np.arange(n), np.arange(n)] = d
    Bd[np.arange(n - 1), np.arange(1, n)] = e
    return jacobi_sv(Bd)


ORC_ESPAN = -11
TRACK_KEEP_ALL = 1


def _track_out(m, n, r, k):
    return (np.zeros((m, k), order="F"), np.zeros(k), np.zeros(max(k - 1, 1)),
            np.zeros((n, k), order="F"), np.zeros(4))


def _track_rank(r, delta, gamma, keep_all):
    return r + 1 if (keep_all and delta > 0 and gamma > 0) else r


def track_complement(A, x):
    """Projection of x onto the orthonormal columns of A and its complement
    (Section 4, eq. (defup), with one reorthogonalization pass when needed):
    returns (xhat, xperp, norm, (s0, s1, s2)); norm 0 means x is taken to lie
    in span(A)."""
    A = _f64(A)
    rows, r = A.shape
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    xhat, xperp, norm, sums = np.zeros(r), np.zeros(rows), np.zeros(1), np.zeros(3)
    st = lib().orc_track_complement(rows, r, _p(A), rows, _p(x), _p(xhat), _p(xperp), _p(norm), _p(sums))
    if st != ORC_OK:
        raise ValueError(f"orc_track_complement failed with status {st}")
    return xhat, xperp, float(norm[0]), tuple(sums)


def track_finish(U, d, e, V, bh, ch, delta, gamma, qb, qc, keep_all: bool = False):
    """The tracking update from given projections b_hat, c_hat, norms delta,
    gamma and unit complements qb, qc (Section 4, eqs. (qrlr)-(bdlrup)):
    returns (U2, d2, e2, V2, info), info = (delta, gamma, removed index or
    -1, output rank)."""
    U, V = _f64(U), _f64(V)
    m, r = U.shape
    n = V.shape[0]
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64) if r > 1 else np.zeros(1)
    bh = np.ascontiguousarray(bh, dtype=np.float64).ravel()
    ch = np.ascontiguousarray(ch, dtype=np.float64).ravel()
    qb = np.ascontiguousarray(qb if qb is not None else np.zeros(m), dtype=np.float64).ravel()
    qc = np.ascontiguousarray(qc if qc is not None else np.zeros(n), dtype=np.float64).ravel()
    k = _track_rank(r, delta, gamma, keep_all)
    U2, d2, e2, V2, info = _track_out(m, n, r, k)
    st = lib().orc_track_finish(m, n, r, _p(U), m, _p(d), _p(e), _p(V), n, _p(bh), _p(ch), float(delta),
                                float(gamma), _p(qb), _p(qc), TRACK_KEEP_ALL if keep_all else 0, _p(U2), m,
                                _p(d2), _p(e2), _p(V2), n, _p(info))
    if st != ORC_OK:
        raise ValueError(f"orc_track_finish failed with status {st}")
    return U2, d2, e2[:k - 1], V2, (info[0], info[1], int(info[2]), int(info[3]))


def track_update(U, d, e, V, b, c, keep_all: bool = False):
    """Subspace-tracking update (Section 4): returns (U2, d2, e2, V2, info)
    with info = (delta, gamma, removed index or -1, output rank).  Raises
    ValueError with the status when r = 1 and a side is not augmented
    (status ORC_ESPAN)."""
    U, V = _f64(U), _f64(V)
    m, r = U.shape
    n = V.shape[0]
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64) if r > 1 else np.zeros(1)
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    c = np.ascontiguousarray(c, dtype=np.float64).ravel()
    U2, d2, e2, V2, info = _track_out(m, n, r, r + 1)
    st = lib().orc_track_update(m, n, r, _p(U), m, _p(d), _p(e), _p(V), n, _p(b), _p(c),
                                TRACK_KEEP_ALL if keep_all else 0, _p(U2), m, _p(d2), _p(e2),
                                _p(V2), n, _p(info))
    if st != ORC_OK:
        raise ValueError(f"orc_track_update failed with status {st}")
    k = int(info[3])
    return (np.asfortranarray(U2[:, :k]), d2[:k], e2[:k - 1], np.asfortranarray(V2[:, :k]),
            (info[0], info[1], int(info[2]), k))


def set_mutation(k: int) -> None:
    lib().orc_set_mutation(k)


# ---- orthogonality monitor and correction (test infrastructure) -----------
# The paper reorthogonalizes its factors "only a few times" without saying
# how.  The reading used here: the drift of a factor X is the Frobenius norm
# of E = X^T X - I, and the correction is one Newton-Schulz step towards the
# orthogonal polar factor of X, X <- X - X E / 2 (the nearest orthogonal
# matrix; from a drift e the step leaves a drift of order e^2).  Plain
# numpy products, fp64.

def orth_gram(X):
    X = np.asarray(X, dtype=np.float64)
    return X.T @ X - np.eye(X.shape[1])


def orth_error(X) -> float:
    return float(np.sqrt(np.sum(orth_gram(X) ** 2)))


def reorth_step(X):
    X = np.asarray(X, dtype=np.float64)
    return X - (X @ orth_gram(X)) / 2.0


# ---- truncated bidiagonal approximation (Section 1.3, eqs. (trBD), (errtrBD)) --

def truncated_bd(Q, d, e, P, r: int):
    """Best rank-r truncated bidiagonal approximation of A = Q Bd P^T: keep
    the r columns i of Bd with the largest t_i = d_i^2 + e_{i-1}^2 (each
    product and the sum rounded on their own; e_0 = 0; ties keep the lower
    index), so that A_r = Qr Pr^T with Qr(:, j) = d_i q_i + e_{i-1} q_{i-1}
    and Pr(:, j) = p_i, i = idx[j] in the selection order; the squared
    Frobenius error is the sum of the dropped t_i (ascending i).
    Returns (idx, err2, Qr, Pr)."""
    Q = np.asarray(Q, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.shape[0]
    t = d * d
    t[1:] = t[1:] + e * e
    idx = np.argsort(-t, kind="stable")[:r]
    keep = np.zeros(n, dtype=bool)
    keep[idx] = True
    err2 = 0.0
    for i in range(n):
        if not keep[i]:
            err2 = err2 + float(t[i])
    Qr = np.empty((Q.shape[0], r), order="F")
    Pr = np.empty((P.shape[0], r), order="F")
    for j, i in enumerate(idx):
        Qr[:, j] = d[i] * Q[:, i] if i == 0 else d[i] * Q[:, i] + e[i - 1] * Q[:, i - 1]
        Pr[:, j] = P[:, i]
    return idx.astype(np.int64), err2, Qr, Pr


# ---- Householder bidiagonal update, BHU (Section 3.3, Theorem 1, Algorithm 1) --
#
# Readings taken here (the paper leaves them open):
# - house(x) for a column x(k:m) or a row x(k+1:n): when the entries to be
#   annihilated are already all zero the reflector is the identity (its
#   essential vector is zero and the leading entry is kept); otherwise
#   alpha = -sign(x_1) ||x|| (sign(0) = +1) and y = (x - alpha e_1) / ||x - alpha e_1||,
#   so H = I - 2 y y^T with ||y|| = 1 as the compact forms (eq. QP) assume.
# - Left reflectors k = 1..n-1 when m = n and k = 1..n when m > n (column n
#   has entries below the diagonal only when m > n); right reflectors
#   w_{k+1} for k = 1..n-2, each zeroing row k right of entry k+1.
# - The row reflector of step k is computed from row k of A_{k,k-1} (the
#   printed e_{k+1} index is read as the row that holds the entries
#   w_{k+1} annihilates).
# - The last bidiagonal entries not produced as a reflector's leading value
#   (e_{n-1}, and d_n when m = n) are read from column n of the final
#   representation.

def _bd_mul(d, e, x, m):
    """B x for the m x n upper bidiagonal B (diagonal d, superdiagonal e)."""
    n = len(d)
    y = np.zeros(m)
    y[:n] = d * x
    y[: n - 1] += e * x[1:]
    return y


def _bd_tmul(d, e, y):
    """B^T y (y of length m)."""
    n = len(d)
    x = d * y[:n]
    x[1:] += e * y[: n - 1]
    return x


def _house(x):
    """(alpha, y) for x: y unit with (I - 2 y y^T) x = alpha e_1, or y = 0 and
    alpha = x_1 when x(2:) is already zero."""
    x = np.asarray(x, dtype=np.float64)
    if not np.any(x[1:] != 0.0):
        return float(x[0]), np.zeros_like(x)
    nrm = float(np.sqrt(np.sum(x * x)))
    alpha = -nrm if x[0] >= 0.0 else nrm
    y = x.copy()
    y[0] -= alpha
    return alpha, y / float(np.sqrt(np.sum(y * y)))


def bhu_repr(d, e, b, c, Y, W):
    """The factors (U, M, V) of Theorem 1 for A = B + b c^T after the left
    reflectors in the columns of Y (m x i) and the right ones in W (n x j):
    Q_i^T A P_j = B - U M^{-1} V^T with U = [b, Y, B W], V = [c, B^T Y, W]
    and M = [[-1, 0, c^T W], [Y^T b, T^T / 2, Y^T B W], [0, 0, R / 2]],
    T and R the unit upper triangular matrices of eq. (TR)."""
    m, i = Y.shape
    n, j = W.shape
    BW = np.zeros((m, j))  # B W
    BW[:n] = d[:, None] * W
    BW[:n - 1] += e[:, None] * W[1:]
    BtY = d[:, None] * Y[:n]  # B^T Y
    BtY[1:] += e[:, None] * Y[:n - 1]
    T = np.eye(i) + np.triu(2.0 * (Y.T @ Y), 1)
    R = np.eye(j) + np.triu(2.0 * (W.T @ W), 1)
    M = np.zeros((1 + i + j, 1 + i + j))
    M[0, 0] = -1.0
    M[0, 1 + i:] = c @ W
    M[1:1 + i, 0] = Y.T @ b
    M[1:1 + i, 1:1 + i] = 0.5 * T.T
    M[1:1 + i, 1 + i:] = Y.T @ BW
    M[1 + i:, 1 + i:] = 0.5 * R
    U = np.column_stack([b, Y, BW])
    V = np.column_stack([c, BtY, W])
    return U, M, V


def bhu_bidiag(d, e, b, c, m: int):
    """Algorithm 1 on B + b c^T (B the m x n upper bidiagonal (d, e); b of
    length m, c of length n).  Each step takes column k (then row k) of the
    current A_{kk} from the representation of Theorem 1, never forming A.
    Returns (d+, e+, Y, W): the new bidiagonal and the unit essential vectors
    (Y m x n_left, W n x n_right) so that B + b c^T = Q_k Bd+ P_k^T with
    Q_k = I - 2 Y T^{-1} Y^T and P_k = I - 2 W R^{-1} W^T (eq. QP)."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).ravel()
    c = np.asarray(c, dtype=np.float64).ravel()
    n = len(d)
    kl = n - 1 if m == n else n
    kr = n - 2
    Y = np.zeros((m, 0))
    W = np.zeros((n, 0))
    dp = np.zeros(n)
    ep = np.zeros(n - 1)

    def column(k):  # column k (0-based) of the current A
        U, M, V = bhu_repr(d, e, b, c, Y, W)
        ek = np.zeros(n)
        ek[k] = 1.0
        return _bd_mul(d, e, ek, m) - U @ np.linalg.solve(M, V[k, :])

    def row(k):  # row k (0-based) of the current A
        U, M, V = bhu_repr(d, e, b, c, Y, W)
        ek = np.zeros(m)
        ek[k] = 1.0
        return _bd_tmul(d, e, ek) - V @ np.linalg.solve(M.T, U[k, :])

    for k in range(kl):
        a = column(k)
        alpha, y = _house(a[k:])
        dp[k] = alpha
        yk = np.zeros(m)
        yk[k:] = y
        Y = np.column_stack([Y, yk])
        if k >= kr:
            continue
        ar = row(k)
        beta, w = _house(ar[k + 1:])
        ep[k] = beta
        wk = np.zeros(n)
        wk[k + 1:] = w
        W = np.column_stack([W, wk])
    last = column(n - 1)
    ep[n - 2] = last[n - 2]
    if m == n:
        dp[n - 1] = last[n - 1]
    return dp, ep, Y, W


def bhu_update(Q, d, e, P, b, c):
    """Rank-1 update of A = Q Bd P^T by Algorithm 1: returns (Q+, d+, e+, P+)
    with Q+ Bd+ P+^T = A + b c^T, Q+ = Q Q_k and P+ = P P_k (eq. QP)."""
    Q = np.asarray(Q, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    m, n = Q.shape[0], P.shape[0]
    bb = Q.T @ np.asarray(b, dtype=np.float64).ravel()
    cc = P.T @ np.asarray(c, dtype=np.float64).ravel()
    dp, ep, Y, W = bhu_bidiag(d, e, bb, cc, m)
    T = np.eye(Y.shape[1]) + np.triu(2.0 * (Y.T @ Y), 1)
    R = np.eye(W.shape[1]) + np.triu(2.0 * (W.T @ W), 1)
    Qk = np.eye(m) - 2.0 * Y @ np.linalg.solve(T, Y.T)
    Pk = np.eye(n) - 2.0 * W @ np.linalg.solve(R, W.T) if W.shape[1] else np.eye(n)
    return Q @ Qk, dp, ep, P @ Pk
