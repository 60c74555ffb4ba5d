"""Seeded synthetic workloads for the bidiagonal-update path.

This module only draws inputs: initial factorizations A = Q Bd P^T and the
update vectors b, c.  It holds none of the update method's arithmetic, and
both the GPU library and the CPU oracle consume the same bytes it returns.

The shapes and value distributions follow the update model of Section 1
(A+ = A + B C^T), the zero-start streams of the applications in Section 4,
and the recommendation-style ratings of Section 4.2.  No dataset from the
paper is available; every input here is synthetic.

RNG: numpy PCG64 (``numpy.random.default_rng``) with explicit seeds.
Orthogonal factors come from LAPACK's Householder QR of N(0,1) matrices
(``numpy.linalg.qr``), with no sign normalisation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Factorization:
    Q: np.ndarray  # m x m, column-major, orthogonal
    d: np.ndarray  # n
    e: np.ndarray  # n - 1
    P: np.ndarray  # n x n, column-major, orthogonal

    @property
    def m(self) -> int:
        return self.Q.shape[0]

    @property
    def n(self) -> int:
        return self.P.shape[0]

    def dense(self) -> np.ndarray:
        """A = Q Bd P^T (test-side reference; plain numpy)."""
        Bd = np.zeros((self.m, self.n))
        Bd[np.arange(self.n), np.arange(self.n)] = self.d
        Bd[np.arange(self.n - 1), np.arange(1, self.n)] = self.e
        return self.Q @ Bd @ self.P.T

    def frob(self) -> float:
        return float(math.sqrt(float(self.d @ self.d + self.e @ self.e)))


def orthogonal(rng: np.random.Generator, k: int) -> np.ndarray:
    """Q factor of the Householder QR of a k x k N(0,1) matrix."""
    G = rng.standard_normal((k, k))
    Q, _ = np.linalg.qr(G)
    return np.asfortranarray(Q)


def factorization(m: int, n: int, seed: int, d_dist: str = "uniform") -> Factorization:
    """Q0, P0 orthogonal; d ~ U(1,10) ("uniform") or log-uniform on
    [1e-3, 1e2] ("loguniform"); e ~ U(0,1)."""
    if m < n or n < 2:
        raise ValueError("need m >= n >= 2")
    rng = np.random.default_rng(seed)
    Q = orthogonal(rng, m)
    P = orthogonal(rng, n)
    if d_dist == "uniform":
        d = rng.uniform(1.0, 10.0, n)
    elif d_dist == "loguniform":
        d = np.exp(rng.uniform(math.log(1e-3), math.log(1e2), n))
    else:
        raise ValueError(d_dist)
    e = rng.uniform(0.0, 1.0, n - 1)
    return Factorization(Q, d, e, P)


def zero_start(m: int, n: int) -> Factorization:
    """A0 = 0 with Q0 = I, P0 = I, Bd0 = 0 (the streams of Section 4 start so)."""
    return Factorization(np.asfortranarray(np.eye(m)), np.zeros(n), np.zeros(n - 1),
                         np.asfortranarray(np.eye(n)))


def gaussian_updates(m: int, n: int, count: int, seed: int, scale_b: float | None = None,
                     scale_c: float | None = None, r: int = 1):
    """`count` rank-r updates (B m x r, C n x r), column-major.
    Default scaling b ~ N(0,1)/sqrt(m), c ~ N(0,1)/sqrt(n)."""
    rng = np.random.default_rng(seed)
    sb = (1.0 / math.sqrt(m)) if scale_b is None else scale_b
    sc = (1.0 / math.sqrt(n)) if scale_c is None else scale_c
    out = []
    for _ in range(count):
        B = np.asfortranarray(rng.standard_normal((m, r)) * sb)
        C = np.asfortranarray(rng.standard_normal((n, r)) * sc)
        out.append((B, C))
    return out


# ---- named workloads -------------------------------------------------------

def tiny(seed: int = 1000):
    """m = n = 200; d ~ U(1,10), e ~ U(0,1); 10 rank-1 updates
    b ~ N(0,1)/sqrt(m), c ~ N(0,1)/sqrt(n)."""
    f = factorization(200, 200, seed)
    ups = gaussian_updates(200, 200, 10, seed + 1)
    return f, ups


def one_stream(seed: int = 2000, count: int = 200, m: int = 4000, n: int = 2000):
    """m = 4000, n = 2000; d log-uniform on [1e-3, 1e2]; updates
    b, c ~ N(0,1) with the product b c^T scaled (on b) by 1e-2 ||A||_F / sqrt(m n)."""
    f = factorization(m, n, seed, d_dist="loguniform")
    scale = 1e-2 * f.frob() / math.sqrt(m * n)
    ups = gaussian_updates(m, n, count, seed + 1, scale_b=scale, scale_c=1.0)
    return f, ups


def square(n: int, seed: int):
    """Square stream with the tiny-config construction at size n."""
    return factorization(n, n, seed)


def batched_sizes(count: int = 256, seed: int = 3000, lo: int = 128, hi: int = 2048):
    """n = round(exp(U(ln lo, ln hi))) per stream."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(count)]


def ratings(users: int = 10000, items: int = 2000, density: float = 0.01,
            zipf_s: float = 1.1, seed: int = 4000) -> np.ndarray:
    """Integer ratings 1..5 at the given density; user uniform, item drawn
    from a Zipf(s) law truncated to `items` ranks, duplicates rejected."""
    rng = np.random.default_rng(seed)
    ranks = np.arange(1, items + 1, dtype=np.float64)
    pz = ranks ** (-zipf_s)
    pz /= pz.sum()
    target = int(round(density * users * items))
    A = np.zeros((users, items))
    filled = 0
    while filled < target:
        k = target - filled
        us = rng.integers(0, users, k)
        its = rng.choice(items, size=k, p=pz)
        vals = rng.integers(1, 6, k).astype(np.float64)
        for uu, ii, vv in zip(us, its, vals):
            if A[uu, ii] == 0.0 and filled < target:
                A[uu, ii] = vv
                filled += 1
    return np.asfortranarray(A)


def rating_row(rng: np.random.Generator, items: int, nnz: int, zipf_s: float = 1.1) -> np.ndarray:
    """A fresh user row with `nnz` ratings drawn as in `ratings`."""
    ranks = np.arange(1, items + 1, dtype=np.float64)
    pz = ranks ** (-zipf_s)
    pz /= pz.sum()
    row = np.zeros(items)
    its = rng.choice(items, size=min(nnz, items), replace=False, p=pz)
    row[its] = rng.integers(1, 6, len(its)).astype(np.float64)
    return row


def tracking_state(m: int, n: int, r: int, seed: int):
    """Thin tracked factors for subspace tracking (Section 4): U (m x r) and
    V (n x r) with orthonormal columns (Q factors of the Householder QR of
    N(0,1) matrices), d ~ U(1, 10) sorted descending (a dominant subspace),
    e ~ U(0, 1).  Returns (U, d, e, V), column-major."""
    if r < 1 or m < r or n < r:
        raise ValueError("need m, n >= r >= 1")
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    d = np.sort(rng.uniform(1.0, 10.0, r))[::-1].copy()
    e = rng.uniform(0.0, 1.0, max(r - 1, 0))
    return np.asfortranarray(U), d, e, np.asfortranarray(V)


def tracking_update(m: int, n: int, seed: int, scale: float = 1.0):
    """One streaming rank-1 update b c^T: b ~ N(0,1) scale / sqrt(m),
    c ~ N(0,1) / sqrt(n)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(m) * scale / math.sqrt(m), rng.standard_normal(n) / math.sqrt(n))


def zero_start_tracking(m: int, n: int, r: int):
    """The zero start of the paper's streaming experiments (Section 4): A0 = 0,
    U0 = I_m(:, 1:r), V0 = I_n(:, 1:r), B0 = 0.  Returns (U, d, e, V)."""
    U = np.asfortranarray(np.eye(m)[:, :r])
    V = np.asfortranarray(np.eye(n)[:, :r])
    return U, np.zeros(r), np.zeros(max(r - 1, 0)), V


def link_stream(m: int, n: int, steps: int, seed: int, density: float = 0.05):
    """A link-prediction-shaped update stream (Section 4): at step h, b_h has
    entries in {0, 1} (each 1 with probability density) and c_h = e_{h mod n}.
    Returns a list of (b, c)."""
    rng = np.random.default_rng(seed)
    out = []
    for h in range(steps):
        b = (rng.random(m) < density).astype(np.float64)
        c = np.zeros(n)
        c[h % n] = 1.0
        out.append((b, c))
    return out


def bidiagonal_factors(A: np.ndarray, seed: int = 0):
    """A starting factorization A = Q [B; 0] P^T of a tall matrix (m >= n):
    Householder QR A = Q1 [R; 0] (LAPACK, through numpy), then Golub-Kahan
    bidiagonalization of R from p1 = e1 (Section 2's recurrences
    R P = W B, R^T W = P B^T) with two passes of full reorthogonalization
    against all earlier vectors, and Q = Q1 diag(W, I).  A breakdown (a zero
    d_k or e_k) continues from a random unit vector orthogonal to the earlier
    ones, with that entry of B exactly 0.  Input construction only: it
    shares nothing with the update method.  Returns (Q, d, e, P)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n or n < 2:
        raise ValueError("need m >= n >= 2")
    rng = np.random.default_rng(seed)
    Q1, R = np.linalg.qr(A, mode="complete")
    R = np.ascontiguousarray(R[:n])
    scale = max(np.linalg.norm(R), 1.0)
    W = np.zeros((n, n))
    P = np.zeros((n, n))
    d = np.zeros(n)
    e = np.zeros(n - 1)

    def orth(x, basis):
        for _ in range(2):
            x = x - basis @ (basis.T @ x)
        return x

    def fresh(basis):
        while True:
            x = orth(rng.standard_normal(basis.shape[0]), basis)
            nx = np.linalg.norm(x)
            if nx > 1e-8:
                return x / nx

    p = np.zeros(n)
    p[0] = 1.0
    for k in range(n):
        P[:, k] = p
        w = R @ p - (e[k - 1] * W[:, k - 1] if k > 0 else 0.0)
        w = orth(w, W[:, :k])
        nw = np.linalg.norm(w)
        if nw <= 1e-13 * scale:
            d[k] = 0.0
            W[:, k] = fresh(W[:, :k])
        else:
            d[k] = nw
            W[:, k] = w / nw
        if k + 1 < n:
            p = R.T @ W[:, k] - d[k] * P[:, k]
            p = orth(p, P[:, :k + 1])
            npn = np.linalg.norm(p)
            if npn <= 1e-13 * scale:
                e[k] = 0.0
                p = fresh(P[:, :k + 1])
            else:
                e[k] = npn
                p = p / npn
    Q = Q1.copy(order="F")
    Q[:, :n] = Q1[:, :n] @ W
    return Q, d, e, np.asfortranarray(P)
