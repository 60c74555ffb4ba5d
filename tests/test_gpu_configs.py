"""The workload configurations at their own sizes, against the oracle.

  * one stream, m = 4000, n = 2000, 200 rank-1 updates: every update in
    lockstep (the GPU's projections u, v feed the oracle's pass on 64 tracked
    rows of Q and P; d and e are compared bit for bit after every update,
    the tracked rows at checkpoints), then the dense invariants and the
    singular values of Bd against a dense SVD of A+;
  * recommendation-shaped, 10000 users x 2000 items: the initial
    factorization from the ratings (workloads.bidiagonal_factors), row
    replacements r = 1, 4, 8 at a time and a mean adjustment, in lockstep as
    rank-1 passes, and the same calls as rank-r updates on a twin handle
    (bit-identical, reading 9);
  * mixed sizes, n log-uniform on [128, 2048] in one batch: eight sampled
    streams against the oracle (rank-4 steps on the smaller ones, lockstep
    rank-1 on the larger);
  * served mix with n = 512 ... 8192: every stream served equals the same
    updates on a lone handle.
"""
from concurrent.futures import ThreadPoolExecutor

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


def _de(h):
    d = np.empty(h.n)
    e = np.empty(h.n - 1)
    h.read_into(d=d, e=e)
    return d, e


class _Lockstep:
    """The oracle's continuation of a GPU handle on a few tracked rows.

    The rows are split into groups that the oracle passes on concurrent
    threads (its C entry points release the interpreter lock); each group
    regenerates the same rotations, so every group's d, e must agree."""

    def __init__(self, f, qr, pr, groups=1):
        self.m, self.n = f.Q.shape[0], f.P.shape[0]
        self.qr, self.pr = qr, pr
        self.gq = np.array_split(np.arange(len(qr)), groups)
        self.gp = np.array_split(np.arange(len(pr)), groups)
        self.Qr, self.Pr = f.Q[qr].copy(), f.P[pr].copy()
        self.d, self.e = f.d.copy(), f.e.copy()
        self.pool = ThreadPoolExecutor(groups) if groups > 1 else None

    def step(self, oracle, u, v):
        one = lambda g: oracle.bgu_pass_rows(self.m, self.n, self.Qr[self.gq[g]], self.d, self.e,
                                             self.Pr[self.gp[g]], u, v)
        outs = list(self.pool.map(one, range(len(self.gq)))) if self.pool else [one(0)]
        for g, (Qg, dg, eg, Pg) in enumerate(outs):
            _eq(f"oracle group {g} d", dg, outs[0][1])
            _eq(f"oracle group {g} e", eg, outs[0][2])
            self.Qr[self.gq[g]] = Qg
            self.Pr[self.gp[g]] = Pg
        self.d, self.e = outs[0][1], outs[0][2]

    def pass_(self, oracle, h, b, c, tag):
        u, v = h.project(b, c)
        self.step(oracle, u, v)
        h.update(b, c)
        d, e = _de(h)
        _eq(f"{tag} d", d, self.d)
        _eq(f"{tag} e", e, self.e)

    def rows(self, h, tag):
        Q, d, e, P = h.read()
        _eq(f"{tag} Q rows", Q[self.qr], self.Qr)
        _eq(f"{tag} P rows", P[self.pr], self.Pr)
        return Q, d, e, P

    def close(self):
        if self.pool:
            self.pool.shutdown()


# ---- one stream, 4000 x 2000, 200 updates --------------------------------------------

@pytest.fixture(scope="module")
def one_stream(bdu):
    f, ups = W.one_stream()
    rng = np.random.default_rng(74)
    qr = np.sort(rng.choice(f.m, 64, replace=False))
    pr = np.sort(rng.choice(f.n, 64, replace=False))
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    st = {"f": f, "ups": ups, "h": h, "ls": _Lockstep(f, qr, pr, groups=8), "done": 0, "A": f.dense()}
    yield st
    st["ls"].close()
    h.close()


def _run(oracle, st, upto):
    h, ls = st["h"], st["ls"]
    for k in range(st["done"], upto):
        B, C = st["ups"][k]
        ls.pass_(oracle, h, B[:, 0], C[:, 0], f"update {k}")
        st["A"] += B @ C.T
        if (k + 1) % 50 == 0:
            ls.rows(h, f"update {k}")
    st["done"] = upto


def test_one_stream_updates_0_to_99_lockstep(bdu, oracle, one_stream):
    _run(oracle, one_stream, 100)


def test_one_stream_updates_100_to_199_lockstep_and_invariants(bdu, oracle, one_stream):
    assert one_stream["done"] == 100, "runs after the first half"
    _run(oracle, one_stream, 200)
    f, A = one_stream["f"], one_stream["A"]
    m, n = f.m, f.n
    Q, d, e, P = one_stream["h"].read()
    Bd = np.zeros((n, n))
    Bd[np.arange(n), np.arange(n)] = d
    Bd[np.arange(n - 1), np.arange(1, n)] = e
    rec = np.linalg.norm(A - Q[:, :n] @ Bd @ P.T) / np.linalg.norm(A)
    assert rec <= 1e-12, rec
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-12 * np.sqrt(m)
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 1e-12 * np.sqrt(n)
    # singular values of Bd against a dense SVD of A+ (normwise, 1e-11 sigma_1)
    sa = np.linalg.svd(A, compute_uv=False)
    sb = np.linalg.svd(Bd, compute_uv=False)
    assert np.max(np.abs(sa - sb)) <= 1e-11 * sa[0]


# ---- recommendation-shaped, 10000 x 2000 ----------------------------------------------

def test_rating_stream_full_size(bdu, oracle):
    users, items = 10000, 2000
    A = W.ratings(users, items, seed=4000)
    Q0, d0, e0, P0 = W.bidiagonal_factors(A, seed=4001)
    f = W.Factorization(Q0, d0, e0, P0)
    del Q0
    rng = np.random.default_rng(4002)
    qr = np.sort(rng.choice(users, 32, replace=False))
    pr = np.sort(rng.choice(items, 32, replace=False))
    h1 = bdu.Handle(f.Q, f.d, f.e, f.P)   # rank-1 passes, in lockstep with the oracle
    hr = bdu.Handle(f.Q, f.d, f.e, f.P)   # the same calls as rank-r updates
    ls = _Lockstep(f, qr, pr, groups=4)
    calls = [1] * 8 + [4] * 3 + ["mean"] + [8] * 2
    passes = 0
    try:
        for ci, r in enumerate(calls):
            if r == "mean":  # subtract the row means: A <- A - (A e / n) e^T
                B = np.asfortranarray((-(A @ np.ones(items)) / items)[:, None])
                C = np.asfortranarray(np.ones((items, 1)))
            else:  # replace r users' rows
                who = rng.choice(users, r, replace=False)
                B = np.zeros((users, r), order="F")
                C = np.zeros((items, r), order="F")
                for k, i in enumerate(who):
                    B[i, k] = 1.0
                    C[:, k] = W.rating_row(rng, items, nnz=20) - A[i]
            A += B @ C.T
            hr.update(B, C)
            for k in range(B.shape[1]):
                ls.pass_(oracle, h1, B[:, k].copy(), C[:, k].copy(), f"call {ci} pass {k}")
                passes += 1
        Q1, d1, e1, P1 = ls.rows(h1, "end")
        Qr, dr, er, Prr = hr.read()
        for nm, x, y in zip("QdeP", (Qr, dr, er, Prr), (Q1, d1, e1, P1)):
            _eq(f"rank-r vs rank-1 {nm}", x, y)
        Bd = np.zeros((items, items))
        Bd[np.arange(items), np.arange(items)] = d1
        Bd[np.arange(items - 1), np.arange(1, items)] = e1
        rows = Q1[qr, :items] @ Bd @ P1.T
        assert np.linalg.norm(rows - A[qr]) <= 1e-12 * np.linalg.norm(A)
        assert passes == 8 + 12 + 1 + 16
    finally:
        ls.close()
        h1.close()
        hr.close()


# ---- mixed sizes in one batch ------------------------------------------------------

def _reflector_pair(rng, n):
    """A dense orthogonal matrix in milliseconds: the product of two
    Householder reflections."""
    M = np.eye(n)
    for _ in range(2):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        M = M - 2.0 * np.outer(M @ v, v)
    return np.asfortranarray(M)


def test_mixed_size_batch_sampled_streams(bdu, oracle):
    sizes = W.batched_sizes(count=256, seed=3000)
    rng = np.random.default_rng(3001)
    small = sorted({n for n in sizes if n <= 400})[:6]
    large = sorted({n for n in sizes if n >= 1500})[-2:]
    others = [n for n in sizes if n not in small and n not in large][:24]
    hs, refs, lock, batch = [], {}, {}, None
    try:
        for i, n in enumerate(small + large + others):
            if n in small or n in large:
                f = W.factorization(n, n, 3100 + i)
            else:
                Q = _reflector_pair(rng, n)
                f = W.Factorization(Q, rng.uniform(1, 10, n), rng.uniform(0, 1, n - 1), _reflector_pair(rng, n))
            hs.append(bdu.Handle(f.Q, f.d, f.e, f.P))
            if n in small:
                refs[i] = oracle.State(f.Q, f.d, f.e, f.P)
            elif n in large:
                lock[i] = _Lockstep(f, np.sort(rng.choice(n, 4, replace=False)),
                                    np.sort(rng.choice(n, 4, replace=False)))
        batch = bdu.Batch(hs, max_rank=4)
        for step in range(3):
            Bs, Cs, ranks = [], [], []
            for i, h in enumerate(hs):
                r = 4 if (i in refs and step != 1) else 1
                (B, C), = W.gaussian_updates(h.m, h.n, 1, 3200 + 100 * step + i, r=r)
                Bs.append(B)
                Cs.append(C)
                ranks.append(r)
            proj = {i: hs[i].project(Bs[i][:, 0], Cs[i][:, 0]) for i in lock}
            batch.update(Bs, Cs, ranks)
            batch.sync()
            for i, ref in refs.items():
                oracle.bgu_update(ref, Bs[i], Cs[i])
                for nm, x, y in zip("QdeP", hs[i].read(), (ref.Q, ref.d, ref.e, ref.P)):
                    _eq(f"step {step} stream {i} (n = {hs[i].n}) {nm}", x, y)
            for i, ls in lock.items():
                ls.step(oracle, *proj[i])
                d, e = _de(hs[i])
                _eq(f"step {step} stream {i} (n = {hs[i].n}) d", d, ls.d)
                _eq(f"step {step} stream {i} (n = {hs[i].n}) e", e, ls.e)
        for i, ls in lock.items():
            ls.rows(hs[i], f"stream {i}")
        assert len(refs) + len(lock) >= 8
    finally:
        if batch is not None:
            batch.close()
        for h in hs:
            h.close()


# ---- served mix up to n = 8192 --------------------------------------------------------

def test_served_mix_with_large_streams_equals_alone(bdu):
    sizes = [512, 1024, 2048, 4096, 8192]
    rng = np.random.default_rng(6000)
    srv = bdu.Server(budget_bytes=200 << 30, queue_cap=8, max_batch=8)
    sids, alone, plan = [], [], []
    try:
        for i, n in enumerate(sizes):
            Q, P = _reflector_pair(rng, n), _reflector_pair(rng, n)
            d, e = rng.uniform(1, 10, n), rng.uniform(0, 1, n - 1)
            sids.append(srv.open(Q, d, e, P))
            alone.append(bdu.Handle(Q, d, e, P))
            for k, r in enumerate((1, 2, 1)):
                (B, C), = W.gaussian_updates(n, n, 1, 6100 + 10 * i + k, r=r)
                plan.append((i, k, B, C))
        # submit in an interleaving that keeps each stream's own order
        queues = {i: [p for p in plan if p[0] == i] for i in range(len(sizes))}
        tickets = []
        while any(queues.values()):
            i = int(rng.choice([j for j in queues if queues[j]]))
            _, _, B, C = queues[i].pop(0)
            tickets.append(srv.submit(sids[i], B, C))
            alone[i].update(B, C)
        for t in tickets:
            srv.wait(t)
        st = srv.stats()
        assert st["completed"] == len(plan) and st["failed"] == 0
        for i, sid in enumerate(sids):
            got, one = srv.read(sid), alone[i].read()
            for nm, x, y in zip("QdeP", got, one):
                _eq(f"n = {sizes[i]} {nm} served vs alone", x, y)
            eq, ep = alone[i].orth_error()
            assert eq <= 1e-12 * np.sqrt(sizes[i]) and ep <= 1e-12 * np.sqrt(sizes[i])
    finally:
        srv.close()
        for h in alone:
            h.close()
