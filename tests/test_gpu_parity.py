"""GPU parity: the HIP path through the C ABI against the CPU oracle.

The library and the oracle follow the same schedule and the same rounding
(sequential fma projections; r = sqrt(fma(a,a,b*b)); c, s by IEEE division;
fma(c,x,-(s*y)), fma(s,x,c*y)), so d, e, Q, P and every rotation must agree
exactly (== on values; the sign of a zero is not compared).  At the full
4000 x 2000 size the oracle checks d, e and sampled rows of Q and P after
the first update, and invariants after the whole stream.
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
    assert bad.size == 0, (f"{name}: {bad.size} of {x.size} differ, first at {bad[0]}: "
                           f"{x.ravel()[bad[0]]!r} vs {y.ravel()[bad[0]]!r}, "
                           f"max |diff| {np.max(np.abs(x - y)):.3e}")


def test_rotation_primitive_bit_exact(bdu, oracle):
    rng = np.random.default_rng(40)
    k = 20000
    a = rng.standard_normal(k) * 10.0 ** rng.integers(-300, 300, k)
    b = rng.standard_normal(k) * 10.0 ** rng.integers(-300, 300, k)
    a[::97] = 0.0
    b[::89] = 0.0
    a[1::53] = rng.standard_normal(len(a[1::53]))
    b[1::53] = rng.standard_normal(len(b[1::53]))
    for mode in (1, 2):
        c, s, r = bdu.givens_device(a, b, mode)
        ref = np.array([oracle.givens(x, y, mode) for x, y in zip(a, b)])
        _eq(f"c mode {mode}", c, ref[:, 0])
        _eq(f"s mode {mode}", s, ref[:, 1])
        _eq(f"r mode {mode}", r, ref[:, 2])


def test_rotation_primitive_fast_range_bit_exact(bdu, oracle):
    """Magnitudes inside the generator's fast range [2^-370, 2^370] in whole
    wavefronts of 64 (which then take the shortened square root and
    divisions), and wavefronts with one lane on or just past a bound."""
    rng = np.random.default_rng(41)
    k = 64 * 400
    a = rng.standard_normal(k) * 10.0 ** rng.uniform(-100, 100, k)
    b = rng.standard_normal(k) * 10.0 ** rng.uniform(-100, 100, k)
    lo, hi = 2.0 ** -370, 2.0 ** 370
    edges = [lo, np.nextafter(lo, 0.0), hi, np.nextafter(hi, np.inf), -lo, -hi]
    for w in range(0, k // 64, 5):
        x = edges[(w // 5) % len(edges)]
        if (w // 5) % 2:
            a[64 * w + w % 64] = x
        else:
            b[64 * w + (3 * w) % 64] = x
    for mode in (1, 2):
        c, s, r = bdu.givens_device(a, b, mode)
        ref = np.array([oracle.givens(x, y, mode) for x, y in zip(a, b)])
        _eq(f"c mode {mode}", c, ref[:, 0])
        _eq(f"s mode {mode}", s, ref[:, 1])
        _eq(f"r mode {mode}", r, ref[:, 2])


@pytest.mark.parametrize("m,n", [(2, 2), (64, 64), (65, 63), (200, 200), (4000, 2000)])
def test_projection_bit_exact(bdu, oracle, m, n):
    f = W.factorization(m, n, 41)
    rng = np.random.default_rng(42)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    u, v = h.project(b, c)
    h.close()
    _eq("u", u, oracle.project(f.Q, b))
    _eq("v", v, oracle.project(f.P, c))


PASS_SHAPES = [(2, 2), (3, 2), (3, 3), (4, 3), (5, 5), (12, 12), (14, 12), (13, 12), (65, 64),
               (130, 97), (200, 200), (257, 191), (300, 300)]


@pytest.mark.parametrize("m,n", PASS_SHAPES)
def test_pass_from_projections_bit_exact(bdu, oracle, m, n):
    """One pass from the oracle's projections: d, e, Q, P and every rotation."""
    f = W.factorization(m, n, 43)
    rng = np.random.default_rng(44)
    u, v = rng.standard_normal(m), rng.standard_normal(n)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update_projected(u, v)
    Q, d, e, P = h.read()
    side, idx, c, s = h.last_rotations()
    h.close()
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    _, tr, _ = oracle.bgu_pass(ref, u, v, flags=oracle.CHECK_PHASES, trace_cap=10 ** 7)
    _eq("side", side, tr["side"])
    _eq("idx", idx, tr["i"])
    _eq("c", c, tr["c"])
    _eq("s", s, tr["s"])
    _eq("d", d, ref.d)
    _eq("e", e, ref.e)
    _eq("Q", Q, ref.Q)
    _eq("P", P, ref.P)


def test_tiny_stream_bit_exact(bdu, oracle):
    """m = n = 200, 10 rank-1 updates, each projected independently on both sides."""
    f, ups = W.tiny()
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    for k, (B, C) in enumerate(ups):
        h.update(B, C)
        oracle.bgu_update(ref, B, C, flags=oracle.CHECK_PHASES)
        Q, d, e, P = h.read()
        _eq(f"d after update {k}", d, ref.d)
        _eq(f"e after update {k}", e, ref.e)
    _eq("Q", Q, ref.Q)
    _eq("P", P, ref.P)
    h.close()


@pytest.mark.parametrize("m,n,r", [(70, 53, 3), (128, 128, 4), (97, 96, 8)])
def test_rank_r_bit_exact(bdu, oracle, m, n, r):
    f = W.factorization(m, n, 45)
    (B, C), = W.gaussian_updates(m, n, 1, 46, r=r)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update(B, C)
    Q, d, e, P = h.read()
    h.close()
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_update(ref, B, C)
    for nm, x, y in [("d", d, ref.d), ("e", e, ref.e), ("Q", Q, ref.Q), ("P", P, ref.P)]:
        _eq(nm, x, y)


def test_tiling_does_not_change_results(bdu):
    m, n = 150, 131
    f = W.factorization(m, n, 47)
    (B, C), = W.gaussian_updates(m, n, 1, 48, r=2)
    outs = []
    saved = bdu.get_tiling()
    try:
        for tk in [(6, 1, 1), (12, 1, 1), (12, 2, 2), (12, 4, 2), (6, 4, 1), (12, 8, 2), (6, 8, 1), (12, 4, 1),
                   (12, 3, 1), (12, 7, 1), (12, 15, 1), (12, 3, 2), (12, 7, 2), (18, 5, 1)]:
            bdu.set_tiling(*tk)
            h = bdu.Handle(f.Q, f.d, f.e, f.P)
            h.update(B, C)
            outs.append(h.read())
            h.close()
    finally:
        bdu.set_tiling(*saved)
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            _eq("tiling", x, y)


STAGED = [(12, 3, 1), (12, 7, 1), (12, 15, 1), (12, 3, 2), (12, 7, 2), (18, 3, 1), (18, 5, 1), (18, 7, 1)]


@pytest.mark.parametrize("tk", STAGED)
@pytest.mark.parametrize("m,n", [(2, 2), (14, 12), (65, 64), (257, 191), (300, 300)])
def test_staged_applier_bit_exact(bdu, oracle, tk, m, n):
    """The staged applier (memory wavefront + compute wavefronts): one pass from
    the oracle's projections, d, e, Q and P exactly."""
    f = W.factorization(m, n, 80 + m)
    rng = np.random.default_rng(81 + n)
    u, v = rng.standard_normal(m), rng.standard_normal(n)
    saved = bdu.get_tiling()
    bdu.set_tiling(*tk)
    try:
        h = bdu.Handle(f.Q, f.d, f.e, f.P)
    finally:
        bdu.set_tiling(*saved)
    assert h.tiling() == tk
    h.update_projected(u, v)
    got = h.read()
    h.close()
    st = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_pass(st, u.copy(), v.copy())
    for nm, x, y in zip("QdeP", got, (st.Q, st.d, st.e, st.P)):
        _eq(f"{tk} {nm}", x, y)


def test_batched_equals_one_by_one(bdu, oracle):
    shapes = [(200, 200), (97, 64), (130, 130), (65, 64), (300, 257), (2, 2)]
    hs, hs1, refs, ups = [], [], [], []
    for i, (m, n) in enumerate(shapes):
        f = W.factorization(m, n, 50 + i)
        hs.append(bdu.Handle(f.Q, f.d, f.e, f.P))
        hs1.append(bdu.Handle(f.Q, f.d, f.e, f.P))
        refs.append(oracle.State(f.Q, f.d, f.e, f.P))
        ups.append(W.gaussian_updates(m, n, 3, 60 + i, r=1 + i % 3))
    for step in range(3):
        Bs = [u[step][0] for u in ups]
        Cs = [u[step][1] for u in ups]
        bdu.update_batched(hs, Bs, Cs)
        for h1, ref, B, C in zip(hs1, refs, Bs, Cs):
            h1.update(B, C)
            oracle.bgu_update(ref, B, C)
    for h, h1, ref in zip(hs, hs1, refs):
        got, one = h.read(), h1.read()
        for nm, x, y, z in zip("QdeP", got, one, (ref.Q, ref.d, ref.e, ref.P)):
            _eq(f"batched {nm} vs plain", x, y)
            _eq(f"batched {nm} vs oracle", x, z)
        h.close()
        h1.close()


@pytest.mark.parametrize("m,n", [(6, 6), (40, 40), (9, 6), (130, 70)])
def test_zero_start(bdu, oracle, m, n):
    f = W.zero_start(m, n)
    rng = np.random.default_rng(70)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    h.update(b, c)
    Q, d, e, P = h.read()
    h.close()
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_update(ref, b, c)
    for nm, x, y in [("d", d, ref.d), ("e", e, ref.e), ("Q", Q, ref.Q), ("P", P, ref.P)]:
        _eq(nm, x, y)
    nc = np.linalg.norm(c)
    tail = b[n - 1] * nc if m == n else np.linalg.norm(b) * nc
    assert abs(d[n - 1] - tail) <= 1e-13 * abs(tail)


def test_already_bidiagonal(bdu):
    n = 33
    f = W.factorization(n, n, 71)
    d0 = np.arange(1.0, n + 1)
    e0 = np.arange(2.0, n + 1)
    u = np.zeros(n); u[n - 2], u[n - 1] = 3.0, -5.0
    v = np.zeros(n); v[n - 1] = 0.5
    h = bdu.Handle(f.Q, d0, e0, f.P)
    h.update_projected(u, v)
    Q, d, e, P = h.read()
    side, idx, c, s = h.last_rotations()
    h.close()
    assert np.all(c == 1.0) and np.all(s == 0.0)
    _eq("Q", Q, f.Q)
    _eq("P", P, f.P)
    d_ref, e_ref = d0.copy(), e0.copy()
    d_ref[n - 1] += -2.5
    e_ref[n - 2] += 1.5
    _eq("d", d, d_ref)
    _eq("e", e, e_ref)


def test_device_pointers(bdu, oracle):
    import torch
    m, n = 120, 90
    f = W.factorization(m, n, 72)
    (B, C), = W.gaussian_updates(m, n, 1, 73, r=2)
    dev = torch.device("cuda:0")
    tQ = torch.from_numpy(f.Q.T.copy()).to(dev).T  # column-major on the device
    tP = torch.from_numpy(f.P.T.copy()).to(dev).T
    h = bdu.Handle(tQ, torch.from_numpy(f.d).to(dev), torch.from_numpy(f.e).to(dev), tP)
    tB = torch.from_numpy(B.T.copy()).to(dev).T
    tC = torch.from_numpy(C.T.copy()).to(dev).T
    h.update(tB, tC)
    oQ = torch.empty((m, m), dtype=torch.float64, device=dev).T.contiguous().T
    od = torch.empty(n, dtype=torch.float64, device=dev)
    h.read_into(Q=oQ, d=od)
    h.close()
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_update(ref, B, C)
    _eq("Q (device)", oQ.cpu().numpy(), ref.Q)
    _eq("d (device)", od.cpu().numpy(), ref.d)


def test_one_stream_full_size(bdu, oracle):
    """m = 4000, n = 2000, 200 updates.  First update: d, e and 64 sampled rows
    of Q and P match the oracle exactly.  After all 200: reconstruction,
    orthogonality and the Frobenius norm hold."""
    f, ups = W.one_stream()
    m, n = f.m, f.n
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    B, C = ups[0]
    h.update(B, C)
    Q1, d1, e1, P1 = h.read()
    u = oracle.project(f.Q, B[:, 0])
    v = oracle.project(f.P, C[:, 0])
    rng = np.random.default_rng(74)
    qr = np.sort(rng.choice(m, 64, replace=False))
    pr = np.sort(rng.choice(n, 64, replace=False))
    Qr, d, e, Pr = oracle.bgu_pass_rows(m, n, f.Q[qr], f.d, f.e, f.P[pr], u, v)
    _eq("d", d1, d)
    _eq("e", e1, e)
    _eq("Q rows", Q1[qr], Qr)
    _eq("P rows", P1[pr], Pr)
    Aplus = f.dense() + B @ C.T
    for B, C in ups[1:]:
        h.update(B, C)
        Aplus += B @ C.T
    Q, d, e, P = h.read()
    h.close()
    Bd = np.zeros((m, n))
    Bd[np.arange(n), np.arange(n)] = d
    Bd[np.arange(n - 1), np.arange(1, n)] = e
    rec = np.linalg.norm(Aplus - Q @ Bd @ P.T) / np.linalg.norm(Aplus)
    assert rec <= 1e-12, rec
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-12 * np.sqrt(m)
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 1e-12 * np.sqrt(n)
    assert abs(np.sqrt(d @ d + e @ e) - np.linalg.norm(Aplus)) <= 1e-13 * np.linalg.norm(Aplus)


@pytest.mark.parametrize("m,n", [(700, 5), (513, 2), (260, 3), (1030, 64)])
def test_spike_heavy_shapes(bdu, oracle, m, n):
    """m much larger than n: the spike dominates the left rotations."""
    f = W.factorization(m, n, 90 + n)
    (B, C), = W.gaussian_updates(m, n, 1, 91 + n, r=2)
    ref = oracle.State(f.Q, f.d, f.e, f.P)
    oracle.bgu_update(ref, B, C)
    saved = bdu.get_tiling()
    try:
        for tk in [(12, 7, 1), (12, 8, 1), (6, 1, 1), (12, 3, 2)]:
            bdu.set_tiling(*tk)
            h = bdu.Handle(f.Q, f.d, f.e, f.P)
            h.update(B, C)
            for nm, x, y in zip("QdeP", h.read(), (ref.Q, ref.d, ref.e, ref.P)):
                _eq(f"{tk} {nm}", x, y)
            h.close()
    finally:
        bdu.set_tiling(*saved)


def test_nonfinite_inputs_are_rejected(bdu, oracle):
    m, n = 60, 50
    f = W.factorization(m, n, 95)
    (B, C), = W.gaussian_updates(m, n, 1, 96, r=2)
    bdu.set_finite_check(True)
    try:
        h = bdu.Handle(f.Q, f.d, f.e, f.P)
        before = h.read()
        for bad in ("B", "C"):
            Bb, Cb = B.copy(order="F"), C.copy(order="F")
            (Bb if bad == "B" else Cb)[3, 1] = np.nan if bad == "B" else np.inf
            with pytest.raises(bdu.BduError) as ei:
                h.update(Bb, Cb)
            assert ei.value.status == bdu.BDU_ENONFINITE
            for nm, x, y in zip("QdeP", h.read(), before):
                _eq(f"unchanged after bad {bad}: {nm}", x, y)
        u = np.ones(m)
        u[7] = -np.inf
        with pytest.raises(bdu.BduError):
            h.update_projected(u, np.ones(n))
        h.update(B, C)  # finite inputs still go through
        ref = oracle.State(f.Q, f.d, f.e, f.P)
        oracle.bgu_update(ref, B, C)
        for nm, x, y in zip("QdeP", h.read(), (ref.Q, ref.d, ref.e, ref.P)):
            _eq(f"after a good update: {nm}", x, y)
        g = W.factorization(m, n, 97)
        d_bad = g.d.copy()
        d_bad[0] = np.nan
        with pytest.raises(bdu.BduError) as ei:
            bdu.Handle(g.Q, d_bad, g.e, g.P)
        assert ei.value.status == bdu.BDU_ENONFINITE
        h2 = bdu.Handle(g.Q, g.d, g.e, g.P)
        b2 = h2.read()
        Bb = B.copy(order="F")
        Bb[0, 0] = np.nan
        with pytest.raises(bdu.BduError) as ei:
            bdu.update_batched([h2, h], [B, Bb], [C, C])
        assert ei.value.status == bdu.BDU_ENONFINITE
        for nm, x, y in zip("QdeP", h2.read(), b2):
            _eq(f"batch member unchanged: {nm}", x, y)
        h.close()
        h2.close()
    finally:
        bdu.set_finite_check(False)


def test_plain_bench_configuration_full_size(bdu, oracle):
    """The benchmark's plain leg: one stream at m = n = 2048 with tiling
    (12, 15, 1), the pass in eight segments; d, e and 32 sampled rows of Q
    and P against the oracle, bit for bit."""
    n = 2048
    f = W.factorization(n, n, 710)
    rng = np.random.default_rng(711)
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    saved = bdu.get_tiling()
    bdu.set_tiling(12, 15, 1)
    try:
        h = bdu.Handle(f.Q, f.d, f.e, f.P)
    finally:
        bdu.set_tiling(*saved)
    assert len(bdu.plan_segments(n, n)[0]) == 8
    h.update(b.reshape(n, 1), c.reshape(n, 1))
    Q1, d1, e1, P1 = h.read()
    h.close()
    u = oracle.project(f.Q, b)
    v = oracle.project(f.P, c)
    qr = np.sort(rng.choice(n, 32, replace=False))
    pr = np.sort(rng.choice(n, 32, replace=False))
    Qr, d, e, Pr = oracle.bgu_pass_rows(n, n, f.Q[qr], f.d, f.e, f.P[pr], u, v)
    _eq("d", d1, d)
    _eq("e", e1, e)
    _eq("Q rows", Q1[qr], Qr)
    _eq("P rows", P1[pr], Pr)
