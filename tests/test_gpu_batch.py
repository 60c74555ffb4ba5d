"""Batches (bdu_batch_*): a fixed set of streams updated step after step.

Every step of a batch must leave each stream exactly where the oracle's
sequential rank-r update leaves it, whatever the mix of shapes, applier
tilings and per-step ranks (0 = no update) in the batch; from the second
step on the launches are a replayed HIP graph, so each replay is checked,
with unrelated eager work between replays.
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
                           f"{x.ravel()[bad[0]]!r} vs {y.ravel()[bad[0]]!r}")


SHAPES = [(120, 120), (97, 64), (64, 64), (150, 131), (33, 20), (2, 2), (200, 200)]
TILINGS = [(12, 7, 1), (12, 4, 2), (6, 2, 1), (12, 8, 1), (6, 4, 2), (12, 1, 1), (12, 7, 1)]


def _streams(bdu, oracle, seed):
    hs, refs = [], []
    saved = bdu.get_tiling()
    try:
        for i, ((m, n), tk) in enumerate(zip(SHAPES, TILINGS)):
            bdu.set_tiling(*tk)
            f = W.factorization(m, n, seed + i)
            hs.append(bdu.Handle(f.Q, f.d, f.e, f.P))
            refs.append(oracle.State(f.Q, f.d, f.e, f.P))
    finally:
        bdu.set_tiling(*saved)
    return hs, refs


def _check(hs, refs, what):
    for i, (h, ref) in enumerate(zip(hs, refs)):
        for nm, x, y in zip("QdeP", h.read(), (ref.Q, ref.d, ref.e, ref.P)):
            _eq(f"{what}, stream {i} {nm}", x, y)


@pytest.mark.parametrize("eager", [False, True])
def test_batch_steps_replayed_graph_match_oracle(bdu, oracle, eager):
    hs, refs = _streams(bdu, oracle, 300)
    other = bdu.Handle(*(lambda f: (f.Q, f.d, f.e, f.P))(W.factorization(80, 80, 399)))
    (ob, oc), = W.gaussian_updates(80, 80, 1, 398)
    batch = bdu.Batch(hs, max_rank=3, eager=eager)
    rng = np.random.default_rng(301)
    try:
        for step in range(6):
            ranks = rng.integers(0, 4, len(hs))
            ranks[step % len(hs)] = 3  # every step has a full-rank stream
            Bs, Cs = [], []
            for i, ((m, n), r) in enumerate(zip(SHAPES, ranks)):
                if r == 0:
                    Bs.append(None)
                    Cs.append(None)
                    continue
                (B, C), = W.gaussian_updates(m, n, 1, 1000 * step + i, r=int(r))
                Bs.append(B)
                Cs.append(C)
                oracle.bgu_update(refs[i], B, C)
            batch.update(Bs, Cs, [int(r) for r in ranks])
            other.update(ob, oc)  # unrelated eager work between replays
            batch.sync()
            _check(hs, refs, f"step {step} ranks {list(ranks)}")
            info = batch.info()
            assert info["steps"] == step + 1
            assert info["groups"] == 6  # (12,7,1) (12,4,2) (6,2,1) (12,8,1) (6,4,2) (12,1,1)
            assert info["graph"] == (1 if step >= 1 and not eager else 0)
    finally:
        batch.close()
        other.close()
        for h in hs:
            h.close()


def test_batch_with_stage_timing_runs_eagerly(bdu, oracle):
    hs, refs = _streams(bdu, oracle, 320)
    batch = bdu.Batch(hs, max_rank=2)
    try:
        for step in range(3):
            if step == 1:
                bdu.timing_enable(True)
            Bs, Cs = [], []
            for i, (m, n) in enumerate(SHAPES):
                (B, C), = W.gaussian_updates(m, n, 1, 2000 * step + i, r=1 + (i + step) % 2)
                Bs.append(B)
                Cs.append(C)
                oracle.bgu_update(refs[i], B, C)
            batch.update(Bs, Cs)
            batch.sync()
        t = bdu.timing_read()
        assert t["apply"][1] >= 2 * 6  # steps 1 and 2: two passes, six tiling groups
        assert batch.info()["graph"] == 0  # the graph is only captured with timing off
        _check(hs, refs, "timed steps")
    finally:
        bdu.timing_enable(False)
        batch.close()
        for h in hs:
            h.close()


def test_batch_member_calls_are_ordered_after_the_batch(bdu, oracle):
    """A plain update of a member right after a batch step (no sync) sees the step."""
    hs, refs = _streams(bdu, oracle, 340)
    batch = bdu.Batch(hs, max_rank=1)
    try:
        for step in range(3):
            Bs, Cs = [], []
            for i, (m, n) in enumerate(SHAPES):
                (B, C), = W.gaussian_updates(m, n, 1, 3000 * step + i)
                Bs.append(B)
                Cs.append(C)
                oracle.bgu_update(refs[i], B, C)
            batch.update(Bs, Cs)
            (B, C), = W.gaussian_updates(*SHAPES[0], 1, 3500 + step)
            hs[0].update(B, C)
            oracle.bgu_update(refs[0], B, C)
        _check(hs, refs, "batch then plain")
    finally:
        batch.close()
        for h in hs:
            h.close()


def test_batch_rejects_bad_arguments(bdu):
    f = W.factorization(20, 20, 360)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    try:
        with pytest.raises(bdu.BduError) as ei:
            bdu.Batch([h, h])
        assert ei.value.status == bdu.BDU_EINVAL
        b = bdu.Batch([h], max_rank=1)
        (B, C), = W.gaussian_updates(20, 20, 1, 361, r=2)
        with pytest.raises(bdu.BduError) as ei:
            b.update([B], [C])  # rank 2 > max_rank 1
        assert ei.value.status == bdu.BDU_EINVAL
        b.close()
    finally:
        h.close()


SUPPORTED = [(k0, nw, rpl) for k0 in (6, 12) for nw in (1, 2, 4, 8) for rpl in (1, 2)
             if (k0, nw, rpl) != (6, 8, 2)] + [(12, 3, 1), (12, 7, 1), (12, 15, 1), (12, 3, 2), (12, 7, 2),
                                               (18, 3, 1), (18, 5, 1), (18, 7, 1)]


def test_autotune_records_the_tiling_auto_handles_use(bdu, oracle):
    m, n = 150, 131
    res = bdu.autotune(m, n, 3)
    assert (res["k0"], res["nw"], res["rpl"]) in SUPPORTED
    assert res["us_per_step"] > 0
    saved = bdu.get_tiling()
    bdu.set_tiling_auto()
    try:
        assert bdu.get_tiling() == (0, 0, 0)
        f = W.factorization(m, n, 370)
        h = bdu.Handle(f.Q, f.d, f.e, f.P)
        assert h.tiling() == (res["k0"], res["nw"], res["rpl"])
        (B, C), = W.gaussian_updates(m, n, 1, 371, r=2)
        h.update(B, C)
        ref = oracle.State(f.Q, f.d, f.e, f.P)
        oracle.bgu_update(ref, B, C)
        for nm, x, y in zip("QdeP", h.read(), (ref.Q, ref.d, ref.e, ref.P)):
            _eq(f"auto-tiled {nm}", x, y)
        h.close()
        g = W.factorization(41, 40, 372)  # no entry for this shape: the default tiling
        h2 = bdu.Handle(g.Q, g.d, g.e, g.P)
        assert h2.tiling() == (12, 7, 1)
        h2.close()
    finally:
        bdu.set_tiling(*saved)


@pytest.mark.parametrize("tk", [(12, 7, 1), (12, 15, 1)])
def test_bench_launch_configuration_full_size(bdu, oracle, tk):
    """The benchmark's batched configuration: 64 streams at m = n = 2048 in
    one batch with the tilings its autotuner picks, passes in segments, the
    step replayed from the captured graph (an empty step first makes the
    real one the first replay).  Three streams are checked against the
    oracle: d, e and 16 sampled rows of Q and P, bit for bit."""
    n, S = 2048, 64
    f = W.factorization(n, n, 700)
    rng = np.random.default_rng(701)
    bs = [rng.standard_normal(n) for _ in range(S)]
    cs = [rng.standard_normal(n) for _ in range(S)]
    saved = bdu.get_tiling()
    bdu.set_tiling(*tk)
    try:
        hs = [bdu.Handle(f.Q, f.d, f.e, f.P) for _ in range(S)]
    finally:
        bdu.set_tiling(*saved)
    batch = bdu.Batch(hs, max_rank=1)
    batch.update([None] * S, [None] * S, ranks=[0] * S)
    batch.update(bs, cs)
    batch.sync()
    assert batch.info()["graph"] == 1
    for s in (0, S // 2, S - 1):
        Q1, d1, e1, P1 = hs[s].read()
        u = oracle.project(f.Q, bs[s])
        v = oracle.project(f.P, cs[s])
        qr = np.sort(rng.choice(n, 16, replace=False))
        pr = np.sort(rng.choice(n, 16, replace=False))
        Qr, d, e, Pr = oracle.bgu_pass_rows(n, n, f.Q[qr], f.d, f.e, f.P[pr], u, v)
        _eq(f"{tk} stream {s} d", d1, d)
        _eq(f"{tk} stream {s} e", e1, e)
        _eq(f"{tk} stream {s} Q rows", Q1[qr], Qr)
        _eq(f"{tk} stream {s} P rows", P1[pr], Pr)
    batch.close()
    for h in hs:
        h.close()
