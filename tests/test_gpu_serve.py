"""The served form: admission, bounded queues, continuous batching.

A stream's result must not depend on what else is being served: after a
mixed, interleaved load every stream equals both the oracle's sequential
updates and the same updates applied to a lone handle.
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
    assert bad.size == 0, f"{name}: {bad.size} of {x.size} differ, first at {bad[0]}"


SHAPES = [(90, 90), (120, 77), (64, 64), (150, 150), (33, 20)]


def test_mixed_load_equals_alone_and_oracle(bdu, oracle):
    srv = bdu.Server(budget_bytes=1 << 34, queue_cap=64, max_batch=8)
    rng = np.random.default_rng(500)
    sids, alone, refs, plan = [], [], [], []
    try:
        for i, (m, n) in enumerate(SHAPES):
            f = W.factorization(m, n, 510 + i)
            sids.append(srv.open(f.Q, f.d, f.e, f.P))
            alone.append(bdu.Handle(f.Q, f.d, f.e, f.P))
            refs.append(oracle.State(f.Q, f.d, f.e, f.P))
        # 6 requests per stream, ranks 1-3, submitted in a random interleaving
        for i, (m, n) in enumerate(SHAPES):
            for k in range(6):
                (B, C), = W.gaussian_updates(m, n, 1, 5000 + 10 * i + k, r=1 + (k + i) % 3)
                plan.append((i, k, B, C))
        order = rng.permutation(len(plan))
        per_stream = {i: [] for i in range(len(SHAPES))}
        for j in order:
            per_stream[plan[j][0]].append(plan[j])
        # keep each stream's own order k = 0..5 (the queue is FIFO per stream)
        for i in per_stream:
            per_stream[i].sort(key=lambda x: x[1])
        cursor = {i: 0 for i in per_stream}
        tickets = []
        for j in order:
            i = plan[j][0]
            _, k, B, C = per_stream[i][cursor[i]]
            cursor[i] += 1
            tickets.append(srv.submit(sids[i], B, C))
            alone[i].update(B, C)
            oracle.bgu_update(refs[i], B, C)
        lats = [srv.wait(t) for t in tickets]
        assert all(x >= 0 for x in lats)
        st = srv.stats()
        assert st["completed"] == len(plan) and st["failed"] == 0 and st["pending"] == 0
        assert st["batched_passes"] == sum(B.shape[1] for _, _, B, _ in plan)
        for i, sid in enumerate(sids):
            got, one = srv.read(sid), alone[i].read()
            for nm, x, y, z in zip("QdeP", got, one, (refs[i].Q, refs[i].d, refs[i].e, refs[i].P)):
                _eq(f"stream {i} {nm} served vs alone", x, y)
                _eq(f"stream {i} {nm} served vs oracle", x, z)
    finally:
        srv.close()
        for h in alone:
            h.close()


def test_paused_arrivals_form_one_round(bdu, oracle):
    """Requests for all streams queued while paused run as a single batched round."""
    srv = bdu.Server(budget_bytes=1 << 34, queue_cap=4, max_batch=16)
    try:
        sids, refs = [], []
        for i, (m, n) in enumerate(SHAPES):
            f = W.factorization(m, n, 530 + i)
            sids.append(srv.open(f.Q, f.d, f.e, f.P))
            refs.append(oracle.State(f.Q, f.d, f.e, f.P))
        srv.pause(True)
        for i, (m, n) in enumerate(SHAPES):
            (B, C), = W.gaussian_updates(m, n, 1, 540 + i)
            srv.submit(sids[i], B, C, detach=True)
            oracle.bgu_update(refs[i], B, C)
        assert srv.stats()["pending"] == len(SHAPES)
        srv.pause(False)
        srv.drain()
        st = srv.stats()
        assert st["rounds"] == 1 and st["batched_passes"] == len(SHAPES) and st["completed"] == len(SHAPES)
        for i, sid in enumerate(sids):
            for nm, x, y in zip("QdeP", srv.read(sid), (refs[i].Q, refs[i].d, refs[i].e, refs[i].P)):
                _eq(f"stream {i} {nm}", x, y)
    finally:
        srv.close()


def test_queue_cap_and_budget_admission(bdu):
    m = n = 64
    one = bdu.footprint_bytes(m, n)
    srv = bdu.Server(budget_bytes=2 * one + one // 2, queue_cap=2, max_batch=4)
    try:
        f = W.factorization(m, n, 550)
        a = srv.open(f.Q, f.d, f.e, f.P)
        b = srv.open(f.Q, f.d, f.e, f.P)
        with pytest.raises(bdu.BduError) as ei:
            srv.open(f.Q, f.d, f.e, f.P)
        assert ei.value.status == bdu.BDU_ENOMEM
        st = srv.stats()
        assert st["rejected_memory"] == 1 and st["streams"] == 2 and st["bytes_in_use"] == 2 * one
        srv.pause(True)
        (B, C), = W.gaussian_updates(m, n, 1, 551)
        t1 = srv.submit(a, B, C)
        t2 = srv.submit(a, B, C)
        with pytest.raises(bdu.BduError) as ei:
            srv.submit(a, B, C)
        assert ei.value.status == bdu.BDU_EBUSY
        t3 = srv.submit(b, B, C)  # the other stream's queue is independent
        assert not srv.poll(t1)
        srv.pause(False)
        for t in (t1, t2, t3):
            srv.wait(t)
        st = srv.stats()
        assert st["rejected_busy"] == 1 and st["completed"] == 3
        srv.close_stream(b)  # returns its budget: a new stream fits again
        c = srv.open(f.Q, f.d, f.e, f.P)
        assert srv.stats()["streams"] == 2 and c != b
    finally:
        srv.close()


def test_rounds_batch_passes_so_short_requests_finish_first(bdu, oracle):
    """A rank-1 request queued beside a rank-3 one finishes after the first round."""
    srv = bdu.Server(budget_bytes=1 << 34, queue_cap=4, max_batch=16)
    try:
        fa, fb = W.factorization(80, 80, 560), W.factorization(70, 60, 561)
        a = srv.open(fa.Q, fa.d, fa.e, fa.P)
        b = srv.open(fb.Q, fb.d, fb.e, fb.P)
        (Ba, Ca), = W.gaussian_updates(80, 80, 1, 562, r=3)
        (Bb, Cb), = W.gaussian_updates(70, 60, 1, 563, r=1)
        srv.pause(True)
        ta = srv.submit(a, Ba, Ca)
        tb = srv.submit(b, Bb, Cb)
        srv.pause(False)
        lb = srv.wait(tb)
        la = srv.wait(ta)
        st = srv.stats()
        assert st["rounds"] == 3 and st["batched_passes"] == 4
        assert lb < la
        ra, rb = oracle.State(fa.Q, fa.d, fa.e, fa.P), oracle.State(fb.Q, fb.d, fb.e, fb.P)
        oracle.bgu_update(ra, Ba, Ca)
        oracle.bgu_update(rb, Bb, Cb)
        for sid, ref in ((a, ra), (b, rb)):
            for nm, x, y in zip("QdeP", srv.read(sid), (ref.Q, ref.d, ref.e, ref.P)):
                _eq(f"stream {sid} {nm}", x, y)
    finally:
        srv.close()


@pytest.mark.parametrize("classes,rounds", [([], 8), ([100], 9)])
def test_size_classes_run_their_own_rounds(bdu, oracle, classes, rounds):
    """A rank-8 request on a large stream and a rank-1 request on a small
    one: with one class the small pass rides in the first of the large
    stream's eight rounds; with the two streams in different classes it
    runs in a round of its own, concurrently, and waits for none of them.
    Results are bit-identical either way."""
    srv = bdu.Server(budget_bytes=1 << 34, queue_cap=4, max_batch=16, classes=classes)
    try:
        fa, fb = W.factorization(300, 280, 570), W.factorization(64, 50, 571)
        assert srv.class_of(280) == len(classes) and srv.class_of(50) == 0
        a = srv.open(fa.Q, fa.d, fa.e, fa.P)
        b = srv.open(fb.Q, fb.d, fb.e, fb.P)
        (Ba, Ca), = W.gaussian_updates(300, 280, 1, 572, r=8)
        (Bb, Cb), = W.gaussian_updates(64, 50, 1, 573, r=1)
        srv.pause(True)
        ta = srv.submit(a, Ba, Ca)
        tb = srv.submit(b, Bb, Cb)
        srv.pause(False)
        srv.wait(ta)
        srv.wait(tb)
        st = srv.stats()
        assert st["rounds"] == rounds and st["batched_passes"] == 9 and st["completed"] == 2
        ra, rb = oracle.State(fa.Q, fa.d, fa.e, fa.P), oracle.State(fb.Q, fb.d, fb.e, fb.P)
        oracle.bgu_update(ra, Ba, Ca)
        oracle.bgu_update(rb, Bb, Cb)
        for sid, ref in ((a, ra), (b, rb)):
            for nm, x, y in zip("QdeP", srv.read(sid), (ref.Q, ref.d, ref.e, ref.P)):
                _eq(f"stream {sid} {nm}", x, y)
    finally:
        srv.close()


def test_streams_open_and_close_while_other_classes_run(bdu, oracle):
    """Membership changes rebuild a class's batch between its rounds; the
    other classes keep serving, and every stream ends equal to the oracle."""
    srv = bdu.Server(budget_bytes=1 << 34, queue_cap=8, max_batch=16, classes=[64, 128])
    try:
        shapes = [(60, 40), (100, 90), (200, 150), (50, 50)]
        fs = [W.factorization(m, n, 580 + i) for i, (m, n) in enumerate(shapes)]
        refs = [oracle.State(f.Q, f.d, f.e, f.P) for f in fs]
        sids = [srv.open(f.Q, f.d, f.e, f.P) for f in fs[:3]]
        tickets = []
        for k in range(4):
            for i in range(3):
                m, n = shapes[i]
                (B, C), = W.gaussian_updates(m, n, 1, 590 + 10 * k + i, r=1 + (k + i) % 2)
                tickets.append(srv.submit(sids[i], B, C))
                oracle.bgu_update(refs[i], B, C)
            if k == 1:  # a fourth stream joins class 0 mid-load
                sids.append(srv.open(fs[3].Q, fs[3].d, fs[3].e, fs[3].P))
            if k >= 1:
                m, n = shapes[3]
                (B, C), = W.gaussian_updates(m, n, 1, 700 + k)
                tickets.append(srv.submit(sids[3], B, C))
                oracle.bgu_update(refs[3], B, C)
        for t in tickets:
            srv.wait(t)
        for i, sid in enumerate(sids):
            for nm, x, y in zip("QdeP", srv.read(sid), (refs[i].Q, refs[i].d, refs[i].e, refs[i].P)):
                _eq(f"stream {i} {nm}", x, y)
        srv.close_stream(sids[0])  # class 0 rebuilt without it; stream 3 still served
        (B, C), = W.gaussian_updates(50, 50, 1, 710)
        srv.wait(srv.submit(sids[3], B, C))
        oracle.bgu_update(refs[3], B, C)
        for nm, x, y in zip("QdeP", srv.read(sids[3]), (refs[3].Q, refs[3].d, refs[3].e, refs[3].P)):
            _eq(f"stream 3 after close {nm}", x, y)
        assert srv.stats()["failed"] == 0
    finally:
        srv.close()


def test_concurrent_clients_across_classes(bdu):
    """Three client threads submit to streams of three size classes while the
    main thread opens, updates, reads and closes streams of a fourth; every
    stream ends equal to the same updates on a lone handle."""
    import threading

    srv = bdu.Server(budget_bytes=1 << 34, queue_cap=3, max_batch=16, classes=[64, 128, 256])
    shapes = [(50, 40), (60, 60), (120, 100), (110, 90), (250, 200), (240, 240)]
    fs = [W.factorization(m, n, 810 + i) for i, (m, n) in enumerate(shapes)]
    sids = [srv.open(f.Q, f.d, f.e, f.P) for f in fs]
    alone = [bdu.Handle(f.Q, f.d, f.e, f.P) for f in fs]
    plans = {i: [W.gaussian_updates(m, n, 1, 820 + 10 * i + k, r=1 + (k % 3))[0] for k in range(8)]
             for i, (m, n) in enumerate(shapes)}
    errors = []

    def client(idx):
        try:
            tickets = []
            for k in range(8):
                for i in idx:
                    B, C = plans[i][k]
                    while True:
                        try:
                            tickets.append(srv.submit(sids[i], B, C))
                            break
                        except bdu.BduError as err:
                            if err.status != bdu.BDU_EBUSY:
                                raise
            for t in tickets:
                srv.wait(t)
        except Exception as exc:  # reported by the main thread
            errors.append(exc)

    threads = [threading.Thread(target=client, args=([0, 1],)), threading.Thread(target=client, args=([2, 3],)),
               threading.Thread(target=client, args=([4, 5],))]
    try:
        for t in threads:
            t.start()
        for k in range(4):  # meanwhile: a stream of the largest class opens, updates, reads and closes
            f = W.factorization(300, 280, 850 + k)
            sid = srv.open(f.Q, f.d, f.e, f.P)
            lone = bdu.Handle(f.Q, f.d, f.e, f.P)
            (B, C), = W.gaussian_updates(300, 280, 1, 860 + k, r=2)
            srv.wait(srv.submit(sid, B, C))
            lone.update(B, C)
            for nm, x, y in zip("QdeP", srv.read(sid), lone.read()):
                _eq(f"transient stream {k} {nm}", x, y)
            srv.close_stream(sid)
            lone.close()
        for t in threads:
            t.join(timeout=240)
        assert not errors, errors
        for i, updates in plans.items():
            for B, C in updates:
                alone[i].update(B, C)
        for i, sid in enumerate(sids):
            for nm, x, y in zip("QdeP", srv.read(sid), alone[i].read()):
                _eq(f"stream {i} (n = {shapes[i][1]}) {nm}", x, y)
        st = srv.stats()
        assert st["failed"] == 0 and st["completed"] == 6 * 8 + 4
    finally:
        srv.close()
        for h in alone:
            h.close()
