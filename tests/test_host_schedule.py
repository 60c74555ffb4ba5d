"""Host-side logic of the GPU library (no device needed).

- The schedule the device decodes in closed form is the oracle's rotation
  sequence, rotation for rotation (side, index, phase).
- The generation ticks respect every data dependency: two rotations that
  touch a common entry of the working matrix, of u or of v run at ticks in
  schedule order.  Entry sets are derived here from the rotation windows,
  independently of the library's conservative row intervals.
- The library exports every function its header declares.
"""
import bisect
import os
import re

import numpy as np
import pytest

from paper_2509_02840_amd import bdu
from paper_2509_02840_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SHAPES = [(2, 2), (3, 2), (3, 3), (4, 3), (5, 5), (7, 4), (12, 12), (14, 12), (13, 12), (30, 20),
          (31, 31), (45, 40), (64, 64), (65, 64), (100, 37)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_decoded_schedule_is_the_oracle_sequence(oracle, m, n):
    side, idx, ph, tick = bdu.plan_rotations(m, n)
    f = W.factorization(m, n, 1)
    st = oracle.State(f.Q, f.d, f.e, f.P)
    rng = np.random.default_rng(3)
    cnt, tr, _ = oracle.bgu_pass(st, rng.standard_normal(m), rng.standard_normal(n),
                                 flags=oracle.NO_QP, trace_cap=10 ** 6)
    keep = side != 2
    assert np.count_nonzero(side == 2) == 1  # the fold
    assert np.array_equal(side[keep], tr["side"])
    assert np.array_equal(idx[keep], tr["i"])
    assert np.array_equal(ph[keep], tr["phase"])
    stats = bdu.plan_stats(m, n)
    assert stats["left"] == cnt[0] and stats["right"] == cnt[1] and stats["spike"] == cnt[2]


def _cells(side, i, m, n, N):
    """Entries a step reads and writes: ('W', r, c), ('u', i), ('v', j).  The
    windows are those the schedule can make nonzero (columns i-1..i+3 of a
    left rotation, rows j-2..j+2 of a right one), which the oracle pin
    test_rotation_windows_hold_every_nonzero checks."""
    out = []
    if side == 0:  # left rotation on rows i, i+1
        for c in range(max(1, i - 1), min(n, i + 3) + 1):
            if i + 1 <= N:
                out += [("W", i, c), ("W", i + 1, c)]
        out += [("u", i), ("u", i + 1)]
    elif side == 1:  # right rotation on columns i, i+1
        for r in range(max(1, i - 2), min(N, i + 2) + 1):
            out += [("W", r, i), ("W", r, i + 1)]
        out += [("v", i), ("v", i + 1)]
    else:  # fold: (N-1, n), (N, n), u_{N-1}, u_N, v_n
        out = [("W", N - 1, n), ("W", N, n), ("u", N - 1), ("u", N), ("v", n)]
    return out


@pytest.mark.parametrize("m,n", [(12, 12), (14, 12), (31, 31), (45, 40), (64, 64), (100, 37), (90, 90)])
def test_generation_ticks_respect_dependencies(m, n):
    side, idx, ph, tick = bdu.plan_rotations(m, n)
    N = n if m == n else n + 1
    last = {}
    for s, i, p, t in zip(side, idx, ph, tick):
        if p == 0:
            assert t == -1  # the spike runs before generation
            continue
        for cell in _cells(int(s), int(i), m, n, N):
            prev = last.get(cell, -1)
            assert t > prev, (s, i, p, t, cell, prev)
            last[cell] = t


def test_ticks_are_parallel():
    """Generation runs many chains at once: far fewer ticks than rotations."""
    st = bdu.plan_stats(2048, 2048)
    assert st["ticks"] * 50 < st["left"] + st["right"]


def test_library_exports_every_declared_function():
    hdr = open(os.path.join(ROOT, "include", "bdu.h")).read()
    names = re.findall(r"^\w[\w\s\*]*?\b(bdu_\w+)\s*\(", hdr, flags=re.M)
    assert len(names) >= 15
    L = bdu.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_invalid_arguments_fail_without_a_device():
    import ctypes
    L = bdu.lib()
    h = ctypes.c_void_p()
    one = np.ones(4)
    assert L.bdu_create(2, 3, one.ctypes.data, one.ctypes.data, one.ctypes.data, one.ctypes.data,
                        ctypes.byref(h)) == bdu.BDU_EINVAL  # m < n
    assert L.bdu_create(1, 1, one.ctypes.data, one.ctypes.data, one.ctypes.data, one.ctypes.data,
                        ctypes.byref(h)) == bdu.BDU_EINVAL  # n < 2
    assert L.bdu_create(4, 4, None, one.ctypes.data, one.ctypes.data, one.ctypes.data,
                        ctypes.byref(h)) == bdu.BDU_EINVAL
    assert L.bdu_update(None, one.ctypes.data, one.ctypes.data, 1) == bdu.BDU_EINVAL
    assert L.bdu_update_batched(None, None, None, None, 0) == bdu.BDU_EINVAL
    assert L.bdu_set_tiling(7, 1, 1) == bdu.BDU_EINVAL
    assert L.bdu_set_tiling(12, 4, 3) == bdu.BDU_EINVAL
    assert L.bdu_plan_stats(3, 4, None) == bdu.BDU_EINVAL
    assert bdu.lib().bdu_strerror(bdu.BDU_ENOMEM) == b"out of device memory"


def test_footprint_grows_with_size():
    a, b = bdu.footprint_bytes(512, 512), bdu.footprint_bytes(1024, 1024)
    assert 2.5 * a < b < 4.5 * a
    assert b > 16 * 1024 * 1024  # Q and P alone


def test_tuning_table_round_trip(tmp_path):
    """The autotuner's table is plain text; loading validates every line."""
    good = tmp_path / "tune.txt"
    good.write_text("# comment\n2048 2048 12 8 1 280000.0\n4000 2000 12 4 2 1500.5\n")
    assert bdu.tune_load(str(good)) == 2
    out = tmp_path / "saved.txt"
    bdu.tune_save(str(out))
    rows = [ln.split() for ln in out.read_text().splitlines() if not ln.startswith("#")]
    assert ["2048", "2048", "12", "8", "1"] in [r[:5] for r in rows]
    assert ["4000", "2000", "12", "4", "2"] in [r[:5] for r in rows]
    for bad in ("2048 2048 7 8 1 1.0\n", "10 20 12 8 1 1.0\n", "2048 2048 12\n", "6 6 6 8 2 1.0\n"):
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        with pytest.raises(bdu.BduError):
            bdu.tune_load(str(p))
    with pytest.raises(bdu.BduError):
        bdu.tune_load(str(tmp_path / "missing.txt"))


def test_plan_queries_in_auto_tiling_mode(tmp_path):
    """Schedule queries resolve the per-shape tiling in "auto" mode (no 0-wide blocks)."""
    saved = bdu.get_tiling()
    f = tmp_path / "t.txt"
    f.write_text("64 64 6 2 1 10.0\n")
    bdu.tune_load(str(f))
    try:
        bdu.set_tiling_auto()
        a = bdu.plan_stats(64, 64)   # tuned entry
        b = bdu.plan_stats(65, 64)   # default tiling
        side, idx, ph, tick = bdu.plan_rotations(64, 64)
        assert a["left"] + a["right"] + 1 == len(side)  # plus the fold
        assert b["chains"] > 0 and bdu.footprint_bytes(64, 64) > 0
    finally:
        bdu.set_tiling(*saved)


def _staged_protocol_violations(K0, NW, lmax, RC=15):
    """Replay the staged applier's LDS column hand-overs front by front (a
    barrier after every front) and return every read that does not see its
    value's write across a barrier, or that is not separated by a barrier
    from the slot's next write.  Ring j feeds compute wavefront j (ring 0
    from the memory wavefront, ring NW to it).  Compute wavefront w reads
    columns 0..3 at its first front and 3f+4..3f+6 at every front f (a front
    early); the memory wavefront writes columns 0..6 before the first barrier
    and 3F+7..3F+9 at front F, and stores the columns the last wavefront
    finished at F-1.  (The coefficients reach the compute wavefronts by
    scalar loads, outside LDS.)"""
    U = S = K0 + 3
    lam_hi = lmax + 1
    fend = lmax // 3 + K0 + 1
    Fend = fend + (NW - 1) * S
    nfront = -(-(Fend + 1) // S) * S
    flush_end = lam_hi // 3 + K0 - 1
    nchunk = nfront // U
    events = {}  # (ring, slot) -> list of (F, order, kind, value)

    def put(ring, slot, F, kind, value, order):
        events.setdefault((ring, slot), []).append((F, order, kind, value))

    PRO = -1  # the memory wavefront's prologue, before the first barrier
    for lam in range(7):
        put(0, lam % RC, PRO, "w", lam, 0)
    for F in range(nfront):
        for k in range(3):
            lam = 3 * F + 7 + k
            put(0, lam % RC, F, "w", lam, 0)
        for k in range(3):
            lam = 3 * (F - 1 - (NW - 1) * S - K0 + 1) + k
            if 0 <= lam <= lam_hi:
                put(NW, lam % RC, F, "r", lam, 1)
    for w in range(NW):
        live_end = min(w + (flush_end + U) // U, nchunk)
        for f in range(0, live_end * U - w * S):
            F = w * S + f
            lams = ([0, 1, 2, 3] if f == 0 else []) + [3 * f + 4, 3 * f + 5, 3 * f + 6]
            for lam in lams:
                if lam <= lam_hi + 6:
                    put(w, lam % RC, F, "r", lam, 1)
            for k in range(3):
                lam = 3 * (f - K0 + 1) + k
                if lam >= 0:
                    put(w + 1, lam % RC, F, "w", lam, 0)
    def barrier_between(a, b):  # the barrier after some front B, a <= B < b
        return a < b

    bad = []
    for key, ev in events.items():
        ev.sort(key=lambda x: (x[0], x[1]))
        writes = [e for e in ev if e[2] == "w"]
        for F, _, kind, value in ev:
            if kind != "r":
                continue
            mine = [wr for wr in writes if wr[3] == value]
            if not mine:
                if value <= lam_hi:
                    bad.append((key, F, value, "never written"))
                continue
            Fw = mine[-1][0]
            if not (Fw == PRO or barrier_between(Fw, F)):
                bad.append((key, F, value, f"written at {Fw} without a barrier before the read"))
            later = [wr for wr in writes if (wr[0], wr[1]) > (Fw, 0) and wr[3] != value]
            if later and not barrier_between(F, later[0][0]):
                bad.append((key, F, value, f"slot rewritten at {later[0][0]} without a barrier after the read"))
    return bad


@pytest.mark.parametrize("K0,NW,RC", [(12, 3, 15), (12, 7, 15), (12, 15, 15), (18, 3, 21), (18, 5, 21), (18, 7, 21)])
@pytest.mark.parametrize("lmax", [0, 1, 2, 5, 17, 40, 100, 257])
def test_staged_lds_protocol_is_race_free(K0, NW, RC, lmax):
    assert _staged_protocol_violations(K0, NW, lmax, RC=RC) == []


def _pipelined_launch_violations(K0, NW, blocks, ncols, RC=15, margin=None):
    """Replay one launch of the staged applier over plan blocks (rows base,
    lmax, nfront, phase, start, off) the way the kernel runs them back to
    back: every wavefront runs one barrier per front of T chunks of U fronts;
    compute wavefront w is live in block b from chunk rel_b + w for C_b
    chunks; the memory wavefront's load side follows the block of its last
    prologue, its store side the oldest block not yet written back.  Returns
    the violations of: (1) LDS: every read of a column a block needs sees
    the write of that column across a barrier, with no other write to the
    slot from that write's front to the read's; (2) device memory: every
    load of a column comes at least `margin` fronts after every earlier
    block's store of it, and every store after every earlier block's load
    and store of it; (3) barriers: no wavefront would need to go back in
    time (its idle count would be negative)."""
    U = S = K0 + 3
    DL = U // 3
    margin = DL + 3 if margin is None else margin
    bl = [tuple(int(x) for x in r) for r in blocks if r[1] >= 0]
    if not bl:
        return []
    start0 = bl[0][4]
    views = []
    for base, lmax, nfront, phase, start, off in bl:
        desc = phase == 1
        lam_hi = lmax + 1
        views.append(dict(rel=start - start0, nfront=nfront, lam_hi=lam_hi, C=(lam_hi // 3 + K0 - 1 + U) // U,
                          dir=-1 if desc else 1, col0=base - 1,
                          lam_lo=max(base - ncols, 0) if desc else 0))
    T = max(v["rel"] + v["nfront"] // U for v in views)
    bad = []
    ev = {}    # (ring, slot) -> [(G, wave, order, kind, value)]
    mem = {}   # matrix column -> [(G, order, kind, block)]

    def lds(ring, lam, G, wave, order, kind, value):
        ev.setdefault((ring, lam % RC), []).append((G, wave, order, kind, value))

    def col(v, lam):
        return v["col0"] + v["dir"] * lam

    def valid(v, lam):
        c = col(v, lam)
        return 0 <= lam <= v["lam_hi"] and 0 <= c < ncols

    def mload(b, lam, G, order):
        v = views[b]
        if valid(v, lam):
            mem.setdefault(col(v, lam), []).append((G, order, "load", b))

    # memory wavefront (wave NW)
    def prologue(b, G):
        for lam in range(7):
            lds(0, lam, G, NW, 5, "w", (b, lam))
            mload(b, lam, G, 5)
        for j in range(DL):
            for k in range(3):
                mload(b, 3 * j + 7 + k, G, 6)
    L = St = 0
    prologue(0, -1)
    nxt = 1
    next_pro = views[1]["rel"] * U - 1 if len(views) > 1 else -2
    for G in range(T * U):
        v = views[L]
        Fl = G - v["rel"] * U
        if Fl < v["C"] * U - 1:
            for k in range(3):
                lds(0, 3 * Fl + 7 + k, G, NW, 0, "w", (L, 3 * Fl + 7 + k))
                mload(L, 3 * (Fl + DL) + 7 + k, G, 1)
        if St < len(views):
            vs = views[St]
            Fs = G - vs["rel"] * U
            for k in range(3):
                lam = 3 * (Fs - 1 - (NW - 1) * S - K0 + 1) + k
                if vs["lam_lo"] <= lam <= vs["lam_hi"]:
                    lds(NW, lam, G, NW, 2, "r", (St, lam))
                    if valid(vs, lam):
                        mem.setdefault(col(vs, lam), []).append((G, 3, "store", St))
            if Fs >= vs["lam_hi"] // 3 + (NW - 1) * S + K0:
                St += 1
        if G == next_pro:
            L = nxt
            prologue(L, G)
            nxt += 1
            next_pro = views[nxt]["rel"] * U - 1 if nxt < len(views) else -2
    if nxt < len(views):
        bad.append(("prologue never reached", nxt))
    if St < len(views):
        bad.append(("blocks not written back", St))
    # compute wavefronts
    for w in range(NW):
        cur = 0
        for b, v in enumerate(views):
            nlive = min(v["C"], v["nfront"] // U - w)
            if v["rel"] + w < cur:
                bad.append(("barrier count", w, b))
            cur = v["rel"] + w + nlive
            for f in range(nlive * U):
                G = (v["rel"] + w) * U + f
                lams = ([0, 1, 2, 3] if f == 0 else []) + [3 * f + 4, 3 * f + 5, 3 * f + 6]
                for lam in lams:
                    if lam <= v["lam_hi"]:
                        lds(w, lam, G, w, 1, "r", (b, lam))
                for k in range(3):
                    lam = 3 * (f - K0 + 1) + k
                    if lam >= 0:
                        lds(w + 1, lam, G, w, 3, "w", (b, lam))
        if cur > T:
            bad.append(("barrier count at the end", w))
    # (1) LDS hand-overs: the slot's last write before the read's front is
    # the value's, every write at that front comes from one wavefront (in
    # its program order), and nothing writes the slot at the read's front
    for key, es in ev.items():
        writes = sorted(e for e in es if e[3] == "w")
        fronts = [wr[0] for wr in writes]
        for G, wave, order, kind, value in es:
            if kind != "r":
                continue
            j = bisect.bisect_left(fronts, G) - 1
            if j < 0 or writes[j][4] != value:
                bad.append(("not the slot's last write", key, G, value, writes[j][4] if j >= 0 else None))
                continue
            Gw = fronts[j]
            same = writes[bisect.bisect_left(fronts, Gw):j + 1]
            if any(wr[1] != writes[j][1] for wr in same):
                bad.append(("two wavefronts write the slot in one front", key, Gw, value))
            if bisect.bisect_right(fronts, G) != bisect.bisect_left(fronts, G):
                bad.append(("slot written in the read's front", key, G, value))
    # (2) device memory: each access of a block against every access of an
    # earlier block to the same column, whatever their order in time
    for c, es in mem.items():
        for G, o, kind, b in es:
            for G2, o2, kind2, b2 in es:
                if b2 >= b:
                    continue
                if kind == "load" and kind2 == "store" and G < G2 + margin:
                    bad.append(("load too soon after an earlier block's store", c, b, G, b2, G2))
                if kind == "store" and (G, o) <= (G2, o2):
                    bad.append(("store before an earlier block's access", c, b, G, b2, G2))
    return bad


_PIPE_TILINGS = [(12, 3, 1, 15), (12, 7, 1, 15), (12, 15, 1, 15), (18, 3, 1, 21), (18, 5, 1, 21), (18, 7, 1, 21)]


@pytest.mark.parametrize("k0,nw,rpl,RC", _PIPE_TILINGS)
@pytest.mark.parametrize("m,n", [(40, 40), (130, 97), (257, 191), (420, 150), (900, 900)])
def test_pipelined_staged_launches_are_race_free(k0, nw, rpl, RC, m, n):
    """Every launch the plan makes (the whole pass, each phase, each
    segment) on both sides replays without an LDS race, a device-memory
    reordering or a barrier mismatch."""
    saved = bdu.get_tiling()
    try:
        bdu.set_tiling(k0, nw, rpl)
        tcut, bcut, _ = bdu.plan_segments(m, n)
        for side, ncols in ((0, m), (1, n)):
            blocks = bdu.plan_blocks(m, n, side)
            nb1 = int(np.sum(blocks[:, 3] == 1))
            parts = [(0, len(blocks)), (0, nb1), (nb1, len(blocks))]
            prev = 0
            for c in bcut:
                parts.append((prev, int(c)))
                prev = int(c)
            for a, b in parts:
                assert _pipelined_launch_violations(k0, nw, blocks[a:b], ncols, RC=RC) == [], (side, a, b)
    finally:
        bdu.set_tiling(*saved)


def test_plan_blocks_boundary():
    """bdu_plan_blocks: argument errors, and the layout the kernels read
    (phase-1 blocks first, slots back to back, start chunks non-decreasing
    and at least the previous block's live chunks apart)."""
    L = bdu.lib()
    assert L.bdu_plan_blocks(5, 6, 0, None, 0) == bdu.BDU_EINVAL   # m < n
    assert L.bdu_plan_blocks(6, 6, 2, None, 0) == bdu.BDU_EINVAL   # side
    assert L.bdu_plan_blocks(6, 6, 0, None, -1) == bdu.BDU_EINVAL  # cap
    assert L.bdu_plan_blocks(6, 6, 0, None, 3) == bdu.BDU_EINVAL   # no room
    saved = bdu.get_tiling()
    try:
        for k0, nw in ((12, 15), (12, 7), (18, 5)):
            bdu.set_tiling(k0, nw, 1)
            U = k0 + 3
            K = k0 * nw
            for side in (0, 1):
                b = bdu.plan_blocks(300, 260, side)
                st = bdu.plan_stats(300, 260)
                ph = b[:, 3]
                assert list(ph) == sorted(ph)
                assert np.all(b[1:, 5] == b[:-1, 5] + b[:-1, 2] * K)
                assert b[-1, 5] + b[-1, 2] * K == st["left_slots" if side == 0 else "right_slots"]
                assert np.all(b[:, 2] % U == 0)
                live = [(b[i, 4], ((b[i, 1] + 1) // 3 + k0 - 1 + U) // U) for i in range(len(b)) if b[i, 1] >= 0]
                for (s0, c0), (s1, _) in zip(live, live[1:]):
                    assert s1 >= s0 + c0
    finally:
        bdu.set_tiling(*saved)


def test_pipelined_checker_sees_a_reordering():
    """Blocks started one chunk after the previous one's live chunks, ignoring
    the device-memory order, would load columns before they are stored."""
    saved = bdu.get_tiling()
    try:
        bdu.set_tiling(12, 15, 1)
        blocks = bdu.plan_blocks(600, 600, 1).copy()
        U = 15
        s = 0
        for r in blocks:
            if r[1] < 0:
                continue
            r[4] = s
            s += ((r[1] + 1) // 3 + 12 - 1 + U) // U
        bad = _pipelined_launch_violations(12, 15, blocks, 600)
        assert any(b[0].startswith("load too soon") for b in bad)
    finally:
        bdu.set_tiling(*saved)


def test_staged_protocol_checker_sees_a_race():
    """A ring of 9 columns (three fronts) would be rewritten in the front of
    its last read."""
    assert _staged_protocol_violations(12, 7, 100, RC=9) != []


def test_finite_check_switch_validates_its_argument():
    assert bdu.lib().bdu_set_finite_check(2) == bdu.BDU_EINVAL
    assert bdu.lib().bdu_set_finite_check(0) == bdu.BDU_OK


def test_tracking_rejects_bad_sizes_without_a_device():
    import ctypes
    L = bdu.lib()
    h = ctypes.c_void_p()
    U = np.zeros((4, 3), order="F")
    d = np.ones(3)
    e = np.ones(2)
    V = np.zeros((5, 3), order="F")
    # r > m
    assert L.bdu_track_create(2, 5, 3, U.ctypes.data, d.ctypes.data, e.ctypes.data, V.ctypes.data,
                              ctypes.byref(h)) == bdu.BDU_EINVAL
    # r > n
    assert L.bdu_track_create(4, 2, 3, U.ctypes.data, d.ctypes.data, e.ctypes.data, V.ctypes.data,
                              ctypes.byref(h)) == bdu.BDU_EINVAL
    # r = 0
    assert L.bdu_track_create(4, 5, 0, U.ctypes.data, d.ctypes.data, e.ctypes.data, V.ctypes.data,
                              ctypes.byref(h)) == bdu.BDU_EINVAL
    # e missing with r > 1
    assert L.bdu_track_create(4, 5, 3, U.ctypes.data, d.ctypes.data, None, V.ctypes.data,
                              ctypes.byref(h)) == bdu.BDU_EINVAL
    assert L.bdu_track_update(None, None, None) == bdu.BDU_EINVAL
    assert L.bdu_track_last(None, None, None, None) == bdu.BDU_EINVAL
    assert L.bdu_track_orth_error(None, None, None) == bdu.BDU_EINVAL
    assert L.bdu_track_reorthogonalize(None, 0.0, None, None) == bdu.BDU_EINVAL
    assert L.bdu_track_set_drift_check(None, 5, 1e-12) == bdu.BDU_EINVAL
    assert L.bdu_track_drift_stats(None, None, None, None, None) == bdu.BDU_EINVAL
    assert L.bdu_strerror(bdu.BDU_ESPAN) == b"rank-1 tracker with an update vector in the span of its basis"


def test_orthogonality_calls_reject_a_null_handle():
    L = bdu.lib()
    assert L.bdu_orth_error(None, None, None) == bdu.BDU_EINVAL
    assert L.bdu_reorthogonalize(None, 0.0, None, None) == bdu.BDU_EINVAL


def test_truncated_bd_rejects_bad_ranks_without_a_device():
    L = bdu.lib()
    assert L.bdu_truncated_bd(None, 1, None, None, None, None) == bdu.BDU_EINVAL


@pytest.mark.parametrize("m,n", [(2, 2), (3, 2), (8, 6), (17, 13), (65, 65), (300, 257), (2048, 2048), (4096, 2048)])
def test_split_tick_separates_the_phases(m, n):
    """A split pass generates ticks [0, split) and then [split, ticks): every
    rotation of phase 1 and the fold (Section 3.4) must lie in the first part
    and every phase-2 rotation in the second, so that the first part's
    rotations can be applied while the second part is generated."""
    side, idx, ph, tick = bdu.plan_rotations(m, n)
    split = bdu.plan_stats(m, n)["split"]
    assert 0 < split < bdu.plan_stats(m, n)["ticks"]
    first = (ph == 1) | (ph == 3)
    assert np.all(tick[first] < split)
    assert np.all(tick[ph == 2] >= split)
    assert tick[first].max() == split - 1


def test_split_switch_validates_its_argument():
    assert bdu.lib().bdu_set_split_pass(3) == bdu.BDU_EINVAL
    assert bdu.lib().bdu_set_split_pass(-1) == bdu.BDU_EINVAL
    assert bdu.lib().bdu_set_split_pass(2) == bdu.BDU_OK


@pytest.mark.parametrize("m,n", [(2, 2), (3, 2), (8, 6), (17, 13), (65, 65), (300, 257), (1000, 999),
                                 (2048, 2048), (4096, 2048)])
def test_segments_apply_only_generated_blocks(m, n):
    """Segment k's application covers the applier blocks below bcut[k]
    (phase-1 blocks, then phase-2 blocks): every rotation of those blocks must
    have been generated before tcut[k], the tick segment k's generation stops
    at; the segments cover the pass exactly, in increasing ticks and blocks."""
    side, idx, ph, tick = bdu.plan_rotations(m, n)
    tcut, bcut, blk = bdu.plan_segments(m, n)
    st = bdu.plan_stats(m, n)
    assert len(tcut) >= 1
    assert tcut[-1] == st["ticks"] and bcut[-1] > blk.max()
    assert np.all(np.diff(tcut) > 0) and np.all(np.diff(bcut) > 0)
    rot = (ph == 1) | (ph == 2)
    assert np.all(blk[rot] >= 0) and np.all(blk[~rot] == -1)
    for k in range(len(tcut)):
        inside = rot & (blk < bcut[k])
        assert np.all(tick[inside] < tcut[k]), k
    # phase-1 blocks come before phase-2 blocks
    assert blk[ph == 1].max() < blk[ph == 2].min()
