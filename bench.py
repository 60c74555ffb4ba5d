"""Benchmark: FP64 rank-1 bidiagonal updates per second on one MI355X.

Workload (square streams, m = n = 2048, the tiny-config construction at
that size): Q0, P0 are Haar orthogonal (Householder-QR factors of N(0,1)
matrices, signed-column-permuted per stream), d ~ U(1,10), e ~ U(0,1); every
update is b ~ N(0,1)/sqrt(m), c ~ N(0,1)/sqrt(n).

- batched (the reported value): S streams in one batch (bdu_batch_*); one
  step is one rank-1 update of every stream, queued with one
  bdu_batch_update call and waited for.  value = S * steps / time.  The
  applier tiling is autotuned on S synthetic streams beforehand (untimed).
- plain: one stream, one bdu_update per rank-1 update, timed beside it, with
  the tiling autotuned on one stream.

A step runs the whole path: projection, generation, and accumulation into Q
and P.  Inputs are resident in device memory before the timed region.  The
applier (the dominant kernel) is timed live with HIP events on the stream it
runs on; its roofline figure is the FP64 vector ALU peak.  The CPU baseline
is the test oracle on a bounded sample (one rank-1 update of one stream).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 rank-1 updates/sec + p50/p99 latency, batched vs plain, n=2048"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 128 FP64 flop/clk x 2.4 GHz

# HBM bytes of one applier launch (the average over a pass's launches, one
# per segment of the pass) for the tiling the batched autotuner picks, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of this script
# (profiles/apply_staged_kernel_n2048_s64_traffic.md), each scaled by what
# the counter reads for a plain 1 GiB device copy (bench.py --copy-probe).
# Valid only for the sources with this digest and the workload named;
# otherwise the traffic is reported as null.
TRAFFIC_SOURCES = ["paper_2509_02840_amd/csrc/kernels.hip", "paper_2509_02840_amd/csrc/primitives.h",
                   "paper_2509_02840_amd/csrc/schedule.h", "paper_2509_02840_amd/csrc/device.h",
                   "paper_2509_02840_amd/csrc/plan.cpp", "paper_2509_02840_amd/csrc/bdu.cpp"]
MEASURED_TRAFFIC = {"sha256": "cef9529b2487179606c055ab0defff1f899c18220473f652ba7bd510cd4d777e", "n": 2048, "streams": 64,
                    "bytes": {(12, 15, 1): 27503370709.8, (12, 7, 1): 54759873861.9}}


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n: int, streams: int, tiling) -> float | None:
    t = MEASURED_TRAFFIC
    if (n, streams) != (t["n"], t["streams"]) or tuple(tiling) not in t["bytes"]:
        return None
    return t["bytes"][tuple(tiling)] if sources_digest() == t["sha256"] else None


class StreamFactory:
    """Seeded initial factorizations on the device.

    Q0 and P0 are Haar-distributed orthogonal matrices: the Q factors of a
    Householder QR of N(0,1) matrices (LAPACK, computed once on the host),
    each stream taking its own random signed column permutation of them.
    d ~ U(1, 10), e ~ U(0, 1) are drawn per stream."""

    def __init__(self, torch, gen, n: int, seed: int):
        from paper_2509_02840_amd import workloads as W

        rng = np.random.default_rng(seed)
        dev = torch.device("cuda:0")
        self.torch, self.gen, self.n, self.dev = torch, gen, n, dev
        self.Qb = torch.from_numpy(np.ascontiguousarray(W.orthogonal(rng, n))).to(dev)
        self.Pb = torch.from_numpy(np.ascontiguousarray(W.orthogonal(rng, n))).to(dev)

    def _signed_perm(self, B):
        torch, n = self.torch, self.n
        perm = torch.randperm(n, generator=self.gen, device=self.dev)
        sgn = torch.randint(0, 2, (n,), generator=self.gen, device=self.dev).to(torch.float64) * 2.0 - 1.0
        return (B[:, perm] * sgn).T.contiguous().T  # column-major

    def make(self):
        torch, n = self.torch, self.n
        Q = self._signed_perm(self.Qb)
        P = self._signed_perm(self.Pb)
        d = 1.0 + 9.0 * torch.rand(n, generator=self.gen, dtype=torch.float64, device=self.dev)
        e = torch.rand(n - 1, generator=self.gen, dtype=torch.float64, device=self.dev)
        return Q, d, e, P


def make_updates(torch, gen, n: int, count: int):
    dev = torch.device("cuda:0")
    b = torch.randn((count, n), generator=gen, dtype=torch.float64, device=dev) / math.sqrt(n)
    c = torch.randn((count, n), generator=gen, dtype=torch.float64, device=dev) / math.sqrt(n)
    return b, c


def applier_flops(bdu, m: int, n: int) -> float:
    """Algorithmic flops of one rank-1 accumulation: 6 per rotation per row."""
    st = bdu.plan_stats(m, n)
    return 6.0 * (m * st["left"] + n * st["right"])


def host_cpu() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_threads() -> int:
    """Threads for the all-cores leg: the CPUs this process may run on,
    capped by OMP_NUM_THREADS where it is set (a share of a shared host)."""
    usable = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(usable, int(cap))) if cap.isdigit() and int(cap) > 0 else usable


def oracle_rows_split_seconds(O, Q, d, e, P, b, c, threads: int) -> float:
    """One rank-1 update by the oracle, as it stands, split over threads:
    the projections by columns of Q and P (every entry is the oracle's own
    sequential sum), the pass by rows of Q and P (each thread regenerates
    the same rotations and applies them to its rows; the oracle's C entry
    points release the interpreter lock).  The row groups are gathered
    before the clock starts."""
    from concurrent.futures import ThreadPoolExecutor

    m, n = Q.shape[0], P.shape[0]
    gq = [g for g in np.array_split(np.arange(m), threads) if len(g)]
    gp = [g for g in np.array_split(np.arange(n), threads) if len(g)]
    Qg = [np.asfortranarray(Q[g]) for g in gq]
    Pg = [np.asfortranarray(P[g]) for g in gp] + [np.zeros((0, n), order="F")] * (len(gq) - len(gp))
    cq = [(g[0], g[-1] + 1) for g in gq]
    cp = [(g[0], g[-1] + 1) for g in gp]
    with ThreadPoolExecutor(threads) as pool:
        t0 = time.perf_counter()
        u = np.concatenate(list(pool.map(lambda s: O.project(Q[:, s[0]:s[1]], b), cq)))
        v = np.concatenate(list(pool.map(lambda s: O.project(P[:, s[0]:s[1]], c), cp)))
        list(pool.map(lambda k: O.bgu_pass_rows(m, n, Qg[k], d, e, Pg[k], u, v), range(len(gq))))
        return time.perf_counter() - t0


def cpu_baseline(Q, d, e, P, b, c, what: str, single_sample: int = 1) -> dict:
    """The oracle, as it stands, on one rank-1 update of one stream, in two
    modes: all host threads with the rows split (the reported value) and a
    single thread.  With single_sample = k > 1 the single thread runs the
    pass on the first 1/k of the rows of Q and P and is extrapolated:
    projection + generation (a pass on no rows) + k x (the sample's rows)."""
    from oracle import oracle as O

    m, n = Q.shape[0], P.shape[0]
    T = cpu_threads()
    all_s = oracle_rows_split_seconds(O, Q, d, e, P, b, c, T)
    if single_sample <= 1:
        st = O.State(Q, d, e, P)
        t0 = time.perf_counter()
        O.bgu_update(st, b, c)
        single = time.perf_counter() - t0
        how = f"the whole update, measured ({single:.1f} s)"
    else:
        k = single_sample
        Qs, Ps = np.asfortranarray(Q[: m // k]), np.asfortranarray(P[: n // k])
        none = np.zeros((0, m), order="F"), np.zeros((0, n), order="F")
        t0 = time.perf_counter()
        u, v = O.project(Q, b), O.project(P, c)
        t1 = time.perf_counter()
        O.bgu_pass_rows(m, n, none[0], d, e, none[1], u, v)
        t2 = time.perf_counter()
        O.bgu_pass_rows(m, n, Qs, d, e, Ps, u, v)
        t3 = time.perf_counter()
        gen = t2 - t1
        single = (t1 - t0) + gen + k * ((t3 - t2) - gen)
        how = (f"extrapolated from a pass on 1/{k} of the rows of Q and P ({t3 - t2:.1f} s; "
               f"projection {t1 - t0:.2f} s, generation {gen:.2f} s)")
    return {"value": 1.0 / all_s, "unit": "rank-1 updates/s", "cores": T, "kind": "oracle",
            "sample": f"one rank-1 update of {what}, rows of Q and P split over {T} threads ({all_s:.1f} s)",
            "single_thread": {"value": 1.0 / single, "unit": "rank-1 updates/s", "cores": 1,
                              "sample": f"one rank-1 update of {what}, one thread: {how}"},
            "host": host_cpu()}


def copy_probe(torch) -> int:
    """A plain device copy of known size: under the FETCH_SIZE / WRITE_SIZE
    counters it gives the factor between counted and true HBM bytes."""
    n = 1 << 27  # 2^27 doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_launch": 8 * n, "copy_probe_bytes_written_per_launch": 8 * n,
                      "launches": 3}))
    return 0


def householder_pair(torch, gen, n: int):
    """A dense orthogonal n x n matrix (I - 2 v v^T)(I - 2 w w^T), v, w random
    unit vectors, built on the GPU.  For throughput runs over many sizes: the
    update's work does not depend on the factors' values."""
    dev = torch.device("cuda:0")
    v = torch.randn(n, 1, generator=gen, dtype=torch.float64, device=dev)
    w = torch.randn(n, 1, generator=gen, dtype=torch.float64, device=dev)
    v /= v.norm()
    w /= w.norm()
    eye = torch.eye(n, dtype=torch.float64, device=dev)
    H = (eye - 2.0 * (v @ v.T)) @ (eye - 2.0 * (w @ w.T))
    return H.T.contiguous().T  # column-major


def random_stream(torch, gen, n: int):
    Q = householder_pair(torch, gen, n)
    P = householder_pair(torch, gen, n)
    d = 1.0 + 9.0 * torch.rand(n, generator=gen, dtype=torch.float64, device="cuda:0")
    e = torch.rand(n - 1, generator=gen, dtype=torch.float64, device="cuda:0")
    return Q, d, e, P


def hetero(torch, bdu, args) -> int:
    """Mixed sizes in one batch: S square streams, n = round(exp(U(ln 128, ln 2048))),
    each taking 32 rank-1 and 8 rank-4 updates in a seeded random order; a
    step updates every stream once (one batch step, max rank 4)."""
    S = args.hetero_streams
    rng = np.random.default_rng(args.seed)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(args.seed)
    sizes = [int(round(math.exp(rng.uniform(math.log(128), math.log(2048))))) for _ in range(S)]
    orders = [rng.permutation([1] * 32 + [4] * 8) for _ in range(S)]
    hs = []
    for n in sizes:
        Q, d, e, P = random_stream(torch, gen, n)
        hs.append(bdu.Handle(Q, d, e, P))
        del Q, P
    torch.cuda.empty_cache()
    nsteps = len(orders[0])
    batch = bdu.Batch(hs, max_rank=4)

    def inputs(k):
        Bs, Cs = [], []
        for n, o in zip(sizes, orders):
            r = int(o[k])
            Bs.append(torch.randn((r, n), generator=gen, dtype=torch.float64, device="cuda:0").T / math.sqrt(n))
            Cs.append(torch.randn((r, n), generator=gen, dtype=torch.float64, device="cuda:0").T / math.sqrt(n))
        return Bs, Cs, [int(o[k]) for o in orders]

    steps_in = [inputs(k) for k in range(nsteps)]  # resident before timing
    batch.update(*steps_in[0])  # warm-up step
    batch.sync()
    lat = []
    total_r1 = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, nsteps):
        Bs, Cs, rs = steps_in[k]
        ta = time.perf_counter()
        batch.update(Bs, Cs, rs)
        batch.sync()
        lat.append(time.perf_counter() - ta)
        total_r1 += sum(rs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del steps_in
    info = batch.info()
    batch.close()
    tilings = sorted({h.tiling() for h in hs})
    for h in hs:
        h.close()
    print(json.dumps({
        "metric": "FP64 rank-1-equivalent updates/sec, heterogeneous batch",
        "value": total_r1 / dt, "unit": "rank-1 updates/s", "steps": nsteps - 1,
        "ms_per_step": 1e3 * dt / (nsteps - 1), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)), "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{S} square streams, n log-uniform on [128, 2048], 32 rank-1 + 8 rank-4 "
                               "updates per stream in random order, one batch step per update",
                   "n_min": min(sizes), "n_max": max(sizes), "n_median": int(np.median(sizes)),
                   "tilings": [list(t) for t in tilings], "graph": bool(info["graph"])}}))
    return 0


def serve(torch, bdu, args) -> int:
    """Served load: R resident square streams, n uniform over {512, ..., 8192};
    requests arrive as a Poisson process, uniform over the streams, rank
    1/2/4/8 with probability 0.6/0.2/0.1/0.1, Gaussian b, c.  Requests that
    find their stream's queue full are rejected.  Two runs: one at the given
    rate (saturating at the default) during which new streams arrive as a
    Poisson process (2/s by default) and are admitted while the device-memory
    budget allows (else refused and counted), then, on the streams resident
    by then, a search for the highest sustainable rate, starting at 0.9 x the accepted
    request rate of the first run and stepping down by 0.85: a rate is
    sustainable when at most 1 % of its arrivals are rejected and its p99
    latency is not growing (the second half of the window, drain included,
    within 1.25 x the first half's p99 + 50 ms).  Each run reports accepted rank-1-equivalent updates/s (arrival window
    and drain) and the latency of its completed requests."""
    rng = np.random.default_rng(args.seed)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(args.seed)
    R = args.serve_streams
    srv = bdu.Server(budget_bytes=int(args.serve_budget_gb * 2 ** 30), queue_cap=args.serve_queue,
                     max_batch=R)
    sizes = [int(x) for x in rng.choice([int(v) for v in args.serve_sizes.split(",")], R)]
    sids = []
    for n in sizes:
        Q, d, e, P = random_stream(torch, gen, n)
        try:
            sids.append(srv.open(Q, d, e, P))
        except bdu.BduError as err:
            if err.status != bdu.BDU_ENOMEM:
                raise
            sids.append(None)
        del Q, P
    torch.cuda.empty_cache()
    live = [(sid, n) for sid, n in zip(sids, sizes) if sid is not None]
    admission = srv.stats()
    # pre-drawn update vectors per size and rank, in host memory as a client
    # would send them (the server copies its inputs)
    ranks = [1, 2, 4, 8]
    size_set = sorted(set(int(v) for v in args.serve_sizes.split(",")))
    pool = {(n, r): (np.asfortranarray(rng.standard_normal((n, r)) / math.sqrt(n)),
                     np.asfortranarray(rng.standard_normal((n, r)) / math.sqrt(n)))
            for n in size_set for r in ranks}
    torch.cuda.synchronize()

    def run(rate: float, seconds: float, halves: bool, stream_rate: float = 0.0) -> dict:
        """Poisson arrivals at `rate` for `seconds`, then a drain; new
        streams (n uniform over the sizes) arrive at `stream_rate` and are
        admitted while the budget allows.  With halves, the latency
        statistics are read at half time and again after the drain, so the
        two halves' p99 can be compared."""
        srv.reset_stats()
        submitted = busy = accepted_r1 = opened = refused = 0
        first_half = None
        t0 = time.perf_counter()
        next_t = t0
        next_s = t0 + rng.exponential(1.0 / stream_rate) if stream_rate > 0 else float("inf")
        while True:
            now = time.perf_counter()
            if now - t0 >= seconds:
                break
            if now >= next_s:
                n = int(rng.choice(size_set))
                Q, d, e, P = random_stream(torch, gen, n)
                try:
                    live.append((srv.open(Q, d, e, P), n))
                    opened += 1
                except bdu.BduError as err:
                    if err.status != bdu.BDU_ENOMEM:
                        raise
                    refused += 1
                del Q, P
                next_s += rng.exponential(1.0 / stream_rate)
                continue
            if halves and first_half is None and now - t0 >= seconds / 2:
                first_half = srv.stats()
                srv.reset_stats()
            if now < next_t:
                time.sleep(min(next_t - now, 0.01))
                continue
            next_t += rng.exponential(1.0 / rate)
            sid, n = live[rng.integers(len(live))]
            r = int(rng.choice(ranks, p=[0.6, 0.2, 0.1, 0.1]))
            B, C = pool[(n, r)]
            try:
                srv.submit(sid, B, C, detach=True)
                submitted += 1
                accepted_r1 += r
            except bdu.BduError as err:
                if err.status != bdu.BDU_EBUSY:
                    raise
                busy += 1
        t_arrivals = time.perf_counter() - t0
        srv.drain()
        t_all = time.perf_counter() - t0
        st = srv.stats()
        out = {"rate": rate, "value": accepted_r1 / t_all, "requests_per_s": submitted / t_all,
               "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"], "max_ms": st["max_ms"],
               "requests_accepted": submitted, "requests_rejected_busy": busy, "rounds": st["rounds"],
               "mean_round_size": st["batched_passes"] / max(st["rounds"], 1),
               "arrival_window_s": t_arrivals, "drain_s": t_all - t_arrivals,
               "streams_opened": opened, "streams_rejected_memory": refused, "streams_resident": st["streams"],
               "budget_bytes_in_use": st["bytes_in_use"]}
        if halves and first_half is not None:
            out["first_half_p99_ms"] = first_half["p99_ms"]
            out["first_half_p50_ms"] = first_half["p50_ms"]
            out["rounds"] += first_half["rounds"]
        print(f"serve: rate {rate:.3g}/s accepted {submitted} rejected {busy} p50 {st['p50_ms']:.1f} ms "
              f"p99 {st['p99_ms']:.1f} ms drain {t_all - t_arrivals:.2f} s", file=sys.stderr, flush=True)
        return out

    first = run(args.serve_rate, args.serve, False, args.serve_stream_rate)
    tried = []
    sustain = None
    if args.serve_search:
        # stable: at most 1 % of arrivals rejected, and the second half's
        # p99 (through the drain) within 1.25 x the first half's + 50 ms
        rate = 0.9 * first["requests_per_s"]
        for _ in range(args.serve_search):
            x = run(rate, args.serve, True)
            tried.append({k: x.get(k) for k in ("rate", "requests_accepted", "requests_rejected_busy", "drain_s",
                                                 "first_half_p99_ms", "p50_ms", "p99_ms")})
            offered = x["requests_accepted"] + x["requests_rejected_busy"]
            if ("first_half_p99_ms" in x and x["requests_rejected_busy"] <= 0.01 * max(offered, 1)
                    and x["p99_ms"] <= 1.25 * x["first_half_p99_ms"] + 50.0):
                sustain = x
                break
            rate *= 0.85
    srv.close()
    line = {
        "metric": "FP64 served rank-1-equivalent updates/sec, p50/p99 latency of completed requests",
        "value": first["value"], "unit": "rank-1 updates/s", "dtype": "f64", "data": "synthetic",
        "p50_ms": first["p50_ms"], "p99_ms": first["p99_ms"], "mean_ms": first["mean_ms"], "max_ms": first["max_ms"],
        "config": {"workload": f"{R} resident square streams, n uniform over {{{args.serve_sizes}}}, new streams "
                               f"Poisson({args.serve_stream_rate}/s) admitted under the budget, update arrivals "
                               f"Poisson {args.serve_rate}/s for {args.serve} s, ranks 1/2/4/8 w.p. .6/.2/.1/.1",
                   "streams_admitted": len(live), "streams_rejected_memory": admission["rejected_memory"],
                   "budget_gb": args.serve_budget_gb, "queue_cap": args.serve_queue,
                   "size_classes": "n <= 1024, <= 2048, <= 4096, larger"},
        "requests_accepted": first["requests_accepted"], "requests_rejected_busy": first["requests_rejected_busy"],
        "streams_opened_during_run": first["streams_opened"],
        "streams_rejected_memory_during_run": first["streams_rejected_memory"],
        "streams_resident_at_end": first["streams_resident"], "budget_bytes_in_use_at_end": first["budget_bytes_in_use"],
        "rounds": first["rounds"], "mean_round_size": first["mean_round_size"],
        "arrival_window_s": first["arrival_window_s"], "drain_included_s": first["arrival_window_s"] + first["drain_s"],
        "sustainable": sustain, "sustainable_search": tried,
    }
    print(json.dumps(line))
    return 0


def track(torch, bdu, args) -> int:
    """Subspace tracking (Section 4) on the recommendation shape: a thin
    rank-r factorization of a users x items matrix (U, V Haar-like thin
    orthonormal factors, d ~ U(1,10) descending, e ~ U(0,1)), updated with
    b ~ N(0,1)/sqrt(m), c ~ N(0,1)/sqrt(n) and truncated back to rank r after
    each update.  One update per call, each waited for (latency); inputs
    resident on the device before the timed region."""
    from paper_2509_02840_amd import workloads as W

    m, n, r = args.track_m, args.track_n, args.track_r
    U, d, e, V = W.tracking_state(m, n, r, args.seed)
    t = bdu.Tracker(U, d, e, V)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(args.seed)
    total = args.warmup + args.track_steps
    bs = torch.randn((total, m), generator=gen, dtype=torch.float64, device="cuda:0") / math.sqrt(m)
    cs = torch.randn((total, n), generator=gen, dtype=torch.float64, device="cuda:0") / math.sqrt(n)
    for k in range(args.warmup):
        t.update(bs[k], cs[k])
    t.sync()
    bdu.timing_enable(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, total):
        ta = time.perf_counter()
        t.update(bs[k], cs[k])
        t.sync()
        lat.append(time.perf_counter() - ta)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = bdu.timing_read()
    bdu.timing_enable(False)
    t.close()
    line = {
        "metric": "FP64 subspace-tracking rank-1 updates/sec + p50/p99 latency",
        "value": args.track_steps / dt, "unit": "rank-1 updates/s", "steps": args.track_steps,
        "ms_per_step": 1e3 * dt / args.track_steps, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)), "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"rank-{r} subspace tracking of a {m} x {n} users x items matrix, one rank-1 "
                               "update per call, truncated back to rank r",
                   "m": m, "n": n, "r": r},
        "middle_stage_ms_per_step": {k: v[0] / args.track_steps for k, v in stages.items()},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        bh, ch = W.tracking_update(m, n, args.seed + 1)
        c0 = time.perf_counter()
        O.track_update(U, d, e, V, bh, ch)
        cdt = time.perf_counter() - c0
        line["cpu_baseline"] = {"value": 1.0 / cdt, "unit": "rank-1 updates/s", "cores": 1, "kind": "oracle",
                                "sample": f"one tracking update at this shape, single thread ({1e3 * cdt:.0f} ms)"}
    print(json.dumps(line))
    return 0


def recsys(torch, bdu, args) -> int:
    """The recommendation-shaped stream (users x items, Section 4's rating
    experiments on synthetic data): integer ratings 1..5 at 1% density with
    Zipf(1.1) item popularity; the starting factorization A = Q Bd P^T from
    the ratings (Householder QR, then Golub-Kahan on R; host, untimed, its
    time reported).  Then calls of rank r = 1, 4, 8 in turn, each replacing
    r users' rows (b_k = e_i, c_k = new row - old row, 20 new ratings), with
    the row-mean adjustment (b = -A e / n, c = e) as every 50th call.  The
    calls are drawn, and the dense rating matrix followed, on the host
    beforehand; B and C are resident on the device before the timed region.
    One bdu_update per call, each waited for.  value = rank-1 passes per
    second over the timed calls of all three ranks."""
    from paper_2509_02840_amd import workloads as W

    m, n = args.recsys_users, args.recsys_items
    t0 = time.perf_counter()
    A = W.ratings(m, n, seed=args.seed)
    Q, d, e, P = W.bidiagonal_factors(A, seed=args.seed + 1)
    init_s = time.perf_counter() - t0
    rng = np.random.default_rng(args.seed + 2)
    dev = torch.device("cuda:0")
    ranks = [1, 4, 8]
    calls = []  # (rank label, timed, B, C) with B, C on the device
    first = None
    k_all = 0
    for r in ranks:
        for k in range(args.warmup + args.recsys_steps):
            k_all += 1
            if k_all % 50 == 0:
                B = (-(A @ np.ones(n)) / n)[:, None]
                C = np.ones((n, 1))
                A += B @ C.T
                label = "mean"
            else:
                who = rng.choice(m, r, replace=False)
                B = np.zeros((m, r))
                C = np.zeros((n, r))
                for j, i in enumerate(who):
                    B[i, j] = 1.0
                    C[:, j] = W.rating_row(rng, n, nnz=20) - A[i]
                    A[i] += C[:, j]
                label = r
            if first is None:
                first = (B[:, 0].copy(), C[:, 0].copy())
            col = lambda X: torch.from_numpy(np.ascontiguousarray(X.T)).to(dev).T  # column-major
            calls.append((label, k >= args.warmup, col(B), col(C)))
    h = bdu.Handle(Q, d, e, P)
    torch.cuda.synchronize()
    for label, timed, B, C in calls:
        if not timed:
            h.update(B, C)
    h.sync()
    bdu.timing_enable(True)
    lat = {r: [] for r in ranks + ["mean"]}
    passes = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for label, timed, B, C in calls:
        if not timed:
            continue
        ta = time.perf_counter()
        h.update(B, C)
        h.sync()
        lat[label].append(time.perf_counter() - ta)
        passes += B.shape[1]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = bdu.timing_read()
    bdu.timing_enable(False)
    h.close()
    apply_ms, apply_launches = stages["apply"]
    avg_apply_s = apply_ms / 1e3 / max(apply_launches, 1)
    flops_per_launch = passes * applier_flops(bdu, m, n) / max(apply_launches, 1)
    achieved = flops_per_launch / avg_apply_s / 1e12
    pct = lambda xs, q: 1e3 * float(np.percentile(xs, q)) if xs else None
    line = {
        "metric": "FP64 rank-1 updates/sec + p50/p99 latency, recommendation stream",
        "value": passes / dt, "unit": "rank-1 updates/s", "n_gpus": 1, "steps": len(calls) - args.warmup * 3,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / passes, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{m} users x {n} items ratings 1..5 at 1% density (Zipf 1.1 items); calls "
                               f"replacing r users' rows, r = 1, 4, 8 ({args.recsys_steps} timed calls each), "
                               "row-mean adjustment every 50th call",
                   "m": m, "n": n, "ranks": ranks, "initial_factorization_s": init_s},
        "per_rank": {str(r): {"calls": len(lat[r]), "p50_ms": pct(lat[r], 50), "p99_ms": pct(lat[r], 99),
                              "passes_per_s": (len(lat[r]) * (1 if r == "mean" else r)) / max(sum(lat[r]), 1e-30)}
                     for r in lat},
        "stage_ms_per_pass": {k: v[0] / passes for k, v in stages.items()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_launch": flops_per_launch, "avg_launch_ms": avg_apply_s * 1e3},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(Q, d, e, P, first[0], first[1], f"the {m} x {n} rating stream",
                                            single_sample=8)
    print(json.dumps(line))
    return 0


def orth(torch, bdu, args) -> int:
    """Orthogonality monitor and correction at m = n = args.n: drift
    measurement (X^T X - I on the FP64 matrix cores) and one Newton-Schulz
    step on both factors of one stream, each call waited for.  Flops per
    factor of size k (ld rows): gram 2 ld k^2 on the blocks computed (the
    upper half and the diagonal blocks, mirrored), update 2 ld k^2."""
    n = args.n
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(args.seed)
    Q, d, e, P = random_stream(torch, gen, n)
    h = bdu.Handle(Q, d, e, P)
    del Q, P
    h.orth_error()  # scratch allocation and warm-up
    h.reorthogonalize(0.0)
    k = args.orth_steps
    t0 = time.perf_counter()
    for _ in range(k):
        eq, ep = h.orth_error()
    t_mon = (time.perf_counter() - t0) / k
    t0 = time.perf_counter()
    for _ in range(k):
        h.reorthogonalize(0.0)
    h.sync()
    t_fix = (time.perf_counter() - t0) / k
    h.close()
    ld = (n + 127) // 128 * 128
    nb = (n + 63) // 64
    gram_flops = 2.0 * ld * (64 * 64) * (nb * (nb + 1) // 2)  # upper blocks incl. the diagonal
    upd_flops = 2.0 * ld * n * n
    print(json.dumps({
        "metric": "orthogonality monitor / Newton-Schulz correction, one stream, both factors",
        "n": n, "monitor_ms": 1e3 * t_mon, "correction_ms": 1e3 * t_fix, "drift_q": eq, "drift_p": ep,
        "monitor_tflops_wall": 2 * gram_flops / t_mon / 1e12,
        "correction_tflops_wall": 2 * (gram_flops + upd_flops) / t_fix / 1e12,
        "flops": {"gram_per_factor": gram_flops, "update_per_factor": upd_flops},
        "dtype": "f64", "data": "synthetic"}))
    return 0


def bhu_stream_bytes(m: int, n: int) -> float:
    """Algorithmic bytes the Householder update streams at m x n: per step k
    (0-based) the column reads Rv (j x j triangle), W (n x j), Y (m x i)
    twice and S (i x i triangle); the reflector bookkeeping reads Y (m x k)
    and S (k x k triangle); the row (k < n - 2) reads S (triangle), Y, W
    twice and Rv (triangle), W and Rv again, with i = k, j = min(k, n - 2).
    Vectors are counted too (a few per product)."""
    kl = n - 1 if m == n else n
    kr = n - 2
    tri = lambda k: k * (k + 1) / 2
    tot = 0.0
    for k in range(kl + 1):  # the last pass is the final column
        i, j = min(k, kl), min(k, kr)
        tot += tri(j) + n * j + 2 * m * i + tri(i) + 4 * (m + n)
        if k == kl:
            break
        tot += m * k + tri(k) + 2 * m
        if k < kr:
            tot += tri(k + 1) + m * (k + 1) + 2 * n * j + tri(j) + n * k + tri(k) + 4 * (m + n)
    return 8.0 * tot


def bhu(torch, bdu, args) -> int:
    """Householder bidiagonal update (Algorithm 1) of one stream at
    m = n = args.n, each update waited for, beside the Givens update of the
    same stream; the oracle's Householder update at n = 256 as the CPU
    baseline (its dense solves make larger sizes take minutes)."""
    n = args.n
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(args.seed)
    out = {}
    for size in (n, 256):
        Q, d, e, P = random_stream(torch, gen, size)
        hh = bdu.Handle(Q, d, e, P)
        hg = bdu.Handle(Q, d, e, P)
        del Q, P
        k = args.bhu_steps
        bs, cs = make_updates(torch, gen, size, k + 1)
        hh.update_householder(bs[0], cs[0])
        hh.sync()
        lat = []
        for t in range(1, k + 1):
            ta = time.perf_counter()
            hh.update_householder(bs[t], cs[t])
            hh.sync()
            lat.append(time.perf_counter() - ta)
        glat = []
        for t in range(1, k + 1):
            ta = time.perf_counter()
            hg.update(bs[t], cs[t])
            hg.sync()
            glat.append(time.perf_counter() - ta)
        hh.close()
        hg.close()
        out[size] = (float(np.median(lat)), float(np.median(glat)))
    t_bhu, t_bgu = out[n]
    byts = bhu_stream_bytes(n, n)
    line = {
        "metric": "FP64 Householder (BHU) rank-1 updates/sec, one stream",
        "value": 1.0 / t_bhu, "unit": "updates/s", "n": n, "ms_per_update": 1e3 * t_bhu,
        "givens_ms_per_update": 1e3 * t_bgu, "n256_ms_per_update": 1e3 * out[256][0],
        "roofline": {"bound": "hbm", "achieved": byts / t_bhu / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": byts / t_bhu / 1e9 / 8000.0, "traffic": None,
                     "kernel": "whole update (reflector products)", "bytes_per_update": byts},
        "dtype": "f64", "data": "synthetic", "config": {"workload": f"one stream, m = n = {n}, BHU rank-1 updates"},
    }
    if not args.no_cpu_baseline:
        sys.path.insert(0, ROOT)
        from oracle import oracle as O
        from paper_2509_02840_amd import workloads as W
        f = W.factorization(256, 256, args.seed)
        rng = np.random.default_rng(args.seed)
        b, c = rng.standard_normal(256), rng.standard_normal(256)
        t0 = time.perf_counter()
        O.bhu_update(f.Q, f.d, f.e, f.P, b, c)
        tc = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / tc, "unit": "updates/s", "cores": 1, "kind": "oracle",
                                "sample": "one oracle Householder update at m = n = 256 (compare n256_ms_per_update)"}
    print(json.dumps(line))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--streams", type=int, default=64)
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiling", type=str, default=None,
                    help="applier tiling K0,NW,RPL (default: autotuned for the batched workload)")
    ap.add_argument("--no-autotune", action="store_true", help="use the library's default tiling")
    ap.add_argument("--graph-steps", type=int, default=3,
                    help="extra batched steps replayed as a HIP graph after the timed region")
    ap.add_argument("--hetero", action="store_true",
                    help="instead: the mixed-size batch workload (prints its own JSON line)")
    ap.add_argument("--hetero-streams", type=int, default=256)
    ap.add_argument("--serve", type=float, default=0.0,
                    help="instead: serve Poisson arrivals for this many seconds (prints its own JSON line)")
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-sizes", type=str, default="512,1024,2048,4096,8192")
    ap.add_argument("--serve-rate", type=float, default=20000.0)
    ap.add_argument("--serve-queue", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-stream-rate", type=float, default=2.0,
                    help="new streams per second (Poisson) during the --serve run, admitted under the budget")
    ap.add_argument("--serve-search", type=int, default=6,
                    help="after the --serve run, at most this many lower rates tried for the sustainable one")
    ap.add_argument("--orth", action="store_true",
                    help="time the orthogonality monitor and correction at m = n = --n")
    ap.add_argument("--orth-steps", type=int, default=10)
    ap.add_argument("--bhu", action="store_true",
                    help="instead: the Householder update (Algorithm 1) beside the Givens one (prints its own JSON line)")
    ap.add_argument("--bhu-steps", type=int, default=4)
    ap.add_argument("--track", action="store_true",
                    help="subspace tracking (Section 4) instead of the full-factorization benchmark")
    ap.add_argument("--track-m", type=int, default=10000)
    ap.add_argument("--track-n", type=int, default=2000)
    ap.add_argument("--track-r", type=int, default=64)
    ap.add_argument("--track-steps", type=int, default=200)
    ap.add_argument("--recsys", action="store_true",
                    help="instead: the recommendation-shaped stream (prints its own JSON line)")
    ap.add_argument("--recsys-users", type=int, default=10000)
    ap.add_argument("--recsys-items", type=int, default=2000)
    ap.add_argument("--recsys-steps", type=int, default=100)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent streams would shard across GPUs with no communication)",
              file=sys.stderr)
        return 2

    import torch

    if args.copy_probe:
        return copy_probe(torch)
    from paper_2509_02840_amd import bdu

    torch.cuda.set_device(0)
    if args.track:
        return track(torch, bdu, args)
    if args.recsys:
        return recsys(torch, bdu, args)
    if args.orth:
        return orth(torch, bdu, args)
    if args.bhu:
        return bhu(torch, bdu, args)
    if args.hetero:
        return hetero(torch, bdu, args)
    if args.serve > 0:
        return serve(torch, bdu, args)
    n = args.n
    tune = plain_tune = None
    if args.tiling:
        bdu.set_tiling(*[int(x) for x in args.tiling.split(",")])
    elif not args.no_autotune:
        # untimed: every applier tiling on one stream (the plain leg's
        # workload: latency favours deeper pipelines per panel), then on S
        # synthetic streams of this shape (the batched leg's)
        t0 = time.perf_counter()
        plain_tune = bdu.autotune(n, n, 1)
        plain_tune["seconds"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        tune = bdu.autotune(n, n, args.streams)
        tune["seconds"] = time.perf_counter() - t0
        bdu.set_tiling_auto()
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(args.seed)

    factory = StreamFactory(torch, gen, n, args.seed)

    # ---- plain: one stream, one update per call --------------------------
    Q, d, e, P = factory.make()
    if plain_tune:
        bdu.set_tiling(plain_tune["k0"], plain_tune["nw"], plain_tune["rpl"])
    h = bdu.Handle(Q, d, e, P)
    plain_tiling = h.tiling()
    if plain_tune:
        bdu.set_tiling_auto()
    del Q, P
    pb, pc = make_updates(torch, gen, n, args.warmup + args.plain_steps)
    torch.cuda.synchronize()
    for k in range(args.warmup):
        h.update(pb[k], pc[k])
    h.sync()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.plain_steps):
        ta = time.perf_counter()
        h.update(pb[k], pc[k])
        h.sync()
        lat.append(time.perf_counter() - ta)
    torch.cuda.synchronize()
    plain_time = time.perf_counter() - t0
    plain_ups = args.plain_steps / plain_time
    h.close()
    del pb, pc

    # ---- batched: S streams, one update of every stream per step -----------
    S = args.streams
    hs = []
    for _ in range(S):
        Q, d, e, P = factory.make()
        hs.append(bdu.Handle(Q, d, e, P))
        del Q, P
    tiling = hs[0].tiling()
    torch.cuda.empty_cache()
    steps = args.warmup + args.steps
    ub = [make_updates(torch, gen, n, steps) for _ in range(S)]
    batch = bdu.Batch(hs, max_rank=1)
    step_inputs = lambda k: ([ub[s][0][k] for s in range(S)], [ub[s][1][k] for s in range(S)])
    torch.cuda.synchronize()
    for k in range(args.warmup):
        batch.update(*step_inputs(k))
    batch.sync()
    # timed region: stage events bracket every launch, so the steps run as
    # eager launches (events cannot sit between the nodes of a replayed graph)
    bdu.timing_enable(True)
    step_lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, steps):
        ta = time.perf_counter()
        batch.update(*step_inputs(k))
        batch.sync()
        step_lat.append(time.perf_counter() - ta)
    torch.cuda.synchronize()
    batched_time = time.perf_counter() - t0
    stages = bdu.timing_read()
    bdu.timing_enable(False)
    # after the timed region: the same steps replayed as a HIP graph
    graph_ms = None
    if args.graph_steps > 0:
        batch.update(*step_inputs(args.warmup))  # captures the graph
        batch.sync()
        tg = time.perf_counter()
        for j in range(args.graph_steps):
            batch.update(*step_inputs(args.warmup + j % args.steps))
        batch.sync()
        graph_ms = 1e3 * (time.perf_counter() - tg) / args.graph_steps
        assert batch.info()["graph"] == 1
    batch.close()
    for x in hs:
        x.close()

    value = S * args.steps / batched_time
    # a split pass applies phase 1 and phase 2 in two launches, each with
    # its share of the rotations (about half): flops per launch are the
    # step's divided by the launches per step
    apply_ms, apply_launches = stages["apply"]
    avg_apply_s = apply_ms / 1e3 / max(apply_launches, 1)
    launches_per_step = max(apply_launches, 1) / args.steps
    flops_per_launch = S * applier_flops(bdu, n, n) / launches_per_step
    achieved = flops_per_launch / avg_apply_s / 1e12
    k0, nw, rpl = tiling

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rank-1 updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * batched_time / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched BGU rank-1 updates, {S} square streams m=n={n}, "
                               f"one update per stream per step; plain = 1 stream",
                   "m": n, "n": n, "streams": S, "rank": 1, "tiling": [k0, nw, rpl],
                   "autotune": tune, "plain_tiling": list(plain_tiling), "plain_autotune": plain_tune},
        "plain_updates_per_s": plain_ups,
        "batched_over_plain": value / plain_ups,
        "p50_ms": 1e3 * float(np.percentile(step_lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(step_lat, 99)),
        "plain_p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "plain_p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "graph_replay_ms_per_step": graph_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(n, S, (k0, nw, rpl)),
                     "kernel": f"apply_staged_kernel<{k0}, {nw}, {rpl}>" if nw in (3, 5, 7, 15)
                     else f"apply_kernel<{k0}, {nw}, {rpl}>",
                     "flops_per_launch": flops_per_launch, "launches_per_step": launches_per_step,
                     "avg_launch_ms": avg_apply_s * 1e3},
    }
    if not args.no_cpu_baseline:
        from paper_2509_02840_amd import workloads as W

        f = W.factorization(n, n, args.seed)
        (B, C), = W.gaussian_updates(n, n, 1, args.seed + 1)
        out["cpu_baseline"] = cpu_baseline(f.Q, f.d, f.e, f.P, B[:, 0], C[:, 0], f"one {n}x{n} stream")
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
