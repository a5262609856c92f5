#!/usr/bin/env python3
"""Benchmark of the RANLUX++ generator hot path on one MI355X.

One bench step is one pass of the plain hot path over the many-streams
workload: seed 65 536 streams (ids 0..65535, luxury p = 2048) on the GPU by
exponentiation, then draw 4096 float64 uniforms per stream (2^28 doubles,
2 GiB) into a stream-major [65536, 4096] array in HBM.  The value reported is
doubles/s over whole steps.

Order of the GPU work:
  cold       the headline step from a cold start (W untimed, K timed steps,
             the first GPU work of the process): the chip's power management
             boosts, cuts the clock hard and recovers over the first ~50 ms of
             this load, and these steps fall in that swing
  legs       the other measurements below, each its own timed region
  settle     --settle untimed steps of the headline load (default 100,
             about 45 ms), so the headline does not inherit the clock the
             last leg left behind
  headline   W untimed warm-up steps, then exactly K timed steps, at the
             clock the chip holds under this load (`value`, `roofline`)

Legs (reported beside the headline in the same JSON line):
  ceilings   a plain 2 GiB device fill and a 1 GiB copy: the write and copy
             rates this GPU reaches, beside the published 8 TB/s
  rates      instruction-rate microbenchmarks (vector multiply-adds, carries,
             float64 adds, int8 matrix-core ops) against the chip's capacity
  u64        the same step writing the 48-bit integers instead of doubles
  normal     the same streams as standard normals (Box-Muller on field pairs)
  f32        the same streams writing float32, one RANLUX number each
             (8192 per stream: the same 2 GiB), checked against the doubles
  lcg52      the legacy conversion (52 raw LCG bits per double, 11 per
             step; biased, for comparison only), 4096 per stream
             (each of these four also alternates its kernel with the
             headline kernel, `same_clock`: kernel times at one clock)
  levels     the same shape with records of five luxury levels in one call
             (p = RLX_P_RECORD), in level blocks and shuffled
  single     one stream (id 1), 2^20 doubles plus the state after each step
  skip       2^20 seeded states, each skipped by a log-uniform offset in
             [1, 2^64) generator steps
  step_valu  the headline step with the vector-ALU generator step instead of
             the matrix-core one (same values)
  batch      8192 requests in one fused launch replayed from a HIP graph
  serve      the request loop: capacity, then Poisson loads relative to it
  cpu_baseline  the CPU oracle (Python integers) on a bounded sample of the
             many-streams workload, on a process pool; its values are also
             compared bit for bit with the GPU's output of the same streams.
  cpu_native the C++ CPU baseline (unsigned __int128, one thread per core of
             the box's share) on the many-streams, single-stream, skip and
             batch workloads, before any GPU work

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
(defaults K = 200, W = 100)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P = 2048
N_STREAMS = 65536
DRAWS = 4096
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
SIMDS = 256 * 4                   # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9                  # peak engine clock
VALU_WAVE_ISSUE = SIMDS * CLOCK_HZ / 4   # wave64 vector instructions per second (4 cycles each)
INT8_PEAK_OPS = 5.0e15            # dense int8 matrix-core peak, published
MFMA_OPS = 2 * 32 * 32 * 32       # operations of one v_mfma_i32_32x32x32_i8
MATRIX_OPS_PER_DOUBLE = 2 * 73 * 73 / 12   # a step's contraction: 72 input bytes + the constant
                                           # column by 73 output digits, per 12 doubles
KERNEL_SOURCES = ("paper_2106_02504_amd/csrc/rlx.hip", "include/rlx_arith.hpp",
                  "paper_2106_02504_amd/csrc/rlx_device.hpp", "include/rlx_mfma.hpp")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a pool of processes

def _oracle_chunk(args):
    lo, hi, p, count = args
    import numpy as np
    import oracle as O
    out = np.empty((hi - lo, count), dtype=np.uint64)
    for r, sid in enumerate(range(lo, hi)):
        vals, _, _ = O.draws(O.seed(sid, p), 0, p, count)
        out[r] = vals
    return lo, out


def _oracle_windows(args):
    sid, p, count, windows = args
    import oracle as O
    x0 = O.seed(sid, p)
    return [(w, O.window(x0, p, w, n)) for w, n in windows]


def batch_sample(reqs, k=24, width=512):
    """Requests of the batched workload checked against the oracle: their
    first and last `width` values."""
    import random
    rng = random.Random(44)
    idx = sorted(set([0, len(reqs) - 1] + rng.sample(range(len(reqs)), k)))
    out = []
    for i in idx:
        r = reqs[i]
        n = min(r.count, width)
        wins = [(0, n)] + ([(r.count - n, n)] if r.count > n else [])
        out.append((i, (r.stream_id, r.p, r.count, wins)))
    return out


def serve_sample(n_requests: int, k=16, width=512):
    """Requests of the serving leg's check run compared with the oracle:
    their first and last `width` values.  The server hands each request the
    next window of its stream in admission order (arrival order, index order
    for ties), and the leg serves the same request list (the same stream ids
    and counts) five times after a warm-up: three Poisson loads, the timed
    capacity run and an untimed check run with every request arriving at
    once, so every start is known in advance from the counts alone (the
    order of the middle runs -- capacity first, then the Poisson loads --
    does not change any cursor at the check run)."""
    import random
    import workloads
    warm = workloads.serve_requests(64, 1.0, seed=6)
    runs = workloads.serve_requests(n_requests, 1.0)
    cursor = {}
    for r in warm:
        cursor[r.stream_id] = cursor.get(r.stream_id, 0) + r.count
    for _ in range(4):                        # the Poisson runs and the capacity run
        for r in runs:
            cursor[r.stream_id] = cursor.get(r.stream_id, 0) + r.count
    starts = []
    for r in runs:                            # the check run
        starts.append(cursor.get(r.stream_id, 0))
        cursor[r.stream_id] = starts[-1] + r.count
    rng = random.Random(45)
    out = []
    for i in sorted(rng.sample(range(len(runs)), k)):
        r = runs[i]
        n = min(r.count, width)
        rel = [0] + ([r.count - n] if r.count > n else [])
        out.append((i, (r.stream_id, P, r.count, [(starts[i] + o, n) for o in rel])))
    return out


def oracle_checks(items, workers: int):
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_windows, [a for _, a in items])
    return {i: r for (i, _), r in zip(items, res)}


def cpu_baseline(n_streams: int, workers: int):
    import numpy as np
    chunk = max(1, n_streams // (workers * 8))
    tasks = [(lo, min(n_streams, lo + chunk), P, DRAWS) for lo in range(0, n_streams, chunk)]
    res = np.empty((n_streams, DRAWS), dtype=np.uint64)
    ctx = mp.get_context("fork")  # forked before any GPU use in this process
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        for lo, arr in pool.imap_unordered(_oracle_chunk, tasks):
            res[lo:lo + arr.shape[0]] = arr
    dt = time.perf_counter() - t0
    return res, dt


def cpu_native_leg(workers: int, ref=None, batch_reqs=None, reps: int = 5) -> dict:
    """The C++ CPU baseline (paper_2106_02504_amd.cpu: nine 64-bit words,
    unsigned __int128 products, `workers` std::threads) on the survey's
    configurations: C2 in full (65536 streams x 4096 doubles, seeding
    included), C1 block-split over the threads (one stream, 2^20 doubles),
    C3 (2^20 states seeded and skipped by log-uniform offsets) and C4 (the
    8192-request batch).  Each is the median of `reps` timed runs (steady
    clock).  Run before any GPU work; values of the first C2 streams are
    compared with the oracle's."""
    import statistics
    import numpy as np
    import workloads
    from paper_2106_02504_amd import cpu as rcpu

    def median_time(fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts), r

    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    res = {"kind": "native C++ (unsigned __int128, std::thread)", "cores": workers,
           "host": {"os_cpu_count": os.cpu_count(), "affinity": affinity}, "timing": f"median of {reps} runs"}
    dt, out = median_time(lambda: rcpu.generate(N_STREAMS, 0, DRAWS, P, nthreads=workers))
    res["many_streams"] = {"value": N_STREAMS * DRAWS / dt, "unit": "doubles/s", "seconds": dt,
                           "workload": "65536 streams (ids 0..65535) x 4096 doubles, p=2048, seeding included"}
    if ref is not None:
        got = (out[: ref.shape[0]] * 2.0 ** 48).astype(np.uint64)
        res["many_streams"]["bit_exact_vs_oracle"] = bool(np.array_equal(got, ref))
    del out
    dt, _ = median_time(lambda: rcpu.generate_split(1, 1 << 20, P, nthreads=workers))
    res["single"] = {"value": (1 << 20) / dt, "unit": "doubles/s", "seconds": dt,
                     "workload": "1 stream (id 1), 2^20 doubles, steps split over the threads by skip"}
    n3 = 1 << 20
    offs = workloads.skip_offsets(n3)
    t_seed, x = median_time(lambda: rcpu.seed(n3, 0, P, nthreads=workers))
    ts = []
    for _ in range(reps):
        y = x.copy()
        t0 = time.perf_counter()
        rcpu.skip(y, offs, P, nthreads=workers)
        ts.append(time.perf_counter() - t0)
    dt = statistics.median(ts)
    res["skip"] = {"value": n3 / dt, "unit": "states/s", "seconds": dt, "seed_seconds": t_seed,
                   "workload": "2^20 states, offsets log-uniform in [1, 2^64) steps"}
    del x, y
    if batch_reqs is not None:
        ids = [r.stream_id for r in batch_reqs]
        counts = [r.count for r in batch_reqs]
        ps = [r.p for r in batch_reqs]
        dt, (out, _) = median_time(lambda: rcpu.generate_requests(ids, [0] * len(batch_reqs), counts, ps,
                                                                   nthreads=workers))
        res["batch"] = {"value": out.shape[0] / dt, "unit": "doubles/s", "seconds": dt,
                        "workload": "8192 requests, own stream each, p over five levels, log-uniform counts"}
        del out
    return res


# ---------------------------------------------------------------------------

def sources_sha() -> str:
    """Hash of the generate kernel's sources with comments and blank space
    removed, so that only code changes invalidate the counter summary."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_counters(kernel: str) -> dict:
    """The committed rocprofv3 counter summary of `kernel` (HBM bytes, VALU
    instructions per launch), if it was taken on the current kernel sources;
    otherwise an empty dict."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        doc = json.load(open(path))
    except (OSError, ValueError):
        return {}
    ent = doc.get(kernel)
    if not ent or ent.get("sources_sha") != sources_sha():
        return {}
    return ent


def kernel_record(kind: int) -> str:
    """Name of the headline kernel's entry in profiles/traffic.json."""
    return "k_generate_f64_many_streams_" + ("mfma" if kind == 0 else "valu")


def compute_side(counters: dict, gen_ms: float, total: int, kind: int) -> dict:
    """The headline kernel against the compute units, from the committed
    counter run on the current sources (rocprofv3 SQ_INSTS_VALU,
    SQ_INSTS_MFMA): vector instructions issued against the issue capacity of
    1024 SIMDs at 2.4 GHz in the measured kernel time, and int8 matrix-core
    operations against the published dense peak, both executed and
    algorithmic (72 bytes + the constant column by 73 output digits per
    step, 12 doubles per step)."""
    out = {"note": "executed instructions per launch from profiles/traffic.json (same kernel sources); "
                   "null when those counters were taken on other sources"}
    valu = counters.get("valu_insts_per_launch")
    mfma = counters.get("mfma_insts_per_launch")
    sec = gen_ms * 1e-3
    out["valu"] = None if not valu else {
        "insts_per_launch": valu, "frac_of_issue_at_2.4GHz": round(valu / (VALU_WAVE_ISSUE * sec), 4)}
    if kind == 0:
        algo = MATRIX_OPS_PER_DOUBLE * total / sec
        out["matrix_int8"] = {"algorithmic_ops_per_s": algo, "algorithmic_frac": round(algo / INT8_PEAK_OPS, 4),
                              "peak_ops_per_s": INT8_PEAK_OPS}
        if mfma:
            ex = mfma * MFMA_OPS / sec
            out["matrix_int8"].update(executed_ops_per_s=ex, executed_frac=round(ex / INT8_PEAK_OPS, 4),
                                      mfma_insts_per_launch=mfma)
    return out


def rates_leg(rlx, torch, dev) -> dict:
    """Issue rates of the instruction kinds the kernels use (rlx_test_rates:
    independent chains, 8 waves per SIMD), against the chip's capacity at
    2.4 GHz: wave64 vector instructions per 4 cycles per SIMD, and the
    published dense int8 matrix-core peak."""
    n_threads = SIMDS * 8 * 64
    res = {"waves_per_simd": 8}
    for kind, (name, per_iter) in rlx.RATE_KINDS.items():
        iters = 1024 if kind == 3 else 4096
        out = torch.empty(n_threads, dtype=torch.int32, device=dev)
        for _ in range(2):
            rlx.test_rates(kind, iters, n_threads, out)
        torch.cuda.synchronize()
        times = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            rlx.test_rates(kind, iters, n_threads, out)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        t = sorted(times)[len(times) // 2]
        wave_insts = n_threads / 64 * per_iter * iters
        ent = {"insts_per_iteration": per_iter, "seconds": t, "wave_insts_per_s": wave_insts / t}
        if kind == 3:
            ent["ops_per_s"] = wave_insts * MFMA_OPS / t
            ent["frac_of_int8_peak"] = round(ent["ops_per_s"] / INT8_PEAK_OPS, 4)
        else:
            ent["frac_of_issue_at_2.4GHz"] = round(wave_insts / t / VALU_WAVE_ISSUE, 4)
        res[name] = ent
    return res


SETTLE_STEPS = 100   # steps of this load after which the chip's clock has settled


def device_info(torch, dev) -> dict:
    """What the runtime reports for the GPU the bench ran on (the roofline
    peaks use the published figures: 256 CUs, 2.4 GHz, 8 TB/s)."""
    pr = torch.cuda.get_device_properties(dev)
    info = {"name": pr.name, "compute_units": pr.multi_processor_count,
            "memory_gib": round(pr.total_memory / 2 ** 30, 1)}
    for attr in ("gcnArchName", "clock_rate", "L2_cache_size"):
        if hasattr(pr, attr):
            info[attr] = getattr(pr, attr)
    return info


def timed(fn, stream, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def paired_kernel_ms(torch, stream, fa, fb, reps: int = 10) -> dict:
    """Kernel durations of two launches alternated a, b, a, b, ... (HIP
    events on the launch stream), so both see the same clock: medians of
    each and their ratio."""
    import statistics
    ta, tb = [], []
    fa()
    fb()
    for _ in range(reps):
        for f, acc in ((fa, ta), (fb, tb)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            f()
            e1.record(stream)
            acc.append((e0, e1))
    torch.cuda.synchronize()
    a = statistics.median(x.elapsed_time(y) for x, y in ta)
    b = statistics.median(x.elapsed_time(y) for x, y in tb)
    return {"kernel_ms": a, "f64_kernel_ms": b, "ratio_to_f64": a / b, "reps": reps,
            "note": "kernel alternated with the headline f64 kernel on its own records (same clock)"}


def batch_leg(rlx, torch, np, dev, reqs, checks, args, plain=None):
    """8192 requests (own stream each, p uniform over 5 levels, log-uniform
    counts in [1, 2^20]) in one fused launch; lanes per segment and
    segment length from the autotuner; also replayed from a HIP graph."""
    from paper_2106_02504_amd import autotune
    n = len(reqs)
    st = rlx.new_states(n, device=dev)
    by_p = {}
    for r in reqs:
        by_p.setdefault(r.p, []).append(r.stream_id)
    for p, ids in by_p.items():
        sub = rlx.new_states(len(ids), device=dev)
        rlx.init_streams(sub, p, ids=torch.tensor(ids, dtype=torch.int64, device=dev))
        st[torch.tensor(ids, device=dev)] = sub
    req = rlx.requests_array([r.stream_id for r in reqs], 0, [r.count for r in reqs], [r.p for r in reqs])
    total = int(req["count"].sum())
    out = torch.empty(total, dtype=torch.float64, device=dev)
    if args.batch_config:
        g, sb = (int(v) for v in args.batch_config.split(":"))
        tuned = {"lanes": g, "seg_blocks": sb, "cached": None, "fixed": True}
    else:
        tuned = autotune.tune(req, st, out)
    plan = rlx.Plan(req, lanes=tuned["lanes"], seg_blocks=tuned["seg_blocks"], device=dev)
    # the same launch captured in a HIP graph (the form a serving or training
    # loop replays); direct launches and replays are timed alternately, one
    # at a time with HIP events, and the medians reported
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.generate_f64(st, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.generate_f64(st, out)
    g.replay()
    torch.cuda.synchronize()
    reps = max(20, args.steps // 4)
    direct, replay, ref = [], [], []
    seq = [(lambda: plan.generate_f64(st, out), direct), (g.replay, replay)]
    if plain is not None:
        # the plain headline kernel in the same alternation: the batch's
        # rate relative to it at the same clock
        seq.append((plain[0], ref))
    for _ in range(reps):
        for fn, acc in seq:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            acc.append(e0.elapsed_time(e1))
    ms = float(np.median(direct))
    gms = float(np.median(replay))
    exact = None
    if checks is not None:
        exact = True
        for i, wins in checks.items():
            o = int(req["out_offset"][i])
            for w, vals in wins:
                got = (out[o + w:o + w + len(vals)] * 2.0 ** 48).to(torch.int64).cpu().numpy()
                exact &= got.view(np.uint64).tolist() == vals
    info = plan.info()
    plan.close()
    same = None
    if plain is not None:
        pms = float(np.median(ref))
        same = {"plain_kernel_ms": pms, "plain_doubles_per_s": plain[1] / (pms * 1e-3),
                "fraction_of_plain": (total / (gms * 1e-3)) / (plain[1] / (pms * 1e-3)),
                "note": "the plain many-streams kernel alternated with the batch launches (same clock)"}
    return {"value": total / (gms * 1e-3), "unit": "doubles/s", "graph_replay_ms": gms, "same_clock": same,
            "direct_ms": ms, "direct_value": total / (ms * 1e-3), "reps": reps,
            "timing": "value from HIP-graph replays; direct launches and replays alternate, medians of each",
            "lanes_per_segment": tuned["lanes"], "seg_blocks": tuned["seg_blocks"],
            "draws_per_lane": 12 * tuned["seg_blocks"] // tuned["lanes"],
            "autotune": {"cached": tuned.get("cached"), "table": tuned.get("table")},
            "requests": n, "values": total, "segments": info["segments"], "items": info["items"],
            "bit_exact_sample": exact,
            "workload": "8192 requests, own stream each (id r), p uniform over {24,218,404,794,2048}, "
                        "counts floor(2^(20U)) in [1, 2^20], one fused launch"}


def serve_leg(rlx, torch, np, dev, args, checks=None):
    """Poisson arrivals of requests of log-uniform size 10^3..10^8 from a pool
    of 10^6 streams (p = 2048).  The server's capacity is measured first (the
    same requests all arriving at once); the loads are then 0.5, 0.8 and 0.95
    of that capacity divided by the mean request size."""
    import workloads
    from paper_2106_02504_amd.serve import Server
    mean_n = workloads.mean_serve_size()
    srv = Server(pool=workloads.SERVE["pool"], p=P, arena_values=1 << 31, slots=3, lanes=args.serve_lanes,
                 seg_blocks=args.serve_seg, device=dev)
    res = {"pool": workloads.SERVE["pool"], "p": P, "arena_values": 1 << 31, "slots": 3,
           "lanes_per_segment": args.serve_lanes, "seg_blocks": args.serve_seg,
           "mean_request": mean_n, "runs": []}
    # warm-up: the first launches load the kernels' code and fill the plans
    warm = workloads.serve_requests(64, 1.0, seed=6)
    srv.run([0.0] * len(warm), [r.stream_id for r in warm], [r.count for r in warm])
    # capacity: the requests all arriving at once
    reqs = workloads.serve_requests(args.serve_requests, 1.0)
    st = srv.run([0.0] * len(reqs), [r.stream_id for r in reqs], [r.count for r in reqs])
    summ = st.summary()
    cap = summ["doubles_per_s"]
    res["capacity"] = {"doubles_per_s": cap, "batches": summ["batches"], "makespan_s": summ["makespan_s"]}
    for frac in (0.5, 0.8, 0.95):
        lam = frac * cap / mean_n
        reqs = workloads.serve_requests(args.serve_requests, lam)
        st = srv.run([r.arrival_s for r in reqs], [r.stream_id for r in reqs], [r.count for r in reqs])
        summ = st.summary()
        summ.pop("starts", None)
        res["runs"].append(dict(load=frac, load_of="measured capacity", rate_per_s=lam, **summ))
    reqs = workloads.serve_requests(args.serve_requests, 1.0)
    # check run (untimed: the copies synchronise): the same load again, with
    # sampled requests compared with oracle windows computed in the CPU leg
    if checks is None:
        res["capacity"].update(bit_exact_sample=None, sample=None)
        srv.close()
        return res
    seen = {}

    def grab(i, view):
        if i in checks:
            seen[i] = [(w, (view[w - int(st0[i]):w - int(st0[i]) + len(v)] * 2.0 ** 48).to(torch.int64)
                        .cpu().numpy().view(np.uint64).tolist()) for w, v in checks[i]]

    st0 = {i: min(w for w, _ in wins) for i, wins in checks.items()}   # offset 0 starts the request
    st = srv.run([0.0] * len(reqs), [r.stream_id for r in reqs], [r.count for r in reqs], on_complete=grab)
    starts = st.summary()["starts"]
    exact = all(i in seen and all(got == want for (_, got), (_, want) in zip(seen[i], checks[i]))
                for i in checks) and all(int(starts[i]) == st0[i] for i in checks)
    res["capacity"].update(bit_exact_sample=exact,
                           sample=f"check run after the Poisson runs: first and last 512 values of {len(checks)} "
                                  f"requests against the oracle")
    srv.close()
    return res


def engine_leg(rlx, torch, dev, args):
    """The paper's GPU benchmark form (section 4.2): 1024 x 128 threads, each
    summing 10^6 doubles from its own generator, here through the device-side
    engine.  Uniform start (every stream at position 0) against staggered
    start (stream i at position i, so threads advance at different times)."""
    n = 1024 * 128
    draws = args.engine_draws
    res = {"threads": n, "draws_per_thread": draws, "p": P,
           "paper_context": "RTX 2070 SUPER: 11.8 s uniform, more than 80 s staggered (10^6 draws)"}
    for name, stagger in (("uniform", False), ("staggered", True)):
        st = rlx.new_states(n, device=dev)

        def reset():
            rlx.init_streams(st, P, id0=0)
            if stagger:
                rlx.skip_values(st, torch.arange(n, dtype=torch.int64, device=dev), P)
        reset()
        rlx.test_engine(st, 1000, P, "sum")  # warm-up
        times = []
        for _ in range(3):
            reset()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            rlx.test_engine(st, draws, P, "sum")
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        t = min(times)
        res[name] = {"seconds": t, "doubles_per_s": n * draws / t}
        del st
    res["staggered_over_uniform"] = res["staggered"]["seconds"] / res["uniform"]["seconds"]
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=SETTLE_STEPS)
    ap.add_argument("--settle", type=int, default=SETTLE_STEPS,
                    help="untimed steps of the headline load right before the headline's warm-up")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-streams", type=int, default=16384)
    ap.add_argument("--legs",
                    default="cpu_native,ceilings,rates,u64,normal,f32,lcg52,levels,single,skip,step_valu,engine,batch,serve",
                    help="extra legs to time (comma list or 'none')")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-lanes", type=int, default=64, help="lanes per segment of the server's plans")
    ap.add_argument("--serve-seg", type=int, default=8192, help="steps per segment of the server's plans")
    ap.add_argument("--engine-draws", type=int, default=10 ** 6,
                    help="draws per thread in the device-engine leg (the paper's 10^6)")
    ap.add_argument("--lanes", type=int, default=0, help="force lanes per stream (0 = library's pick)")
    ap.add_argument("--step-kernel", choices=("mfma", "valu"), default="mfma",
                    help="generator step of the headline: int8 matrix cores (default) or vector ALU")
    ap.add_argument("--batch-config", default="",
                    help="LANES:SEG_BLOCKS for the batch leg instead of autotuning (e.g. 32:4096)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU (--gpus {args.gpus} requested): the streams are independent, "
              "so several GPUs would each run this workload on their own range of stream ids with no "
              "exchange; run it with --gpus 1", file=sys.stderr)
        return 2

    import workloads
    wanted = set() if args.legs == "none" else set(args.legs.split(","))
    batch_reqs = workloads.batch_requests() if "batch" in wanted else None
    cpu = None
    checks = None
    serve_checks = None
    if not args.no_cpu:
        if batch_reqs is not None:
            checks = oracle_checks(batch_sample(batch_reqs), min(16, os.cpu_count() or 1))
        if "serve" in wanted:
            serve_checks = oracle_checks(serve_sample(args.serve_requests), min(16, os.cpu_count() or 1))
        workers = min(16, os.cpu_count() or 1)
        ref, cpu_dt = cpu_baseline(args.cpu_streams, workers)
        cpu = {"value": args.cpu_streams * DRAWS / cpu_dt, "unit": "doubles/s", "cores": workers,
               "kind": "oracle",
               "sample": f"first {args.cpu_streams} of the 65536 streams x {DRAWS} doubles, p={P} "
                         f"({args.cpu_streams * DRAWS} doubles, {cpu_dt:.1f} s wall on {workers} processes, "
                         f"about {cpu_dt * workers:.0f} CPU-seconds)"}
    cpu_native = None
    if "cpu_native" in wanted:
        cpu_native = cpu_native_leg(min(16, os.cpu_count() or 1), None if args.no_cpu else ref, batch_reqs)

    import numpy as np
    import torch
    import paper_2106_02504_amd as rlx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    kind = rlx.STEP_MFMA if args.step_kernel == "mfma" else rlx.STEP_VALU
    rlx.set_step_kernel(kind)
    rlx.prepare(P)
    rlx.set_lanes_per_stream(args.lanes)
    lanes = rlx.lanes_per_stream(N_STREAMS, DRAWS)
    st = rlx.new_states(N_STREAMS, device=dev)
    out = torch.empty((N_STREAMS, DRAWS), dtype=torch.float64, device=dev)
    total = N_STREAMS * DRAWS
    bytes_per_launch = total * 8 + N_STREAMS * 80 * 2

    def run_steps(warmup: int, steps: int) -> dict:
        """W untimed then K timed steps (seeding + generation); wall time
        per step between device synchronisations, and the two kernels' mean
        durations from HIP events on the launch stream."""
        ev, ev_init = [], []

        def step():
            i0 = torch.cuda.Event(enable_timing=True)
            i0.record(stream)
            rlx.init_streams(st, P, id0=0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rlx.generate_f64(st, DRAWS, P, out=out)
            e1.record(stream)
            ev.append((e0, e1))
            ev_init.append((i0, e0))

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev.clear()
        ev_init.clear()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        gen = [a.elapsed_time(b) for a, b in ev]
        return {"value": total / wall, "ms_per_step": wall * 1e3, "kernel_ms": float(np.mean(gen)),
                "kernel_ms_min": float(np.min(gen)), "kernel_ms_max": float(np.max(gen)),
                "init_ms": float(np.mean([a.elapsed_time(b) for a, b in ev_init])),
                "hbm_frac": bytes_per_launch / (float(np.mean(gen)) * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # cold: the same steps as the headline, as the first GPU work of the
    # process (inside the power-management swing of the first ~50 ms)
    cold = run_steps(args.warmup, args.steps)

    # bit-exact check of the sampled streams against the oracle's values
    bit_exact = None
    if cpu is not None:
        got = (out[: args.cpu_streams] * 2.0 ** 48).to(torch.int64).cpu().numpy().view(np.uint64)
        bit_exact = bool(np.array_equal(got, ref))
        cpu["bit_exact_vs_gpu"] = bit_exact

    legs = {}
    # the headline kernel on records and an output of its own, alternated
    # with each width's kernel for a same-clock comparison
    st_ref = rlx.new_states(N_STREAMS, device=dev)
    rlx.init_streams(st_ref, P, id0=0)
    out_ref = torch.empty_like(out)

    def f64_ref():
        rlx.generate_f64(st_ref, DRAWS, P, out=out_ref)

    if "ceilings" in wanted:
        # what plain device fills and copies reach on this GPU: the achievable
        # side of the published 8 TB/s (the generate kernel writes 2 GiB)
        buf = torch.empty(1 << 28, dtype=torch.float64, device=dev)      # 2 GiB
        half = buf[: 1 << 27]
        other = buf[1 << 27:]
        dt_fill = timed(lambda: buf.fill_(0.5), stream, 50, 20, torch)
        dt_copy = timed(lambda: other.copy_(half), stream, 50, 20, torch)
        legs["ceilings"] = {"fill_2GiB_gbs": (1 << 31) / dt_fill / 1e9,
                            "copy_1GiB_read_plus_write_gbs": (1 << 31) / dt_copy / 1e9}
        del buf, half, other
    if "rates" in wanted:
        legs["rates"] = rates_leg(rlx, torch, dev)
    if "u64" in wanted:
        outu = torch.empty((N_STREAMS, DRAWS), dtype=torch.int64, device=dev)

        def step_u():
            rlx.init_streams(st, P, id0=0)
            rlx.generate_u64(st, DRAWS, P, out=outu)
        dt = timed(step_u, stream, max(5, args.steps // 2), 2, torch)
        legs["u64"] = {"value": total / dt, "unit": "values/s", "ms_per_step": dt * 1e3,
                       "same_bits_as_f64": bool(torch.equal(outu.to(torch.float64) * 2.0 ** -48, out))}
        legs["u64"]["same_clock"] = paired_kernel_ms(
            torch, stream, lambda: rlx.generate_u64(st, DRAWS, P, out=outu), f64_ref)
        del outu
    if "single" in wanted:
        st1 = rlx.new_states(1, device=dev)
        out1 = torch.empty((1, 1 << 20), dtype=torch.float64, device=dev)
        tr1 = torch.zeros((1, (11 + (1 << 20)) // 12 + 1, 9), dtype=torch.int64, device=dev)
        ev1 = []

        def step_1():
            rlx.init_streams(st1, P, id0=1)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rlx.generate_f64_trace(st1, 1 << 20, P, out=out1, trace=tr1)
            e1.record(stream)
            ev1.append((e0, e1))
        dt = timed(step_1, stream, 50, 10, torch)
        torch.cuda.synchronize()
        k1 = float(np.median([a.elapsed_time(b) for a, b in ev1[-50:]]))
        ev1.clear()
        # the same stream in one lane: the latency of a generator step
        rlx.set_lanes_per_stream(1)
        dt1 = timed(step_1, stream, 1, 1, torch)
        rlx.set_lanes_per_stream(args.lanes)
        steps1 = (1 << 20) // 12 + 1
        legs["single"] = {"value": (1 << 20) / dt, "unit": "doubles/s", "ms_per_step": dt * 1e3,
                          # the generate call alone (its kernel and, for a record that
                          # spans several waves, the skip launch advancing it)
                          "call_ms": k1, "call_value": (1 << 20) / (k1 * 1e-3),
                          "lanes_per_stream": rlx.lanes_per_stream(1, 1 << 20),
                          "one_lane_ms": dt1 * 1e3, "one_lane_us_per_generator_step": dt1 * 1e6 / steps1,
                          "workload": "1 stream (id 1), p=2048, 2^20 doubles + state after each step"}
    if "skip" in wanted:
        n3 = 1 << 20
        st3 = rlx.new_states(n3, device=dev)
        offs = torch.from_numpy(workloads.skip_offsets(n3).view(np.int64)).to(dev)
        rlx.init_streams(st3, P, id0=0)

        def step_3():
            rlx.skip(st3, offs, P)
        dt = timed(step_3, stream, 10, 2, torch)
        legs["skip"] = {"value": n3 / dt, "unit": "states/s", "ms_per_step": dt * 1e3,
                        "workload": "2^20 states, offsets log-uniform in [1, 2^64) steps"}
        del st3, offs
    if "normal" in wanted:
        outn = torch.empty((N_STREAMS, DRAWS), dtype=torch.float64, device=dev)

        def step_n():
            rlx.init_streams(st, P, id0=0)
            rlx.generate_normal_f64(st, DRAWS, P, out=outn)
        dt = timed(step_n, stream, max(5, args.steps // 5), 2, torch)
        flat = outn.view(-1)
        legs["normal"] = {"value": total / dt, "unit": "normals/s", "ms_per_step": dt * 1e3,
                          "mean": float(flat.mean()), "var": float(flat.var()),
                          "workload": "many-streams shape, Box-Muller on field pairs"}
        del flat
        legs["normal"]["same_clock"] = paired_kernel_ms(
            torch, stream, lambda: rlx.generate_normal_f64(st, DRAWS, P, out=outn), f64_ref)
        del outn
    if "f32" in wanted:
        outf = torch.empty((N_STREAMS, 2 * DRAWS), dtype=torch.float32, device=dev)

        def step_f():
            rlx.init_streams(st, P, id0=0)
            rlx.generate_f32(st, 2 * DRAWS, P, out=outf)
        dt = timed(step_f, stream, max(5, args.steps // 2), 2, torch)
        # the pair of floats at position j reassembles the 48-bit value j
        lo = (outf[:, 0::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
        hi = (outf[:, 1::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
        same = bool(torch.equal(lo + (hi << 24), (out * 2.0 ** 48).to(torch.int64)))
        del lo, hi
        legs["f32"] = {"value": 2 * total / dt, "unit": "floats/s", "ms_per_step": dt * 1e3,
                       "gb_per_s": 2 * total * 4 / dt / 1e9, "pairs_equal_f64_bits": same,
                       "workload": f"many-streams shape, {2 * DRAWS} float32 per stream (24 per step)"}
        legs["f32"]["same_clock"] = paired_kernel_ms(
            torch, stream, lambda: rlx.generate_f32(st, 2 * DRAWS, P, out=outf), f64_ref)
        del outf
    if "lcg52" in wanted:
        out52 = torch.empty((N_STREAMS, DRAWS), dtype=torch.float64, device=dev)

        def step_52():
            rlx.init_streams(st, P, id0=0)
            rlx.generate_f64_lcg52(st, DRAWS, P, out=out52)
        dt = timed(step_52, stream, max(5, args.steps // 2), 2, torch)
        legs["lcg52"] = {"value": total / dt, "unit": "doubles/s", "ms_per_step": dt * 1e3,
                         "multiples_of_2^-52": bool(((out52 * 2.0 ** 52).frac() == 0).all()),
                         "workload": "many-streams shape, legacy raw-LCG doubles (11 per step)"}
        legs["lcg52"]["same_clock"] = paired_kernel_ms(
            torch, stream, lambda: rlx.generate_f64_lcg52(st, DRAWS, P, out=out52), f64_ref)
        del out52
    if "levels" in wanted:
        # records of the five batch levels in one call (p = RLX_P_RECORD):
        # the many-streams shape with the records in level blocks (waves of
        # one level) and shuffled (nearly every wave mixes levels)
        import workloads
        lv = workloads.LUXURY_LEVELS
        stl = rlx.new_states(N_STREAMS, device=dev)
        per = N_STREAMS // len(lv)
        for k, pl in enumerate(lv):
            hi = N_STREAMS if k == len(lv) - 1 else (k + 1) * per
            rlx.init_streams(stl[k * per:hi], pl, id0=k * per)
        gen = torch.Generator().manual_seed(9)
        sts = stl[torch.randperm(N_STREAMS, generator=gen).to(dev)].contiguous()
        outl = torch.empty_like(out)
        legs["levels"] = {
            "workload": f"65536 streams x {DRAWS} doubles, levels {list(lv)} in blocks of {per}, "
                        "p = RLX_P_RECORD",
            "blocks": paired_kernel_ms(torch, stream, lambda: rlx.generate_f64(stl, DRAWS, rlx.P_RECORD, out=outl),
                                       f64_ref),
            "shuffled": paired_kernel_ms(torch, stream,
                                         lambda: rlx.generate_f64(sts, DRAWS, rlx.P_RECORD, out=outl), f64_ref,
                                         reps=3)}
        for k in ("blocks", "shuffled"):
            legs["levels"][k]["doubles_per_s"] = total / (legs["levels"][k]["kernel_ms"] * 1e-3)
        del stl, sts, outl
    if "step_valu" in wanted:
        # the headline step with the other generator-step kernel (and its own
        # lane choice): same values, different instruction mix
        other = rlx.STEP_VALU if kind == rlx.STEP_MFMA else rlx.STEP_MFMA
        ref_out = out.clone()
        rlx.set_step_kernel(other)
        rlx.set_lanes_per_stream(0)
        alt = run_steps(max(5, args.warmup // 2), max(5, args.steps // 2))
        legs["step_valu" if other == rlx.STEP_VALU else "step_mfma"] = dict(
            alt, unit="doubles/s", lanes_per_stream=rlx.lanes_per_stream(N_STREAMS, DRAWS),
            same_values=bool(torch.equal(out, ref_out)))
        del ref_out
        rlx.set_step_kernel(kind)
        rlx.set_lanes_per_stream(args.lanes)
    if "engine" in wanted:
        legs["engine"] = engine_leg(rlx, torch, dev, args)

    if "batch" in wanted:
        del out
        legs["batch"] = batch_leg(rlx, torch, np, dev, batch_reqs, checks, args, plain=(f64_ref, total))
        out = torch.empty((N_STREAMS, DRAWS), dtype=torch.float64, device=dev)
    del f64_ref, st_ref, out_ref

    if "serve" in wanted:
        legs["serve"] = serve_leg(rlx, torch, np, dev, args, serve_checks)

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # settle: untimed steps of the headline load itself, so that the clock
    # the headline sees is the one the chip holds under this load rather
    # than whatever the last leg left behind; then the headline: W untimed
    # warm-up steps and exactly K timed steps
    for _ in range(args.settle):
        rlx.init_streams(st, P, id0=0)
        rlx.generate_f64(st, DRAWS, P, out=out)
    torch.cuda.synchronize()
    head = run_steps(args.warmup, args.steps)
    value = head["value"]
    gen_ms = head["kernel_ms"]

    # rates relative to the headline
    if "ceilings" in legs:
        legs["ceilings"]["generate_fraction_of_fill"] = (bytes_per_launch / (gen_ms * 1e-3) / 1e9
                                                         / legs["ceilings"]["fill_2GiB_gbs"])
    if "serve" in legs:
        legs["serve"]["capacity"]["fraction_of_plain"] = legs["serve"]["capacity"]["doubles_per_s"] / value
    if "batch" in legs:
        legs["batch"]["fraction_of_plain"] = legs["batch"]["value"] / value

    # roofline of the generation kernel: output doubles + state read/write
    achieved_gbs = bytes_per_launch / (gen_ms * 1e-3) / 1e9
    counters = measured_counters(kernel_record(kind))
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": counters.get("hbm_bytes_per_launch"),
                "kernel": f"k_generate<f64> ({args.step_kernel} step, {lanes} lanes per stream)",
                "kernel_ms": round(gen_ms, 4), "algorithmic_bytes_per_launch": bytes_per_launch,
                "traffic_note": "HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, each scaled by the "
                                "same counter on a plain device copy (profiles/traffic.json); null unless those "
                                "counters were taken on the current kernel sources"}
    # the compute side: the matrix cores' int8 operations and the vector ALU
    # issue, from the committed counter run on the same sources
    compute = compute_side(counters, gen_ms, total, kind)

    rec = {
        "metric": "doubles/sec (1 GPU, bit-exact vs oracle), plain vs batched; p99 request latency",
        "value": value,
        "unit": "doubles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "many-streams: 65536 streams seeded with ids 0..65535 by skip-ahead "
                               "seeding, p=2048, 4096 float64 per stream (2^28 doubles) stream-major in HBM",
                   "streams": N_STREAMS, "draws_per_stream": DRAWS, "p": P, "output": "float64",
                   "lanes_per_stream": lanes, "step_kernel": args.step_kernel},
        "bit_exact": bit_exact,
        "init_ms": round(head["init_ms"], 4),
        "device": device_info(torch, dev),
        "roofline": roofline,
        "compute": compute,
        "cold": dict(cold, note="the same W + K steps as the first GPU work of the process, before the legs: "
                                "inside the power-management swing of the first ~50 ms of this load"),
        "order": "cold, legs, settle, headline: the headline is timed after the legs and after "
                 f"{args.settle} untimed steps of its own load, at the clock the chip holds under it",
        "settle_steps": args.settle,
        "cpu_baseline": cpu,
        "cpu_native": cpu_native,
        "legs": legs,
        "kernel_sources_sha": sources_sha(),
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
