"""Serving loop: every request's values are the same alone and in the mix.

The loop assigns each request the next window of its stream in arrival
order; whatever batches, slots and overlaps the run produces, request k must
hold exactly the values of that window (checked against a one-request plan
run alone, and against the oracle on a sample).  Admission never lets the
admitted outputs exceed the arena.
"""
import random

import numpy as np
import pytest
import torch

import oracle as O
import paper_2106_02504_amd as rlx
from paper_2106_02504_amd.serve import Server

pytestmark = pytest.mark.gpu


def fifo_starts(stream_id, count, arrival):
    order = np.argsort(arrival, kind="stable")
    cur = {}
    start = np.zeros(len(count), dtype=np.uint64)
    for r in order:
        s = int(stream_id[r])
        start[r] = cur.get(s, 0)
        cur[s] = cur.get(s, 0) + int(count[r])
    return start


@pytest.mark.parametrize("slots,arena", [(1, 1 << 18), (3, 1 << 16), (4, 1 << 22)])
def test_serve_results_equal_alone(slots, arena):
    rng = np.random.default_rng(slots)
    n = 300
    p = 218
    pool = 64
    arrival = np.cumsum(rng.exponential(1.0 / 20000.0, size=n))
    stream_id = rng.integers(0, pool, size=n).astype(np.uint64)
    count = np.floor(10.0 ** (1 + 3.5 * rng.random(n))).astype(np.uint64)
    srv = Server(pool=pool, p=p, arena_values=arena, slots=slots, lanes=8, seg_blocks=64)
    stats, outs = srv.run(arrival, stream_id, count, keep_outputs=True)
    start = fifo_starts(stream_id, count, arrival)
    assert np.array_equal(stats.extra["starts"], start)
    assert stats.arena_peak_values <= arena
    assert np.isfinite(stats.latencies_ms).all() and (stats.latencies_ms >= -1.0).all()
    # alone: each request as a one-request plan over the same records
    st = srv.states
    for k in range(n):
        req = rlx.requests_array([int(stream_id[k])], [int(start[k])], [int(count[k])], p)
        out = torch.empty(int(count[k]), dtype=torch.float64, device=st.device)
        plan = rlx.Plan(req, lanes=4, seg_blocks=16)
        plan.generate_f64(st, out)
        assert np.array_equal(outs[k], out.cpu().numpy()), k
        plan.close()
    # oracle on a sample
    for k in random.Random(slots).sample(range(n), 12):
        x0 = O.seed(int(stream_id[k]), p)
        exp = O.window(x0, p, int(start[k]), int(count[k]))
        assert (outs[k] * 2.0 ** 48).astype(np.int64).tolist() == exp
    srv.close()


@pytest.mark.parametrize("batch_values", (1, 5000, 1 << 30))
def test_serve_batch_cap_does_not_change_values(batch_values):
    # the cap on a batch's values only changes how requests are grouped:
    # with one request per batch (cap 1), small batches, or no cap, every
    # request still gets its window of its stream
    rng = np.random.default_rng(7)
    n, p, pool = 120, 404, 16
    arrival = np.zeros(n)                      # all at once: admission order = index
    stream_id = rng.integers(0, pool, size=n).astype(np.uint64)
    count = np.floor(10.0 ** (1 + 3 * rng.random(n))).astype(np.uint64)
    srv = Server(pool=pool, p=p, arena_values=1 << 20, slots=3, lanes=16, seg_blocks=32,
                 batch_values=batch_values)
    stats, outs = srv.run(arrival, stream_id, count, keep_outputs=True)
    start = fifo_starts(stream_id, count, arrival)
    assert np.array_equal(stats.extra["starts"], start)
    if batch_values == 1:
        assert stats.batches == n
    for k in random.Random(batch_values).sample(range(n), 10):
        exp = O.window(O.seed(int(stream_id[k]), p), p, int(start[k]), int(count[k]))
        assert (outs[k] * 2.0 ** 48).astype(np.int64).tolist() == exp, k
    srv.close()


def test_serve_full_size_sampled():
    """The serving workload at its real size: a pool of 10^6 streams at
    p = 2048, request sizes floor(10^(3 + 5 U)) (up to 10^8 values), Poisson
    arrivals; 150 requests.  Requests of at most 10^5 values are checked
    whole against the oracle, larger ones on their first, last and eight
    random windows of 1024 values; every request's start is its stream's
    cursor in arrival order."""
    import workloads
    reqs = workloads.serve_requests(150, 20000.0, seed=11)
    arrival = np.array([r.arrival_s for r in reqs])
    stream_id = np.array([r.stream_id for r in reqs], dtype=np.uint64)
    count = np.array([r.count for r in reqs], dtype=np.uint64)
    p = 2048
    srv = Server(pool=workloads.SERVE["pool"], p=p, arena_values=1 << 30, slots=3, lanes=64, seg_blocks=8192)
    rng = random.Random(12)
    got = {}

    def check(r, view):
        c = int(count[r])
        if c <= 100_000:
            got[r] = [(0, view.cpu().numpy())]
        else:
            w = 1024
            offs = [0, c - w] + [rng.randrange(c - w) for _ in range(8)]
            got[r] = [(o, view[o:o + w].cpu().numpy()) for o in offs]

    stats = srv.run(arrival, stream_id, count, on_complete=check)
    start = fifo_starts(stream_id, count, arrival)
    assert np.array_equal(stats.extra["starts"], start)
    assert sorted(got) == list(range(len(reqs)))
    assert int(count.max()) > 10 ** 7                     # the large end of the size range is present
    checked = 0
    for r in range(len(reqs)):
        x0 = O.seed(int(stream_id[r]), p)
        for o, vals in got[r]:
            exp = O.window(x0, p, int(start[r]) + o, len(vals))
            assert (vals * 2.0 ** 48).astype(np.int64).tolist() == exp, (r, o)
            checked += len(vals)
    assert checked > 10 ** 5
    srv.close()


def test_serve_zero_size_and_oversize_requests():
    # zero-value requests are served (empty output, cursor unchanged) in the
    # mix; a request larger than the arena is refused before anything runs
    n, p, pool = 40, 24, 4
    stream_id = np.array([k % pool for k in range(n)], dtype=np.uint64)
    count = np.array([0 if k % 5 == 0 else 100 + 37 * k for k in range(n)], dtype=np.uint64)
    arrival = np.zeros(n)
    srv = Server(pool=pool, p=p, arena_values=1 << 14, slots=2, lanes=8, seg_blocks=16)
    with pytest.raises(ValueError):
        srv.run([0.0], [0], [(1 << 14) + 1])
    assert int(srv.cursor.sum()) == 0             # the refused request moved nothing
    stats, outs = srv.run(arrival, stream_id, count, keep_outputs=True)
    start = fifo_starts(stream_id, count, arrival)
    assert np.array_equal(stats.extra["starts"], start)
    assert np.isfinite(stats.latencies_ms).all()
    for k in range(n):
        assert outs[k].size == int(count[k])
        if count[k]:
            exp = O.window(O.seed(int(stream_id[k]), p), p, int(start[k]), int(count[k]))
            assert (outs[k] * 2.0 ** 48).astype(np.int64).tolist() == exp, k
    # a batch made only of zero-value requests completes too
    stats = srv.run(np.zeros(3), [1, 2, 3], [0, 0, 0])
    assert stats.batches >= 1 and np.isfinite(stats.latencies_ms).all()
    srv.close()


def test_serve_snapshot_restore_continues_the_streams():
    # a server stopped after some requests and restored in a new server
    # (cursors saved as raw bytes) hands out the same windows as one server
    # that serves every request
    rng = np.random.default_rng(21)
    n, p, pool = 80, 794, 8
    stream_id = rng.integers(0, pool, size=n).astype(np.uint64)
    count = np.floor(10.0 ** (1 + 3 * rng.random(n))).astype(np.uint64)
    arrival = np.zeros(n)
    one = Server(pool=pool, p=p, arena_values=1 << 18, slots=2, lanes=8, seg_blocks=32)
    _, ref = one.run(arrival, stream_id, count, keep_outputs=True)
    one.close()
    a = Server(pool=pool, p=p, arena_values=1 << 18, slots=2, lanes=8, seg_blocks=32)
    _, first = a.run(arrival[:30], stream_id[:30], count[:30], keep_outputs=True)
    snap = a.snapshot()
    raw = snap["cursor"].tobytes()
    a.close()
    b = Server(pool=pool, p=p, arena_values=1 << 18, slots=3, lanes=16, seg_blocks=64)
    b.restore({"p": p, "pool": pool, "cursor": np.frombuffer(raw, dtype=np.uint64)})
    _, rest = b.run(arrival[30:], stream_id[30:], count[30:], keep_outputs=True)
    for k in range(n):
        got = first[k] if k < 30 else rest[k - 30]
        assert np.array_equal(got, ref[k]), k
    with pytest.raises(ValueError):
        b.restore({"p": 24, "pool": pool, "cursor": snap["cursor"]})
    b.close()


def test_serve_cancelled_requests_take_no_values():
    # requests cancelled before admission get nothing and move no cursor:
    # the others get exactly the windows they would get without them
    rng = np.random.default_rng(31)
    n, p, pool = 60, 218, 6
    stream_id = rng.integers(0, pool, size=n).astype(np.uint64)
    count = np.floor(10.0 ** (1 + 3 * rng.random(n))).astype(np.uint64)
    arrival = np.zeros(n)
    cancel = np.full(n, np.nan)
    cancel[::4] = 0.0                              # due before the first admission
    cancel[1::8] = 1e9                             # far in the future: served
    srv = Server(pool=pool, p=p, arena_values=1 << 16, slots=2, lanes=8, seg_blocks=32)
    stats, outs = srv.run(arrival, stream_id, count, keep_outputs=True, cancel_s=cancel)
    gone = np.zeros(n, dtype=bool)
    gone[::4] = True
    assert stats.extra["cancelled"] == int(gone.sum())
    assert np.isnan(stats.latencies_ms[gone]).all() and np.isfinite(stats.latencies_ms[~gone]).all()
    assert stats.values == int(count[~gone].sum())
    kept = np.flatnonzero(~gone)
    start = fifo_starts(stream_id[kept], count[kept], arrival[kept])
    assert np.array_equal(stats.extra["starts"][kept], start)
    assert int(srv.cursor.sum()) == int(count[kept].sum())
    for j, k in enumerate(kept):
        exp = O.window(O.seed(int(stream_id[k]), p), p, int(start[j]), int(count[k]))
        assert (outs[k] * 2.0 ** 48).astype(np.int64).tolist() == exp, k
    assert all(outs[k] is None for k in np.flatnonzero(gone))
    summ = stats.summary()
    assert summ["requests"] == kept.size and np.isfinite(summ["p99_ms"])
    srv.close()
