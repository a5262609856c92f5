"""Serving: a request loop over a device-resident pool of stream records.

Each request asks for `count` uniform doubles from stream `stream_id` of the
pool.  Records stay at their seeds on the device; the server keeps, on the
host, a cursor per stream (values already handed out).  Admission is first in
first out: a request is admitted when its output fits in the free part of an
output arena on the device, it is assigned the window
[cursor, cursor + count) of its stream and the cursor advances.  Its values
are therefore fixed by the arrival order alone -- the same whether it runs
alone or in a mix, and whatever batch it lands in.

Continuous batching: whenever one of `slots` HIP streams is idle, the
admitted-but-not-launched requests, up to `batch_values` values, form one
batch (a Plan on that slot, re-planned in place) and are launched on it; the
cap keeps a next batch ready behind a running one.  Requests that arrive while
other batches run are admitted as arena space and slots free up, and the
batches on different slots overlap on the device.  Completion is observed
with HIP events; latency is arrival -> completion of the request's batch,
on the GPU clock relative to a reference event recorded at time zero.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import Plan, init_streams, new_states, requests_array


class Arena:
    """First-fit allocator of contiguous ranges of an output buffer."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free = [(0, capacity)]  # sorted, coalesced (offset, length)
        self.used = 0

    def alloc(self, n: int):
        for k, (o, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (o + n, ln - n)
                self.used += n
                return o
        return None

    def release(self, off: int, n: int) -> None:
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


@dataclass
class _Batch:
    slot: int
    ids: np.ndarray        # request indices
    offset: int            # arena offset of the batch
    length: int            # values
    done: torch.cuda.Event
    launched_s: float


@dataclass
class ServeStats:
    latencies_ms: np.ndarray
    completion_s: np.ndarray
    values: int
    makespan_s: float
    batches: int
    max_inflight: int
    max_batch_requests: int
    arena_peak_values: int
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        # cancelled requests have no latency (NaN) and are left out
        lat = self.latencies_ms[np.isfinite(self.latencies_ms)]
        if lat.size == 0:
            lat = np.zeros(1)
        return {"requests": int(np.isfinite(self.latencies_ms).sum()), "values": int(self.values),
                "doubles_per_s": self.values / self.makespan_s if self.makespan_s > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                "makespan_s": self.makespan_s, "batches": self.batches, "max_inflight": self.max_inflight,
                "max_batch_requests": self.max_batch_requests, "arena_peak_values": self.arena_peak_values,
                **self.extra}


class Server:
    """Request loop over `pool` streams (seed ids 0..pool-1) at luxury p."""

    def __init__(self, pool: int = 1_000_000, p: int = 2048, arena_values: int = 1 << 31,
                 slots: int = 3, lanes: int = 64, seg_blocks: int = 8192, device="cuda",
                 batch_values: int | None = None):
        # lanes / seg_blocks: 64 lanes per segment of 8192 steps measured the
        # highest capacity on requests of 10^3..10^8 values (whole-wave
        # segments write the longest contiguous runs).  batch_values caps the
        # values of one batch (default: half an arena share per slot) so that
        # the next batch is planned and queued while one runs, instead of
        # waiting for a full arena to drain; a larger single request still
        # goes alone.  With 3 slots, arena/6 per batch measured the lowest
        # p99 at 0.8 load (3.2 ms against 3.5 ms at arena/3, capacity 0.89 of
        # the plain kernel either way).
        self.device = torch.device(device)
        self.batch_values = batch_values if batch_values else max(1, arena_values // (2 * slots))
        self.p = p
        self.pool = pool
        self.states = new_states(pool, device=self.device)
        init_streams(self.states, p, id0=0)
        self.arena = torch.empty(arena_values, dtype=torch.float64, device=self.device)
        self.arena_values = arena_values
        self.lanes, self.seg_blocks = lanes, seg_blocks
        self.slots = slots
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # plans sized for a full arena plus one segment per request
        cap = arena_values // (12 * seg_blocks) + 65536
        empty = requests_array(np.zeros(0, dtype=np.uint64), 0, np.zeros(0, dtype=np.uint64), p)
        self.plans = []
        for s in self.streams:
            with torch.cuda.stream(s):
                self.plans.append(Plan(empty, lanes=lanes, seg_blocks=seg_blocks, capacity_segments=cap,
                                       device=self.device))
        torch.cuda.synchronize(self.device)
        self.cursor = np.zeros(pool, dtype=np.uint64)

    def close(self):
        for pl in self.plans:
            pl.close()

    def snapshot(self) -> dict:
        """Everything that fixes the values of later requests: the level, the
        pool size and the per-stream cursors (the device records stay at
        their seeds, so they need not be saved).  Plain numbers and a numpy
        array, safe to store as raw bytes; call it between runs."""
        return {"p": self.p, "pool": self.pool, "cursor": self.cursor.copy()}

    def restore(self, snap: dict) -> None:
        """Continue from a snapshot of a server with the same level and pool:
        later requests get the values they would have had on that server."""
        if int(snap["p"]) != self.p or int(snap["pool"]) != self.pool:
            raise ValueError("snapshot of a different level or pool size")
        cur = np.asarray(snap["cursor"], dtype=np.uint64)
        if cur.shape != self.cursor.shape:
            raise ValueError("snapshot cursor array does not match the pool")
        self.cursor = cur.copy()

    def run(self, arrival_s, stream_id, count, keep_outputs: bool = False, max_batch: int = 4096,
            on_complete=None, cancel_s=None):
        """Serve the requests (arrival times in seconds from now, stream ids,
        counts), in real time.  Returns ServeStats (and, with keep_outputs,
        a list of host arrays holding each request's values).  on_complete,
        if given, is called as on_complete(request index, device view of its
        values) when its batch has finished, before the arena space is
        reused (the view is only valid during the call).  cancel_s, if
        given, holds a deadline per request (seconds from now; inf or NaN for
        none): a request still waiting for admission at its deadline is
        dropped -- it gets no values, its stream's cursor does not move, and
        its latency, start and output stay empty (NaN, 0, None).  A request
        already admitted is served."""
        arrival_s = np.asarray(arrival_s, dtype=np.float64)
        stream_id = np.asarray(stream_id, dtype=np.uint64)
        count = np.asarray(count, dtype=np.uint64)
        n = arrival_s.size
        order = np.argsort(arrival_s, kind="stable")
        if np.any(count > self.arena_values):
            raise ValueError("a request is larger than the output arena")
        start = np.zeros(n, dtype=np.uint64)
        done_ms = np.full(n, np.nan)
        outputs = [None] * n if keep_outputs else None
        arena = Arena(self.arena_values)
        waiting: deque = deque()
        inflight: list[_Batch] = []
        free_slots = deque(range(self.slots))
        nxt = 0
        batches = max_inflight = max_breq = peak = 0
        cancel = None
        if cancel_s is not None:
            cancel = np.asarray(cancel_s, dtype=np.float64).copy()
            if cancel.shape != (n,):
                raise ValueError("cancel_s needs one deadline per request")
            cancel[np.isnan(cancel)] = np.inf
        cancelled = np.zeros(n, dtype=bool)

        torch.cuda.synchronize(self.device)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.streams[0])
        ref.synchronize()
        t0 = time.perf_counter()
        while nxt < n or waiting or inflight:
            now = time.perf_counter() - t0
            # arrivals
            while nxt < n and arrival_s[order[nxt]] <= now:
                waiting.append(int(order[nxt]))
                nxt += 1
            # cancellations of requests not yet admitted
            if cancel is not None and waiting:
                keep = deque()
                for r in waiting:
                    if cancel[r] <= now:
                        cancelled[r] = True
                    else:
                        keep.append(r)
                waiting = keep
            # completions
            still = []
            for b in inflight:
                if b.done.query():
                    t_ms = ref.elapsed_time(b.done)
                    done_ms[b.ids] = t_ms
                    if keep_outputs:
                        offs = 0
                        host = self.arena[b.offset:b.offset + b.length].cpu().numpy()
                        for r in b.ids:
                            c = int(count[r])
                            outputs[r] = host[offs:offs + c].copy()
                            offs += c
                    if on_complete is not None:
                        offs = b.offset
                        for r in b.ids:
                            c = int(count[r])
                            on_complete(int(r), self.arena[offs:offs + c])
                            offs += c
                    arena.release(b.offset, b.length)
                    free_slots.append(b.slot)
                else:
                    still.append(b)
            inflight = still
            # admission + launch: FIFO while the batch fits in the arena
            if free_slots and waiting:
                ids = []
                need = 0
                while waiting and len(ids) < max_batch:
                    r = waiting[0]
                    c = int(count[r])
                    if arena.used + need + c > self.arena_values:
                        break
                    if ids and need + c > self.batch_values:
                        break
                    ids.append(r)
                    need += c
                    waiting.popleft()
                off = arena.alloc(need) if ids else None
                if ids and off is None:
                    # fragmented: put them back and wait for completions
                    for r in reversed(ids):
                        waiting.appendleft(r)
                    ids = []
                if ids:
                    ids = np.asarray(ids, dtype=np.int64)
                    sid = stream_id[ids]
                    cnt = count[ids]
                    # cursors advance in admission order (requests of one
                    # stream inside a batch take consecutive windows)
                    st = np.empty(ids.size, dtype=np.uint64)
                    for k, (s_, c_) in enumerate(zip(sid.tolist(), cnt.tolist())):
                        st[k] = self.cursor[s_]
                        self.cursor[s_] += np.uint64(c_)
                    start[ids] = st
                    outoff = np.empty(ids.size, dtype=np.uint64)
                    outoff[0] = off
                    if ids.size > 1:
                        outoff[1:] = off + np.cumsum(cnt[:-1], dtype=np.uint64)
                    req = requests_array(sid, st, cnt, self.p, outoff)
                    slot = free_slots.popleft()
                    with torch.cuda.stream(self.streams[slot]):
                        self.plans[slot].update(req)
                        self.plans[slot].generate_f64(self.states, self.arena)
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(self.streams[slot])
                    inflight.append(_Batch(slot, ids, off, need, ev, now))
                    batches += 1
                    max_breq = max(max_breq, ids.size)
                    peak = max(peak, arena.used)
                    max_inflight = max(max_inflight, len(inflight))
            elif not free_slots or (not waiting and inflight):
                time.sleep(0)  # yield; completions are polled
        torch.cuda.synchronize(self.device)
        values = int(count[~cancelled].sum())
        lat = done_ms - arrival_s * 1e3
        served = np.isfinite(done_ms)
        makespan = float(done_ms[served].max()) * 1e-3 - float(arrival_s.min()) if served.any() else 0.0
        stats = ServeStats(lat, done_ms * 1e-3, values, makespan, batches, max_inflight, max_breq, peak,
                           extra={"starts": start, "cancelled": int(cancelled.sum())})
        return (stats, outputs) if keep_outputs else stats
