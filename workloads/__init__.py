"""Seeded synthetic workloads for the RANLUX++ hot path.

These generators only draw the *inputs* (stream ids, skip offsets, request
sizes, luxury levels, arrival times) from numpy's PCG64 with fixed seeds.  They
hold none of the generator's arithmetic, so both the CPU oracle (in tests) and
the GPU library consume the same inputs without sharing any computation.

Workloads (the paper measures on no dataset; all inputs are synthetic):

* ``single``   one stream, id 1, p = 2048, 2^20 draws (plus the state after
                every generator step).
* ``many``     65 536 streams with ids 0..65535, p = 2048, 4096 draws each.
* ``skip``     2^20 streams, ids 0..2^20-1, each advanced by an offset drawn
                log-uniform in [1, 2^64) generator steps.
* ``batch``    8192 requests, p uniform over {24, 218, 404, 794, 2048}, draw
                counts log-uniform in [1, 2^20].
* ``serve``    Poisson arrivals of requests of log-uniform size 10^3..10^8
                against a pool of 10^6 streams at p = 2048.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LUXURY_LEVELS = (24, 218, 404, 794, 2048)

SINGLE = dict(stream_id=1, p=2048, draws=1 << 20)
MANY = dict(n_streams=65536, p=2048, draws=4096)
SKIP = dict(n_streams=1 << 20, p=2048)
BATCH = dict(n_requests=8192, max_draws=1 << 20)
SERVE = dict(pool=1_000_000, p=2048, min_exp=3, max_exp=8)


def skip_offsets(n: int, seed: int = 3) -> np.ndarray:
    """Per-stream skip offsets, log-uniform in [1, 2^64): bit length L uniform
    in {1..64}, then k uniform in [2^(L-1), 2^L).  Returned as uint64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(1, 65, size=n, dtype=np.int64)
    # k = 2^(L-1) + uniform integer in [0, 2^(L-1)): 64 random bits, masked
    r = rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)
    out = np.empty(n, dtype=np.uint64)
    for L in range(1, 65):
        sel = bits == L
        if not sel.any():
            continue
        top = np.uint64(1) << np.uint64(L - 1)
        mask = top - np.uint64(1)
        out[sel] = top | (r[sel] & mask)
    return out


@dataclass
class BatchRequest:
    stream_id: int      # the request's own stream (seeded with this id)
    p: int              # luxury level
    count: int          # number of doubles


def batch_requests(n: int = BATCH["n_requests"], max_draws: int = BATCH["max_draws"],
                   seed: int = 4) -> list[BatchRequest]:
    """Request r: p uniform over LUXURY_LEVELS, count = floor(2^(20 U))
    clamped to [1, max_draws], stream id r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ps = rng.integers(0, len(LUXURY_LEVELS), size=n)
    u = rng.random(n)
    lg = int(np.log2(max_draws))
    counts = np.clip(np.floor(np.exp2(lg * u)).astype(np.int64), 1, max_draws)
    return [BatchRequest(r, LUXURY_LEVELS[int(ps[r])], int(counts[r])) for r in range(n)]


@dataclass
class ServeRequest:
    arrival_s: float    # arrival time, seconds from the start
    stream_id: int      # which pool stream the numbers come from
    count: int          # number of doubles


def serve_requests(n: int, rate_per_s: float, pool: int = SERVE["pool"],
                   min_exp: float = SERVE["min_exp"], max_exp: float = SERVE["max_exp"],
                   seed: int = 5) -> list[ServeRequest]:
    """Poisson arrivals (exponential gaps at `rate_per_s`), size
    floor(10^(min_exp + (max_exp - min_exp) U)), stream uniform in the pool."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    u = rng.random(n)
    sizes = np.floor(10.0 ** (min_exp + (max_exp - min_exp) * u)).astype(np.int64)
    ids = rng.integers(0, pool, size=n)
    return [ServeRequest(float(t[i]), int(ids[i]), int(sizes[i])) for i in range(n)]


def mean_serve_size(min_exp: float = SERVE["min_exp"], max_exp: float = SERVE["max_exp"]) -> float:
    """E[10^(min + (max-min) U)] = (10^max - 10^min) / ((max - min) ln 10)."""
    return (10.0 ** max_exp - 10.0 ** min_exp) / ((max_exp - min_exp) * np.log(10.0))
