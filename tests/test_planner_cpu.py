"""Host logic without a GPU: the batched planner (through its dry-run entry
point) and the serving arena.  Segments must tile every request's window
exactly once, respect the segment length, keep one luxury level per work
item and come out in decreasing-cost item order."""
import random

import numpy as np
import pytest

import paper_2106_02504_amd as rlx
from paper_2106_02504_amd.serve import Arena


def check_plan(req, lanes, seg):
    segs, n_items, total = rlx.plan_dry_run(req, lanes, seg)
    assert total == int(req["count"].sum())
    covered = {}
    per_item = 64 // lanes
    for r in segs:
        state, block, jbase, lo, hi, w = (int(v) for v in r)
        jbase = jbase - (1 << 64) if jbase >= 1 << 63 else jbase
        nb, slot = w & 0xFFFFFFFF, w >> 32
        assert 1 <= nb <= seg
        for j in range(max(lo, jbase), min(hi, jbase + 12 * nb)):
            covered[j] = covered.get(j, 0) + 1
    expect = {}
    for q in req:
        for j in range(int(q["out_offset"]), int(q["out_offset"] + q["count"])):
            expect[j] = 1
    assert covered == expect           # every output index exactly once
    assert n_items >= -(-len(segs) // per_item)
    return segs, n_items


@pytest.mark.parametrize("lanes,seg", [(1, 1), (4, 3), (8, 64), (16, 2048), (64, 5)])
def test_planner_tiles_every_request_once(lanes, seg):
    rng = random.Random(lanes * 31 + seg)
    n = 40
    counts = [rng.choice([0, 1, 11, 12, 13, rng.randrange(1, 3000)]) for _ in range(n)]
    starts = [rng.choice([0, 5, 12, rng.randrange(0, 10 ** 6)]) for _ in range(n)]
    ps = [rng.choice([24, 218, 2048]) for _ in range(n)]
    req = rlx.requests_array(list(range(n)), starts, counts, ps)
    segs, _ = check_plan(req, lanes, seg)
    # block arithmetic: the first segment of a request starts at start // 12
    for k, q in enumerate(req):
        if q["count"] == 0:
            continue
        mine = [r for r in segs if int(r[0]) == k]
        assert min(int(r[1]) for r in mine) == int(q["start"]) // 12


def test_planner_errors():
    req = rlx.requests_array([0], [0], [10], 24)
    with pytest.raises(rlx.RlxError):
        rlx.plan_dry_run(req, lanes=3)
    with pytest.raises(rlx.RlxError):
        rlx.plan_dry_run(req, lanes=8, seg_blocks=0)
    bad = req.copy()
    bad["p"] = 10
    with pytest.raises(rlx.RlxError):
        rlx.plan_dry_run(bad)
    many = rlx.requests_array([0] * 17, 0, [1] * 17, [24 + k for k in range(17)])
    with pytest.raises(rlx.RlxError):
        rlx.plan_dry_run(many)
    empty = rlx.requests_array(np.zeros(0, dtype=np.uint64), 0, np.zeros(0, dtype=np.uint64), 24)
    segs, items, total = rlx.plan_dry_run(empty)
    assert segs.shape == (0, 6) and items == 0 and total == 0


def test_planner_item_order_and_levels():
    import workloads
    reqs = workloads.batch_requests(n=512)
    req = rlx.requests_array([r.stream_id for r in reqs], 0, [r.count for r in reqs], [r.p for r in reqs])
    segs, n_items = check_plan(req, 16, 512)
    # items hold one level each; costs (first = longest segment) never increase
    pos, costs = 0, []
    slots = (segs[:, 5] >> np.uint64(32)).astype(np.int64)
    nbs = (segs[:, 5] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    while pos < len(segs):
        k = 1
        while k < 4 and pos + k < len(segs) and slots[pos + k] == slots[pos] and nbs[pos + k] <= nbs[pos]:
            k += 1
        costs.append(nbs[pos])
        pos += k
    assert all(costs[i] >= costs[i + 1] for i in range(len(costs) - 1))


def test_arena_first_fit():
    a = Arena(100)
    x = a.alloc(40)
    y = a.alloc(40)
    assert (x, y) == (0, 40) and a.alloc(30) is None
    a.release(x, 40)
    assert a.alloc(30) == 0
    a.release(y, 40)
    a.release(0, 30)
    assert a.free == [(0, 100)] and a.used == 0


# --- property test: any request set, any launch shape ---------------------------

from hypothesis import given, settings, strategies as st_  # noqa: E402


@settings(max_examples=60, deadline=None)
@given(data=st_.data(),
       lanes=st_.sampled_from([1, 2, 4, 8, 16, 32, 64]),
       seg=st_.integers(min_value=1, max_value=300))
def test_planner_tiles_any_request_set(data, lanes, seg):
    n = data.draw(st_.integers(min_value=0, max_value=25))
    counts = data.draw(st_.lists(st_.integers(min_value=0, max_value=4000), min_size=n, max_size=n))
    starts = data.draw(st_.lists(st_.integers(min_value=0, max_value=(1 << 40)), min_size=n, max_size=n))
    ps = data.draw(st_.lists(st_.sampled_from([24, 25, 218, 404, 2048]), min_size=n, max_size=n))
    gaps = data.draw(st_.lists(st_.integers(min_value=0, max_value=50), min_size=n, max_size=n))
    offs, o = [], 0
    for c, g in zip(counts, gaps):          # disjoint output windows with gaps
        o += g
        offs.append(o)
        o += c
    req = rlx.requests_array(list(range(n)), starts, counts, ps, out_offset=offs)
    if n == 0:
        req = np.zeros(0, dtype=rlx.REQUEST_DTYPE)
    segs, n_items = check_plan(req, lanes, seg)
    # one luxury level per item: segments of an item are consecutive rows
    per_item = 64 // lanes
    slots = [int(r[5]) >> 32 for r in segs]
    assert len(segs) <= n_items * per_item
    for k, q in enumerate(req):
        if q["count"] == 0:
            continue
        mine = [r for r in segs if int(r[0]) == k]
        assert min(int(r[1]) for r in mine) == int(q["start"]) // 12
    assert len(set(slots)) <= len(set(ps)) if n else True
