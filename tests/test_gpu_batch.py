"""Batched generation (fused kernel + planner) against the oracle and
against the plain kernel, bit for bit.

A request is a window [start, start + count) of one stream, counted from
field 0 of the record's current step; the batch must produce exactly those
values whatever the segmentation, the lanes per segment, the order in which
waves pick up work, or whether the launch is replayed from a HIP graph.
"""
import random

import numpy as np
import pytest
import torch

import oracle as O
import paper_2106_02504_amd as rlx
from rlx_util import records_to_tensor, tensor_to_records

pytestmark = pytest.mark.gpu

DEV = "cuda"
LUX = (24, 218, 404, 794, 2048)


def make_records(ids_and_p):
    return records_to_tensor([(O.seed(i, p), 0, p) for i, p in ids_and_p])


def expected(recs, req):
    """Oracle values of every request, as one flat list per request."""
    out = []
    for r in req:
        x, pos, p = recs[int(r["state"])]
        out.append(O.window(x, p, int(r["start"]), int(r["count"])))
    return out


def small_batch(rng, n_states=12, n_req=60, max_count=3000):
    ids_p = [(i + 5, LUX[i % len(LUX)]) for i in range(n_states)]
    recs = [(O.seed(i, p), 0, p) for i, p in ids_p]
    states = [rng.randrange(n_states) for _ in range(n_req)]
    counts = [rng.choice([0, 1, 11, 12, 13, 25, rng.randrange(1, max_count)]) for _ in range(n_req)]
    starts = [rng.choice([0, 1, 5, 12, 13, rng.randrange(0, 10 ** 6), rng.getrandbits(60)]) for _ in range(n_req)]
    ps = [recs[s][2] for s in states]
    req = rlx.requests_array(states, starts, counts, ps)
    return recs, req


@pytest.mark.parametrize("lanes,seg", [(1, 5), (2, 3), (8, 7), (8, 2048), (16, 40), (64, 1), (64, 100)])
def test_batch_matches_oracle_windows(lanes, seg):
    rng = random.Random(lanes * 1000 + seg)
    recs, req = small_batch(rng)
    st = records_to_tensor(recs)
    before = st.clone()
    total = int(req["count"].sum())
    out = torch.full((total,), -1, dtype=torch.int64, device=DEV)
    plan = rlx.Plan(req, lanes=lanes, seg_blocks=seg)
    plan.generate_u64(st, out)
    got = out.cpu().numpy()
    exp = expected(recs, req)
    for k, r in enumerate(req):
        o, c = int(r["out_offset"]), int(r["count"])
        assert got[o:o + c].tolist() == exp[k], (k, int(r["start"]), c)
    assert torch.equal(st, before)          # records are only read
    assert rlx.check_errors() == 0
    info = plan.info()
    assert info["values"] == total
    plan.close()


def test_batch_f64_equals_plain_kernel():
    # each request's values equal what the plain kernel writes at those positions
    rng = random.Random(7)
    p = 2048
    n = 40
    st = make_records([(i, p) for i in range(n)])
    counts = [rng.randrange(1, 20000) for _ in range(n)]
    starts = [rng.randrange(0, 500) for _ in range(n)]
    req = rlx.requests_array(list(range(n)), starts, counts, p)
    out = torch.empty(int(req["count"].sum()), dtype=torch.float64, device=DEV)
    plan = rlx.Plan(req, lanes=8, seg_blocks=64)
    plan.generate_f64(st, out)
    for k in range(n):
        one = st[k:k + 1].clone()
        ref = rlx.generate_f64(one, starts[k] + counts[k], p)[0, starts[k]:]
        o = int(req["out_offset"][k])
        assert torch.equal(out[o:o + counts[k]], ref), k
    plan.close()


def test_one_shot_batch_helper_all_dtypes():
    # rlx.batch plans, runs and frees in one call; the three output forms
    # agree with each other and with the oracle windows
    rng = random.Random(31)
    recs, req = small_batch(rng, n_req=40, max_count=2000)
    st = records_to_tensor(recs)
    u = rlx.batch(st, req, dtype=torch.int64)
    f = rlx.batch(st, req, lanes=8, seg_blocks=64)
    h = rlx.batch(st, req, lanes=64, seg_blocks=16, dtype=torch.float32)
    total = int(req["count"].sum())
    assert u.shape == (total,) and f.shape == (total,) and h.shape == (2 * total,)
    assert torch.equal(u.to(torch.float64) * 2.0 ** -48, f)
    lo = (h[0::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
    hi = (h[1::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
    assert torch.equal(lo + (hi << 24), u)
    got = u.cpu().numpy()
    exp = expected(recs, req)
    for k in range(0, len(req), 3):
        o, c = int(req["out_offset"][k]), int(req["count"][k])
        assert got[o:o + c].tolist() == exp[k], k
    with pytest.raises(ValueError):
        rlx.batch(st, req, dtype=torch.float16)


def test_plan_update_and_graph_replays():
    rng = random.Random(11)
    p = 404
    n = 64
    st = make_records([(i, p) for i in range(n)])

    def new_requests(seed):
        r = random.Random(seed)
        counts = [r.randrange(1, 3000) for _ in range(n)]
        starts = [r.randrange(0, 10 ** 5) for _ in range(n)]
        return rlx.requests_array(list(range(n)), starts, counts, p)

    cap_vals = 64 * 3000
    out = torch.zeros(cap_vals, dtype=torch.int64, device=DEV)
    req0 = new_requests(0)
    plan = rlx.Plan(req0, lanes=8, seg_blocks=16, capacity_segments=4096)
    # capture the launch in a graph
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.generate_u64(st, out)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.generate_u64(st, out)
    recs = tensor_to_records(st)
    for rep in range(4):
        req = new_requests(100 + rep)
        plan.update(req)
        torch.cuda.synchronize()
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays
        eager = torch.zeros_like(out)
        plan.generate_u64(st, eager)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        got = out.cpu().numpy()
        for k in rng.sample(range(n), 6):
            o, c = int(req["out_offset"][k]), int(req["count"][k])
            x, _, _ = recs[k]
            assert got[o:o + c].tolist() == O.window(x, p, int(req["start"][k]), c)
    plan.close()


def test_plan_errors():
    st = make_records([(1, 24)])
    req = rlx.requests_array([0], [0], [10], 24)
    req["reserved"] = 1
    with pytest.raises(rlx.RlxError):
        rlx.Plan(req)
    req = rlx.requests_array([0] * 17, [0] * 17, [1] * 17, [24 + k for k in range(17)])
    with pytest.raises(rlx.RlxError):
        rlx.Plan(req)  # more than 16 luxury levels
    with pytest.raises(rlx.RlxError):
        rlx.Plan(rlx.requests_array([0], [0], [1], 24), lanes=3)
    # a request whose p differs from its record's p is flagged and skipped
    rlx.check_errors()
    req = rlx.requests_array([0], [0], [10], 218)
    out = torch.full((10,), -1, dtype=torch.int64, device=DEV)
    plan = rlx.Plan(req, lanes=4, seg_blocks=2)
    plan.generate_u64(st, out)
    assert rlx.check_errors() == 0x1
    assert (out.cpu().numpy() == -1).all()
    # capacity exceeded on update
    plan2 = rlx.Plan(rlx.requests_array([0], [0], [12], 24), lanes=4, seg_blocks=1, capacity_segments=2)
    with pytest.raises(rlx.RlxError):
        plan2.update(rlx.requests_array([0], [0], [1000], 24))
    # the binding refuses a launch whose requests read past the records or
    # write past `out` (the library itself cannot know those lengths)
    plan3 = rlx.Plan(rlx.requests_array([0, 1], [0, 0], [5, 5], 24), lanes=4, seg_blocks=2)
    with pytest.raises(ValueError):
        plan3.generate_u64(st, torch.empty(10, dtype=torch.int64, device=DEV))
    st2 = make_records([(1, 24), (2, 24)])
    with pytest.raises(ValueError):
        plan3.generate_u64(st2, torch.empty(9, dtype=torch.int64, device=DEV))
    out3 = plan3.generate_u64(st2, torch.empty(10, dtype=torch.int64, device=DEV))
    assert out3.cpu().tolist() == O.window(O.seed(1, 24), 24, 0, 5) + O.window(O.seed(2, 24), 24, 0, 5)
    plan.close()
    plan2.close()
    plan3.close()


def test_batch_workload_sampled():
    """8192 requests, each its own stream (id r) with p uniform over the five
    levels and log-uniform counts in [1, 2^20]"""
    import workloads
    reqs = workloads.batch_requests()
    n = len(reqs)
    st = rlx.new_states(n)
    ids_by_p = {}
    for r in reqs:
        ids_by_p.setdefault(r.p, []).append(r.stream_id)
    for p, ids in ids_by_p.items():
        idx = torch.tensor(ids, device=DEV)
        sub = rlx.new_states(len(ids))
        rlx.init_streams(sub, p, ids=torch.tensor(ids, dtype=torch.int64, device=DEV))
        st[idx] = sub
    req = rlx.requests_array([r.stream_id for r in reqs], 0, [r.count for r in reqs], [r.p for r in reqs])
    out = torch.empty(int(req["count"].sum()), dtype=torch.float64, device=DEV)
    plan = rlx.Plan(req, lanes=8, seg_blocks=2048)
    plan.generate_f64(out=out, states=st)
    torch.cuda.synchronize()
    rng = random.Random(12)
    for k in [0, n - 1] + rng.sample(range(n), 30):
        r = reqs[k]
        o, c = int(req["out_offset"][k]), r.count
        x0 = O.seed(r.stream_id, r.p)
        if c <= 3000:
            exp = O.window(x0, r.p, 0, c)
            got = (out[o:o + c] * 2.0 ** 48).to(torch.int64).cpu().numpy().tolist()
            assert got == exp, k
        else:
            for w in (0, c // 2, c - 600):
                exp = O.window(x0, r.p, w, 600)
                got = (out[o + w:o + w + 600] * 2.0 ** 48).to(torch.int64).cpu().numpy().tolist()
                assert got == exp, (k, w)
    assert bool(((out >= 0) & (out < 1)).all())
    plan.close()


def test_batch_offsets_beyond_2pow32():
    # requests written past element 2^32 of a 34 GB output, one of them
    # across the index 2^32 itself: offsets are 64-bit end to end
    p = 794
    st = make_records([(3, p), (4, p)])
    base = 1 << 32
    req = rlx.requests_array([0, 1, 0], [0, 123456, 5000], [1000, 777, 50000], p,
                             out_offset=[base - 500, base + 1000, 7])
    out = torch.full((base + 2000,), -1.0, dtype=torch.float64, device=DEV)
    plan = rlx.Plan(req, lanes=16, seg_blocks=64)
    plan.generate_f64(st, out)
    torch.cuda.synchronize()
    for (s, start, c, o) in ((0, 0, 1000, base - 500), (1, 123456, 777, base + 1000), (0, 5000, 50000, 7)):
        got = (out[o:o + c] * 2.0 ** 48).to(torch.int64).cpu().numpy().tolist()
        assert got == O.window(O.seed(3 + s, p), p, start, c), (s, o)
    assert float(out[base + 500]) == -1.0 and float(out[6]) == -1.0
    plan.close()
    del out
    torch.cuda.empty_cache()
