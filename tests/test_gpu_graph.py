"""The plain path inside a captured HIP graph: after one eager call has built
the level's tables and the device error word, rlx_init_streams and
rlx_generate_f64 allocate, synchronise and clear nothing, so a graph that
captured them replays them.  Each replay is checked against eager runs (with
eager work and synchronisations between the replays) and against the oracle
on sampled streams."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import paper_2106_02504_amd as rlx

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                                      # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def test_graph_of_a_whole_step_replays_the_same_values():
    # seeding + generation, as one benchmark step: every replay re-seeds, so
    # every replay writes the same values
    p, n, count = 2048, 1000, 300
    st = rlx.new_states(n)
    out = torch.empty((n, count), dtype=torch.float64, device="cuda")

    def step():
        rlx.init_streams(st, p, id0=5)
        rlx.generate_f64(st, count, p, out=out)

    g = _capture(step)
    ref_st = rlx.new_states(n)
    rlx.init_streams(ref_st, p, id0=5)
    ref = rlx.generate_f64(ref_st, count, p)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        assert torch.equal(st, ref_st), rep
        junk = rlx.generate_f64(rlx.init_streams(rlx.new_states(64), p), 50, p)   # eager work between
        torch.cuda.synchronize()
        del junk
    got = out.cpu().numpy()
    for i in random.Random(3).sample(range(n), 6):
        vals, _, _ = O.draws(O.seed(5 + i, p), 0, p, count)
        assert (got[i] * 2.0 ** 48).astype(np.int64).tolist() == vals, i


def test_graph_of_generation_continues_the_streams():
    # generation alone: the records advance on every replay, so replay k
    # writes values [k count, (k + 1) count) of every stream
    p, n, count = 218, 512, 250                    # 250 = 20 steps + 10 values: positions move
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=100)
    torch.cuda.synchronize()
    out = torch.empty((n, count), dtype=torch.float64, device="cuda")
    g = _capture(lambda: rlx.generate_f64(st, count, p, out=out))   # the warm-up call is window 0
    sample = random.Random(4).sample(range(n), 5)
    seeds = {i: O.seed(100 + i, p) for i in sample}
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for i in sample:
            exp = O.window(seeds[i], p, (rep + 1) * count, count)
            assert (got[i] * 2.0 ** 48).astype(np.int64).tolist() == exp, (rep, i)
        torch.cuda.synchronize()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_capture_before_a_level_is_prepared_is_refused_then_replays_after_prepare():
    # p = 333 is used by no other test, so its tables do not exist yet: a
    # capture that would have to build them (allocate and wait on the
    # capturing stream) gets RLX_ECAPTURE and enqueues nothing; after
    # rlx_prepare the same capture replays, each replay continuing the streams
    from rlx_util import records_to_tensor
    p, n, count = 333, 300, 100
    st = records_to_tensor([(O.seed(40 + i, p), 0, p) for i in range(n)])
    out = torch.empty((n, count), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(rlx.RlxError) as err:
        with torch.cuda.graph(g):
            rlx.generate_f64(st, count, p, out=out)
    assert err.value.code == 5 and "rlx_prepare" in str(err.value)
    torch.cuda.synchronize()
    assert torch.equal(st, records_to_tensor([(O.seed(40 + i, p), 0, p) for i in range(n)]))
    rlx.prepare(p)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rlx.generate_f64(st, count, p, out=out)
    sample = random.Random(5).sample(range(n), 5)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for i in sample:
            exp = O.window(O.seed(40 + i, p), p, rep * count, count)
            assert (got[i] * 2.0 ** 48).astype(np.int64).tolist() == exp, (rep, i)
