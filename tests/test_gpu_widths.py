"""GPU parity of the other output widths against the oracle, bit for bit:
float32 from single RANLUX numbers (rlx_generate_f32, its plan and engine
forms) and the legacy 52-bit doubles from raw LCG bits
(rlx_generate_f64_lcg52).  Every starting position, ragged counts, counts
shorter than a step, several lane counts per record, odd row offsets (rows
of 2 mod 4 floats start 8 bytes off a 16-byte boundary), bad records and
the many-streams workload at full size (sampled rows plus properties that
hold for every value)."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from oracle import widths as W
import paper_2106_02504_amd as rlx
from rlx_util import records_to_tensor, tensor_to_records

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture
def lanes_reset():
    yield
    rlx.set_lanes_per_stream(0)


def staggered(n, p, seed, npos=12):
    rng = random.Random(seed)
    return [(O.seed(rng.randrange(1 << 30), p), rng.randrange(npos), p) for _ in range(n)]


# --- float32 ---------------------------------------------------------------------

@pytest.mark.parametrize("G", (0, 1, 4, 64, 256))
@pytest.mark.parametrize("p", (24, 2048))
def test_f32_matches_oracle(p, G, lanes_reset):
    recs = staggered(41, p, 7 + G)
    rlx.set_lanes_per_stream(G)
    for count in (2, 22, 24, 26, 2 * (12 * 9 + 5)):
        st = records_to_tensor(recs)
        got = rlx.generate_f32(st, count, p).cpu().numpy().astype(np.float64)
        after = tensor_to_records(st)
        for i in range(0, 41, 4):
            x, pos, _ = recs[i]
            want, x2, pos2 = W.draws_f32(x, pos, p, count)
            assert got[i].tolist() == want, (count, i)
            assert after[i] == (x2, pos2, p)


def test_f32_equals_split_u64_and_moves_records_alike():
    p = 404
    recs = staggered(300, p, 3)
    a = records_to_tensor(recs)
    b = a.clone()
    f = rlx.generate_f32(a, 2 * 131, p)
    u = rlx.generate_u64(b, 131, p)
    assert torch.equal(a, b)
    lo = (f[:, 0::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
    hi = (f[:, 1::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
    assert torch.equal(lo + (hi << 24), u)


def test_f32_rejects_odd_counts_and_flags_bad_records():
    p = 2048
    st = records_to_tensor([(O.seed(1, p), 0, p)])
    with pytest.raises(rlx.RlxError):
        rlx.generate_f32(st, 3, p)
    bad = records_to_tensor([(5, 12, p), (O.M, 0, p), (7, 3, p)])
    rlx.check_errors()
    out = torch.full((3, 6), -1.0, dtype=torch.float32, device=DEV)
    rlx.generate_f32(bad, 6, p, out=out)
    assert rlx.check_errors() == 0x6
    o = out.cpu().numpy()
    assert (o[:2] == -1.0).all()
    assert o[2].astype(np.float64).tolist() == W.draws_f32(7, 3, p, 6)[0]


def test_f32_many_streams_workload_sampled():
    """65 536 streams (ids 0..65535), p = 2048, 8192 floats each"""
    p, n, count = 2048, 65536, 8192
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=0)
    f = rlx.generate_f32(st, count, p)
    rng = random.Random(41)
    sample = [0, 1, 255, 65535] + rng.sample(range(n), 6)
    fh = f[torch.tensor(sample, device=DEV)].cpu().numpy().astype(np.float64)
    for r, i in enumerate(sample):
        want, x2, pos2 = W.draws_f32(O.seed(i, p), 0, p, count)
        assert fh[r].tolist() == want, i
    # every value is a multiple of 2^-24 in [0, 1)
    assert bool(((f >= 0) & (f < 1)).all())
    assert bool(((f.to(torch.float64) * 2.0 ** 24).frac() == 0).all())
    recs = tensor_to_records(st[torch.tensor(sample, device=DEV)])
    for i, r in zip(sample, recs):
        assert r == O.state_at(O.seed(i, p), p, count // 2) + (p,)


def test_f32_plan_matches_u64_plan():
    p = 794
    n = 20
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=100)
    rng = random.Random(5)
    req = np.zeros(60, dtype=rlx.REQUEST_DTYPE)
    off = 0
    for k in range(60):
        c = rng.choice((1, 7, 12, 13, 250, 1000))
        req[k] = (rng.randrange(n), rng.randrange(5000), c, off, p, 0)
        off += c + rng.randrange(3)
    plan = rlx.Plan(req, lanes=8, seg_blocks=64, device=DEV)
    try:
        f = torch.full((2 * off,), -1.0, dtype=torch.float32, device=DEV)
        u = torch.full((off,), -1, dtype=torch.int64, device=DEV)
        plan.generate_f32(st, f)
        plan.generate_u64(st, u)
        with pytest.raises(ValueError):
            plan.generate_f32(st, f[:-2])
    finally:
        plan.close()
    lo = (f[0::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
    hi = (f[1::2].to(torch.float64) * 2.0 ** 24).to(torch.int64)
    written = u >= 0
    assert torch.equal((lo + (hi << 24))[written], u[written])
    assert bool((f.view(-1, 2)[~written] == -1.0).all())
    r = req[3]
    want, _, _ = W.draws_f32(*O.state_at(O.seed(100 + int(r["state"]), p), p, int(r["start"])), p, 2 * int(r["count"]))
    o = int(r["out_offset"])
    assert f[2 * o: 2 * o + 2 * int(r["count"])].cpu().numpy().astype(np.float64).tolist() == want


def test_f32_engine_equals_bulk():
    p = 2048
    recs = staggered(150, p, 12)
    a = records_to_tensor(recs)
    b = a.clone()
    got = rlx.test_engine(a, 45, p, "f32")
    bulk = rlx.generate_f32(b, 90, p)
    torch.cuda.synchronize()
    assert torch.equal(got, bulk) and torch.equal(a, b)
    want, _, _ = W.draws_f32(recs[9][0], recs[9][1], p, 90)
    assert got[9].cpu().numpy().astype(np.float64).tolist() == want


# --- legacy 52-bit doubles --------------------------------------------------------

@pytest.mark.parametrize("kind", (rlx.STEP_MFMA, rlx.STEP_VALU))
@pytest.mark.parametrize("G", (0, 1, 2, 16, 64, 1024))
def test_lcg52_matches_oracle(G, kind, lanes_reset):
    p = 218
    recs = staggered(37, p, 20 + G, npos=11)
    rlx.set_lanes_per_stream(G)
    rlx.set_step_kernel(kind)
    try:
        for count in (1, 10, 11, 12, 11 * 40 + 3):
            st = records_to_tensor(recs)
            got = rlx.generate_f64_lcg52(st, count, p).cpu().numpy()
            after = tensor_to_records(st)
            for i in range(0, 37, 3):
                x, pos, _ = recs[i]
                want, x2, pos2 = W.draws_lcg52(x, pos, p, count)
                assert got[i].tolist() == want, (count, i)
                assert after[i] == (x2, pos2, p)
    finally:
        rlx.set_step_kernel(rlx.STEP_MFMA)


def test_lcg52_flags_bad_records():
    p = 2048
    bad = records_to_tensor([(5, 11, p), (5, 12, p), (O.M, 0, p), (9, 0, 218), (7, 10, p)])
    before = bad.clone()
    rlx.check_errors()
    out = torch.full((5, 4), -1.0, dtype=torch.float64, device=DEV)
    rlx.generate_f64_lcg52(bad, 4, p, out=out)
    assert rlx.check_errors() == 0x7
    o = out.cpu().numpy()
    assert (o[:4] == -1.0).all()
    assert torch.equal(bad[:4], before[:4])
    assert o[4].tolist() == W.draws_lcg52(7, 10, p, 4)[0]


@pytest.mark.parametrize("G", (8, 32, 64))
def test_lcg52_whole_window_pair_stores(G, lanes_reset):
    # records at position 0 with 4096-value rows: whole waves of whole
    # windows on 128-byte lines take the 16-byte pair stores; an odd
    # position, rows that are not multiples of 128 bytes and a ragged count
    # take the per-value stores; every value against the oracle
    p = 2048
    rlx.set_lanes_per_stream(G)
    for pos, count in ((0, 4096), (0, 1000), (1, 4096), (0, 4096 + 11)):
        recs = [(O.seed(100 + i, p), pos, p) for i in range(24)]
        st = records_to_tensor(recs)
        got = rlx.generate_f64_lcg52(st, count, p).cpu().numpy()
        after = tensor_to_records(st)
        for i in range(24):
            want, x2, pos2 = W.draws_lcg52(recs[i][0], pos, p, count)
            assert got[i].tolist() == want, (G, pos, count, i)
            assert after[i] == (x2, pos2, p)


def test_lcg52_many_streams_workload_sampled():
    p, n, count = 2048, 65536, 4096
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=0)
    f = rlx.generate_f64_lcg52(st, count, p)
    rng = random.Random(52)
    sample = [0, 1, 65535] + rng.sample(range(n), 5)
    fh = f[torch.tensor(sample, device=DEV)].cpu().numpy()
    for r, i in enumerate(sample):
        assert fh[r].tolist() == W.draws_lcg52(O.seed(i, p), 0, p, count)[0], i
    assert bool(((f >= 0) & (f < 1)).all())
    assert bool(((f * 2.0 ** 52).frac() == 0).all())
