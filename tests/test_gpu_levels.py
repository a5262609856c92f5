"""GPU parity of the calls with per-record luxury levels (p = RLX_P_RECORD):
records of several levels in one generate or skip call, each against the
oracle at its own level, in waves that share one level (the matrix-core
step) and in waves that mix levels (lane-by-lane generic multiplication),
plus records of a level that was never prepared (flagged, untouched)."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from oracle import gauss as G
from oracle import widths as Wd
import paper_2106_02504_amd as rlx
from rlx_util import records_to_tensor, tensor_to_records

pytestmark = pytest.mark.gpu

LEVELS = (24, 218, 404, 794, 2048)


@pytest.fixture(scope="module", autouse=True)
def prepared():
    for p in LEVELS:
        rlx.prepare(p)
    yield
    rlx.set_lanes_per_stream(0)
    rlx.check_errors()


def records(n, seed, levels=LEVELS, sort=False, npos=12):
    rng = random.Random(seed)
    recs = [(O.seed(rng.randrange(1 << 30), p), rng.randrange(npos), p)
            for p in (rng.choice(levels) for _ in range(n))]
    if sort:
        recs.sort(key=lambda r: r[2])
    return recs


@pytest.mark.parametrize("sort", (False, True))
@pytest.mark.parametrize("G", (0, 1, 8, 32, 64, 256))
def test_generate_f64_each_record_at_its_level(G, sort):
    # unsorted: nearly every wave mixes levels; sorted: most waves share one
    # (G = 256 is capped at 64 lanes per record)
    rlx.set_lanes_per_stream(G)
    recs = records(150, 7 + G, sort=sort)
    for count in (1, 13, 500):
        st = records_to_tensor(recs)
        got = (rlx.generate_f64(st, count, rlx.P_RECORD) * 2.0 ** 48).to(torch.int64).cpu().numpy()
        after = tensor_to_records(st)
        for i in range(0, 150, 7):
            x, pos, p = recs[i]
            want, x2, pos2 = O.draws(x, pos, p, count)
            assert got[i].tolist() == want, (G, sort, count, i, p)
            assert after[i] == (x2, pos2, p)
    assert rlx.check_errors() == 0


@pytest.mark.parametrize("G", (16, 32, 64))
def test_alternating_levels_per_half_wave(G):
    # records alternate between two levels: at G = 32 each half-wave is one
    # record, so every wave runs the step with a different multiplier per
    # half; at G = 64 a wave is one record; at G = 16 a half-wave holds two
    # records of different levels (the lane-by-lane path)
    rlx.set_lanes_per_stream(G)
    recs = [(O.seed(500 + i, (24, 2048)[i % 2]), (5 * i) % 12, (24, 2048)[i % 2]) for i in range(40)]
    st = records_to_tensor(recs)
    count = 1000
    got = (rlx.generate_f64(st, count, rlx.P_RECORD) * 2.0 ** 48).to(torch.int64).cpu().numpy()
    after = tensor_to_records(st)
    for i in range(40):
        x, pos, p = recs[i]
        want, x2, pos2 = O.draws(x, pos, p, count)
        assert got[i].tolist() == want, (G, i, p)
        assert after[i] == (x2, pos2, p)
    assert rlx.check_errors() == 0


def test_uniform_waves_many_streams_shape():
    # 4096 streams in five level blocks of 819 (waves of one level at G = 32,
    # but for the one straddling each block boundary), 4096
    # values: the matrix-core path; every 97th row against the oracle
    rlx.set_lanes_per_stream(0)
    n, count = 4096, 4096
    st = rlx.new_states(n)
    per = n // len(LEVELS)
    bounds = [k * per for k in range(len(LEVELS))] + [n]
    for k, p in enumerate(LEVELS):
        rlx.init_streams(st[bounds[k]:bounds[k + 1]], p, id0=bounds[k])
    got = rlx.generate_u64(st, count, rlx.P_RECORD).cpu().numpy()
    for i in range(0, n, 97):
        p = LEVELS[min(i // per, len(LEVELS) - 1)]
        assert got[i].tolist() == O.draws(O.seed(i, p), 0, p, count)[0], (i, p)
    assert rlx.check_errors() == 0


def test_other_widths_at_record_levels():
    recs = records(40, 11)
    st_a, st_b, st_c = (records_to_tensor(recs) for _ in range(3))
    f = rlx.generate_f32(st_a, 2 * 50, rlx.P_RECORD).cpu().numpy()
    z = rlx.generate_normal_f64(st_b, 50, rlx.P_RECORD).cpu().numpy()
    u = rlx.generate_u64(st_c, 50, rlx.P_RECORD).cpu().numpy()
    for i in range(0, 40, 3):
        x, pos, p = recs[i]
        assert f[i].astype(np.float64).tolist() == Wd.draws_f32(x, pos, p, 100)[0], i
        want = np.array(G.normals(x, pos, p, 50)[0])
        assert np.all(np.abs(z[i] - want) <= 2.0 ** -49 * np.abs(want) + 2.0 ** -70), i
        assert u[i].tolist() == O.draws(x, pos, p, 50)[0], i
    assert tensor_to_records(st_a) == tensor_to_records(st_b) == tensor_to_records(st_c)


def test_unprepared_level_is_flagged_and_left_alone():
    rlx.check_errors()
    recs = records(20, 13)
    recs[5] = (O.seed(3, 777), 0, 777)     # a level no call has prepared
    st = records_to_tensor(recs)
    out = torch.full((20, 30), -1.0, dtype=torch.float64, device="cuda")
    rlx.generate_f64(st, 30, rlx.P_RECORD, out=out)
    err = rlx.check_errors()
    assert err & 0x1
    o = out.cpu().numpy()
    assert (o[5] == -1.0).all()
    after = tensor_to_records(st)
    assert after[5] == recs[5]
    for i in (0, 4, 6, 19):
        x, pos, p = recs[i]
        assert ((o[i] * 2.0 ** 48).astype(np.int64)).tolist() == O.draws(x, pos, p, 30)[0]


def test_skip_each_record_at_its_level():
    rng = random.Random(17)
    recs = records(300, 19)
    ks = [rng.randrange(1 << rng.randrange(1, 64)) for _ in recs]
    st = records_to_tensor(recs)
    steps = torch.tensor(np.array(ks, dtype=np.uint64).view(np.int64), device="cuda")
    rlx.skip(st, steps, rlx.P_RECORD)
    after = tensor_to_records(st)
    for i in range(0, 300, 11):
        x, pos, p = recs[i]
        assert after[i] == (O.skip(x, ks[i], p), pos, p), i
    # by values, the same records
    st2 = records_to_tensor(recs)
    rlx.skip_values(st2, 1000, rlx.P_RECORD)
    after2 = tensor_to_records(st2)
    for i in range(0, 300, 13):
        x, pos, p = recs[i]
        want_x, want_pos = O.state_at(x, p, pos + 1000)
        assert after2[i] == (want_x, want_pos, p), i
    assert rlx.check_errors() == 0
