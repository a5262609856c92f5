"""GPU parity of the device-side engine (include/rlx_engine.h), driven by a
kernel written as user code (rlx_test_engine, one thread per record).

Every value is compared bit for bit with the oracle, and with the library's
bulk entry points on the same records (the two interfaces must agree
exactly, including the normals, which use the same device functions on the
same exact arguments).  Records written back are compared exactly.  Staggered
starting positions (record i at position i mod 12) exercise the lazy,
wave-synchronised advance.
"""
import random

import numpy as np
import pytest
import torch

import oracle as O
from oracle import gauss as G
import paper_2106_02504_amd as rlx
from rlx_util import records_to_tensor, tensor_to_records, u64_list

pytestmark = pytest.mark.gpu


def staggered_records(n, p, seed):
    rng = random.Random(seed)
    return [(O.seed(rng.randrange(1 << 30), p), i % 12, p) for i in range(n)]


@pytest.mark.parametrize("p", (24, 2048))
def test_engine_draws_match_oracle_and_bulk(p):
    recs = staggered_records(300, p, p)
    count = 107
    a = records_to_tensor(recs)
    b = a.clone()
    got = rlx.test_engine(a, count, p, "f64")
    bulk = rlx.generate_f64(b, count, p)
    torch.cuda.synchronize()
    assert torch.equal(got, bulk)
    assert torch.equal(a, b)
    got = got.cpu().numpy()
    after = tensor_to_records(a)
    for i in (0, 1, 11, 12, 150, 299):
        x, pos, _ = recs[i]
        want, x2, pos2 = O.draws_f64(x, pos, p, count)
        assert got[i].tolist() == want, i
        assert after[i] == (x2, pos2, p)


def test_engine_u48_matches_bulk():
    p = 218
    recs = staggered_records(130, p, 5)
    a = records_to_tensor(recs)
    b = a.clone()
    got = rlx.test_engine(a, 61, p, "u48")
    bulk = rlx.generate_u64(b, 61, p)
    torch.cuda.synchronize()
    assert torch.equal(got, bulk) and torch.equal(a, b)
    vals, _, _ = O.draws(recs[7][0], recs[7][1], p, 61)
    assert u64_list(got[7]) == vals


def test_engine_seed_equals_init_streams():
    p = 404
    n = 200
    a = rlx.new_states(n)
    got = rlx.test_engine(a, 13, p, "seed")
    b = rlx.new_states(n)
    rlx.init_streams(b, p, id0=0)
    bulk = rlx.generate_f64(b, 13, p)
    torch.cuda.synchronize()
    assert torch.equal(got, bulk) and torch.equal(a, b)
    for i in (0, 1, 77, 199):
        want, _, _ = O.draws_f64(O.seed(i, p), 0, p, 13)
        assert got[i].cpu().tolist() == want


def test_engine_skip_equals_skip_then_draw():
    # record i skips i generator steps, then draws; staggered positions are
    # kept by the skip
    p = 794
    recs = staggered_records(140, p, 8)
    a = records_to_tensor(recs)
    got = rlx.test_engine(a, 30, p, "skip").cpu().numpy()
    after = tensor_to_records(a)
    for i in (0, 1, 13, 139):
        x, pos, _ = recs[i]
        want, x2, pos2 = O.draws_f64(O.skip(x, i, p), pos, p, 30)
        assert got[i].tolist() == want
        assert after[i] == (x2, pos2, p)


def test_engine_normals_equal_bulk_normals():
    p = 2048
    recs = staggered_records(100, p, 9)
    a = records_to_tensor(recs)
    b = a.clone()
    got = rlx.test_engine(a, 50, p, "normal")
    bulk = rlx.generate_normal_f64(b, 50, p)
    torch.cuda.synchronize()
    assert torch.equal(got, bulk) and torch.equal(a, b)
    want, _, _ = G.normals(recs[3][0], recs[3][1], p, 50)
    err = np.abs(got[3].cpu().numpy() - np.asarray(want))
    assert np.all(err <= 2.0 ** -49 * np.abs(want) + 2.0 ** -70)


def test_engine_divergent_calls():
    # lanes draw in bursts of 1..3 values under per-lane branches: the lazy
    # wave-synchronised advance must still give every lane its own sequence
    p = 2048
    recs = staggered_records(200, p, 11)
    a = records_to_tensor(recs)
    b = a.clone()
    got = rlx.test_engine(a, 77, p, "divergent")
    bulk = rlx.generate_f64(b, 77, p)
    torch.cuda.synchronize()
    assert torch.equal(got, bulk) and torch.equal(a, b)
    for i in (0, 1, 2, 65, 199):
        want, _, _ = O.draws_f64(recs[i][0], recs[i][1], p, 77)
        assert got[i].cpu().tolist() == want


def test_engine_sum_in_draw_order():
    # the paper's GPU benchmark form: each thread sums its draws in order
    p = 2048
    recs = staggered_records(70, p, 10)
    a = records_to_tensor(recs)
    b = a.clone()
    sums = rlx.test_engine(a, 500, p, "sum").cpu().numpy()
    vals = rlx.generate_f64(b, 500, p).cpu().numpy()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for i in range(70):
        s = 0.0
        for v in vals[i]:
            s += float(v)
        assert sums[i] == s


def test_engine_rejects_bad_records_and_args():
    p = 2048
    recs = [(O.seed(1, p), 3, p), (O.M, 0, p), (O.seed(2, p), 12, p)]
    a = records_to_tensor(recs)
    before = a.clone()
    out = rlx.test_engine(a, 5, p, "f64")
    torch.cuda.synchronize()
    # the bad records (x = m, pos = 12) are left alone by the kernel
    assert torch.equal(a[1:], before[1:])
    assert out[0].cpu().tolist() == O.draws_f64(O.seed(1, p), 3, p, 5)[0]
    with pytest.raises(rlx.RlxError):
        rlx.test_engine(a, 5, 23, "f64")
    t = rlx.get_tables(p)
    assert t.windows and t.folded and t.windows16 and t.p == p
