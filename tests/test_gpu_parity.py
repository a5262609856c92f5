"""GPU parity: every kernel of librlx.so against the CPU oracle, bit for bit.

Sizes are chosen so that the oracle finishes in seconds while the launches
still span several 256-lane blocks with a ragged last block; edge cases
(empty calls, counts shorter than a step, every starting position, crafted
operands for the rare branches) are included.
"""
import random

import numpy as np
import pytest
import torch

import oracle as O
import paper_2106_02504_amd as rlx
from rlx_util import (ints_to_words, records_to_tensor, tensor_to_records, u64_list,
                      words_to_ints)

pytestmark = pytest.mark.gpu

DEV = "cuda"
LUX = (24, 218, 404, 794, 2048)


def dev_words(values):
    return torch.from_numpy(ints_to_words(values)).to(DEV)


def host_ints(t):
    return words_to_ints(t.cpu().numpy())


# --- generic arithmetic (test-only exports) -----------------------------------

def crafted_operands(rng):
    m = O.M
    pairs = [(2 ** 288 + 1, 2 ** 288 - 1), (m - 1, m - 1), (2 ** 300, 2 ** 276), (0, rng.randrange(m)),
             (1, rng.randrange(m)), (2 ** 576 - 1, 2 ** 576 - 1), (m, m), (m + 5, 2 ** 576 - 2),
             (2 ** 575, 2), (2 ** 240, 2 ** 336)]
    # products landing on chosen residues: y = t * x^-1 mod m
    for t in (0, 1, m - 1, m - 2, 2 ** 240 - 2, 2 ** 336 - 1, 2 ** 336, 2 ** 576 - 2 ** 240 - 1, 2 ** 544):
        x = rng.randrange(1, m)
        pairs.append((x, t * pow(x, -1, m) % m))
    # all-ones words
    ones = sum(0xFFFFFFFF << (32 * k) for k in range(0, 18, 2))
    pairs.append((ones, ones))
    return pairs


def test_mulmod_random_and_crafted():
    rng = random.Random(101)
    pairs = crafted_operands(rng)
    pairs += [(rng.getrandbits(576), rng.getrandbits(576)) for _ in range(3000)]
    pairs += [(rng.randrange(O.M), rng.randrange(O.M)) for _ in range(1000)]
    x = dev_words([a for a, _ in pairs])
    y = dev_words([b for _, b in pairs])
    got = host_ints(rlx.test_mulmod(x, y))
    for (a, b), g in zip(pairs, got):
        assert g == a * b % O.M, (hex(a), hex(b))


def test_pow_matches_oracle():
    rng = random.Random(102)
    bases = [O.A, 2, O.M - 1, 1, 0] + [rng.randrange(O.M) for _ in range(300)]
    exps = [0, 1, 2, 2 ** 96, 2 ** 192 - 1] + [rng.getrandbits(rng.randrange(1, 193)) for _ in range(300)]
    b = dev_words(bases)
    e = torch.from_numpy(ints_to_words(exps, 3)).to(DEV)
    got = host_ints(rlx.test_pow(b, e))
    for base, ex, g in zip(bases, exps, got):
        assert g == pow(base, ex, O.M)


def crafted_states(rng, n_random):
    m = O.M
    xs = [0, 1, 2, m - 1, m - 2, 2 ** 336 - 1, 2 ** 336, 2 ** 336 + 1, 2 ** 240 - 1, 2 ** 240,
          2 ** 576 - 2 ** 240, (m - 1) // 2, 2 ** 575, m - 2 ** 240]

    def setw(x, k, v):
        return (x & ~(0xFFFFFFFF << (32 * k))) | (v << (32 * k))

    for _ in range(200):
        x = rng.randrange(m)
        xs.append(setw(x, 17, (x >> 304) & 0xFFFFFFFF))                       # equal top words
        xs.append(setw(setw(setw(x, 7, 0xFFFFFFFF), 8, 0xFFFFFFFF), 9, 0xFFFFFFFF))  # long carry
        xs.append(setw(x, 0, (-((x >> 336) & 0xFFFFFFFF)) & 0xFFFFFFFF))         # D' word 0 = 0
        xs.append(setw(setw(x, 17, 0xFFFFFFFE), 16, 0xFFFFFFFF))
    xs = [x for x in xs if x < m]
    xs += [rng.randrange(m) for _ in range(n_random)]
    return xs


def test_to_ranlux_random_and_crafted():
    rng = random.Random(103)
    xs = crafted_states(rng, 3000)
    d, carry = rlx.test_to_ranlux(dev_words(xs))
    dg = host_ints(d)
    cg = carry.cpu().numpy().tolist()
    for x, dd, cc in zip(xs, dg, cg):
        nums, c = O.to_ranlux(x)
        assert dd == O.RANLUX.pack(nums), hex(x)
        assert cc == c


# --- seeding and skipping -----------------------------------------------------

@pytest.mark.parametrize("p", LUX)
def test_init_streams_id_range(p):
    n = 700  # three blocks, ragged
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=0)
    got = tensor_to_records(st)
    for i in range(0, n, 7 if p != 2048 else 1):
        assert got[i] == (O.seed(i, p), 0, p), i


def test_init_streams_id_list_and_offsets():
    rng = random.Random(104)
    ids = [0, 1, 2 ** 64 - 1, 2 ** 63, 12345678901234567] + [rng.getrandbits(64) for _ in range(300)]
    st = rlx.new_states(len(ids))
    idt = torch.from_numpy(np.array(ids, dtype=np.uint64).view(np.int64)).to(DEV)
    rlx.init_streams(st, 2048, ids=idt)
    got = tensor_to_records(st)
    for i, sid in enumerate(ids):
        assert got[i] == (O.seed(sid, 2048), 0, 2048)
    st2 = rlx.new_states(10)
    rlx.init_streams(st2, 218, id0=2 ** 64 - 10)
    assert tensor_to_records(st2)[9] == (O.seed(2 ** 64 - 1, 218), 0, 218)


@pytest.mark.parametrize("p", (24, 2048))
def test_skip_per_stream_offsets(p):
    rng = random.Random(105 + p)
    n = 600
    ks = [0, 1, 15, 16, 255, 256, 2 ** 64 - 1, 2 ** 63] + [rng.getrandbits(rng.randrange(1, 65)) for _ in range(n - 8)]
    recs = [(rng.randrange(O.M), rng.randrange(12), p) for _ in range(n)]
    st = records_to_tensor(recs)
    kt = torch.from_numpy(np.array(ks, dtype=np.uint64).view(np.int64)).to(DEV)
    rlx.skip(st, kt, p)
    got = tensor_to_records(st)
    for (x, pos, _), k, g in zip(recs, ks, got):
        assert g == (O.skip(x, k, p), pos, p)
    # one offset for all
    rlx.skip(st, 5, p)
    got2 = tensor_to_records(st)
    for g, g2 in zip(got, got2):
        assert g2 == (O.skip(g[0], 5, p), g[1], p)
    assert rlx.check_errors() == 0


# --- generation -----------------------------------------------------------------

def oracle_draws(recs, count):
    outs, finals = [], []
    for x, pos, p in recs:
        v, x2, pos2 = O.draws(x, pos, p, count)
        outs.append(v)
        finals.append((x2, pos2, p))
    return outs, finals


@pytest.mark.parametrize("p", LUX)
@pytest.mark.parametrize("count", (1, 11, 12, 13, 100, 257))
def test_generate_u64_every_pos(p, count):
    rng = random.Random(p * 1000 + count)
    n = 300  # two blocks, ragged
    recs = [(O.seed(i + 1, p) if i % 3 else rng.randrange(O.M), i % 12, p) for i in range(n)]
    st = records_to_tensor(recs)
    out = rlx.generate_u64(st, count, p)
    exp, fin = oracle_draws(recs, count)
    got = out.cpu().numpy()
    for i in range(n):
        assert got[i].tolist() == exp[i], (i, recs[i][1])
    assert tensor_to_records(st) == fin


@pytest.mark.parametrize("p", (24, 2048))
def test_generate_f64_matches_u64_and_oracle(p):
    n, count = 257, 145
    recs = [(O.seed(i, p), 0, p) for i in range(n)]
    st_a = records_to_tensor(recs)
    st_b = st_a.clone()
    f = rlx.generate_f64(st_a, count, p)
    u = rlx.generate_u64(st_b, count, p)
    assert torch.equal(st_a, st_b)
    assert torch.equal(f, u.to(torch.float64) * 2.0 ** -48)
    assert bool(((f >= 0) & (f < 1)).all())
    exp, _ = oracle_draws(recs[:40], count)
    fh = f.cpu().numpy()
    for i in range(40):
        assert fh[i].tolist() == [O.field_to_double(v) for v in exp[i]]


def test_generate_general_path_equals_fast_path():
    rng = random.Random(106)
    p = 794
    recs = [(x, rng.randrange(12), p) for x in crafted_states(rng, 600)]
    st_a = records_to_tensor(recs)
    st_b = st_a.clone()
    a = rlx.generate_u64(st_a, 61, p)
    b = rlx.test_generate_u64_general(st_b, 61, p)
    assert torch.equal(a, b) and torch.equal(st_a, st_b)
    exp, fin = oracle_draws(recs, 61)
    assert a.cpu().numpy().tolist() == exp
    assert tensor_to_records(st_a) == fin


def test_generate_crafted_step_results():
    # states whose next step lands on chosen results (top word all ones, m - 1, ...)
    rng = random.Random(107)
    p = 2048
    ap = O.multiplier(p)
    inv = pow(ap, -1, O.M)
    targets = [O.M - 1, O.M - 2, 0 + 1, 2 ** 576 - 2 ** 240 - 5, 2 ** 576 - 2 ** 241, 2 ** 544 - 1,
               (2 ** 576 - 2 ** 240) // 3] + [O.M - 1 - rng.randrange(2 ** 300) for _ in range(60)]
    recs = [(t * inv % O.M, 0, p) for t in targets]
    st = records_to_tensor(recs)
    out = rlx.generate_u64(st, 36, p)
    exp, fin = oracle_draws(recs, 36)
    assert out.cpu().numpy().tolist() == exp
    assert tensor_to_records(st) == fin


def test_continuation_split_invariance():
    p = 404
    n = 300
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=50)
    ref_st = st.clone()
    whole = rlx.generate_u64(ref_st, 1000, p)
    parts = []
    for c in (1, 11, 12, 0, 250, 13, 713):
        parts.append(rlx.generate_u64(st, c, p))
    assert torch.equal(torch.cat(parts, dim=1), whole)
    assert torch.equal(st, ref_st)


def test_state_copies_continue_on_the_host():
    # section 4.2: the state is plain words; continue a GPU stream in the oracle
    p = 2048
    st = rlx.new_states(5)
    rlx.init_streams(st, p, id0=9)
    rlx.generate_u64(st, 777, p)
    recs = tensor_to_records(st)
    more = rlx.generate_u64(st, 50, p).cpu().numpy().tolist()
    for (x, pos, _), row in zip(recs, more):
        assert O.draws(x, pos, p, 50)[0] == row


def test_trace_small():
    p = 2048
    st = rlx.new_states(3)
    rlx.init_streams(st, p, id0=1)
    recs = tensor_to_records(st)
    vals, trace = rlx.generate_f64_trace(st, 12 * 20 + 5, p)
    steps = trace.shape[1]
    for i, (x, pos, _) in enumerate(recs):
        row = words_to_ints(trace[i].cpu().numpy())
        xs = [x]
        for _ in range(steps - 1):
            xs.append(O.mulmod(O.multiplier(p), xs[-1]))
        assert row[: (pos + 12 * 20 + 5) // 12 + 1] == xs[: (pos + 12 * 20 + 5) // 12 + 1]


def test_empty_and_error_paths():
    p = 2048
    st = rlx.new_states(4)
    rlx.init_streams(st, p)
    before = st.clone()
    out = rlx.generate_f64(st, 0, p)
    assert out.shape == (4, 0) and torch.equal(st, before)
    # a record with the wrong p, one with pos 12, one with x = m
    bad = records_to_tensor([(5, 0, 218), (5, 12, 2048), (O.M, 0, 2048), (7, 3, 2048)])
    rlx.check_errors()
    out = torch.full((4, 5), -1, dtype=torch.int64, device=DEV)
    rlx.generate_u64(bad, 5, p, out=out)
    flags = rlx.check_errors()
    assert flags == 0x7
    o = out.cpu().numpy()
    assert (o[:3] == -1).all()
    assert o[3].tolist() == O.draws(7, 3, 2048, 5)[0]
    assert rlx.check_errors() == 0
    with pytest.raises(rlx.RlxError):
        rlx.generate_u64(st, 5, 23)


# --- the workloads at full size, sampled ----------------------------------------

def test_single_stream_workload_full():
    """one stream, id 1, p = 2048, 2^20 doubles and the state after every step"""
    p, count = 2048, 1 << 20
    st = rlx.new_states(1)
    rlx.init_streams(st, p, id0=1)
    vals, trace = rlx.generate_f64_trace(st, count, p)
    u = (vals * 2.0 ** 48).to(torch.int64).cpu().numpy()[0]
    exp, x_end, pos_end = O.draws(O.seed(1, p), 0, p, count)
    assert u.tolist() == exp
    assert tensor_to_records(st) == [(x_end, pos_end, p)]
    # every one of the 87 382 trace states against the oracle's successive
    # multiplications X_{t+1} = A_p X_t mod m from the seed
    # (the binding sizes the trace for pos = 11: rows past the last state
    # visited stay as allocated, zero)
    tr = trace[0].cpu().numpy()
    nst = count // 12 + 1
    assert not tr[nst:].any()
    got = words_to_ints(tr[:nst])
    a, x = O.multiplier(p), O.seed(1, p)
    for t in range(nst):
        assert got[t] == x, t
        x = a * x % O.M
    for t in (0, 1000, nst - 1):                      # and against skip-ahead
        assert got[t] == O.skip(O.seed(1, p), t, p)


def test_many_streams_workload_sampled():
    """65 536 streams (ids 0..65535), p = 2048, 4096 doubles each"""
    p, n, count = 2048, 65536, 4096
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=0)
    f = rlx.generate_f64(st, count, p)
    rng = random.Random(108)
    sample = [0, 1, 255, 256, 65535] + rng.sample(range(n), 11)
    fh = f.cpu().numpy()
    for i in sample:
        exp, x_end, pos_end = O.draws(O.seed(i, p), 0, p, count)
        assert fh[i].tolist() == [O.field_to_double(v) for v in exp], i
    recs = tensor_to_records(st[torch.tensor(sample, device=DEV)])
    for i, r in zip(sample, recs):
        assert r == O.state_at(O.seed(i, p), p, count) + (p,)
    # every value is in [0, 1) and the u64 variant agrees with the doubles
    assert bool(((f >= 0) & (f < 1)).all())
    st2 = rlx.new_states(n)
    rlx.init_streams(st2, p, id0=0)
    u = rlx.generate_u64(st2, count, p)
    assert torch.equal(u.to(torch.float64) * 2.0 ** -48, f)


def test_skip_workload_sampled():
    """2^20 streams advanced by log-uniform offsets in [1, 2^64)"""
    import workloads
    p, n = 2048, 1 << 20
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=0)
    offs = workloads.skip_offsets(n)
    kt = torch.from_numpy(offs.view(np.int64)).to(DEV)
    rlx.skip(st, kt, p)
    rng = random.Random(109)
    sample = [0, 1, n - 1] + rng.sample(range(n), 40)
    recs = tensor_to_records(st[torch.tensor(sample, device=DEV)])
    for i, r in zip(sample, recs):
        assert r == (O.skip(O.seed(i, p), int(offs[i]), p), 0, p)


# --- lanes per stream: the values never depend on the launch shape --------------

@pytest.fixture
def lanes_reset():
    yield
    rlx.set_lanes_per_stream(0)


@pytest.mark.parametrize("G", (1, 2, 4, 8, 16, 32, 64, 128, 1024, 4096, 16384, 65536))
def test_lanes_per_stream_bit_identical(G, lanes_reset):
    rng = random.Random(200 + G)
    p = 218
    n, count = 37, 12 * 70 + 7
    recs = [(O.seed(i + 3, p), rng.randrange(12), p) for i in range(n)]
    st = records_to_tensor(recs)
    rlx.set_lanes_per_stream(G)
    assert rlx.lanes_per_stream(n, count) == G
    out = rlx.generate_u64(st, count, p)
    exp, fin = oracle_draws(recs, count)
    assert out.cpu().numpy().tolist() == exp
    assert tensor_to_records(st) == fin
    # f64 with trace (all records share pos 0 for the trace layout)
    st2 = records_to_tensor([(O.seed(i + 3, p), 0, p) for i in range(n)])
    vals, trace = rlx.generate_f64_trace(st2, count, p)
    u = (vals * 2.0 ** 48).to(torch.int64).cpu().numpy()
    for i in range(0, n, 5):
        ex, _, _ = O.draws(O.seed(i + 3, p), 0, p, count)
        assert u[i].tolist() == ex
        tr = words_to_ints(trace[i].cpu().numpy())
        x = O.seed(i + 3, p)
        for t in range(count // 12 + 1):
            assert tr[t] == x, (i, t)
            x = O.mulmod(O.multiplier(p), x)


@pytest.mark.parametrize("G", (2, 8, 64, 256))
def test_lanes_short_counts_and_general_path(G, lanes_reset):
    # counts shorter than a lane's share, every pos, and the general branch
    rng = random.Random(300 + G)
    p = 24
    recs = [(x, rng.randrange(12), p) for x in crafted_states(rng, 100)]
    rlx.set_lanes_per_stream(G)
    for count in (1, 5, 12, 13, 40, 12 * G + 1):
        st_a = records_to_tensor(recs)
        st_b = st_a.clone()
        a = rlx.generate_u64(st_a, count, p)
        b = rlx.test_generate_u64_general(st_b, count, p)
        exp, fin = oracle_draws(recs, count)
        assert a.cpu().numpy().tolist() == exp, count
        assert torch.equal(a, b) and torch.equal(st_a, st_b)
        assert tensor_to_records(st_a) == fin


def test_records_spanning_many_waves_advance_after_the_launch():
    """16 streams x 2^24 values at the automatic lane count G = 65536: 2^20
    lanes in 16 384 waves, more than the chip holds at once, so the lanes of
    one record run in several dispatch rounds and every workgroup still has
    blocks to draw (21 steps per lane).  The records must end at position
    2^24 (advanced after every lane has read them), every stream's values
    must match the oracle at its start, end and random windows, and a second
    call must continue from the advanced records.  The same for the legacy
    52-bit doubles, whose records count 11 values per step."""
    import oracle.widths as W
    p, n, count = 2048, 16, 1 << 24
    assert rlx.lanes_per_stream(n, count) == 65536
    rng = random.Random(110)
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=500)
    out = rlx.generate_f64(st, count, p)
    torch.cuda.synchronize()
    recs = tensor_to_records(st)
    for i in range(n):
        x0 = O.seed(500 + i, p)
        assert recs[i] == O.state_at(x0, p, count) + (p,), i
        for j in [0, count - 40] + rng.sample(range(count - 40), 6):
            got = (out[i, j:j + 40] * 2.0 ** 48).to(torch.int64).cpu().numpy().tolist()
            assert got == O.window(x0, p, j, 40), (i, j)
    nxt = rlx.generate_u64(st, 29, p)
    for i in range(n):
        assert u64_list(nxt[i]) == O.window(O.seed(500 + i, p), p, count, 29), i
    del out
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=700)
    out = rlx.generate_f64_lcg52(st, count, p)
    torch.cuda.synchronize()
    recs = tensor_to_records(st)
    for i in range(n):
        x0 = O.seed(700 + i, p)
        steps, pos = divmod(count, 11)
        assert recs[i] == (O.skip(x0, steps, p), pos, p), i
        for j in [0, count - 30] + rng.sample(range(count - 30), 4):
            s0, p0 = divmod(j, 11)
            want = W.draws_lcg52(O.skip(x0, s0, p), p0, p, 30)[0]
            assert out[i, j:j + 30].cpu().numpy().tolist() == want, (i, j)
    del out
    torch.cuda.empty_cache()


def test_output_beyond_2pow32_elements():
    """Two records x (2^31 + 5) doubles: row 1 starts past element 2^31 and
    ends past 2^32 (34 GB of output), so every output offset needs 64 bits.
    Windows at the start, around the 32-bit boundaries and at the end of
    each row are compared with the oracle, and the records after the call."""
    p = 2048
    count = (1 << 31) + 5
    st = rlx.new_states(2)
    rlx.init_streams(st, p, id0=40)
    out = rlx.generate_f64(st, count, p)
    torch.cuda.synchronize()
    flat = out.view(-1)
    for r in range(2):
        x0 = O.seed(40 + r, p)
        for j in (0, (1 << 31) - 30, count - 40):    # windows inside the row, one across index 2^31
            k = r * count + j
            got = (flat[k:k + 35] * 2.0 ** 48).to(torch.int64).cpu().numpy().tolist()
            assert got == O.window(x0, p, j, 35), (r, j)
    # the element at global index 2^32 and its neighbours (row 1)
    k = 1 << 32
    got = (flat[k - 3:k + 3] * 2.0 ** 48).to(torch.int64).cpu().numpy().tolist()
    assert got == O.window(O.seed(41, p), p, k - 3 - count, 6)
    recs = tensor_to_records(st)
    for r in range(2):
        assert recs[r] == O.state_at(O.seed(40 + r, p), p, count) + (p,)
    del out, flat
    torch.cuda.empty_cache()
