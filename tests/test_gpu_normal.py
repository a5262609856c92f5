"""GPU parity of the Gaussian draws (rlx_generate_normal_f64) against the
mpmath Box-Muller oracle.

The device evaluates the transform in binary64 (include/rlx_gauss.hpp: an
exact range reduction for each of log and the angle, series for the rest),
so values are compared under a tolerance rather than bit for bit:

    |gpu - oracle| <= 2^-49 |oracle| + 2^-70

The relative part is 8 ulp of the result: ln(1 - u1), cos and sin are each
within about an ulp (tests/test_host_gauss.py measures the same code built
for the host, whose operations are all correctly rounded, so it computes
the device's bits), sqrt halves the log's error and rounds once, and the
product adds half an ulp; the host build's worst case is 2 ulp, and 8 ulp
leaves a wide margin.  The absolute floor covers the exact zeros of cos and
sin at quarter turns, which the 40-digit oracle returns as values of about
10^-41.

Everything that is exact is compared exactly: the records after the call
(normals consume positions like uniforms do) and the zero of u1 = 0.
"""
import random

import numpy as np
import pytest
import torch

import oracle as O
from oracle import gauss as G
import paper_2106_02504_amd as rlx
from rlx_util import records_to_tensor, tensor_to_records

pytestmark = pytest.mark.gpu

DEV = "cuda"
REL = 2.0 ** -49
ABS = 2.0 ** -70


def assert_close(got, want, what):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    err = np.abs(got - want)
    bound = REL * np.abs(want) + ABS
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (what, int(bad[0]), float(got[bad[0]]), float(want[bad[0]]))


def ulps(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    sp = np.spacing(np.abs(want))
    return float(np.max(np.abs(got - want) / np.maximum(sp, 2.0 ** -1074)))


@pytest.mark.parametrize("p", (24, 2048))
def test_normals_match_oracle_every_position(p):
    # 300 records (two 256-lane blocks, ragged), every starting position,
    # 107 values each (several steps, ragged end)
    rng = random.Random(p)
    recs = []
    for i in range(300):
        x = O.seed(rng.randrange(1 << 20), p)
        recs.append((x, i % 12, p))
    st = records_to_tensor(recs)
    out = rlx.generate_normal_f64(st, 107, p)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    after = tensor_to_records(st)
    worst = 0.0
    for i, (x, pos, _) in enumerate(recs):
        want, x2, pos2 = G.normals(x, pos, p, 107)
        assert_close(got[i], want, ("record", i))
        worst = max(worst, ulps(got[i], want))
        assert after[i] == (x2, pos2, p)
    print(f"max error {worst:.2f} ulp")


def test_normal_advance_equals_uniform_advance():
    p = 404
    recs = [(O.seed(i, p), (5 * i) % 12, p) for i in range(100)]
    a = records_to_tensor(recs)
    b = a.clone()
    rlx.generate_normal_f64(a, 53, p)
    rlx.generate_f64(b, 53, p)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_normals_with_lanes_per_stream():
    # the staged path with G lanes per record gives the same values as G = 1
    p = 2048
    recs = [(O.seed(i, p), i % 12, p) for i in range(70)]
    outs = []
    try:
        for g in (1, 2, 8, 64):
            rlx.set_lanes_per_stream(g)
            st = records_to_tensor(recs)
            outs.append(rlx.generate_normal_f64(st, 1000, p).cpu())
    finally:
        rlx.set_lanes_per_stream(0)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    for i in (0, 33, 69):
        want, _, _ = G.normals(recs[i][0], recs[i][1], p, 1000)
        assert_close(outs[0][i].numpy(), want, ("record", i))


def test_normals_full_size_sampled():
    # the many-streams shape: 65 536 records x 4096 normals; sampled rows
    # against the oracle, moments of the whole output
    p = 2048
    n, count = 65536, 4096
    st = rlx.new_states(n)
    rlx.init_streams(st, p, id0=0)
    out = rlx.generate_normal_f64(st, count, p)
    torch.cuda.synchronize()
    rng = random.Random(9)
    for i in [0, 1, n - 1] + [rng.randrange(n) for _ in range(5)]:
        cols = sorted(rng.sample(range(count), 24))
        want_row, _, _ = G.normals(O.seed(i, p), 0, p, max(cols) + 1)
        assert_close(out[i, cols].cpu().numpy(), [want_row[c] for c in cols], ("row", i))
    flat = out.view(-1)
    mean = float(flat.mean())
    var = float(flat.var())
    size = flat.numel()
    assert abs(mean) < 6.0 / size ** 0.5
    assert abs(var - 1.0) < 6.0 * (2.0 / size) ** 0.5
    assert torch.isfinite(flat).all()
    # the largest |z| is bounded by sqrt(96 ln 2) (u1 <= 1 - 2^-48)
    assert float(flat.abs().max()) <= G.radius((1 << 48) - 1) * (1 + 1e-15)


def test_normal_edge_cases():
    p = 2048
    assert rlx.generate_normal_f64(rlx.new_states(5), 0, p).numel() == 0
    st = records_to_tensor([(O.seed(1, p), 11, p)])
    got = rlx.generate_normal_f64(st, 1, p).cpu().numpy()[0]
    want, x2, pos2 = G.normals(O.seed(1, p), 11, p, 1)
    assert_close(got, want, "single value at pos 11")
    assert tensor_to_records(st)[0] == (x2, pos2, p)
