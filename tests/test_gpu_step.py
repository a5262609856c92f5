"""The two generator-step kernels (sections 2.1, 2.2): one step by A_p^(2^g)
on the matrix cores (int8 contraction of the state's bytes) and on the vector
ALU (32-bit multiply-adds with the reduction folded into the multiplier),
each against the oracle's plain modular product, on random and crafted
states, for every luxury level and the lane counts the generate calls use;
and the generate calls giving bit-identical values and records under either
kernel."""
import random

import pytest
import torch

import oracle as O
import paper_2106_02504_amd as rlx
from rlx_util import ints_to_words, words_to_ints, tensor_to_records

pytestmark = pytest.mark.gpu

LEVELS = (24, 218, 404, 794, 2048)
KINDS = (rlx.STEP_MFMA, rlx.STEP_VALU)


def crafted_states():
    m = O.M
    byte_fill = lambda b: sum(b << (8 * i) for i in range(72))
    vals = [0, 1, 2, 255, 256, m - 1, m - 2, (m - 1) // 2,
            2 ** 575, 2 ** 576 - 2 ** 241,          # large, below m
            2 ** 240 - 1, 2 ** 240, 2 ** 336 - 1, 2 ** 336,
            byte_fill(0x80), byte_fill(0x7F), byte_fill(0x01),   # signed digits 0, -1, -127
            byte_fill(0x80) ^ 1, m - 1 - byte_fill(0x01)]
    vals += [(1 << (8 * i)) for i in range(0, 72, 7)]            # single bytes at awkward offsets
    vals += [((1 << (8 * i)) - 1) for i in (1, 9, 36, 71)]        # runs of 0xFF bytes
    return [v % m for v in vals]


def step_oracle(xs, p, g):
    a = pow(O.multiplier(p), 2 ** g, O.M)
    return [a * x % O.M for x in xs]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("p", LEVELS)
def test_step_kernel_against_oracle(kind, p):
    rng = random.Random(1000 + p)
    xs = crafted_states() + [rng.randrange(O.M) for _ in range(200)]
    x = torch.from_numpy(ints_to_words(xs)).cuda()
    for g in (0, 1, 2, 3, 4, 5, 6, 7, 10, 16, 20, 63):
        got = words_to_ints(rlx.test_step(x, p, g, kind).cpu().numpy())
        assert got == step_oracle(xs, p, g), (kind, p, g)


@pytest.mark.parametrize("kind", KINDS)
def test_step_kernel_general_fold(kind):
    # the exact general fold on every lane gives the same canonical results
    rng = random.Random(7)
    p = 2048
    xs = crafted_states() + [rng.randrange(O.M) for _ in range(100)]
    x = torch.from_numpy(ints_to_words(xs)).cuda()
    for g in (0, 4, 16):
        got = words_to_ints(rlx.test_step(x, p, g, kind, general=True).cpu().numpy())
        assert got == step_oracle(xs, p, g), (kind, g)


def test_step_kernel_ragged_wave():
    # n not a multiple of 64: the matrix-core step still runs whole waves
    # (the lanes past n step a dummy state and store nothing)
    rng = random.Random(9)
    for n in (1, 63, 65, 129):
        xs = [rng.randrange(O.M) for _ in range(n)]
        x = torch.from_numpy(ints_to_words(xs)).cuda()
        got = words_to_ints(rlx.test_step(x, 2048, 4, rlx.STEP_MFMA).cpu().numpy())
        assert got == step_oracle(xs, 2048, 4), n


@pytest.fixture
def kind_reset():
    yield
    rlx.set_step_kernel(rlx.STEP_MFMA)
    rlx.set_lanes_per_stream(0)


@pytest.mark.parametrize("G", [1, 2, 8, 16, 64, 256])
def test_generate_identical_under_both_step_kernels(G, kind_reset):
    p, n, count = 794, 300, 1500
    res = {}
    for kind in KINDS:
        rlx.set_step_kernel(kind)
        assert rlx.step_kernel() == kind
        rlx.set_lanes_per_stream(G)
        st = rlx.new_states(n)
        rlx.init_streams(st, p, id0=11)
        f = rlx.generate_f64(st, count, p)
        u = rlx.generate_u64(st, 77, p)
        fl = rlx.generate_f32(st, 202, p)
        nm = rlx.generate_normal_f64(st, 99, p)
        torch.cuda.synchronize()
        res[kind] = (f.cpu(), u.cpu(), fl.cpu(), nm.cpu(), tensor_to_records(st))
    a, b = res[rlx.STEP_MFMA], res[rlx.STEP_VALU]
    for k in range(4):
        assert torch.equal(a[k], b[k]), (G, k)
    assert a[4] == b[4]
    # and against the oracle on a few streams
    for i in (0, 151, n - 1):
        exp = O.window(O.seed(11 + i, p), p, 0, count)
        assert (a[0][i] * 2.0 ** 48).to(torch.int64).tolist() == exp, (G, i)

