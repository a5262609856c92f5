"""Pins for the other output widths (float32 from single RANLUX numbers, and
the legacy 52-bit doubles from raw LCG bits).

* float32: the values times 2^24 are the subtract-with-borrow recurrence's
  own outputs, run number by number (section 1), with the luxury decimation
  (the last 24 of every p outputs); each value is exact in binary32; 2c
  floats move a stream exactly as c 48-bit draws do.
* legacy: the 11 values of a step reassemble the LCG state that the SWB
  recurrence reaches (via the LCG form X = D - D / 2^336 + c), the top 4
  bits stay unused, and the bias the paper names (top bits of X are 0 more
  often) holds for m.
Planted mistakes (numbers of a pair swapped, digits of X instead of the
RANLUX numbers, 52-bit values taken from the top down, a missed advance)
each fail at least one pin.
"""

import random

import numpy as np
import pytest

import oracle as O
from oracle import widths as W

SWB = O.RANLUX


def swb_numbers(x0, p, steps):
    """The RANLUX numbers a stream delivers in `steps` generator steps, from
    the SWB recurrence alone: the 24 numbers of the start state oldest first,
    then, per step, the last 24 of p new SWB outputs in production order."""
    d, c = SWB.to_ranlux(x0)
    out = SWB.digits(d)
    for _ in range(steps - 1):
        produced = []
        for _ in range(p):
            d, c = SWB.swb_step(d, c)
            produced.append(SWB.digits(d)[-1])
        out += produced[-24:]
    return out


def lcg_states_by_swb(x0, p, steps):
    """LCG states X_0 .. X_{steps-1} of a stream reached by running the SWB
    recurrence p steps at a time and mapping each state to its LCG form."""
    d, c = SWB.to_ranlux(x0)
    xs = []
    for _ in range(steps):
        xs.append(SWB.to_lcg(d, c))
        d, c = SWB.swb_steps(d, c, p)
    return xs


def f32_pins(draws_f32, p=218, seed=4):
    failed = []
    x0 = O.seed(seed, p)
    n = 24 * 4 + 10
    vals, x2, pos2 = draws_f32(x0, 0, p, n)
    want = swb_numbers(x0, p, 5)[:n]
    if [v * 2.0 ** 24 for v in vals] != [float(w) for w in want]:
        failed.append("swb sequence")
    if any(np.float32(v) != v or not (0.0 <= v < 1.0) for v in vals):
        failed.append("binary32 exact")
    _, xa, pa = O.draws(x0, 0, p, n // 2)
    if (x2, pos2) != (xa, pa):
        failed.append("state after 2c floats")
    return failed


def lcg52_pins(draws_lcg52, p=404, seed=6):
    failed = []
    x0 = O.seed(seed, p)
    steps = 4
    vals, x2, pos2 = draws_lcg52(x0, 0, p, 11 * steps)
    xs = lcg_states_by_swb(x0, p, steps + 1)
    for t in range(steps):
        part = vals[11 * t: 11 * t + 11]
        ints = [v * 2.0 ** 52 for v in part]
        if any(i != int(i) or not (0 <= i < 2 ** 52) for i in ints):
            failed.append("52-bit exact")
            break
        if sum(int(i) << (52 * k) for k, i in enumerate(ints)) != xs[t] % (1 << 572):
            failed.append("reassembles X_t")
            break
    if (x2, pos2) != (xs[steps], 0):
        failed.append("state after 11 t values")
    return failed


def test_f32_pins_hold():
    assert f32_pins(W.draws_f32) == []
    assert f32_pins(W.draws_f32, p=24, seed=9) == []


def test_lcg52_pins_hold():
    assert lcg52_pins(W.draws_lcg52) == []
    assert lcg52_pins(W.draws_lcg52, p=24, seed=1) == []


def test_f32_continuation_and_positions():
    rng = random.Random(3)
    p = 794
    x0 = O.seed(11, p)
    full, xe, pe = W.draws_f32(x0, 0, p, 300)
    for _ in range(10):
        c = rng.randrange(0, 150)
        a, x1, p1 = W.draws_f32(x0, 0, p, 2 * c)
        b, x2, p2 = W.draws_f32(x1, p1, p, 300 - 2 * c)
        assert a + b == full and (x2, p2) == (xe, pe)
    u48, _, _ = O.draws(x0, 0, p, 150)
    for j, v in enumerate(u48):
        assert full[2 * j] * 2.0 ** 24 + full[2 * j + 1] * 2.0 ** 48 == float(v) and v < 2 ** 53
    with pytest.raises(ValueError):
        W.draws_f32(x0, 0, p, 3)


def test_lcg52_continuation_and_edges():
    p = 218
    x0 = O.seed(2, p)
    full, xe, pe = W.draws_lcg52(x0, 0, p, 100)
    a, x1, p1 = W.draws_lcg52(x0, 0, p, 37)
    b, x2, p2 = W.draws_lcg52(x1, p1, p, 63)
    assert a + b == full and (x2, p2) == (xe, pe) and p1 == 37 % 11
    assert pe == 100 % 11 and xe == O.skip(x0, 100 // 11, p)
    # seed 0 is X = 1: one value 2^-52, then zeros
    assert W.draws_lcg52(1, 0, p, 11)[0] == [2.0 ** -52] + [0.0] * 10
    with pytest.raises(ValueError):
        W.draws_lcg52(x0, 11, p, 1)


def test_lcg52_top_bits_biased():
    # the paper's reason to drop the conversion: X < m < 2^576, so the top
    # bit of X is 1 for fewer than half of the states
    assert 2 * (O.M - 2 ** 575) < O.M
    assert W.LCG52_VALUES * 52 == 572


# --- planted mistakes ------------------------------------------------------------

def _f32_swapped(x, pos, p, n):
    v, x2, p2 = W.draws_f32(x, pos, p, n)
    return [v[i ^ 1] for i in range(len(v))], x2, p2


def _f32_from_x(x, pos, p, n):
    out = []
    a = O.multiplier(p)
    while len(out) < n:
        nums = [(x >> (24 * j)) & 0xFFFFFF for j in range(24)]
        out += [W.number_to_f32(nums[2 * pos]), W.number_to_f32(nums[2 * pos + 1])]
        pos += 1
        if pos == 12:
            x, pos = O.mulmod(a, x), 0
    return out, x, pos


def _f32_no_advance(x, pos, p, n):
    v, _, _ = W.draws_f32(x, pos, p, n)
    return v, x, pos


def _lcg52_top_down(x, pos, p, n):
    v, x2, p2 = W.draws_lcg52(x, pos, p, n)
    return [v[11 * (i // 11) + 10 - i % 11] for i in range(len(v))], x2, p2


def _lcg52_from_d(x, pos, p, n):
    d, _ = SWB.to_ranlux(x)
    v, x2, p2 = W.draws_lcg52(d, pos, p, n)
    return v, x2, p2


def test_planted_mistakes_are_caught():
    assert f32_pins(_f32_swapped)
    assert f32_pins(_f32_from_x)
    assert f32_pins(_f32_no_advance)
    assert lcg52_pins(_lcg52_top_down)
    assert lcg52_pins(_lcg52_from_d)
