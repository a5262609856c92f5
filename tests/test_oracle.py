"""Pins for the CPU oracle: each test checks the oracle against something the
paper or the mathematics fixes, not against the oracle itself.

* closed forms of m (section 2.2) and of the multiplier a;
* brute force over every state of small subtract-with-borrow generators: one
  SWB step equals one multiplication by a (the LCG equivalence of section 1);
* the 576-bit SWB recurrence run directly, step by step, against the LCG
  form at every luxury level used (p SWB steps = one multiply by a^p);
* skip-ahead against repeated single steps (section 2.4);
* seeding identities; crafted mulmod operands with known residues;
* stream semantics: continuation and windows.
"""

import random

import pytest
import sympy

import oracle as O
from oracle import SwbParams

SMALL = [(3, 5, 2), (2, 6, 3), (4, 3, 1), (1, 7, 3), (2, 5, 2)]
LUX = (24, 218, 404, 794, 2048)


def rnd_x(rng):
    return rng.randrange(O.M)


# --- constants -----------------------------------------------------------------

def test_modulus_closed_form():
    # section 2.2 prints m = 2^576 - 2^240 + 1
    assert O.M == 2 ** 576 - 2 ** 240 + 1
    assert O.NBITS == 576 and O.FIELDS == 12


def test_modulus_is_prime():
    assert sympy.isprime(O.M)


def test_multiplier_closed_form():
    # a = b^-1 mod m written out: 2^576 - 2^552 - 2^240 + 2^216 + 1
    assert O.A == 2 ** 576 - 2 ** 552 - 2 ** 240 + 2 ** 216 + 1
    assert (O.A << 24) % O.M == 1


# --- the SWB <-> LCG equivalence, brute force on small generators --------------

@pytest.mark.parametrize("bbits,r,s", SMALL)
def test_small_canonical_states_exhaustive(bbits, r, s):
    g = SwbParams(bbits, r, s)
    seen = set()
    for x in range(g.m):
        d, c = g.to_ranlux(x)
        assert c in (0, 1) and 0 <= d < g.b ** r
        assert g.to_lcg(d, c) == x
        assert g.swb_step(d, c) == g.to_ranlux(g.a * x % g.m)
        seen.add((d, c))
    assert len(seen) == g.m          # to_ranlux is injective on [0, m)


@pytest.mark.parametrize("bbits,r,s", SMALL)
def test_small_all_states_congruence(bbits, r, s):
    # every SWB state, canonical or not, steps like a multiply by a (mod m)
    g = SwbParams(bbits, r, s)
    for d in range(g.b ** r):
        for c in (0, 1):
            d2, c2 = g.swb_step(d, c)
            assert g.to_lcg(d2, c2) % g.m == g.a * g.to_lcg(d, c) % g.m


def test_small_period_divides_group_order():
    # a has multiplicative order dividing m - 1 when m is prime
    for bbits, r, s in SMALL:
        g = SwbParams(bbits, r, s)
        if sympy.isprime(g.m):
            assert pow(g.a, g.m - 1, g.m) == 1


# --- the same at full size ------------------------------------------------------

def test_ranlux_round_trip_random_and_edges():
    rng = random.Random(11)
    xs = [0, 1, 2, O.M - 1, O.M - 2, 2 ** 336 - 1, 2 ** 336, 2 ** 336 + 1,
          2 ** 240 - 1, 2 ** 240, 2 ** 576 - 2 ** 240, (O.M - 1) // 2]
    xs += [rnd_x(rng) for _ in range(2000)]
    for x in xs:
        nums, c = O.to_ranlux(x)
        assert len(nums) == 24 and all(0 <= v < 2 ** 24 for v in nums)
        assert c in (0, 1)
        assert O.to_lcg(nums, c) == x


def test_swb_steps_equal_multiplier_powers():
    rng = random.Random(12)
    g = O.RANLUX
    for _ in range(5):
        x = rnd_x(rng)
        d, c = g.to_ranlux(x)
        y = x
        for k in range(1, 101):
            d, c = g.swb_step(d, c)
            y = O.mulmod(O.A, y)
            assert (d, c) == g.to_ranlux(y), k


def test_noncanonical_swb_state_becomes_canonical():
    # arbitrary digits and carry: congruent after every step, canonical after r
    rng = random.Random(13)
    g = O.RANLUX
    for _ in range(5):
        d = rng.getrandbits(576)
        c = rng.randrange(2)
        x0 = g.to_lcg(d, c) % O.M
        for k in range(1, 60):
            d, c = g.swb_step(d, c)
            xk = O.mulmod(pow(O.A, k, O.M), x0)
            assert g.to_lcg(d, c) % O.M == xk
            if k >= 24:
                assert (d, c) == g.to_ranlux(xk)


@pytest.mark.parametrize("p", LUX)
def test_luxury_step_equals_p_swb_steps(p):
    rng = random.Random(p)
    g = O.RANLUX
    x = rnd_x(rng)
    d, c = g.to_ranlux(x)
    d, c = g.swb_steps(d, c, p)
    assert (d, c) == g.to_ranlux(O.mulmod(O.multiplier(p), x))


@pytest.mark.parametrize("p", (24, 218, 404))
def test_multiplier_by_repeated_multiplication(p):
    y = 1
    for _ in range(p):
        y = y * O.A % O.M
    assert O.multiplier(p) == y


def test_multiplier_rejects_small_p():
    with pytest.raises(ValueError):
        O.multiplier(23)


# --- mulmod, crafted operands ---------------------------------------------------

def test_mulmod_crafted():
    m = O.M
    # (2^288 + 1)(2^288 - 1) = 2^576 - 1 = m + 2^240 - 2: unreduced value >= m
    assert O.mulmod(2 ** 288 + 1, 2 ** 288 - 1) == 2 ** 240 - 2
    assert O.mulmod(m - 1, m - 1) == 1
    assert O.mulmod(2 ** 300, 2 ** 276) == 2 ** 240 - 1      # 2^576 = m + 2^240 - 1
    rng = random.Random(14)
    for _ in range(50):
        x = rnd_x(rng)
        assert O.mulmod(x, 1) == x and O.mulmod(x, 0) == 0
        assert O.mulmod(x, m - 1) == (m - x) % m
        assert O.mulmod(O.mulmod(x, O.A), 2 ** 24) == x


# --- skip and seed (section 2.4) ------------------------------------------------

def test_skip_equals_single_steps():
    rng = random.Random(15)
    for p in (24, 2048):
        x = rnd_x(rng)
        a_p = O.multiplier(p)
        y = x
        for k in range(0, 300):
            assert O.skip(x, k, p) == y
            y = y * a_p % O.M


def test_skip_composes():
    rng = random.Random(16)
    x = rnd_x(rng)
    for _ in range(20):
        j, k = rng.getrandbits(64), rng.getrandbits(64)
        assert O.skip(O.skip(x, j, 2048), k, 2048) == O.skip(x, j + k, 2048)
    assert O.skip(x, 0, 2048) == x


def test_seed_identities():
    for p in (24, 2048):
        assert O.seed(0, p) == 1
        for i in range(4):
            assert O.seed(i + 1, p) == O.skip(O.seed(i, p), 2 ** 96, p)
            assert O.seed(i, p) == pow(O.seed_multiplier(p), i, O.M)


# --- fields, doubles and streams ------------------------------------------------

def test_fields_repack_to_ranlux_numbers():
    rng = random.Random(17)
    for _ in range(200):
        x = rnd_x(rng)
        f = O.fields(x)
        nums, _ = O.to_ranlux(x)
        assert sum(v << (48 * k) for k, v in enumerate(f)) == sum(v << (24 * j) for j, v in enumerate(nums))
        for v in f:
            d = O.field_to_double(v)
            assert 0.0 <= d < 1.0 and d * 2.0 ** 48 == v


def test_seed_zero_first_step():
    # X = 1: D = floor(2^576 / m) = 1, so the first value is 1 then zeros
    f = O.fields(1)
    assert f == [1] + [0] * 11


def swb_stream(x0, p, n):
    """Draws produced by the SWB recurrence directly: the state's 24 numbers
    are taken in pairs (older number low), then p SWB steps are made."""
    g = O.RANLUX
    d, c = g.to_ranlux(x0)
    out = []
    while len(out) < n:
        nums = g.digits(d)
        out += [nums[2 * k] | (nums[2 * k + 1] << 24) for k in range(12)]
        d, c = g.swb_steps(d, c, p)
    return out[:n]


@pytest.mark.parametrize("p", (24, 218))
def test_draws_equal_direct_swb(p):
    x0 = O.seed(1, p)
    vals, _, _ = O.draws(x0, 0, p, 12 * 25 + 5)
    assert vals == swb_stream(x0, p, 12 * 25 + 5)


def test_draws_continuation_and_windows():
    rng = random.Random(18)
    p = 404
    x0 = O.seed(7, p)
    full, xe, pe = O.draws(x0, 0, p, 500)
    for _ in range(20):
        n1 = rng.randrange(0, 500)
        a, x1, p1 = O.draws(x0, 0, p, n1)
        b, x2, p2 = O.draws(x1, p1, p, 500 - n1)
        assert a + b == full and (x2, p2) == (xe, pe)
        assert O.state_at(x0, p, n1) == (x1, p1)
        assert O.window(x0, p, n1, 500 - n1) == full[n1:]
    assert pe == 500 % 12 and xe == O.skip(x0, 500 // 12, p)


def test_draws_eager_advance():
    x0 = O.seed(3, 24)
    _, x, pos = O.draws(x0, 0, 24, 12)
    assert pos == 0 and x == O.mulmod(O.multiplier(24), x0)
    _, x, pos = O.draws(x0, 5, 24, 0)
    assert (x, pos) == (x0, 5)


def test_state_record_layout():
    rng = random.Random(19)
    x = rnd_x(rng)
    rec = O.state_record(x, 7, 2048)
    assert len(rec) == 10 and rec[9] == 7 + (2048 << 32)
    assert O.parse_record(rec) == (x, 7, 2048)
    assert O.from_limbs(O.to_limbs(x)) == x


# --- planted mistakes: each must be caught by the pins above --------------------

def _equivalence_holds(g):
    for x in range(g.m):
        d, c = g.to_ranlux(x)
        if g.to_lcg(d, c) != x or g.swb_step(d, c) != g.to_ranlux(g.a * x % g.m):
            return False
    return True


def test_planted_mistakes_are_caught():
    base = (3, 5, 2)
    g = SwbParams(*base)
    assert _equivalence_holds(g)
    # wrong multiplier (b instead of b^-1: the other LCG direction)
    bad = SwbParams(*base); bad.a = bad.b
    assert not _equivalence_holds(bad)
    # wrong sign of the short-lag term in the modulus
    bad = SwbParams(*base); bad.m = bad.b ** 5 - bad.b ** 2 - 1; bad.a = pow(bad.b, -1, bad.m)
    assert not _equivalence_holds(bad)
    # wrong lag position in the recurrence (short lag off by one)
    bad = SwbParams(*base); bad.s = 3
    assert not _equivalence_holds(bad)
    # wrong shift in to_lcg / to_ranlux (top numbers off by one digit)
    bad = SwbParams(*base); bad.qshift += bad.bbits
    assert not _equivalence_holds(bad)


# --- stored vectors (written by tests/golden/make_golden.py from the oracle) ----

def test_golden_vectors_reproduce():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_vectors.json")
    doc = json.load(open(path))
    for p, h in doc["multipliers"].items():
        assert O.multiplier(int(p)) == int(h, 16)
    for s in doc["streams"][::7]:
        x0 = O.seed(s["id"], s["p"])
        assert x0 == int(s["seed_x"], 16)
        vals, x1, pos1 = O.draws(x0, 0, s["p"], 40)
        assert [format(v, "x") for v in vals] == s["first40"]
        assert (x1, pos1) == (int(s["x_after40"], 16), s["pos_after40"])
