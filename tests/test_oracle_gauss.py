"""Pins for the Gaussian oracle (Box-Muller on aligned field pairs): special
values where the trigonometric factor or the radius is known exactly, the
identity z0^2 + z1^2 = r^2, the position property of the stream, and the
distribution itself (Kolmogorov-Smirnov against the standard normal CDF).
Planted mistakes (wrong angle scale, radius without the factor -2, swapped
components, unpaired fields) each fail at least one pin."""

import math
import random

import numpy as np
import pytest
import scipy.stats

import oracle as O
from oracle import gauss as G

TWO48 = 1 << 48


def check_pins(bm, radius):
    """Pins on a Box-Muller candidate bm(v1, v2, component) and its radius;
    returns the list of failed pin names."""
    failed = []
    rng = random.Random(7)
    for _ in range(20):
        v1, v2 = rng.randrange(TWO48), rng.randrange(TWO48)
        # u1 = 0: radius 0, both components 0
        if bm(0, v2, 0) != 0.0 or bm(0, v2, 1) != 0.0:
            failed.append("u1=0")
        r = radius(v1)
        # u2 = 0: (r, 0); u2 = 1/4: (0, r); u2 = 1/2: (-r, 0); u2 = 3/4: (0, -r)
        for v2q, c0, c1 in ((0, r, 0.0), (TWO48 // 4, 0.0, r), (TWO48 // 2, -r, 0.0), (3 * TWO48 // 4, 0.0, -r)):
            z0, z1 = bm(v1, v2q, 0), bm(v1, v2q, 1)
            if abs(z0 - c0) > 1e-15 * max(1.0, r) or abs(z1 - c1) > 1e-15 * max(1.0, r):
                failed.append("quarter turns")
        # identity: z0^2 + z1^2 = -2 ln(1 - u1)
        z0, z1 = bm(v1, v2, 0), bm(v1, v2, 1)
        r2 = -2.0 * math.log1p(-v1 / TWO48)
        if abs(z0 * z0 + z1 * z1 - r2) > 1e-13 * max(1.0, r2):
            failed.append("identity")
    # closed form: u1 = 1 - e^-1/2 gives r = 1; u1 = 1 - e^-2 gives r = 2
    for target in (1.0, 2.0):
        v1 = round((1.0 - math.exp(-target * target / 2.0)) * TWO48)
        if abs(radius(v1) - target) > 1e-12:
            failed.append(f"r={target}")
        if abs(bm(v1, 0, 0) - target) > 1e-12:
            failed.append(f"z(r={target})")
    return sorted(set(failed))


def test_box_muller_pins():
    assert check_pins(G.box_muller, G.radius) == []


def test_radius_extremes():
    # largest radius: u1 = 1 - 2^-48, r = sqrt(96 ln 2)
    assert G.radius(TWO48 - 1) == pytest.approx(math.sqrt(96.0 * math.log(2.0)), rel=1e-15)
    assert G.radius(0) == 0.0
    assert G.radius(1) == pytest.approx(math.sqrt(2.0 / TWO48), rel=1e-12)


def test_planted_mistakes_are_caught():
    def half_angle(v1, v2, c):       # angle pi u2 instead of 2 pi u2
        r = G.radius(v1)
        a = math.pi * v2 / TWO48
        return r * (math.cos(a) if c == 0 else math.sin(a))

    def no_minus_two(v1, v2, c):     # r = sqrt(-ln(1 - u1))
        r = math.sqrt(-math.log1p(-v1 / TWO48))
        a = 2 * math.pi * v2 / TWO48
        return r * (math.cos(a) if c == 0 else math.sin(a))

    def swapped(v1, v2, c):          # sin for even, cos for odd
        return G.box_muller(v1, v2, 1 - c)

    def no_log(v1, v2, c):           # r = sqrt(2 u1)
        r = math.sqrt(2 * v1 / TWO48)
        a = 2 * math.pi * v2 / TWO48
        return r * (math.cos(a) if c == 0 else math.sin(a))

    for bm, rad in ((half_angle, G.radius),
                    (no_minus_two, lambda v: math.sqrt(-math.log1p(-v / TWO48))),
                    (swapped, G.radius),
                    (no_log, lambda v: math.sqrt(2 * v / TWO48))):
        assert check_pins(bm, rad), bm.__name__


def test_step_normals_use_aligned_pairs():
    x = O.seed(3, 2048)
    f = O.fields(x)
    z = G.step_normals(x)
    for k in range(12):
        assert z[k] == G.box_muller(f[k & ~1], f[k | 1], k & 1)
    # the pair (2i, 2i+1) shares its radius
    for i in range(6):
        assert z[2 * i] ** 2 + z[2 * i + 1] ** 2 == pytest.approx(G.radius(f[2 * i]) ** 2, rel=1e-14)


def test_normals_are_a_function_of_position():
    p = 218
    x = O.seed(11, p)
    whole, xe, pe = G.normals(x, 0, p, 61)
    # any split point continues with identical values and the same end state
    for cut in (1, 5, 12, 13, 30):
        a, x1, p1 = G.normals(x, 0, p, cut)
        b, x2, p2 = G.normals(x1, p1, p, 61 - cut)
        assert a + b == whole and (x2, p2) == (xe, pe)
    # and the same positions as the uniform draws
    _, xu, pu = O.draws(x, 0, p, 61)
    assert (xu, pu) == (xe, pe)


def test_normal_distribution():
    # 6000 normals from 500 seeded streams: Kolmogorov-Smirnov against N(0, 1)
    z = []
    for sid in range(500):
        z += G.step_normals(O.seed(sid, 2048))
    z = np.asarray(z)
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the pairs are independent: correlation of (z_2i, z_2i+1) is small
    c = np.corrcoef(z[0::2], z[1::2])[0, 1]
    assert abs(c) < 5.0 / math.sqrt(z.size / 2)
