"""Gaussian draws on top of the RANLUX++ uniforms -- CPU oracle.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never does.  It shares no code with the HIP library.

The paper leaves distributions to the framework around the engine (section
2.4 mentions ROOT's ``RandomFunctions`` on top of the engine's uniform draws)
and fixes no algorithm.  The reading taken here is the Box-Muller transform on
aligned pairs of 48-bit fields of one generator step:

* the normal at absolute stream position s uses the two fields of its pair,
  positions s & ~1 and s | 1 (a pair never straddles a step, 12 being even),
  with u1 = v1 2^-48 and u2 = v2 2^-48 in [0, 1);
* r = sqrt(-2 ln(1 - u1)) (1 - u1 lies in (0, 1], so r is finite), and the
  normal is r cos(2 pi u2) for even s and r sin(2 pi u2) for odd s.

So the n-th normal is a function of the stream position alone, and drawing n
normals consumes exactly n positions, like n uniforms.

The transform is evaluated with mpmath at 40 significant digits and rounded
once to the nearest binary64 value, so this oracle is accurate to half an ulp
of the result; a device implementation is compared with it under a tolerance
of a few ulp.
"""

from __future__ import annotations

import mpmath

from .ranluxpp import FIELD_BITS, FIELDS, M, fields, multiplier, mulmod

_DPS = 40


def box_muller(v1: int, v2: int, component: int) -> float:
    """Normal from the 48-bit field pair (v1, v2): r cos(2 pi u2) for
    component 0, r sin(2 pi u2) for component 1, r = sqrt(-2 ln(1 - u1))."""
    with mpmath.workdps(_DPS):
        scale = mpmath.mpf(2) ** -FIELD_BITS
        u1 = mpmath.mpf(v1) * scale
        u2 = mpmath.mpf(v2) * scale
        r = mpmath.sqrt(-2 * mpmath.log(1 - u1))
        angle = 2 * mpmath.pi * u2
        z = r * (mpmath.cos(angle) if component == 0 else mpmath.sin(angle))
        return float(z)


def radius(v1: int) -> float:
    """r = sqrt(-2 ln(1 - v1 2^-48)), rounded once to binary64."""
    with mpmath.workdps(_DPS):
        u1 = mpmath.mpf(v1) * mpmath.mpf(2) ** -FIELD_BITS
        return float(mpmath.sqrt(-2 * mpmath.log(1 - u1)))


def step_normals(x: int) -> list[float]:
    """The 12 normals of one generator step with state X."""
    f = fields(x)
    return [box_muller(f[k & ~1], f[k | 1], k & 1) for k in range(FIELDS)]


def normals(x: int, pos: int, p: int, n: int) -> tuple[list[float], int, int]:
    """n normals from the stream whose current step is X with `pos` positions
    used; returns (values, X', pos') with the same eager advance as the
    uniform draws."""
    if not (0 <= pos < FIELDS):
        raise ValueError("pos must be in [0, 12)")
    if not (0 <= x < M):
        raise ValueError("state must be in [0, m)")
    a_p = multiplier(p)
    out: list[float] = []
    cur = step_normals(x)
    while len(out) < n:
        out.append(cur[pos])
        pos += 1
        if pos == FIELDS:
            x = mulmod(a_p, x)
            pos = 0
            cur = step_normals(x)
    return out, x, pos
