"""Other output widths of RANLUX++ (arXiv 2106.02504, section 2.3) -- CPU
oracle, TEST INFRASTRUCTURE ONLY (see ranluxpp.py for the rules).

Section 2.3 converts each generator step's LCG state back to the 24 RANLUX
numbers (24 bits each, equally distributed) and builds doubles from 48 bits.
Two other widths follow directly from that passage:

* float32 from single RANLUX numbers: each number v gives v * 2^-24, exact
  in binary32 (24-bit significand), 24 values per step, in the order the
  subtract-with-borrow recurrence produced them (oldest first).  The draw
  position of a stream record counts 48-bit fields, so floats come in pairs:
  field k gives numbers 2k and 2k + 1, and 2c floats use c positions.
* the earlier conversion the paper attributes to Sibidanov: 52 bits of the
  LCG state X itself as a double's mantissa.  The paper notes that it is
  biased (X < m < 2^576, so the top bits are 0 slightly more often) and does
  not use it; it is kept for comparison only.  The paper does not fix which
  52 bits; the reading taken here is bits [52k, 52k + 52) of X for
  k = 0..10, low bits first, 11 values per step (the top 4 bits unused), and
  a stream position counting those values (0..10 within a step).
"""

from __future__ import annotations

from .ranluxpp import BBITS, M, mulmod, multiplier, to_ranlux

NUM_MASK = (1 << BBITS) - 1
NUMBERS = 24                    # RANLUX numbers per step
LCG52_BITS = 52
LCG52_VALUES = 576 // LCG52_BITS   # 11 values per step
LCG52_MASK = (1 << LCG52_BITS) - 1


def number_to_f32(v: int) -> float:
    """A RANLUX number (24 bits) -> v * 2^-24 in [0, 1); representable
    exactly in binary32, so the Python float is the float32 value."""
    return v * 2.0 ** -BBITS


def draws_f32(x: int, pos: int, p: int, n: int) -> tuple[list[float], int, int]:
    """n (even) float32 values from the stream at (X, pos): the RANLUX numbers
    of each step oldest first, two per 48-bit position (section 2.3); returns
    (values, X', pos') with pos' = pos + n/2 positions, advanced eagerly as
    the 48-bit draws are."""
    if n % 2:
        raise ValueError("float32 draws come in pairs (one 48-bit position each)")
    if not (0 <= pos < 12) or not (0 <= x < M):
        raise ValueError("bad stream state")
    a_p = multiplier(p)
    out: list[float] = []
    nums, _ = to_ranlux(x)
    while len(out) < n:
        out.append(number_to_f32(nums[2 * pos]))
        out.append(number_to_f32(nums[2 * pos + 1]))
        pos += 1
        if pos == 12:
            x = mulmod(a_p, x)
            pos = 0
            nums, _ = to_ranlux(x)
    return out, x, pos


def lcg52_values(x: int) -> list[int]:
    """The 11 52-bit values of a step taken straight from the LCG state X
    (the legacy conversion, section 2.3): bits [52k, 52k + 52), low first."""
    return [(x >> (LCG52_BITS * k)) & LCG52_MASK for k in range(LCG52_VALUES)]


def lcg52_to_double(v: int) -> float:
    """52-bit value -> v * 2^-52 in [0, 1) (exact)."""
    return v * 2.0 ** -LCG52_BITS


def draws_lcg52(x: int, pos: int, p: int, n: int) -> tuple[list[float], int, int]:
    """n legacy doubles from the stream at (X, pos), pos in [0, 11) counting
    52-bit values of the current step; the step advances by A_p after its
    11th value (eagerly, as the 48-bit draws do)."""
    if not (0 <= pos < LCG52_VALUES) or not (0 <= x < M):
        raise ValueError("bad stream state")
    a_p = multiplier(p)
    out: list[float] = []
    cur = lcg52_values(x)
    while len(out) < n:
        out.append(lcg52_to_double(cur[pos]))
        pos += 1
        if pos == LCG52_VALUES:
            x = mulmod(a_p, x)
            pos = 0
            cur = lcg52_values(x)
    return out, x, pos
