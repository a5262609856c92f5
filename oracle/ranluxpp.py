"""Plain CPU oracle for the RANLUX++ generator (Hahnfeld & Moneta, "A Portable
Implementation of RANLUX++", arXiv 2106.02504).

TEST INFRASTRUCTURE ONLY.  This module is the correctness authority against
which the GPU library is checked bit for bit.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product path
never does.  It shares no code, tables or constants with the HIP library.

Everything here is the plain mathematical definition written with Python's
arbitrary-precision integers (``*``, ``%``, ``//`` and ``pow``), slow and
obviously correct:

* the LCG form of RANLUX: state X in [0, m), m = 2^576 - 2^240 + 1 (paper
  section 2.2), one generator step X <- a^p X mod m where a is the LCG
  multiplier equivalent to one subtract-with-borrow (SWB) step (section 1,
  the equivalence due to Sibidanov, and luxury level p);
* the SWB recurrence itself, for cross-checks (section 1);
* conversion of X back to 24 base-2^24 RANLUX numbers plus carry and the
  inverse (section 2 and 2.3);
* 48-bit fields per double, 12 per generator step (section 2.3);
* seeding and skipping by exponentiation (section 2.4).

Readings where the paper is silent are listed in the functions below (field
order, seeding exponent, eager advance); each is a stated choice, not a
derivation from the paper's text.
"""

from __future__ import annotations

# --- the RANLUX parameters (section 2.2; SWB lags r = 24, s = 10, base 2^24) --

BBITS = 24                      # bits per RANLUX number
B = 1 << BBITS                  # base b
R = 24                          # long lag r: RANLUX numbers in one state
S = 10                          # short lag s
NBITS = BBITS * R               # 576: width of the LCG state
M = B ** R - B ** S + 1         # modulus m = 2^576 - 2^240 + 1 (section 2.2)
A = M - (M - 1) // B            # multiplier a = b^-1 mod m: one SWB step
FIELD_BITS = 48                 # bits per double (section 2.3)
FIELDS = NBITS // FIELD_BITS    # 12 doubles per generator step
FIELD_MASK = (1 << FIELD_BITS) - 1
SEED_SHIFT = 96                 # seed id advances the stream by 2^96 steps
LIMBS = 9                       # uint64_t[9] state words (section 2)


class SwbParams:
    """A subtract-with-borrow generator x_n = x_{n-s} - x_{n-r} - c_{n-1} mod b
    with base b = 2^bbits and its LCG form: modulus m = b^r - b^s + 1 and
    multiplier a = m - (m - 1)/b (the inverse of b mod m).  RANLUX is
    (24, 24, 10); small instances exist so that tests can enumerate every
    state (section 1)."""

    def __init__(self, bbits: int, r: int, s: int):
        assert 0 < s < r
        self.bbits, self.r, self.s = bbits, r, s
        self.b = 1 << bbits
        self.m = self.b ** r - self.b ** s + 1
        self.a = self.m - (self.m - 1) // self.b
        self.width = bbits * r                # bits of the packed numbers
        self.qshift = bbits * (r - s)         # position of the top s numbers

    # -- LCG state X  <->  packed SWB state (D, carry) -------------------------
    def to_ranlux(self, x: int) -> tuple[int, int]:
        """X in [0, m) -> (D, carry).  D = floor(X * b^r / m) holds the r most
        recent SWB numbers as the first r base-b digits of X/m: the newest
        number is the most significant digit, the oldest the least.  The
        carry follows from inverting to_lcg."""
        assert 0 <= x < self.m
        d = (x << self.width) // self.m
        carry = x - d + (d >> self.qshift)
        return d, carry

    def to_lcg(self, d: int, carry: int) -> int:
        """(D, carry) -> X = D - floor(D / b^(r-s)) + carry, the LCG state of
        an SWB state (inverse of to_ranlux on canonical states)."""
        return d - (d >> self.qshift) + carry

    # -- the SWB recurrence itself ---------------------------------------------
    def digits(self, d: int) -> list[int]:
        """Packed D -> list of r numbers, oldest first."""
        return [(d >> (self.bbits * j)) & (self.b - 1) for j in range(self.r)]

    def pack(self, digits: list[int]) -> int:
        return sum(v << (self.bbits * j) for j, v in enumerate(digits))

    def swb_step(self, d: int, carry: int) -> tuple[int, int]:
        """One SWB step on a packed state: the new number is
        x_n = x_{n-s} - x_{n-r} - c_{n-1} mod b with borrow c_n; it becomes the
        newest (most significant) digit and the oldest digit drops out."""
        xs = self.digits(d)                   # xs[r-1] = x_{n-1}, xs[0] = x_{n-r}
        v = xs[self.r - self.s] - xs[0] - carry
        c_new = 1 if v < 0 else 0
        return self.pack(xs[1:] + [v % self.b]), c_new

    def swb_steps(self, d: int, carry: int, k: int) -> tuple[int, int]:
        for _ in range(k):
            d, carry = self.swb_step(d, carry)
        return d, carry


RANLUX = SwbParams(BBITS, R, S)


# --- 576-bit modular arithmetic (sections 2.1 and 2.2) ------------------------

def mulmod(x: int, y: int) -> int:
    """(x * y) mod m, the canonical residue in [0, m): the product of two
    576-bit numbers (section 2.1) reduced modulo m (section 2.2), whose
    final correction always leaves a residue below m."""
    return (x * y) % M


def multiplier(p: int) -> int:
    """A_p = a^p mod m: one generator step at luxury level p equals p SWB
    steps (section 1)."""
    if p < R:
        raise ValueError("luxury level p must be >= 24")
    return pow(A, p, M)


def seed_multiplier(p: int) -> int:
    """B_p = A_p^(2^96) mod m, the factor between consecutive seeds."""
    return pow(multiplier(p), 1 << SEED_SHIFT, M)


def seed(stream_id: int, p: int) -> int:
    """LCG state of stream `stream_id` at draw position 0: X = A_p^(2^96 id)
    applied to X = 1 (section 2.4 seeds by exponentiation; the 2^96 spacing is
    the reading taken here).  Seed 0 is X = 1."""
    if stream_id < 0:
        raise ValueError("stream id must be >= 0")
    return pow(multiplier(p), stream_id << SEED_SHIFT, M)


def skip(x: int, k: int, p: int) -> int:
    """Advance an LCG state by k generator steps without generating:
    X <- A_p^k X mod m (section 2.4)."""
    if k < 0:
        raise ValueError("skip count must be >= 0")
    return mulmod(pow(multiplier(p), k, M), x)


# --- RANLUX numbers and doubles (section 2.3) ---------------------------------

def to_ranlux(x: int) -> tuple[list[int], int]:
    """X -> (24 RANLUX numbers oldest first, carry)."""
    d, carry = RANLUX.to_ranlux(x)
    return RANLUX.digits(d), carry


def to_lcg(numbers: list[int], carry: int) -> int:
    """(24 RANLUX numbers oldest first, carry) -> X."""
    return RANLUX.to_lcg(RANLUX.pack(numbers), carry)


def fields(x: int) -> list[int]:
    """The 12 48-bit values of one generator step.  Field k is bits
    [48k, 48k+48) of the packed RANLUX numbers D = floor(X 2^576 / m), i.e.
    numbers 2k (low half) and 2k+1 (high half), oldest pair first.  The
    paper fixes 48 bits per double but not their order; this is the reading
    taken here."""
    d, _ = RANLUX.to_ranlux(x)
    return [(d >> (FIELD_BITS * k)) & FIELD_MASK for k in range(FIELDS)]


def field_to_double(v: int) -> float:
    """48-bit value -> double in [0, 1): v * 2^-48 (exact in binary64)."""
    return v * 2.0 ** -FIELD_BITS


# --- a stream: LCG state plus position (sections 2 and 2.3) -------------------

def draws(x: int, pos: int, p: int, n: int) -> tuple[list[int], int, int]:
    """Take n 48-bit values from the stream whose current step is X with
    `pos` fields already used; return (values, X', pos').

    The state is kept in canonical eager form: pos in [0, 11], and the step
    is advanced as soon as its 12th field is used, so (X, pos) is a unique
    function of the absolute draw position.  Values of one step are used
    before the generator advances (section 2.3)."""
    if not (0 <= pos < FIELDS):
        raise ValueError("pos must be in [0, 12)")
    if not (0 <= x < M):
        raise ValueError("state must be in [0, m)")
    a_p = multiplier(p)
    out: list[int] = []
    cur = fields(x)
    while len(out) < n:
        out.append(cur[pos])
        pos += 1
        if pos == FIELDS:
            x = mulmod(a_p, x)
            pos = 0
            cur = fields(x)
    return out, x, pos


def draws_f64(x: int, pos: int, p: int, n: int) -> tuple[list[float], int, int]:
    vals, x2, pos2 = draws(x, pos, p, n)
    return [field_to_double(v) for v in vals], x2, pos2


def state_at(x_seed: int, p: int, position: int) -> tuple[int, int]:
    """(X, pos) of a stream at absolute draw `position`, counted from the
    stream state X_seed at pos 0: X = A_p^floor(P/12) X_seed, pos = P mod 12."""
    steps, pos = divmod(position, FIELDS)
    return skip(x_seed, steps, p), pos


def window(x_seed: int, p: int, position: int, n: int) -> list[int]:
    """n draws starting at absolute `position` of the stream that starts at
    X_seed, reached by skipping rather than generating."""
    x, pos = state_at(x_seed, p, position)
    return draws(x, pos, p, n)[0]


# --- the in-memory state record -----------------------------------------------

def to_limbs(x: int) -> list[int]:
    """576-bit X -> nine 64-bit words, least significant first (the paper
    stores uint64_t[9]; the word order is the reading taken here)."""
    return [(x >> (64 * i)) & ((1 << 64) - 1) for i in range(LIMBS)]


def from_limbs(words) -> int:
    return sum(int(w) << (64 * i) for i, w in enumerate(words))


def state_record(x: int, pos: int, p: int) -> list[int]:
    """The 80-byte stream record as ten unsigned 64-bit words: x[0..8], then
    pos in the low and p in the high 32 bits of word 9."""
    return to_limbs(x) + [pos | (p << 32)]


def parse_record(words) -> tuple[int, int, int]:
    w = [int(v) & ((1 << 64) - 1) for v in words]
    return from_limbs(w[:LIMBS]), w[LIMBS] & 0xFFFFFFFF, w[LIMBS] >> 32
