// rlx_arith.hpp -- 576-bit modular arithmetic of RANLUX++ for gfx950 (used by
// librlx.so and by the device-side engine of rlx_engine.h).
//
// Numbers below 2^576 are held as eighteen 32-bit words, least significant
// first.  The modulus is m = 2^576 - 2^240 + 1 (paper, section 2.2).  Two
// multiplications modulo m exist:
//
//  * mulmod_generic(x, y): the full 576 x 576 -> 1152-bit product (section
//    2.1) followed by a reduction that uses only additions, subtractions and
//    shifts and ends with the fix that makes the result smaller than m
//    (section 2.2).  Used for seeding, skipping and table construction, where
//    the multiplier differs per lane.
//
//  * step(): the generator step X <- A X mod m for a multiplier A that is the
//    same for the whole launch.  The reduction is folded into a constant
//    table: C_j = A 2^(o_j) mod m (j < 21), so that with X split into 21
//    limbs l_j of w_j bits at bit offsets o_j, A X = sum_j l_j C_j (mod m).
//    The widths are ten of 28 bits, ten of 27 and one of 26 (576 in all);
//    since sum_j 2^(w_j) <= 2^32, every column sum of products
//    l_j * C_j[k] (32-bit words C_j[k]) stays below 2^64, so the product is
//    378 v_mad_u64_u32 with no carry handling.  One 32-bit word remains
//    above 2^576 and is folded with 2^576 = 2^240 - 1 (mod m).
//
// Both end in the canonical residue.  Rare carries, borrows and the final
// comparison with m take a general branch that is exact for every input; the
// common case is a short straight-line path.  `force_general` sends every
// lane through the general code (used by tests).
//
// The conversion to RANLUX numbers (section 2.3) uses
//   D = floor(X 2^576 / m) = X + q0 - delta,   q0 = floor(X / 2^336),
// where, with D' = X + q0, delta = 1 exactly when D' m > X 2^576, i.e. when
// D' > u 2^240 for u = (X mod 2^336) + q0.  If u >= 2^336 then delta = 0;
// otherwise u = D' mod 2^336 and delta = 1 iff floor(D' / 2^240) > D' mod
// 2^336, or they are equal and D' mod 2^240 != 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RLX_HD __host__ __device__ __forceinline__

namespace rlx {

constexpr int NW = 18;        // 32-bit words of a 576-bit number
constexpr int NL = 21;        // limbs of X in the constant-multiplier step

// width and bit offset of limb j: ten 28-bit, ten 27-bit, one 26-bit limb
RLX_HD constexpr int limb_bits(int j) { return j < 10 ? 28 : (j < 20 ? 27 : 26); }
RLX_HD constexpr int limb_offset(int j) { return j <= 10 ? 28 * j : 280 + 27 * (j - 10); }
static_assert(limb_offset(NL - 1) + limb_bits(NL - 1) == 576, "limbs cover 576 bits");

// m = 2^576 - 2^240 + 1
RLX_HD uint32_t m_word(int k) {
  return k == 0 ? 1u : (k < 7 ? 0u : (k == 7 ? 0xFFFF0000u : 0xFFFFFFFFu));
}

// ---------------------------------------------------------------------------
// word helpers

// a + b + c with carry c in {0, 1} (add-with-carry chains)
RLX_HD uint32_t addc(uint32_t a, uint32_t b, uint32_t& c) {
  unsigned int co;
  const uint32_t r = __builtin_addc(a, b, c, &co);
  c = co;
  return r;
}

// a - b - br with borrow br in {0, 1}
RLX_HD uint32_t subb(uint32_t a, uint32_t b, uint32_t& br) {
  unsigned int bo;
  const uint32_t r = __builtin_subc(a, b, br, &bo);
  br = bo;
  return r;
}

// bits [32 i + s, 32 i + s + 32) of the number w (s in 0..31), reading zeros
// above word n-1.
template <int N>
RLX_HD uint32_t window32(const uint32_t (&w)[N], int i, int s) {
  uint32_t lo = (i < N) ? w[i] : 0u;
  if (s == 0) return lo;
  uint32_t hi = (i + 1 < N) ? w[i + 1] : 0u;
  return (lo >> s) | (hi << (32 - s));
}

// x >= m for a number x < 2^576 held in NW words.
RLX_HD bool geq_m(const uint32_t (&x)[NW]) {
  uint32_t br = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) (void)subb(x[k], m_word(k), br);
  return br == 0;
}

// x <- x - m if x >= m (x < 2^576 < 2m, so one subtraction suffices).
RLX_HD void canonicalize(uint32_t (&x)[NW]) {
  uint32_t r[NW];
  uint32_t br = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) r[k] = subb(x[k], m_word(k), br);
  const bool ge = (br == 0);
#pragma unroll
  for (int k = 0; k < NW; ++k) x[k] = ge ? r[k] : x[k];
}

// x <- x + h 2^240 - h (mod m) for x < 2^576 and h < 2^32, exact and
// canonical: the value x + h (2^240 - 1) is non-negative and below
// 2^576 + 2^272; an overflow above 2^576 is folded once more.
RLX_HD void fold_word_general(uint32_t (&x)[NW], uint32_t h) {
  // t = x + (h << 16) at word 7 - h at word 0, as a signed running sum
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    int64_t add = 0;
    if (k == 7) add = (int64_t)(uint64_t)(h << 16);
    if (k == 8) add = (int64_t)(h >> 16);
    if (k == 0) add = -(int64_t)h;
    acc += (int64_t)x[k] + add;
    x[k] = (uint32_t)acc;
    acc >>= 32;  // arithmetic: carry in {-1, 0, 1}
  }
  // the sum is >= 0, so the final carry is 0 or 1
  uint32_t top = (uint32_t)acc;
  // x + top 2^576 = x + top (2^240 - 1) (mod m); when top = 1, x < 2^272 here
  // and no further overflow occurs.  2^240 enters as 2^16 at word 7.
  uint32_t c = top << 16;
#pragma unroll
  for (int k = 7; k < NW; ++k) x[k] = addc(x[k], 0u, c);
  uint32_t br = top;
#pragma unroll
  for (int k = 0; k < NW; ++k) x[k] = subb(x[k], 0u, br);
  canonicalize(x);
}

// ---------------------------------------------------------------------------
// generic multiplication modulo m (sections 2.1, 2.2)

// p = x * y, 36 words.  Both factors are split into 21 digits of 28 bits
// (the top one 16 bits).  A digit product is below 2^56 and a column holds
// at most 21 of them, so a column plus the carry from below stays under
// 2^61: each column is one chain of multiply-adds into a 64-bit accumulator
// that starts from the previous column's carry, with no carry handling
// inside the chain.  The 41 product digits (28 bits each) are then packed
// into 32-bit words.
constexpr int GD = 21;  // 28-bit digits of a 576-bit number

template <int N>
RLX_HD void digits28(const uint32_t (&w)[N], uint32_t (&d)[GD]) {
#pragma unroll
  for (int j = 0; j < GD; ++j) d[j] = window32(w, (28 * j) >> 5, (28 * j) & 31) & 0x0FFFFFFFu;
}

RLX_HD void mul576(const uint32_t (&x)[NW], const uint32_t (&y)[NW], uint32_t (&p)[2 * NW]) {
  uint32_t a[GD], b[GD];
  digits28(x, a);
  digits28(y, b);
  uint32_t d[2 * GD];  // product digits, base 2^28
  uint64_t acc = 0;
#pragma unroll
  for (int c = 0; c < 2 * GD - 1; ++c) {
    const int ilo = c < GD ? 0 : c - GD + 1;
    const int ihi = c < GD ? c : GD - 1;
#pragma unroll
    for (int i = ilo; i <= ihi; ++i) acc += (uint64_t)a[i] * b[c - i];
    d[c] = (uint32_t)acc & 0x0FFFFFFFu;
    acc >>= 28;
  }
  d[2 * GD - 1] = (uint32_t)acc;
  // word k = bits [32 k, 32 k + 32): digits floor(32 k / 28) and up
#pragma unroll
  for (int k = 0; k < 2 * NW; ++k) {
    const int c = (32 * k) / 28;
    const int s = (32 * k) % 28;
    uint32_t v = d[c] >> s;
    if (c + 1 < 2 * GD) v |= d[c + 1] << (28 - s);
    if (c + 2 < 2 * GD && 56 - s < 32) v |= d[c + 2] << (56 - s);
    p[k] = v;
  }
}

// r = p mod m for p < 2^1152 (36 words).  With L = p mod 2^576 and
// H = p >> 576:  p = L + H 2^240 - H (mod m), applied until the value fits
// in 576 bits, then the final comparison with m.  Each fold is an add-with-
// carry chain (adding H 2^240, i.e. H << 16 from word 7 on) followed by a
// subtract-with-borrow chain; every intermediate is non-negative.
RLX_HD void mod_m(const uint32_t (&p)[2 * NW], uint32_t (&r)[NW]) {
  // T1 = L + H 2^240 - H  (>= 0, < 2^817): 26 words
  uint32_t t1[26];
  {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 26; ++k) {
      const uint32_t l = k < NW ? p[k] : 0u;
      uint32_t hs = 0;  // word k of H << 240
      if (k >= 7) {
        const uint32_t hi = (k - 7 < NW) ? p[NW + k - 7] : 0u;
        const uint32_t lo = (k >= 8 && k - 8 < NW) ? p[NW + k - 8] : 0u;
        hs = (hi << 16) | (lo >> 16);
      }
      t1[k] = k < 7 ? l : addc(l, hs, c);
    }
    uint32_t br = 0;
#pragma unroll
    for (int k = 0; k < 26; ++k) t1[k] = subb(t1[k], k < NW ? p[NW + k] : 0u, br);
  }
  // T2 = T1 mod 2^576 + T1hi 2^240 - T1hi, T1hi = words 18..25 (< 2^241):
  // below 2^577, with the bit above 2^576 in t
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    uint32_t hs = 0;  // word k of T1hi << 240
    if (k >= 7) {
      const uint32_t hi = (k - 7 < 8) ? t1[NW + k - 7] : 0u;
      const uint32_t lo = (k >= 8 && k - 8 < 8) ? t1[NW + k - 8] : 0u;
      hs = (hi << 16) | (lo >> 16);
    }
    r[k] = k < 7 ? t1[k] : addc(t1[k], hs, c);
  }
  uint32_t br = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) r[k] = subb(r[k], k < 8 ? t1[NW + k] : 0u, br);
  const uint32_t t = c - br;  // T2 >= 0, so the borrow never exceeds the carry
  // T3 = T2 mod 2^576 + t (2^240 - 1); when t = 1, T2 mod 2^576 < 2^482, so
  // no further overflow; then < m
  {
    uint32_t cy = t << 16;
#pragma unroll
    for (int k = 7; k < NW; ++k) r[k] = addc(r[k], 0u, cy);
    uint32_t b2 = t;
#pragma unroll
    for (int k = 0; k < NW; ++k) r[k] = subb(r[k], 0u, b2);
  }
  canonicalize(r);
}

RLX_HD void mulmod_generic(const uint32_t (&x)[NW], const uint32_t (&y)[NW], uint32_t (&r)[NW]) {
  uint32_t p[2 * NW];
  mul576(x, y, p);
  mod_m(p, r);
}

// ---------------------------------------------------------------------------
// the generator step with a launch-uniform multiplier

// The 21 limbs of X (widths limb_bits, offsets limb_offset).
RLX_HD void unpack_limbs(const uint32_t (&w)[NW], uint32_t (&l)[NL]) {
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int bit = limb_offset(j);
    l[j] = window32(w, bit >> 5, bit & 31) & ((1u << limb_bits(j)) - 1u);
  }
}

// Row-offset barrier for the generator step: an empty asm that claims to
// modify the (scalar) offset using a word `dep` of the previous row, so the
// table load using the offset cannot move above the arrival of that row.
struct SgprBarrier {
  __device__ __forceinline__ uint32_t operator()(uint32_t v, uint32_t dep) const {
    asm volatile("" : "+s"(v) : "s"(dep));
    return v;
  }
};

// Table words seen through the constant address space: the compiler may
// then read them with scalar loads (it treats the memory as unchanging for
// the whole launch), even when the table address itself was loaded from
// device memory.
typedef const __attribute__((address_space(4))) uint32_t const_u32;

__device__ __forceinline__ const_u32* constant_table(const uint32_t* p) {
  return (const_u32*)p;
}

// Identity map of a table offset; kernels pass one that hides the offset
// from the optimiser (see step()).
struct Plain {
  RLX_HD uint32_t operator()(uint32_t v, uint32_t) const { return v; }
};

// X <- A X mod m.  `tab` holds C_j = A 2^(o_j) mod m, row j = 18 words
// (kernels pass a pointer into the read-only constant address space, so the
// rows are fetched with scalar loads).  Returns through `x` the canonical
// residue.
template <class Launder = Plain, class TabPtr = const uint32_t*>
RLX_HD void step(uint32_t (&x)[NW], TabPtr tab, bool force_general, Launder launder = Launder()) {
  uint32_t l[NL];
  unpack_limbs(x, l);
  uint64_t s[NW];
  // Rows of the table are read with scalar loads one row ahead of the
  // multiply-adds that use them.  Scalar loads complete out of order, so a
  // wave can only wait for all of them; the load of row j + 1 must therefore
  // be issued after the wait for row j and before row j's multiply-adds.  On
  // the GPU `launder` makes the row offset opaque and ties it to a word of
  // the previous row, which enforces exactly that order (and keeps the
  // compiler from hoisting all 396 words into scalar registers at once).
  uint32_t cur[NW];
  {
    const TabPtr row = tab + launder(0u, 0u);
#pragma unroll
    for (int k = 0; k < NW; ++k) cur[k] = row[k];
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    uint32_t nxt[NW];
    if (j + 1 < NL) {
      const TabPtr row = tab + launder((uint32_t)((j + 1) * NW), cur[0]);
#pragma unroll
      for (int k = 0; k < NW; ++k) nxt[k] = row[k];
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const uint64_t prod = (uint64_t)l[j] * cur[k];
      s[k] = j == 0 ? prod : s[k] + prod;
    }
    if (j + 1 < NL) {
#pragma unroll
      for (int k = 0; k < NW; ++k) cur[k] = nxt[k];
    }
  }
  // carry-normalise to 18 words plus the word h above 2^576.  The carry is
  // added as c * one + s[k] with an opaque one, which is a single
  // multiply-add (no zero-extension of c into a register pair).
  const uint32_t one = launder(1u, 0u);
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint64_t v = (uint64_t)c * one + s[k];
    x[k] = (uint32_t)v;
    c = (uint32_t)(v >> 32);
  }
  const uint32_t h = c;
  // fast fold in place: x - h at words 0-1, x + (h << 16) at words 7-9
  const uint32_t w0 = x[0], w1 = x[1], w7 = x[7], w8 = x[8], w9 = x[9];
  uint32_t br = 0;
  x[0] = subb(w0, h, br);
  x[1] = subb(w1, 0u, br);
  uint32_t cy = 0;
  x[7] = addc(w7, h << 16, cy);
  x[8] = addc(w8, h >> 16, cy);
  x[9] = addc(w9, 0u, cy);
  // rare: a borrow or carry that runs further, or a result that may be >= m
  const bool rare = (br | cy) != 0 || x[17] == 0xFFFFFFFFu || force_general;
  if (rare) {
    x[0] = w0; x[1] = w1; x[7] = w7; x[8] = w8; x[9] = w9;
    fold_word_general(x, h);
  }
}

// ---------------------------------------------------------------------------
// conversion to RANLUX numbers (section 2.3)

// d = floor(X 2^576 / m) for canonical X (the 24 RANLUX numbers, oldest in
// the least significant 24 bits).
RLX_HD void to_ranlux_general(const uint32_t (&x)[NW], uint32_t (&d)[NW]) {
  // q0 = X >> 336 (240 bits, 8 words), D' = X + q0
  uint32_t q[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) q[i] = window32(x, 10 + i, 16);
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) d[k] = addc(x[k], k < 8 ? q[k] : 0u, c);
  // e = carry out of bit 336 in (X mod 2^336) + q0
  uint32_t c2 = 0;
  uint32_t top = 0;
#pragma unroll
  for (int k = 0; k < 11; ++k) {
    uint32_t xv = (k < 10) ? x[k] : (x[10] & 0xFFFFu);
    top = addc(xv, k < 8 ? q[k] : 0u, c2);
  }
  const uint32_t e = (top >> 16) & 1u;
  // hi = D' >> 240 and lo = D' mod 2^336 (11 words each); z = [D' mod 2^240 == 0]
  uint32_t zacc = 0;
#pragma unroll
  for (int k = 0; k < 7; ++k) zacc |= d[k];
  zacc |= d[7] & 0xFFFFu;
  uint32_t br = (zacc == 0) ? 1u : 0u;
#pragma unroll
  for (int k = 0; k < 11; ++k) {
    uint32_t hi = window32(d, 7 + k, 16);
    uint32_t lo = (k < 10) ? d[k] : (d[10] & 0xFFFFu);
    (void)subb(hi, lo, br);
  }
  const uint32_t delta = (e == 0 && br == 0) ? 1u : 0u;
  uint32_t b2 = delta;
#pragma unroll
  for (int k = 0; k < NW; ++k) d[k] = subb(d[k], 0u, b2);
}

// Fast path of the conversion: writes words 0..8 of D into dlo (words 9..17
// of D equal those of X) and returns false, or returns true when the general
// code must be used (rare, or force_general).  The fast path applies when the
// carry of X + q0 stops by word 8, the top 32 bits of D' >> 240 and D' mod
// 2^336 differ, and subtracting delta does not borrow past word 0.
RLX_HD bool to_ranlux_fast(const uint32_t (&x)[NW], uint32_t (&dlo)[9], bool force_general) {
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) dlo[k] = addc(x[k], window32(x, 10 + k, 16), c);
  dlo[8] = addc(x[8], 0u, c);
  const uint32_t hi32 = x[17];
  const uint32_t lo32 = window32(x, 9, 16);
  const uint32_t delta = hi32 > lo32 ? 1u : 0u;
  const bool rare = c != 0 || hi32 == lo32 || (delta != 0 && dlo[0] == 0) || force_general;
  dlo[0] -= delta;
  return rare;
}

RLX_HD void to_ranlux(const uint32_t (&x)[NW], uint32_t (&d)[NW], bool force_general) {
  uint32_t dlo[9];
  if (to_ranlux_fast(x, dlo, force_general)) {
    to_ranlux_general(x, d);
  } else {
#pragma unroll
    for (int k = 0; k < NW; ++k) d[k] = k < 9 ? dlo[k] : x[k];
  }
}

// RANLUX carry bit c = X - D + floor(D / 2^336) (0 or 1) for canonical X and
// D = to_ranlux(X).
RLX_HD uint32_t ranlux_carry(const uint32_t (&x)[NW], const uint32_t (&d)[NW]) {
  // X - D + (D >> 336) is 0 or 1: only the lowest word matters once the
  // value is known to be that small.
  uint32_t lo = x[0] - d[0] + window32(d, 10, 16);
  return lo;
}

// X = D - floor(D / 2^336) + c: the inverse of the conversion (D, c) =
// (to_ranlux(X), ranlux_carry(X, D)) on canonical X (the relation behind
// both is 2^576 = m + 2^240 - 1, section 2.3).  Returns false when the
// result leaves [0, 2^576) (a borrow or a carry out), which happens only for
// pairs (D, c) that no canonical X exports to; the caller still has to check
// X < m and the round trip when (D, c) comes from outside.
RLX_HD bool from_ranlux(const uint32_t (&d)[NW], uint32_t c, uint32_t (&x)[NW]) {
  uint32_t br = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) x[k] = subb(d[k], window32(d, 10 + k, 16), br);
  uint32_t cy = c > 1u ? 2u : c;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint64_t v = (uint64_t)x[k] + cy;
    x[k] = (uint32_t)v;
    cy = (uint32_t)(v >> 32);
  }
  return br == 0 && cy == 0;
}

// ---------------------------------------------------------------------------
// 48-bit fields (section 2.3)
//
// Field k of D is bits [48k, 48k + 48): with i = k / 2 it lies in words
// w0 = D[3i], w1 = D[3i + 1], w2 = D[3i + 2] -- the low 48 bits of (w1:w0)
// for even k, bits 16..63 of (w2:w1) for odd k.

// funnel shift: bits [s, s + 32) of (hi:lo)
RLX_HD uint32_t funnel(uint32_t hi, uint32_t lo, int s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
}

RLX_HD uint64_t field_u64_w(uint32_t w0, uint32_t w1, uint32_t w2, int k) {
  if ((k & 1) == 0) return ((uint64_t)(w1 & 0xFFFFu) << 32) | w0;
  return ((uint64_t)(w2 >> 16) << 32) | funnel(w2, w1, 16);
}

// v 2^-48 for the 48-bit field v, as the bits of 1 + v 2^-48 (v in the top 48
// of the 52 mantissa bits) minus 1.0, which is exact.
RLX_HD double field_f64_w(uint32_t w0, uint32_t w1, uint32_t w2, int k) {
  uint32_t blo, bhi;
  if ((k & 1) == 0) {
    blo = w0 << 4;
    bhi = funnel((w1 & 0xFFFFu) | 0x3FF0000u, w0, 28);
  } else {
    blo = funnel(w2, w1, 12) & 0xFFFFFFF0u;
    bhi = funnel(0x3FFu, w2, 12);
  }
  const uint64_t bits = ((uint64_t)bhi << 32) | blo;
  double one_plus;
  __builtin_memcpy(&one_plus, &bits, 8);
  return one_plus - 1.0;
}

RLX_HD uint64_t field_u64(const uint32_t (&d)[NW], int k) {
  const int i = k >> 1;
  return field_u64_w(d[3 * i], d[3 * i + 1], d[3 * i + 2], k);
}

RLX_HD double field_f64(const uint32_t (&d)[NW], int k) {
  const int i = k >> 1;
  return field_f64_w(d[3 * i], d[3 * i + 1], d[3 * i + 2], k);
}

}  // namespace rlx
