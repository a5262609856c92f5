// rlx_device.hpp -- device helpers shared by the kernels of librlx.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlx.h"
#include "rlx_arith.hpp"
#include "rlx_gauss.hpp"

namespace rlx {

// Tables of one luxury level p (device memory owned by the library):
//   T[i][j] = A_p^(j 16^i) mod m, i < 40, j < 16 (18 words each): 4-bit
//             windows of a 160-bit exponent; rows 0..15 serve skips of
//             k < 2^64 steps, rows 24..39 seeds (exponent 2^96 id).  The
//             device-side engine uses T; the kernels use W below.
//   C[g][j] = A_p^(2^g) 2^(o_j) mod m, g < 64, j < 21 (o_j = limb_offset(j)): the folded
//             multiplier of a step by 2^g generator steps (see step()).
//   W[i][j] = A_p^(j 65536^i) mod m, i < 4, and W[4 + i][j] =
//             A_p^(2^96 j 65536^i) mod m, j < 65536 (37.7 MB): 16-bit windows
//             for skips of k < 2^64 steps and for seeds with ids < 2^64, each
//             entry the product of four entries of T (the kernels' own table;
//             the device-side engine of rlx_engine.h uses T).
constexpr int TAB_ROWS = RLX_TAB_ROWS;
constexpr int TAB_COLS = RLX_TAB_COLS;
constexpr int SEED_ROW0 = RLX_SEED_ROW0;  // 2^96 = 16^24
constexpr size_t TAB_WORDS = (size_t)TAB_ROWS * TAB_COLS * NW;
constexpr int FOLD_G = RLX_FOLD_G;
constexpr size_t FOLD_ROW_WORDS = (size_t)NL * NW;  // one folded multiplier
constexpr size_t FOLD_WORDS = (size_t)FOLD_G * FOLD_ROW_WORDS;
constexpr int WIN_BITS = 16;
constexpr int WIN_ROWS = RLX_WIN16_ROWS;
constexpr int WIN_COLS = RLX_WIN16_COLS;
constexpr int WIN_SEED_ROW0 = RLX_WIN16_SEED_ROW0;
static_assert(WIN_COLS == 1 << WIN_BITS, "16-bit windows");
constexpr size_t WIN_WORDS = (size_t)WIN_ROWS * WIN_COLS * NW;
constexpr int BLOCK = 256;
constexpr int FIELDS = 12;
constexpr int WAVE = 64;

// a = 2^576 - 2^552 - 2^240 + 2^216 + 1 = 2^-24 mod m: one subtract-with-
// borrow step of RANLUX (lags 24 and 10, base 2^24) as an LCG multiplier.
__device__ __forceinline__ uint32_t a_word(int k) {
  return k == 0 ? 1u
       : k < 6  ? 0u
       : k == 6 ? 0x01000000u
       : k == 7 ? 0xFFFF0000u
       : k < 17 ? 0xFFFFFFFFu
                : 0xFFFFFEFFu;
}

__device__ __forceinline__ void set_one(uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < NW; ++k) x[k] = k == 0 ? 1u : 0u;
}

__device__ __forceinline__ void load_words(const uint32_t* __restrict__ src, uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < NW; ++k) x[k] = src[k];
}

__device__ __forceinline__ void store_words(uint32_t* __restrict__ dst, const uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < NW; ++k) dst[k] = x[k];
}

__device__ __forceinline__ void copy_words(uint32_t (&dst)[NW], const uint32_t (&src)[NW]) {
#pragma unroll
  for (int k = 0; k < NW; ++k) dst[k] = src[k];
}

// record i: 80 bytes = five 16-byte vectors
__device__ __forceinline__ void load_record(const rlx_state* __restrict__ st, uint64_t i,
                                            uint32_t (&x)[NW], uint32_t& pos, uint32_t& p) {
  const uint4* r = reinterpret_cast<const uint4*>(st + i);
  uint4 v[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = r[q];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[4 * q + 0] = v[q].x; x[4 * q + 1] = v[q].y; x[4 * q + 2] = v[q].z; x[4 * q + 3] = v[q].w;
  }
  x[16] = v[4].x; x[17] = v[4].y;
  pos = v[4].z;
  p = v[4].w;
}

__device__ __forceinline__ void store_record(rlx_state* __restrict__ st, uint64_t i,
                                             const uint32_t (&x)[NW], uint32_t pos, uint32_t p) {
  uint4* r = reinterpret_cast<uint4*>(st + i);
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = make_uint4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
  r[4] = make_uint4(x[16], x[17], pos, p);
}

__device__ __forceinline__ uint32_t check_record(const uint32_t (&x)[NW], uint32_t pos, uint32_t sp,
                                                 uint32_t p) {
  uint32_t bad = 0;
  if (sp != p) bad |= RLX_ERR_BAD_P;
  if (pos > 11) bad |= RLX_ERR_BAD_POS;
  if (geq_m(x)) bad |= RLX_ERR_BAD_X;
  return bad;
}

__device__ __forceinline__ void mulmod_inplace(uint32_t (&x)[NW], const uint32_t (&y)[NW]) {
  uint32_t r[NW];
  mulmod_generic(x, y, r);
  copy_words(x, r);
}

// X <- A^e X by 16-bit windows: one generic multiplication per non-zero
// 16-bit digit of e by the table entry A^(v 65536^i) (rows 0..3 of W,
// section 2.4).  The lanes of a wave take different exponents, so the wave
// runs as many rounds as its longest exponent has digits (at most 4), each
// lane multiplying when its digit is non-zero.  Starting the lanes of a
// record this way (e = lane index, or the segment's first step plus the
// lane index) costs one per-lane multiplication for e < 65536.
__device__ __forceinline__ void skip_windows(uint32_t (&x)[NW], uint64_t e, const uint32_t* __restrict__ W) {
#pragma unroll 1
  for (int b = 0; b < 4 && __any((e >> (WIN_BITS * b)) != 0); ++b) {
    const uint32_t v = (uint32_t)(e >> (WIN_BITS * b)) & (WIN_COLS - 1u);
    if (v != 0) {
      uint32_t y[NW];
      load_words(W + ((size_t)b * WIN_COLS + v) * NW, y);
      mulmod_inplace(x, y);
    }
  }
}

// What a generate kernel writes for each position: the 48-bit integer, the
// double v 2^-48, a standard normal from the position's field pair, or the
// position's two RANLUX numbers as float32 (low number first).
enum class Out { U64, F64, NORMAL, F32 };

__device__ __forceinline__ double bits_to_f64(uint32_t lo, uint32_t hi) {
  const uint64_t b = ((uint64_t)hi << 32) | lo;
  double v;
  __builtin_memcpy(&v, &b, 8);
  return v;
}

__device__ __forceinline__ uint64_t f64_bits(double v) {
  uint64_t b;
  __builtin_memcpy(&b, &v, 8);
  return b;
}

// The doubles of the field pair held in words (w0, w1, w2) (fields 2i and
// 2i + 1 of a step: bits 0..47 and 48..95 of the three words), each v 2^-48.
// With v < 2^48, the bits 0x403 << 52 | v are the double 16 + v 2^-48 (v
// fills the low 48 mantissa bits as it is, no shift), and subtracting 16 is
// exact (both operands lie in [16, 32)).
__device__ __forceinline__ void pair_f64(uint32_t w0, uint32_t w1, uint32_t w2, double& u_even, double& u_odd) {
  const uint32_t e_hi = (w1 & 0xFFFFu) | 0x40300000u;
  const uint32_t o_lo = __builtin_amdgcn_alignbit(w2, w1, 16);
  const uint32_t o_hi = __builtin_amdgcn_alignbit(0x4030u, w2, 16);
  u_even = bits_to_f64(w0, e_hi) - 16.0;
  u_odd = bits_to_f64(o_lo, o_hi) - 16.0;
}

// A RANLUX number (24 bits) as the float v 2^-24: the conversion is exact
// for v < 2^24 and so is the power-of-two scaling.
__device__ __forceinline__ uint32_t number_f32_bits(uint32_t v) {
  const float f = (float)v * 0x1p-24f;
  uint32_t b;
  __builtin_memcpy(&b, &f, 4);
  return b;
}

// Both output values of the field pair held in words (w0, w1, w2).  For
// normals, Box-Muller on the pair (rlx_gauss.hpp): the even position gets
// r cos(2 pi u2) and the odd one r sin(2 pi u2), r = sqrt(-2 ln(1 - u1)).
// For float32 each position holds its two RANLUX numbers (bits 0..23 and
// 24..47 of the field), the older one in the low 32 bits, i.e. first in
// memory; the numbers that straddle a word are gathered by one byte
// permute each (selector byte 0x0C gives zero).
template <Out K>
__device__ __forceinline__ void pair_values(uint32_t w0, uint32_t w1, uint32_t w2, uint64_t& a, uint64_t& b) {
  if constexpr (K == Out::U64) {
    a = ((uint64_t)(w1 & 0xFFFFu) << 32) | w0;
    b = ((uint64_t)(w2 >> 16) << 32) | __builtin_amdgcn_alignbit(w2, w1, 16);
  } else if constexpr (K == Out::F32) {
    const uint32_t n0 = w0 & 0xFFFFFFu;
    const uint32_t n1 = __builtin_amdgcn_perm(w1, w0, 0x0C050403u);  // w0 byte 3, w1 bytes 0, 1
    const uint32_t n2 = __builtin_amdgcn_perm(w2, w1, 0x0C040302u);  // w1 bytes 2, 3, w2 byte 0
    const uint32_t n3 = w2 >> 8;
    a = ((uint64_t)number_f32_bits(n1) << 32) | number_f32_bits(n0);
    b = ((uint64_t)number_f32_bits(n3) << 32) | number_f32_bits(n2);
  } else {
    double u1, u2;
    if constexpr (K == Out::F64) {
      pair_f64(w0, w1, w2, u1, u2);
    } else {
      gauss::box_muller(w0, w1, w2, u1, u2);
    }
    a = f64_bits(u1);
    b = f64_bits(u2);
  }
}

// Values per lane of the LDS staging area: the 12 output values of one
// step, 16-byte aligned.
constexpr int SLOT_VALUES = FIELDS;

// Write the 12 output values of a step to an LDS slot from D's words 0..8
// in `lo` and 9..17 in `hi` (after the fast conversion hi is X itself).
template <Out K, int NLO>
__device__ __forceinline__ void write_values(const uint32_t (&lo)[NLO], const uint32_t (&hi)[NW],
                                             uint64_t* __restrict__ slot) {
  ulonglong2* s2 = reinterpret_cast<ulonglong2*>(slot);
#pragma unroll
  for (int i = 0; i < FIELDS / 2; ++i) {
    const uint32_t w0 = 3 * i < 9 ? lo[(3 * i) % NLO] : hi[3 * i];
    const uint32_t w1 = 3 * i + 1 < 9 ? lo[(3 * i + 1) % NLO] : hi[3 * i + 1];
    const uint32_t w2 = 3 * i + 2 < 9 ? lo[(3 * i + 2) % NLO] : hi[3 * i + 2];
    uint64_t a, b;
    pair_values<K>(w0, w1, w2, a, b);
    s2[i] = make_ulonglong2(a, b);
    // normals: one pair's transform is finished before the next begins, so
    // their temporaries never overlap (the staged generate kernel fits 128
    // VGPRs and 4 waves per SIMD; interleaving all six took 166 and 3)
    if constexpr (K == Out::NORMAL) __builtin_amdgcn_sched_barrier(0);
  }
}

// Convert X (section 2.3) and write the step's 12 output values to this
// lane's LDS slot.  The two branches write separately, so the common one
// reads X's words where they are instead of merging copies.  Per lane, no
// synchronisation: may run under divergent control flow.
template <Out K>
__device__ __forceinline__ void convert_to_lds(const uint32_t (&x)[NW], uint64_t* __restrict__ slot, bool force) {
  uint32_t dlo[9];
  if (!to_ranlux_fast(x, dlo, force)) {
    write_values<K>(dlo, x, slot);
  } else {
    uint32_t d[NW];
    to_ranlux_general(x, d);
    write_values<K>(d, d, slot);
  }
}

template <Out K>
__device__ __forceinline__ uint64_t field_bits(const uint32_t (&d)[NW], int f) {
  const int i = f >> 1;
  uint64_t a, b;
  pair_values<K>(d[3 * i], d[3 * i + 1], d[3 * i + 2], a, b);
  return (f & 1) ? b : a;
}

__device__ __forceinline__ void put_trace(uint64_t* __restrict__ tr, const uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) tr[k] = ((uint64_t)x[2 * k + 1] << 32) | x[2 * k];
}

// LDS writes of a wave become visible to the whole wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-byte store; non-temporal (no cache allocation: the output is written
// once and never read back by the kernel) when NT is set.  Non-temporal
// stores only pay off for whole 128-byte lines per instruction: partial
// lines written that way are merged late and cost far more bandwidth.
template <bool NT>
__device__ __forceinline__ void store_pair(uint64_t* dst, ulonglong2 v) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  u64x2 w;
  w.x = v.x;
  w.y = v.y;
  if constexpr (NT) {
    __builtin_nontemporal_store(w, reinterpret_cast<u64x2*>(dst));
  } else {
    *reinterpret_cast<u64x2*>(dst) = w;
  }
}

// Store the 12 values of this lane's block from LDS.
//
// The gs = 2^LGS lanes of a group (gs <= 64, aligned inside the wave) hold
// consecutive blocks; lane ls holds the group's block ls and has written its
// 12 values to its LDS slot (convert_to_lds), so the group's slots hold its
// 12 gs values in output order.  Value f of the group's block m goes to
// base[u0 + 12 m + f] when 0 <= u0 + 12 m + f < span.  Only lanes with
// `active` set store.  Called by every lane of the wave.
//
// When the group writes its whole window, the values go out as 16-byte
// pairs: lane ls stores pairs q gs + ls, q < 6, so one store instruction
// writes 16 gs contiguous bytes per group.  If the window starts 8 bytes off
// a 16-byte boundary (an odd output offset), the pairs are shifted by one
// value: lane 0 also stores value 0 alone and lane gs - 1 stores the last
// value alone in place of its last pair.  The stores are non-temporal only
// when a group's run is whole 128-byte lines (from gs = 8 on, on a line
// boundary): partial lines written that way are merged late and cost far
// more bandwidth.  Windows cut by the range take single range-checked
// stores.
template <int LGS>
__device__ __forceinline__ void group_store(const uint64_t* __restrict__ stage, uint32_t tid_blk, uint32_t ls,
                                            int64_t u0, uint64_t span, bool active,
                                            uint64_t* __restrict__ base) {
  constexpr uint32_t gs = 1u << LGS;
  wave_sync();
  const uint64_t* grp = stage + (size_t)(tid_blk - ls) * SLOT_VALUES;
  uint64_t* const gdst = base + u0;
  const uintptr_t a = reinterpret_cast<uintptr_t>(gdst);
  const bool whole = u0 >= 0 && (uint64_t)u0 + FIELDS * gs <= span;
  if (gs >= 8 && __all(active && whole && (a & 127) == 0)) {
    // the common case of a whole wave on line boundaries, as one branch: one
    // base address per lane, the six pairs at constant offsets from it
    const ulonglong2* g2 = reinterpret_cast<const ulonglong2*>(grp) + ls;
    uint64_t* const dst = gdst + 2 * ls;
#pragma unroll
    for (uint32_t q = 0; q < FIELDS / 2; ++q) store_pair<true>(dst + 2 * q * gs, g2[q * gs]);
  } else if (active) {
    if (whole) {
      if ((a & 15) == 0) {
        const ulonglong2* g2 = reinterpret_cast<const ulonglong2*>(grp) + ls;
        uint64_t* const dst = gdst + 2 * ls;
        if (gs >= 8 && (a & 127) == 0) {
#pragma unroll
          for (uint32_t q = 0; q < FIELDS / 2; ++q) store_pair<true>(dst + 2 * q * gs, g2[q * gs]);
        } else {
#pragma unroll
          for (uint32_t q = 0; q < FIELDS / 2; ++q) store_pair<false>(dst + 2 * q * gs, g2[q * gs]);
        }
      } else {
        // pairs k = (values 2k + 1, 2k + 2), k < 6 gs - 1, at 16-byte
        // aligned gdst + 2k + 1
        if (ls == 0) gdst[0] = grp[0];
        uint64_t* const dst = gdst + 2 * ls + 1;
        const uint64_t* const src = grp + 2 * ls + 1;
#pragma unroll
        for (uint32_t q = 0; q < FIELDS / 2; ++q) {
          if (q + 1 < FIELDS / 2 || ls + 1 < gs) {
            store_pair<false>(dst + 2 * q * gs, make_ulonglong2(src[2 * q * gs], src[2 * q * gs + 1]));
          } else {
            gdst[FIELDS * gs - 1] = grp[FIELDS * gs - 1];
          }
        }
      }
    } else {
      // running index (no loop-invariant per-q offsets for the compiler to
      // keep in registers): value q goes to base[u], stored when u < span
      uint64_t u = (uint64_t)(u0 + (int64_t)ls);
#pragma unroll
      for (int q = 0; q < FIELDS; ++q) {
        if (u < span) base[u] = grp[q * gs + ls];
        u += gs;
      }
    }
  }
  wave_sync();
}

}  // namespace rlx
