// rlx_device.hpp -- device helpers shared by the kernels of librlx.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlx.h"
#include "rlx_arith.hpp"

namespace rlx {

// Tables of one luxury level p (device memory owned by the library):
//   T[i][j] = A_p^(j 16^i) mod m, i < 40, j < 16 (18 words each): 4-bit
//             windows of a 160-bit exponent; rows 0..15 serve skips of
//             k < 2^64 steps, rows 24..39 serve seeds (exponent 2^96 id).
//   C[g][j] = A_p^(2^g) 2^(o_j) mod m, g < 64, j < 21 (o_j = limb_offset(j)): the folded
//             multiplier of a step by 2^g generator steps (see step()).
constexpr int TAB_ROWS = 40;
constexpr int TAB_COLS = 16;
constexpr int SEED_ROW0 = 24;  // 2^96 = 16^24
constexpr size_t TAB_WORDS = (size_t)TAB_ROWS * TAB_COLS * NW;
constexpr int FOLD_G = 64;
constexpr size_t FOLD_ROW_WORDS = (size_t)NL * NW;  // one folded multiplier
constexpr size_t FOLD_WORDS = (size_t)FOLD_G * FOLD_ROW_WORDS;
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

__device__ __forceinline__ void mulmod_inplace(uint32_t (&x)[NW], const uint32_t (&y)[NW]) {
  uint32_t r[NW];
  mulmod_generic(x, y, r);
  copy_words(x, r);
}

// x <- A^e x for a per-lane exponent e < 2^64: one folded step by A^(2^g)
// for every set bit g of e.  The steps run in increasing g; a bit that no
// lane of the wave has set is skipped by the whole wave.
__device__ __forceinline__ void advance(uint32_t (&x)[NW], uint64_t e, const uint32_t* __restrict__ ctabs,
                                        bool force) {
#pragma unroll 1
  for (uint32_t g = 0; g < 64 && __any((e >> g) != 0); ++g) {
    const bool set = ((e >> g) & 1u) != 0;
    if (__any(set) && set) step(x, constant_table(ctabs + (size_t)g * FOLD_ROW_WORDS), force, SgprBarrier());
  }
}

template <bool F64>
__device__ __forceinline__ uint64_t field_bits_w(uint32_t w0, uint32_t w1, uint32_t w2, int k) {
  if (F64) {
    const double v = field_f64_w(w0, w1, w2, k);
    uint64_t b;
    __builtin_memcpy(&b, &v, 8);
    return b;
  }
  return field_u64_w(w0, w1, w2, k);
}

// Write the 12 fields of one step to this lane's LDS slot.  D's words 0..8
// are lo[0..8] and words 9..17 are hi[9..17] (after the fast conversion hi is
// X itself; after the general one both are D).  Per lane, no synchronisation:
// may run under divergent control flow.
template <bool F64, int NLO>
__device__ __forceinline__ void lds_fields(const uint32_t (&lo)[NLO], const uint32_t (&hi)[NW],
                                           uint64_t* __restrict__ slot) {
#pragma unroll
  for (int f = 0; f < FIELDS; f += 2) {
    const int i = f >> 1;
    const uint32_t w0 = 3 * i < 9 ? lo[(3 * i) % NLO] : hi[3 * i];
    const uint32_t w1 = 3 * i + 1 < 9 ? lo[(3 * i + 1) % NLO] : hi[3 * i + 1];
    const uint32_t w2 = 3 * i + 2 < 9 ? lo[(3 * i + 2) % NLO] : hi[3 * i + 2];
    slot[f] = field_bits_w<F64>(w0, w1, w2, f);
    slot[f + 1] = field_bits_w<F64>(w0, w1, w2, f + 1);
  }
}

// Convert X (section 2.3) and write its 12 fields to this lane's LDS slot.
template <bool F64>
__device__ __forceinline__ void convert_to_lds(const uint32_t (&x)[NW], uint64_t* __restrict__ slot,
                                               bool force) {
  uint32_t dlo[9];
  if (!to_ranlux_fast(x, dlo, force)) {
    lds_fields<F64>(dlo, x, slot);
  } else {
    uint32_t d[NW];
    to_ranlux_general(x, d);
    lds_fields<F64>(d, d, slot);
  }
}

template <bool F64>
__device__ __forceinline__ uint64_t field_bits(const uint32_t (&d)[NW], int f) {
  const int i = f >> 1;
  return field_bits_w<F64>(d[3 * i], d[3 * i + 1], d[3 * i + 2], f);
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

// Store the 12 fields of this lane's block from LDS.
//
// The gs = 2^LGS lanes of a group (gs <= 64, aligned inside the wave) hold
// consecutive blocks; lane ls holds the group's block ls and has written its
// 12 fields to its LDS slot (convert_to_lds).  Field f of the group's block m
// has output index jb + 12 m + f.  After a wave synchronisation lane ls
// stores the group's entries q gs + ls, q < 12: consecutive lanes write
// consecutive 8-byte values.  Only indices in [lo, hi) are written, and only
// by lanes with `active` set.  Called by every lane of the wave.
template <int LGS>
__device__ __forceinline__ void group_store(const uint64_t* __restrict__ stage, uint32_t tid_blk, uint32_t ls,
                                            int64_t jb, int64_t lo, int64_t hi, bool active,
                                            uint64_t* __restrict__ out) {
  constexpr uint32_t gs = 1u << LGS;
  wave_sync();
  const uint64_t* grp = stage + (size_t)(tid_blk - ls) * FIELDS + ls;
  if (active) {
    if (jb >= lo && jb + (int64_t)(FIELDS * gs) <= hi) {
      uint64_t* dst = out + jb + ls;
#pragma unroll
      for (int q = 0; q < FIELDS; ++q) dst[q * gs] = grp[q * gs];
    } else {
      // running index (no loop-invariant per-q offsets for the compiler to
      // keep in registers): u = j - lo, stored when 0 <= u < hi - lo
      const uint64_t span = (uint64_t)(hi - lo);
      uint64_t u = (uint64_t)(jb + (int64_t)ls - lo);
      uint64_t* base = out + lo;
#pragma unroll
      for (int q = 0; q < FIELDS; ++q) {
        if (u < span) base[u] = grp[q * gs];
        u += gs;
      }
    }
  }
  wave_sync();
}

}  // namespace rlx
