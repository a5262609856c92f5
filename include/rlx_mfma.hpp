// rlx_mfma.hpp -- the generator step X <- A X mod m on the int8 matrix cores
// of gfx950 (v_mfma_i32_32x32x32_i8), for a multiplier A that is the same for
// the whole launch.
//
// The product by a constant is a dense contraction (paper, section 2.1: the
// 576 x 576-bit multiply is the larger part of the generator's time).  With
// X = sum_i x_i 256^i (72 bytes x_i) and C_i = A 256^i mod m,
//
//   A X = sum_i x_i C_i  (mod m),
//
// a [72 x 72] matrix of byte digits of the C_i applied to the byte vector of
// X.  The matrix cores multiply signed bytes exactly into 32-bit sums, so:
//
//  * each byte of X enters as the signed digit d_i = x_i - 128 (the byte with
//    its top bit flipped);
//  * each C_i enters as its balanced base-256 digits (in [-128, 127], up to
//    76 of them), and the constant K = 128 sum_i C_i (the exact integer, not
//    reduced) as one more column multiplied by a constant input byte 1, so
//    that sum_i d_i C_i + K = sum_i x_i C_i exactly: a non-negative integer
//    below 72 * 255 * 2^576 < 2^591;
//  * output row r of the product is the digit sum S_r of weight 256^r; every
//    |S_r| < 2^21, so the 32-bit sums are exact, and four rows make the
//    signed 64-bit sum W_w of 32-bit word w (w < 19);
//  * a signed carry chain over W_0..W_18 gives the 19 words of
//    sum_i x_i C_i: 18 words of X' and the word h above 2^576 (h < 2^15),
//    which is folded back with 2^576 = 2^240 - 1 (mod m) as in step()
//    (section 2.2), ending in the canonical residue.
//
// One wave holds 64 independent states (one per lane).  The contraction runs
// as 18 MFMAs of 32 x 32 x 32: three tiles of 32 output rows (73 used) by
// three steps of 32 input bytes (72 used plus the constant) by two tiles of
// 32 states.  The matrix core pairs byte j of lane l's A operand with byte j
// of lane l's B operand for every (l div 32, j), and returns in lane l, value
// 4q + u of a tile, output row 8q + 4 (l div 32) + u of state column l mod 32.
// Each lane's state is split in halves: E = words 0..8 and F = words 9..17.
// In every lane the halves of the inputs are exchanged with the lane 32 away
// (v_permlane32_swap), so that one register file holds, in lanes 0..31, the
// E half of states 0..31 and, in lanes 32..63, their F half (the B operand of
// state tile 0), and the other one the same for states 32..63 (tile 1); the
// A operand's byte (l div 32, j) of each K step is the column of the input
// byte that sits there.  On the output side the halves are exchanged back:
// lanes 0..31 of tile 0 hold the even words of states 0..31, lanes 32..63
// their odd words, and the same for tile 1, so one exchange per word pair
// gives every lane all 19 words of its own state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlx_arith.hpp"

namespace rlx {

typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef int mf_v16i __attribute__((ext_vector_type(16)));

constexpr int MF_FRAGS = 9;         // A operands: 3 output-row tiles x 3 input steps
constexpr int MF_BYTES = 72;        // input bytes of X
constexpr int MF_ROWS = 96;         // output rows (balanced digits) kept per column
constexpr int MF_COLS = MF_BYTES + 1;  // the 72 C_i and K
// words of one luxury level's table: for each g < RLX_FOLD_G (multiplier
// A^(2^g)), MF_FRAGS fragments of 64 lanes x 4 words
constexpr size_t MF_FRAG_WORDS = (size_t)64 * 4;
constexpr size_t MF_LEVEL_WORDS = (size_t)MF_FRAGS * MF_FRAG_WORDS;

// Input column of A-operand byte j of lane half h in input step ks: the byte
// of X that the B operand holds there (0..71), MF_BYTES for K (the constant
// input byte 1), or -1 for a zero column.  Half h = 0 holds E = words 0..8,
// h = 1 holds F = words 9..17, four words per step: word e = 4 ks + j / 4 of
// the half; e = 9 is the register holding the constant 1 (in both halves;
// only h = 0 carries K), e = 10, 11 pad.
RLX_HD constexpr int mf_input_column(int h, int ks, int j) {
  return (4 * ks + j / 4) < 9 ? 4 * (4 * ks + j / 4 + 9 * h) + j % 4
         : ((4 * ks + j / 4) == 9 && j % 4 == 0 && h == 0) ? MF_BYTES
                                                           : -1;
}

// Balanced base-256 digits of the non-negative number in words w[0..n): the
// digits b_r in [-128, 127] with sum_r b_r 256^r equal to it; writes MF_ROWS
// digits (the number must be below 128 * 256^(MF_ROWS - 1)).
template <int N>
RLX_HD void balanced_digits(const uint32_t (&w)[N], int8_t (&d)[MF_ROWS]) {
  int carry = 0;
  for (int r = 0; r < MF_ROWS; ++r) {
    const int byte = (r / 4 < N) ? (int)((w[r / 4] >> (8 * (r % 4))) & 0xFFu) : 0;
    const int v = byte + carry;
    carry = v >= 128;
    d[r] = (int8_t)(v - 256 * carry);
  }
}

// Opaque 32-bit constant: keeps the compiler from turning multiply-adds by
// it into shifts and sign extensions (a multiply-add is one instruction).
__device__ __forceinline__ uint32_t mf_opaque(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// Exchange register a of lanes 32..63 with register b of lanes 0..31.
__device__ __forceinline__ void mf_swap(uint32_t& a, uint32_t& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}

typedef unsigned mf_v2u __attribute__((ext_vector_type(2)));

// The 64-bit value with low word lo and high word hi (a register pair).
__device__ __forceinline__ int64_t mf_pair(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(int64_t, mf_v2u{lo, hi});
}

// Signed 64-bit sum of output rows 4q .. 4q + 3 of a tile (weights 2^0,
// 2^8, 2^16, 2^24), as four multiply-adds (k1 = 1, the first one sign-
// extends).
__device__ __forceinline__ int64_t mf_word(const mf_v16i& s, int q, int32_t k1, int32_t k8, int32_t k16,
                                           int32_t k24) {
  int64_t w = (int64_t)s[4 * q] * k1;
  w = (int64_t)s[4 * q + 1] * k8 + w;
  w = (int64_t)s[4 * q + 2] * k16 + w;
  w = (int64_t)s[4 * q + 3] * k24 + w;
  return w;
}

// Copy a step's A operands (MF_FRAGS x 64 lanes x 16 bytes) from global
// memory into the block's LDS array `dst`; all `nthreads` threads of the
// block call it, then synchronise before the first step.
__device__ __forceinline__ void mf_stage_operands(mf_v4i* __restrict__ dst, const uint32_t* __restrict__ src,
                                                  uint32_t tid, uint32_t nthreads) {
  const mf_v4i* s = reinterpret_cast<const mf_v4i*>(src);
  for (uint32_t k = tid; k < (uint32_t)MF_FRAGS * 64; k += nthreads) dst[k] = s[k];
}

// X <- A X mod m with the A operands of the launch's multiplier delivered by
// `fetch(3 mt + ks)` (output-row tile mt, input step ks: this lane's 16
// bytes; read just before its two MFMAs, from LDS or global memory).  Must
// run with all 64 lanes of the wave active.  Returns the
// canonical residue; `force_general` sends the fold through its general
// branch.
// Operand fetch from an array af[64 f + lane] (LDS, or any memory).
struct MfFromArray {
  const mf_v4i* __restrict__ af;
  uint32_t lane;
  __device__ __forceinline__ mf_v4i operator()(int f) const { return af[64 * f + lane]; }
};

// Operand fetch from global memory through a buffer resource: the
// wave-uniform table address lives in scalar registers and each fetch is one
// buffer load at this lane's 32-bit offset (no 64-bit address per lane).
// dword 3 of the resource is the raw-buffer format word of gfx9 parts.
struct MfFromBuffer {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t off;  // 16 * lane
  __device__ __forceinline__ MfFromBuffer(const uint32_t* table, uint32_t lane)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(table), (short)0,
                                               (int)(MF_LEVEL_WORDS * sizeof(uint32_t)), 0x00020000)),
        off(16u * lane) {}
  __device__ __forceinline__ mf_v4i operator()(int f) const {
    return __builtin_bit_cast(mf_v4i, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 1024 * f, 0));
  }
};

// The step with the A operands of fetch0 for the states of lanes 0..31
// (state tile 0) and those of fetch1 for lanes 32..63 (tile 1): two
// multipliers in one wave, one per half.
template <class Fetch0, class Fetch1>
__device__ __forceinline__ void mfma_step_halves(uint32_t (&x)[NW], const Fetch0& fetch0, const Fetch1& fetch1,
                                                 bool force_general) {
  // signed input digits, halves exchanged across the two lane halves
  uint32_t a[9], b[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    a[k] = x[k] ^ 0x80808080u;
    b[k] = x[9 + k] ^ 0x80808080u;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) mf_swap(a[k], b[k]);
  const mf_v4i b0[3] = {mf_v4i{(int)a[0], (int)a[1], (int)a[2], (int)a[3]},
                        mf_v4i{(int)a[4], (int)a[5], (int)a[6], (int)a[7]}, mf_v4i{(int)a[8], 1, 0, 0}};
  const mf_v4i b1[3] = {mf_v4i{(int)b[0], (int)b[1], (int)b[2], (int)b[3]},
                        mf_v4i{(int)b[4], (int)b[5], (int)b[6], (int)b[7]}, mf_v4i{(int)b[8], 1, 0, 0}};
  const int32_t k1 = (int32_t)mf_opaque(1u), k8 = (int32_t)mf_opaque(256u);
  const int32_t k16 = (int32_t)mf_opaque(65536u), k24 = (int32_t)mf_opaque(1u << 24);
  const mf_v16i zero = {};
  int32_t c = 0;      // signed carry of the chain
  uint32_t h = 0;     // word 18
#pragma unroll
  for (int mt = 0; mt < 3; ++mt) {
    const mf_v4i f0 = fetch0(3 * mt), f1 = fetch0(3 * mt + 1), f2 = fetch0(3 * mt + 2);
    const mf_v4i g0 = fetch1(3 * mt), g1 = fetch1(3 * mt + 1), g2 = fetch1(3 * mt + 2);
    mf_v16i s0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0, b0[0], zero, 0, 0, 0);
    mf_v16i s1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(g0, b1[0], zero, 0, 0, 0);
    s0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f1, b0[1], s0, 0, 0, 0);
    s1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(g1, b1[1], s1, 0, 0, 0);
    s0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f2, b0[2], s0, 0, 0, 0);
    s1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(g2, b1[2], s1, 0, 0, 0);
    // rows 64 + 8q + ... of the last tile are zero from q = 2 on (the
    // digits end at row 75)
    const int nq = mt < 2 ? 4 : 2;
#pragma unroll
    for (int q = 0; q < nq; ++q) {
      const int64_t w0 = mf_word(s0, q, k1, k8, k16, k24);
      const int64_t w1 = mf_word(s1, q, k1, k8, k16, k24);
      uint32_t lo0 = (uint32_t)w0, hi0 = (uint32_t)((uint64_t)w0 >> 32);
      uint32_t lo1 = (uint32_t)w1, hi1 = (uint32_t)((uint64_t)w1 >> 32);
      mf_swap(lo0, lo1);
      mf_swap(hi0, hi1);
      // this lane's state: word 8 mt + 2 q in (lo0, hi0), the next in (lo1, hi1)
      const int e = 8 * mt + 2 * q;
      const int64_t we = mf_pair(lo0, hi0);
      const int64_t te = (int64_t)c * k1 + we;
      c = (int32_t)((uint64_t)te >> 32);
      if (e < NW) {
        x[e] = (uint32_t)te;
      } else {
        h = (uint32_t)te;
      }
      if (e + 1 < NW) {
        const int64_t wo = mf_pair(lo1, hi1);
        const int64_t to = (int64_t)c * k1 + wo;
        c = (int32_t)((uint64_t)to >> 32);
        x[e + 1] = (uint32_t)to;
      }
    }
  }
  // fold h (< 2^15) with 2^576 = 2^240 - 1: x - h at words 0-1, + (h << 16)
  // at words 7-9 (as in step())
  const uint32_t w0 = x[0], w1 = x[1], w7 = x[7], w8 = x[8], w9 = x[9];
  uint32_t br = 0;
  x[0] = subb(w0, h, br);
  x[1] = subb(w1, 0u, br);
  uint32_t cy = 0;
  x[7] = addc(w7, h << 16, cy);
  x[8] = addc(w8, h >> 16, cy);
  x[9] = addc(w9, 0u, cy);
  const bool rare = (br | cy) != 0 || x[17] == 0xFFFFFFFFu || force_general;
  if (rare) {
    x[0] = w0; x[1] = w1; x[7] = w7; x[8] = w8; x[9] = w9;
    fold_word_general(x, h);
  }
}

// The step with one multiplier for the whole wave.
template <class Fetch>
__device__ __forceinline__ void mfma_step(uint32_t (&x)[NW], const Fetch& fetch, bool force_general) {
  mfma_step_halves(x, fetch, fetch, force_general);
}

}  // namespace rlx
