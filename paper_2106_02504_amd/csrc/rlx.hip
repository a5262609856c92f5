// rlx.hip -- RANLUX++ kernels for gfx950 and the C ABI of librlx.so.
//
// Kernels (one lane per stream record unless noted):
//   k_tab_base / k_tab_fill / k_tab_fold / k_tab_win   per-luxury-level tables
//   k_tab_mf_c / k_tab_mf_k / k_tab_mf_frag          matrix-core operands of a step
//   k_init                                 seeding        (section 2.4)
//   k_skip, k_skip_levels                  skip-ahead     (section 2.4)
//   k_generate<U64|F64|NORMAL|F32, trace, LGS, MF> draw values (sections 2.1-2.3)
//   k_generate_levels<K, LGS>              the same for records of several levels
//   k_generate_lcg52<LGS, MF>              legacy raw-LCG doubles (section 2.3)
//   k_test_*                               generic arithmetic for tests
// The batched kernel and its planner are in rlx_batch.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <new>
#include <utility>

#include "rlx.h"
#include "rlx_arith.hpp"
#include "rlx_device.hpp"
#include "rlx_internal.hpp"
#include "rlx_mfma.hpp"

using namespace rlx;

namespace {

// Error word of each device: RLX_ERR_* bits that kernels OR in when they
// reject a record (read and cleared by rlx_check_errors).
__device__ uint32_t g_err_word;

// Staging of rlx_build_tables_static (the C_i words, then their balanced
// digits; see k_tab_mf_c), one copy per device for the life of the process.
// Host code never uses this name as an address: it uses the device address
// that hipGetSymbolAddress returns for the current device (scratch_ptr).
static __device__ __align__(256) uint8_t scratch[RLX_STATIC_SCRATCH_BYTES];
constexpr size_t SCRATCH_CW_BYTES = (size_t)FOLD_G * MF_BYTES * NW * sizeof(uint32_t);
static_assert(RLX_MFMA_ROW_WORDS == MF_LEVEL_WORDS, "operand rows as the header states");
static_assert(SCRATCH_CW_BYTES % 256 == 0, "digit staging stays aligned");
static_assert(SCRATCH_CW_BYTES + (size_t)FOLD_G * MF_COLS * MF_ROWS == RLX_STATIC_SCRATCH_BYTES,
              "the static scratch holds the staging of every folded row");

// ---------------------------------------------------------------------------
// tables

// One lane: A_p = a^p by square-and-multiply, then T[i][1] = T[i-1][1]^16,
// and T[i][0] = 1.
__global__ __launch_bounds__(64) void k_tab_base(uint32_t* __restrict__ T, uint32_t p) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t a[NW], r[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) a[k] = a_word(k);
  set_one(r);
  const int top = 31 - __builtin_clz(p);
  for (int b = top; b >= 0; --b) {
    mulmod_inplace(r, r);
    if ((p >> b) & 1u) mulmod_inplace(r, a);
  }
  uint32_t one[NW];
  set_one(one);
  for (int i = 0; i < TAB_ROWS; ++i) {
    store_words(T + ((size_t)i * TAB_COLS + 0) * NW, one);
    store_words(T + ((size_t)i * TAB_COLS + 1) * NW, r);
    for (int s = 0; s < 4; ++s) mulmod_inplace(r, r);
  }
}

// T[i][j] = T[i][1]^j for 2 <= j < 16, one lane per entry.
__global__ __launch_bounds__(64) void k_tab_fill(uint32_t* __restrict__ T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= TAB_ROWS * (TAB_COLS - 2)) return;
  const int i = t / (TAB_COLS - 2);
  const uint32_t j = 2 + t % (TAB_COLS - 2);
  uint32_t base[NW], r[NW];
  load_words(T + ((size_t)i * TAB_COLS + 1) * NW, base);
  copy_words(r, base);
  const int top = 31 - __builtin_clz(j);
  for (int b = top - 1; b >= 0; --b) {
    mulmod_inplace(r, r);
    if ((j >> b) & 1u) mulmod_inplace(r, base);
  }
  store_words(T + ((size_t)i * TAB_COLS + j) * NW, r);
}

// W[i][j] = prod_q T[r + q][nibble q of j], q < 4, with r = 4i for the skip
// rows (i < 4) and r = 24 + 4 (i - 4) for the seed rows: A_p^(j 65536^i)
// from four hexadecimal windows.  One lane per entry.
__global__ __launch_bounds__(64) void k_tab_win(const uint32_t* __restrict__ T, uint32_t* __restrict__ W) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= WIN_ROWS * WIN_COLS) return;
  const int i = t / WIN_COLS;
  const uint32_t j = (uint32_t)(t % WIN_COLS);
  const int r = i < WIN_SEED_ROW0 ? 4 * i : SEED_ROW0 + 4 * (i - WIN_SEED_ROW0);
  uint32_t y[NW], a[NW];
  load_words(T + ((size_t)r * TAB_COLS + (j & 15u)) * NW, y);
#pragma unroll 1
  for (int q = 1; q < 4; ++q) {
    load_words(T + ((size_t)(r + q) * TAB_COLS + ((j >> (4 * q)) & 15u)) * NW, a);
    mulmod_inplace(y, a);
  }
  store_words(W + (size_t)t * NW, y);
}

// C_g[j] = A_p^(2^g) 2^(o_j) mod m: block g (g < 64) builds the folded
// multiplier of a step by 2^g generator steps, one lane per row j.  A_p^(2^g)
// is a single entry of T: 2^g = v 16^i with v in {1, 2, 4, 8}.
__global__ __launch_bounds__(64) void k_tab_fold(const uint32_t* __restrict__ T, uint32_t* __restrict__ C) {
  const int g = blockIdx.x;
  const int j = threadIdx.x;
  if (j >= NL) return;
  uint32_t a[NW], pw[NW], r[NW];
  load_words(T + ((size_t)(g >> 2) * TAB_COLS + (1u << (g & 3))) * NW, a);
  const int bit = limb_offset(j);
#pragma unroll
  for (int k = 0; k < NW; ++k) pw[k] = (k == (bit >> 5)) ? (1u << (bit & 31)) : 0u;
  mulmod_generic(a, pw, r);
  store_words(C + (size_t)g * FOLD_ROW_WORDS + (size_t)j * NW, r);
}

// Matrix-core operands of a step by 2^g generator steps (rlx_mfma.hpp),
// g < rows (at most RLX_FOLD_G), in three launches:
// C_i = A_p^(2^g) 256^i mod m for i < 72, one lane per (g, i): its words go
// to cw (for the sums of k_tab_mf_k) and its balanced digits to column i of
// bal[g].
__global__ __launch_bounds__(64) void k_tab_mf_c(const uint32_t* __restrict__ T, uint32_t* __restrict__ cw,
                                                 int8_t* __restrict__ bal, int rows) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * MF_BYTES) return;
  const int g = t / MF_BYTES, i = t % MF_BYTES;
  uint32_t a[NW], pw[NW], r[NW];
  load_words(T + ((size_t)(g >> 2) * TAB_COLS + (1u << (g & 3))) * NW, a);
  // The words of 256^i pass through an empty asm so that the multiplication
  // is compiled for arbitrary operands: specialised for these sparse ones
  // (bits only at multiples of 8), the gfx950 code gave wrong products for
  // i = 7, 14, 21, 35, 42, 49 while the same source built for the host was
  // exact.
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    uint32_t v = (k == i / 4) ? (1u << (8 * (i % 4))) : 0u;
    asm volatile("" : "+v"(v));
    pw[k] = v;
  }
  mulmod_generic(a, pw, r);
  store_words(cw + (size_t)t * NW, r);
  int8_t d[MF_ROWS];
  balanced_digits(r, d);
  int8_t* col = bal + ((size_t)g * MF_COLS + i) * MF_ROWS;
  for (int k = 0; k < MF_ROWS; ++k) col[k] = d[k];
}

// K = 128 sum_i C_i as an exact integer (below 2^590, 19 words), one lane
// per g: its balanced digits are column MF_BYTES of bal[g].
__global__ __launch_bounds__(64) void k_tab_mf_k(const uint32_t* __restrict__ cw, int8_t* __restrict__ bal,
                                                 int rows) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows) return;
  uint32_t s[NW + 1];
  for (int k = 0; k <= NW; ++k) s[k] = 0;
  for (int i = 0; i < MF_BYTES; ++i) {
    const uint32_t* c = cw + ((size_t)g * MF_BYTES + i) * NW;
    uint32_t cy = 0;
    for (int k = 0; k < NW; ++k) s[k] = addc(s[k], c[k], cy);
    s[NW] += cy;
  }
  for (int k = NW; k > 0; --k) s[k] = (s[k] << 7) | (s[k - 1] >> 25);
  s[0] <<= 7;
  int8_t d[MF_ROWS];
  balanced_digits(s, d);
  int8_t* col = bal + ((size_t)g * MF_COLS + MF_BYTES) * MF_ROWS;
  for (int k = 0; k < MF_ROWS; ++k) col[k] = d[k];
}

// The A operands: lane l of fragment f = 3 mt + ks of level g holds, in its
// 16 bytes j, the digit of output row 32 mt + (l mod 32) of the input column
// mf_input_column(l div 32, ks, j), zero for a zero column.
__global__ __launch_bounds__(64) void k_tab_mf_frag(const int8_t* __restrict__ bal, uint32_t* __restrict__ M,
                                                    int rows) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * MF_FRAGS * 64) return;
  const int g = t / (MF_FRAGS * 64), f = (t / 64) % MF_FRAGS, l = t % 64;
  const int mt = f / 3, ks = f % 3, h = l / 32, row = 32 * mt + l % 32;
  for (int q = 0; q < 4; ++q) {
    uint32_t word = 0;
    for (int b = 0; b < 4; ++b) {
      const int col = mf_input_column(h, ks, 4 * q + b);
      const int8_t v = col < 0 ? (int8_t)0 : bal[((size_t)g * MF_COLS + col) * MF_ROWS + row];
      word |= (uint32_t)(uint8_t)v << (8 * b);
    }
    M[(size_t)t * 4 + q] = word;
  }
}

// ---------------------------------------------------------------------------
// seeding and skipping (section 2.4)

// X = A_p^(2^96 id) from 1: the product of the seed windows of the non-zero
// 16-bit digits of id (the first one copied, not multiplied: ids < 2^16 are
// a table copy).
__global__ __launch_bounds__(BLOCK) void k_init(rlx_state* __restrict__ st, uint64_t n,
                                                const uint64_t* __restrict__ ids, uint64_t id0,
                                                uint32_t p, const uint32_t* __restrict__ W) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t id = ids ? ids[i] : id0 + i;
  uint32_t x[NW];
  set_one(x);
  bool first = true;
  for (int b = 0; b < 4 && (id >> (WIN_BITS * b)) != 0; ++b) {
    const uint32_t v = (uint32_t)(id >> (WIN_BITS * b)) & (WIN_COLS - 1u);
    if (v == 0) continue;
    const uint32_t* e = W + ((size_t)(WIN_SEED_ROW0 + b) * WIN_COLS + v) * NW;
    uint32_t y[NW];
    load_words(e, y);
    if (first) {
      copy_words(x, y);
      first = false;
    } else {
      mulmod_inplace(x, y);
    }
  }
  store_record(st, i, x, 0u, p);
}

// Record of the block that this thread skips when every record has its own
// offset: the block's records ordered by the number of 16-bit windows of
// their skip (a counting sort in LDS), so that each wave runs about as many
// multiplication rounds as its own records need instead of the longest in
// the block (offsets log-uniform over 64 bits: about 10 rounds per 4 waves
// instead of 16).  Every thread of the block must call it; the order only
// decides which lane handles which record.
__device__ __forceinline__ uint64_t skip_record_index(const uint64_t* __restrict__ steps, uint64_t n,
                                                      int by_values, uint32_t per_step) {
  __shared__ uint32_t cnt[5];
  __shared__ uint32_t order[BLOCK];
  const uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint64_t k = i < n ? steps[i] / (by_values ? per_step : 1u) : 0;
  const uint32_t key = k ? (uint32_t)(64 - __clzll((long long)k) + WIN_BITS - 1) / WIN_BITS : 0u;
  if (threadIdx.x < 5) cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t slot = atomicAdd(&cnt[key], 1u);
  __syncthreads();
  uint32_t base = 0;
  for (uint32_t b = 0; b < key; ++b) base += cnt[b];
  order[base + slot] = threadIdx.x;
  __syncthreads();
  return (uint64_t)blockIdx.x * BLOCK + order[threadIdx.x];
}

// by_values = 0: skip `steps` generator steps (pos unchanged); 1: skip that
// many values of `per_step` values per step (pos + v = per_step k + pos',
// k steps, new pos'): 12 for the 48-bit fields, 11 for the legacy 52-bit
// values, whose records must have pos < 11.
__global__ __launch_bounds__(BLOCK) void k_skip(rlx_state* __restrict__ st, uint64_t n,
                                                const uint64_t* __restrict__ steps, uint64_t steps0,
                                                uint32_t p, const uint32_t* __restrict__ W,
                                                uint32_t* __restrict__ err, int by_values, uint32_t per_step) {
  const uint64_t i = steps ? skip_record_index(steps, n, by_values, per_step)
                           : (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x[NW], pos, sp;
  load_record(st, i, x, pos, sp);
  uint32_t bad = check_record(x, pos, sp, p);
  if (by_values && pos >= per_step) bad |= RLX_ERR_BAD_POS;
  if (bad) {
    atomicOr(err, bad);
    return;
  }
  uint64_t k = steps ? steps[i] : steps0;
  if (by_values) {
    const uint64_t v = k;
    const uint32_t r = pos + (uint32_t)(v % per_step);
    k = v / per_step + r / per_step;
    pos = r % per_step;
  }
  skip_windows(x, k, W);
  store_record(st, i, x, pos, sp);
}

// Records of several luxury levels in one call (p = RLX_P_RECORD): the
// tables of every level prepared on the device, passed by value.  A record
// whose level is not among them is flagged RLX_ERR_BAD_P and left as it is.
constexpr int MAX_RECORD_LEVELS = RLX_MAX_RECORD_LEVELS;
struct LevelSet {
  uint32_t n;
  uint32_t p[MAX_RECORD_LEVELS];
  const uint32_t* C[MAX_RECORD_LEVELS];
  const uint32_t* M[MAX_RECORD_LEVELS];
  const uint32_t* W[MAX_RECORD_LEVELS];
};

// Index of level p in L, or -1.
__device__ __forceinline__ int level_index(const LevelSet& L, uint32_t p) {
  int li = -1;
#pragma unroll
  for (int k = 0; k < MAX_RECORD_LEVELS; ++k)
    if (k < (int)L.n && L.p[k] == p) li = k;
  return li;
}

// L's table pointer of entry li (a chain of selects over the unrolled
// entries, so the by-value argument is never indexed dynamically).
__device__ __forceinline__ const uint32_t* level_ptr(const uint32_t* const (&tab)[MAX_RECORD_LEVELS], int li) {
  const uint32_t* r = tab[0];
#pragma unroll
  for (int k = 1; k < MAX_RECORD_LEVELS; ++k)
    if (k == li) r = tab[k];
  return r;
}

// k_skip with each record's own level.
__global__ __launch_bounds__(BLOCK) void k_skip_levels(rlx_state* __restrict__ st, uint64_t n,
                                                       const uint64_t* __restrict__ steps, uint64_t steps0,
                                                       LevelSet L, uint32_t* __restrict__ err, int by_values,
                                                       uint32_t per_step) {
  const uint64_t i = steps ? skip_record_index(steps, n, by_values, per_step)
                           : (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x[NW], pos, sp;
  load_record(st, i, x, pos, sp);
  const int li = level_index(L, sp);
  uint32_t bad = check_record(x, pos, sp, sp) | (li < 0 ? RLX_ERR_BAD_P : 0u);
  if (by_values && pos >= per_step) bad |= RLX_ERR_BAD_POS;
  if (bad) {
    atomicOr(err, bad);
    return;
  }
  uint64_t k = steps ? steps[i] : steps0;
  if (by_values) {
    const uint64_t v = k;
    const uint32_t r = pos + (uint32_t)(v % per_step);
    k = v / per_step + r / per_step;
    pos = r % per_step;
  }
  skip_windows(x, k, level_ptr(L.W, li));
  store_record(st, i, x, pos, sp);
}

// ---------------------------------------------------------------------------
// generation (sections 2.1-2.3)

// Draw `count` values for every record with G = 2^lg lanes per record.
//
// Block t of a record is the t-th LCG state visited (t = 0 is the state on
// entry, t = nadv the state after the last advance); the value with output
// index j is field (pos + j) mod 12 of block (pos + j) / 12.  Lane l of a
// record starts at block l (X_l = A^l X_0, by windows) and then takes
// blocks l + G, l + 2G, ... with the folded multiplier of A^G, so the G lanes
// of a record hold G consecutive blocks at every iteration.
//
// Staged (G > 1): the gs = 2^LGS = min(G, 64) lanes of a record inside one
// wave pass their blocks through LDS (group_store), so each store
// instruction writes contiguous runs of the output row instead of one value
// per row per lane.  LGS = 0 is G = 1 (direct stores, no staging).
//
// The record is advanced eagerly.  When its G lanes lie in one wave
// (writeback != 0, G <= 64), the lane holding block nadv writes it back with
// pos = (pos + count) mod 12: every lane of the wave read the record at entry,
// before that store in program order.  Lanes of a record that spans several
// waves may be dispatched in different rounds, and nothing orders one wave's
// load after another wave's store, so then no lane writes the record
// (writeback = 0) and the host advances it by a skip launch on the same
// stream after this kernel.
template <Out K, bool TRACE, int LGS, bool MF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(K == Out::NORMAL && LGS == 0 ? 3 : 4))) void k_generate(rlx_state* __restrict__ st, uint32_t n,
                                                    uint64_t count, uint64_t* __restrict__ out,
                                                    uint64_t* __restrict__ trace, uint64_t trace_steps,
                                                    const uint32_t* __restrict__ ctabs,
                                                    const uint32_t* __restrict__ mtabs,
                                                    const uint32_t* __restrict__ W, uint32_t lg,
                                                    uint32_t p, uint32_t* __restrict__ err,
                                                    int force_general, int writeback) {
  // Per-lane state kept across the loop is x plus four 32-bit words (record
  // index, lane, pos, last block): the host limits n < 2^32 and
  // count <= RLX_MAX_COUNT, so record and block indices fit in 32 bits.
  // Everything else is recomputed per iteration, which keeps the registers
  // within 128 (4 waves per SIMD) without spills; normals without staging
  // (one lane per record) need more and run 3 waves per SIMD.
  constexpr bool STAGED = LGS > 0;
  constexpr uint32_t gs = 1u << LGS;  // lanes of a record inside one wave
  __shared__ __align__(16) uint64_t stage[STAGED ? BLOCK * SLOT_VALUES : 2];
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t i = (uint32_t)(tid >> lg);
  const uint32_t l = (uint32_t)tid & ((1u << lg) - 1u);
  const bool force = force_general != 0;

  uint32_t x[NW];
  uint32_t pos = 0, sp = 0;
  bool active = (tid >> lg) < n;
  if (active) {
    load_record(st, i, x, pos, sp);
    const uint32_t bad = check_record(x, pos, sp, p);
    if (bad) {
      if (l == 0) atomicOr(err, bad);
      active = false;
    }
  }
  if (!active) {
    set_one(x);
    pos = 0;
  }
  const uint32_t nadv = (uint32_t)((pos + count) / FIELDS);

  // lane l starts at block l: X_l = A^l X_0 (bits 6 and up of l are the
  // same for the whole wave)
  if (STAGED) skip_windows(x, l, W);
  const uint32_t* __restrict__ ctab = ctabs + (size_t)lg * FOLD_ROW_WORDS;
  // MF: the step's matrix-core A operands for A^G, staged in LDS once per
  // block (9 KB) and read by every step
  __shared__ mf_v4i af[MF ? MF_FRAGS * 64 : 1];
  if constexpr (MF) {
    mf_stage_operands(af, mtabs + (size_t)lg * MF_LEVEL_WORDS, threadIdx.x, BLOCK);
    __syncthreads();
  }

  for (uint32_t k = 0;; ++k) {
    const uint32_t t = l + (k << lg);
    const bool live = active && t <= nadv;
    if (!__any(live)) break;
    if (live) {
      if (TRACE) put_trace(trace + ((uint64_t)i * trace_steps + t) * 9, x);
      if (writeback && t == nadv) store_record(st, i, x, (uint32_t)((pos + count) % FIELDS), p);
    }
    uint64_t* const row = out + (uint64_t)i * count;
    if (!STAGED) {
      uint32_t d[NW];
      to_ranlux(x, d, force);
      if (live) {
        const int64_t jb = (int64_t)((uint64_t)t * FIELDS) - (int64_t)pos;
#pragma unroll
        for (int f = 0; f < FIELDS; ++f) {
          const int64_t j = jb + f;
          if (j >= 0 && (uint64_t)j < count) row[j] = field_bits<K>(d, f);
        }
      }
    } else {
      const uint32_t tid_blk = threadIdx.x;
      const uint32_t ls = l & (gs - 1);
      convert_to_lds<K>(x, stage + (size_t)tid_blk * SLOT_VALUES, force);
      // the group's blocks t - ls .. t - ls + gs - 1 hold output indices
      // from jb on
      const int64_t jb = (int64_t)((uint64_t)(t - ls) * FIELDS) - (int64_t)pos;
      group_store<LGS>(stage, tid_blk, ls, jb, count, active, row);
    }
    if (__any(live && t + (1u << lg) <= nadv)) {
      if constexpr (MF) {
        mfma_step(x, MfFromArray{af, threadIdx.x & 63}, force);
      } else {
        step(x, constant_table(ctab), force, SgprBarrier());
      }
    }
  }
}

// k_generate for records of several levels (p = RLX_P_RECORD), G <= 64 lanes
// per record, so a record's lanes share a wave and write it back in place.
// A wave in which each half (lanes 0..31, 32..63) has live records of one
// level takes the matrix-core step with one multiplier per half (operands
// read through the L1, as the batched kernel does for items of mixed
// levels); with G >= 32 a half is one record, so this is every wave.  A wave
// with mixed levels inside a half multiplies each lane by its own level's
// A^G with the generic multiplication.
template <Out K, int LGS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(K == Out::NORMAL ? 3 : 4))) void k_generate_levels(
    rlx_state* __restrict__ st, uint32_t n, uint64_t count, uint64_t* __restrict__ out, LevelSet L, uint32_t lg,
    uint32_t* __restrict__ err) {
  constexpr bool STAGED = LGS > 0;
  constexpr uint32_t gs = 1u << LGS;
  __shared__ __align__(16) uint64_t stage[STAGED ? BLOCK * SLOT_VALUES : 2];
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t i = (uint32_t)(tid >> lg);
  const uint32_t l = (uint32_t)tid & ((1u << lg) - 1u);

  uint32_t x[NW];
  uint32_t pos = 0, sp = 0;
  int li = -1;
  bool active = (tid >> lg) < n;
  if (active) {
    load_record(st, i, x, pos, sp);
    li = level_index(L, sp);
    const uint32_t bad = check_record(x, pos, sp, sp) | (li < 0 ? RLX_ERR_BAD_P : 0u);
    if (bad) {
      if (l == 0) atomicOr(err, bad);
      active = false;
    }
  }
  if (!active) {
    set_one(x);
    pos = 0;
    li = -1;
  }
  // each half-wave's level when its live records share one (the step takes
  // one multiplier per half: lanes 0..31 and 32..63 are its two state
  // tiles); a half with no live record takes the other half's
  const uint64_t act = __ballot(li >= 0);
  const uint64_t act0 = act & 0xFFFFFFFFull, act1 = act >> 32;
  const int first0 = act0 ? __ffsll((unsigned long long)act0) - 1 : (act1 ? 32 + __ffsll((unsigned long long)act1) - 1 : 0);
  const int first1 = act1 ? 32 + __ffsll((unsigned long long)act1) - 1 : first0;
  const int u0 = __builtin_amdgcn_readfirstlane(__shfl(li, first0));
  const int u1 = __builtin_amdgcn_readfirstlane(__shfl(li, first1));
  const bool uniform = __all(li < 0 || li == ((threadIdx.x & 32) ? u1 : u0));
  const uint32_t nadv = (uint32_t)((pos + count) / FIELDS);
  if (STAGED && active) skip_windows(x, l, level_ptr(L.W, li));

  for (uint32_t k = 0;; ++k) {
    const uint32_t t = l + (k << lg);
    const bool live = active && t <= nadv;
    if (!__any(live)) break;
    if (live && t == nadv) store_record(st, i, x, (uint32_t)((pos + count) % FIELDS), sp);
    uint64_t* const row = out + (uint64_t)i * count;
    if (!STAGED) {
      uint32_t d[NW];
      to_ranlux(x, d, false);
      if (live) {
        const int64_t jb = (int64_t)((uint64_t)t * FIELDS) - (int64_t)pos;
#pragma unroll
        for (int f = 0; f < FIELDS; ++f) {
          const int64_t j = jb + f;
          if (j >= 0 && (uint64_t)j < count) row[j] = field_bits<K>(d, f);
        }
      }
    } else {
      const uint32_t ls = l & (gs - 1);
      convert_to_lds<K>(x, stage + (size_t)threadIdx.x * SLOT_VALUES, false);
      const int64_t jb = (int64_t)((uint64_t)(t - ls) * FIELDS) - (int64_t)pos;
      group_store<LGS>(stage, threadIdx.x, ls, jb, count, active, row);
    }
    if (__any(live && t + (1u << lg) <= nadv)) {
      if (uniform && u0 == u1) {
        // one level for the wave: one operand fetch serves both halves
        mfma_step(x, MfFromBuffer(level_ptr(L.M, u0) + (size_t)lg * MF_LEVEL_WORDS, threadIdx.x & 63), false);
      } else if (uniform) {
        mfma_step_halves(x, MfFromBuffer(level_ptr(L.M, u0) + (size_t)lg * MF_LEVEL_WORDS, threadIdx.x & 63),
                         MfFromBuffer(level_ptr(L.M, u1) + (size_t)lg * MF_LEVEL_WORDS, threadIdx.x & 63), false);
      } else if (active) {
        uint32_t a[NW];
        load_words(level_ptr(L.C, li) + (size_t)lg * FOLD_ROW_WORDS, a);  // C_0 = A^G
        mulmod_inplace(x, a);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Legacy doubles from raw LCG bits, for comparison only (section 2.3 names
// this earlier conversion and drops it as biased): value k of step t is bits
// [52k, 52k + 52) of X_t, k < 11, as v 2^-52, and the record's pos counts
// these values (0..10).  Same lane interleaving as k_generate (lane l takes
// steps l, l + G, ...) and the same write-back rule; no RANLUX conversion.
// A lane's 11 values go through an LDS slot so that each store instruction
// writes a contiguous run of the row.

constexpr int LCG52_VALUES = 11;

// Bits [52k, 52k + 52) of X as the double v 2^-52: 0x3FF << 52 | v is
// 1 + v 2^-52, and subtracting 1 is exact.  k is a constant after unrolling;
// bits past 575 never reach the 52 kept (k = 10 ends at bit 571).
__device__ __forceinline__ double lcg52_value(const uint32_t (&x)[NW], int k) {
  const int b = 52 * k, w = b >> 5, s = b & 31;
  const uint32_t w2 = x[w + 2 < NW ? w + 2 : NW - 1];
  const uint32_t lo = s ? __builtin_amdgcn_alignbit(x[w + 1], x[w], s) : x[w];
  const uint32_t hi = s ? __builtin_amdgcn_alignbit(w2, x[w + 1], s) : x[w + 1];
  return bits_to_f64(lo, (hi & 0xFFFFFu) | 0x3FF00000u) - 1.0;
}

template <int LGS, bool MF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MF ? 4 : 5))) void k_generate_lcg52(
    rlx_state* __restrict__ st, uint32_t n, uint64_t count, double* __restrict__ out,
    const uint32_t* __restrict__ ctabs, const uint32_t* __restrict__ mtabs, const uint32_t* __restrict__ W,
    uint32_t lg, uint32_t p, uint32_t* __restrict__ err, int writeback) {
  constexpr uint32_t gs = 1u << LGS;  // lanes of a record inside one wave
  __shared__ __align__(16) double stage[BLOCK * LCG52_VALUES];
  __shared__ mf_v4i af[MF ? MF_FRAGS * 64 : 1];  // matrix-core operands of A^G, as in k_generate
  const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t i = (uint32_t)(tid >> lg);
  const uint32_t l = (uint32_t)tid & ((1u << lg) - 1u);

  uint32_t x[NW];
  uint32_t pos = 0, sp = 0;
  bool active = (tid >> lg) < n;
  if (active) {
    load_record(st, i, x, pos, sp);
    uint32_t bad = check_record(x, pos, sp, p);
    if (pos == LCG52_VALUES) bad |= RLX_ERR_BAD_POS;
    if (bad) {
      if (l == 0) atomicOr(err, bad);
      active = false;
    }
  }
  if (!active) {
    set_one(x);
    pos = 0;
  }
  const uint32_t nadv = (uint32_t)((pos + count) / LCG52_VALUES);
  skip_windows(x, l, W);
  const uint32_t* __restrict__ ctab = ctabs + (size_t)lg * FOLD_ROW_WORDS;
  if constexpr (MF) {
    mf_stage_operands(af, mtabs + (size_t)lg * MF_LEVEL_WORDS, threadIdx.x, BLOCK);
    __syncthreads();
  }
  const uint32_t ls = l & (gs - 1);
  double* const slot = stage + (size_t)threadIdx.x * LCG52_VALUES;
  const double* const grp = stage + (size_t)(threadIdx.x - ls) * LCG52_VALUES;
  double* const row = out + (uint64_t)i * count;

  for (uint32_t k = 0;; ++k) {
    const uint32_t t = l + (k << lg);
    const bool live = active && t <= nadv;
    if (!__any(live)) break;
    if (writeback && live && t == nadv) store_record(st, i, x, (uint32_t)((pos + count) % LCG52_VALUES), p);
#pragma unroll
    for (int f = 0; f < LCG52_VALUES; ++f) slot[f] = lcg52_value(x, f);
    wave_sync();
    // the group's blocks t - ls .. t - ls + gs - 1 hold values from u0 on.
    // A whole wave of whole windows starting on 128-byte lines stores 16-byte
    // pairs: lane ls takes pairs q gs + ls of the group's 11 gs / 2, so each
    // instruction writes 16 gs contiguous bytes per group (the last one with
    // half the lanes).  Otherwise value q gs + ls goes to row[u0 + q gs + ls]
    // if in range.
    const int64_t u0 = (int64_t)((uint64_t)(t - ls) * LCG52_VALUES) - (int64_t)pos;
    const bool whole = u0 >= 0 && (uint64_t)u0 + LCG52_VALUES * gs <= count;
    const uint64_t a = reinterpret_cast<uint64_t>(out) + ((uint64_t)i * count + (uint64_t)u0) * sizeof(double);
    if (gs >= 8 && __all(active && whole && (a & 127) == 0)) {
      const ulonglong2* g2 = reinterpret_cast<const ulonglong2*>(grp) + ls;
      uint64_t* const dst = reinterpret_cast<uint64_t*>(row + u0) + 2 * ls;
#pragma unroll
      for (uint32_t q = 0; q < (LCG52_VALUES + 1) / 2; ++q) {
        if (q * gs + ls < LCG52_VALUES * gs / 2) store_pair<true>(dst + 2 * q * gs, g2[q * gs]);
      }
    } else if (active) {
      uint64_t u = (uint64_t)(u0 + (int64_t)ls);
#pragma unroll
      for (int q = 0; q < LCG52_VALUES; ++q) {
        if (u < count) row[u] = grp[q * gs + ls];
        u += gs;
      }
    }
    wave_sync();
    if (__any(live && t + (1u << lg) <= nadv)) {
      if constexpr (MF) {
        mfma_step(x, MfFromArray{af, threadIdx.x & 63}, false);
      } else {
        step(x, constant_table(ctab), false, SgprBarrier());
      }
    }
  }
}

// ---------------------------------------------------------------------------
// RANLUX-form state: export and import (section 2)

__device__ __forceinline__ void load9w(const uint64_t* __restrict__ src, uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const uint64_t v = src[k];
    x[2 * k] = (uint32_t)v;
    x[2 * k + 1] = (uint32_t)(v >> 32);
  }
}

__device__ __forceinline__ void store9w(uint64_t* __restrict__ dst, const uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[k] = ((uint64_t)x[2 * k + 1] << 32) | x[2 * k];
}

__global__ __launch_bounds__(BLOCK) void k_export(const rlx_state* __restrict__ st, uint64_t n,
                                                  uint64_t* __restrict__ packed, uint32_t* __restrict__ carry,
                                                  uint32_t* __restrict__ posout, uint32_t* __restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x[NW], pos, sp, d[NW];
  load_record(st, i, x, pos, sp);
  if (geq_m(x)) {
    atomicOr(err, RLX_ERR_BAD_X);
    return;
  }
  to_ranlux(x, d, false);
  store9w(packed + i * 9, d);
  carry[i] = ranlux_carry(x, d);
  if (posout) posout[i] = pos;
}

// X = D - floor(D / 2^336) + c, accepted when X < m and X exports to (D, c).
__global__ __launch_bounds__(BLOCK) void k_import(rlx_state* __restrict__ st, uint64_t n,
                                                  const uint64_t* __restrict__ packed,
                                                  const uint32_t* __restrict__ carry,
                                                  const uint32_t* __restrict__ posin, uint32_t p,
                                                  uint32_t* __restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t d[NW], x[NW];
  load9w(packed + i * 9, d);
  const uint32_t c = carry[i];
  const uint32_t pos = posin ? posin[i] : 0u;
  if (pos > 11) {
    atomicOr(err, RLX_ERR_BAD_POS);
    return;
  }
  // a carry other than 0/1 fails in from_ranlux or in the round trip below
  bool ok = from_ranlux(d, c, x) && !geq_m(x);
  if (ok) {
    uint32_t d2[NW];
    to_ranlux(x, d2, false);
#pragma unroll
    for (int k = 0; k < NW; ++k) ok = ok && d2[k] == d[k];
    ok = ok && ranlux_carry(x, d2) == c;
  }
  if (!ok) {
    atomicOr(err, RLX_ERR_NOT_CANONICAL);
    return;
  }
  store_record(st, i, x, pos, p);
}

// ---------------------------------------------------------------------------
// test kernels: generic arithmetic on arbitrary operands

__device__ __forceinline__ void load9(const uint64_t* __restrict__ src, uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const uint64_t v = src[k];
    x[2 * k] = (uint32_t)v;
    x[2 * k + 1] = (uint32_t)(v >> 32);
  }
}

__device__ __forceinline__ void store9(uint64_t* __restrict__ dst, const uint32_t (&x)[NW]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[k] = ((uint64_t)x[2 * k + 1] << 32) | x[2 * k];
}

__global__ __launch_bounds__(BLOCK) void k_test_mulmod(const uint64_t* __restrict__ xs, const uint64_t* __restrict__ ys,
                              uint64_t* __restrict__ out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x[NW], y[NW], r[NW];
  load9(xs + i * 9, x);
  load9(ys + i * 9, y);
  mulmod_generic(x, y, r);
  store9(out + i * 9, r);
}

__global__ __launch_bounds__(BLOCK) void k_test_pow(const uint64_t* __restrict__ bs, const uint64_t* __restrict__ es,
                           uint64_t* __restrict__ out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t b[NW], r[NW];
  load9(bs + i * 9, b);
  set_one(r);
  for (int w = 2; w >= 0; --w) {
    const uint64_t e = es[i * 3 + w];
    for (int bit = 63; bit >= 0; --bit) {
      mulmod_inplace(r, r);
      if ((e >> bit) & 1u) mulmod_inplace(r, b);
    }
  }
  store9(out + i * 9, r);
}

__global__ __launch_bounds__(BLOCK) void k_test_to_ranlux(const uint64_t* __restrict__ xs, uint64_t* __restrict__ ds,
                                 uint32_t* __restrict__ carry, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x[NW], d[NW];
  load9(xs + i * 9, x);
  if (geq_m(x)) {
#pragma unroll
    for (int k = 0; k < NW; ++k) d[k] = 0xFFFFFFFFu;
    store9(ds + i * 9, d);
    carry[i] = 0xFFFFFFFFu;
    return;
  }
  to_ranlux(x, d, false);
  store9(ds + i * 9, d);
  carry[i] = ranlux_carry(x, d);
}

// One step by the folded multiplier of 2^g steps, with either step kernel,
// on arbitrary states (the matrix-core step needs whole waves: lanes past n
// step x = 1 and store nothing).
template <bool MF>
__global__ __launch_bounds__(BLOCK) void k_test_step(const uint64_t* __restrict__ xs, uint64_t* __restrict__ out,
                                                     uint64_t n, const uint32_t* __restrict__ ctab,
                                                     const uint32_t* __restrict__ mtab, int general) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x[NW];
  if (i < n) {
    load9(xs + i * 9, x);
  } else {
    set_one(x);
  }
  if constexpr (MF) {
    __shared__ mf_v4i af[MF_FRAGS * 64];
    mf_stage_operands(af, mtab, threadIdx.x, BLOCK);
    __syncthreads();
    mfma_step(x, MfFromArray{af, threadIdx.x & 63}, general != 0);
  } else {
    step(x, constant_table(ctab), general != 0, SgprBarrier());
  }
  if (i < n) store9(out + i * 9, x);
}

}  // namespace

// ===========================================================================
// host side

namespace {

std::mutex g_mu;
std::map<std::pair<int, uint32_t>, host::Tables> g_tables;
std::map<int, uint32_t*> g_err;  // address of g_err_word on each device

inline bool grid_for(uint64_t n, dim3* g) {
  const uint64_t blocks = (n + BLOCK - 1) / BLOCK;
  if (blocks > 0x7FFFFFFFull) return false;
  *g = dim3((unsigned)blocks);
  return true;
}

int current_device(int* dev) { return hipGetDevice(dev) == hipSuccess ? RLX_OK : RLX_EHIP; }

}  // namespace

namespace rlx {
namespace host {

int error_word(hipStream_t, uint32_t** out) {
  int dev;
  if (current_device(&dev)) return RLX_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_err.find(dev);
  if (it != g_err.end()) {
    *out = it->second;
    return RLX_OK;
  }
  // the word is a device variable (zero when the code object loads, one per
  // device): finding its address allocates nothing and enqueues nothing, so
  // this is safe on a stream under capture
  uint32_t* w = nullptr;
  if (hipGetSymbolAddress(reinterpret_cast<void**>(&w), HIP_SYMBOL(g_err_word)) != hipSuccess || !w)
    return RLX_EHIP;
  try {
    g_err[dev] = w;
  } catch (const std::bad_alloc&) {
    return RLX_ENOMEM;
  }
  *out = w;
  return RLX_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept in a fixed table: no
// allocation, nothing enqueued.
constexpr int MAX_DEVICES = 64;
uint8_t* g_scratch[MAX_DEVICES];

int scratch_ptr(uint8_t** out) {
  int dev;
  if (current_device(&dev)) return RLX_EHIP;
  if (dev < 0 || dev >= MAX_DEVICES) return RLX_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* a = nullptr;
    if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return RLX_EHIP;
    g_scratch[dev] = static_cast<uint8_t*>(a);
  }
  *out = g_scratch[dev];
  return RLX_OK;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

// The kernels that build the tables of level p on `s`: the 4-bit windows T,
// the folded multipliers C and matrix-core operands M of the first `rows`
// step sizes 2^g, and the 16-bit windows W.  cw and bal are the staging of
// M (FOLD_G * MF_BYTES * NW words and FOLD_G * MF_COLS * MF_ROWS bytes).
// Enqueues only; allocates and waits for nothing.
void launch_table_build(uint32_t p, int rows, uint32_t* T, uint32_t* C, uint32_t* W, uint32_t* M, uint32_t* cw,
                        int8_t* bal, hipStream_t s) {
  k_tab_base<<<1, 64, 0, s>>>(T, p);
  const int fill = TAB_ROWS * (TAB_COLS - 2);
  k_tab_fill<<<(fill + 63) / 64, 64, 0, s>>>(T);
  k_tab_fold<<<rows, 64, 0, s>>>(T, C);
  k_tab_win<<<(WIN_ROWS * WIN_COLS + 63) / 64, 64, 0, s>>>(T, W);
  k_tab_mf_c<<<(rows * MF_BYTES + 63) / 64, 64, 0, s>>>(T, cw, bal, rows);
  k_tab_mf_k<<<(rows + 63) / 64, 64, 0, s>>>(cw, bal, rows);
  k_tab_mf_frag<<<rows * MF_FRAGS, 64, 0, s>>>(bal, M, rows);
}

int tables(uint32_t p, hipStream_t s, Tables* out) {
  int dev;
  if (current_device(&dev)) return RLX_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, p);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    *out = it->second;
    return RLX_OK;
  }
  // building allocates and waits on `s`, which a stream under capture
  // must not do
  if (capturing(s)) return RLX_ECAPTURE;
  Tables t;
  if (hipMalloc(&t.T, TAB_WORDS * sizeof(uint32_t)) != hipSuccess) return RLX_ENOMEM;
  if (hipMalloc(&t.C, FOLD_WORDS * sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(t.T);
    return RLX_ENOMEM;
  }
  // the matrix-core operands, and two staging buffers freed after the build:
  // the words of the C_i and their balanced digits
  uint32_t* cw = nullptr;
  int8_t* bal = nullptr;
  auto release = [&]() {
    (void)hipFree(t.T);
    (void)hipFree(t.C);
    (void)hipFree(t.W);
    (void)hipFree(t.M);
    (void)hipFree(cw);
    (void)hipFree(bal);
  };
  if (hipMalloc(&t.W, WIN_WORDS * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&t.M, (size_t)FOLD_G * MF_LEVEL_WORDS * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&cw, (size_t)FOLD_G * MF_BYTES * NW * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&bal, (size_t)FOLD_G * MF_COLS * MF_ROWS) != hipSuccess) {
    release();
    return RLX_ENOMEM;
  }
  launch_table_build(p, FOLD_G, t.T, t.C, t.W, t.M, cw, bal, s);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    release();
    return RLX_EHIP;
  }
  (void)hipFree(cw);
  (void)hipFree(bal);
  cw = nullptr;
  bal = nullptr;
  try {
    g_tables[key] = t;
  } catch (const std::bad_alloc&) {
    release();
    return RLX_ENOMEM;
  }
  *out = t;
  return RLX_OK;
}

}  // namespace host
}  // namespace rlx

using namespace rlx::host;

namespace {

std::atomic<uint32_t> g_lanes_override{0};
std::atomic<int> g_step_kind{RLX_STEP_MFMA};

// Lanes per record: the largest power of two G <= RLX_MAX_LANES such that
// the launch stays within `target` lanes and every lane still takes at least
// `min_steps` generator steps -- or, while the launch has fewer lanes than
// one wave per SIMD (2^16), at least one step.  A lane pays one windowed
// multiplication per non-zero 16-bit digit of its index at start-up, so G
// trades start-up work against parallelism and against the length of the
// contiguous runs each store instruction writes (16 G bytes per record).
// With the matrix-core step (a cheaper step, so start-up weighs more, but
// waves that each take half as long and leave a shorter tail) the limits
// are 2^21 lanes and 8 steps, which picks G = 32 on the many-streams shape
// (65 536 x 4096: 0.372 ms against 0.411 at G = 16 and 0.427 at G = 64);
// with the vector-ALU step, 2^20 lanes and 16 steps, G = 16 there.  A single
// stream of 2^20 values ran in 32 us at G = 65536 against 68 us at 4096.
uint32_t auto_lanes(uint64_t n, uint64_t count, bool mf) {
  const uint64_t steps = count / FIELDS + 1;
  const uint64_t target = mf ? 1ull << 21 : 1ull << 20, sparse = 1ull << 16;
  const uint64_t min_steps = mf ? 8 : 16;
  uint64_t g = 1;
  for (;;) {
    const uint64_t g2 = g * 2;
    if (g2 > RLX_MAX_LANES || n > target / g2 || steps / g2 == 0) break;
    if (steps / g2 < min_steps && n > sparse / g2) break;
    g = g2;
  }
  return (uint32_t)g;
}

uint32_t lanes_for(uint64_t n, uint64_t count) {
  const uint32_t o = g_lanes_override.load(std::memory_order_relaxed);
  return o ? o : auto_lanes(n, count, g_step_kind.load(std::memory_order_relaxed) == RLX_STEP_MFMA);
}

// Argument checks shared by the generate calls; on success *lg is log2 of
// the lanes per record and *grid covers n << lg lanes.
int generate_args(const rlx_state* states, uint64_t n, uint64_t count, const void* out, uint32_t p,
                  uint32_t* lg, dim3* grid, bool record_levels = false) {
  if (!states || !out) return RLX_EINVAL;
  if (record_levels ? p != RLX_P_RECORD : !valid_p(p)) return RLX_EINVAL;
  if (!aligned(states, 16) || !aligned(out, 8)) return RLX_EINVAL;
  if (n > RLX_MAX_STREAMS || count > RLX_MAX_COUNT) return RLX_EINVAL;
  if (count > UINT64_MAX / 8 / n) return RLX_EINVAL;
  uint32_t G = lanes_for(n, count);
  if (record_levels && G > 64) G = 64;  // a record's lanes in one wave
  *lg = (uint32_t)__builtin_ctz(G);
  if (n > (UINT64_MAX >> *lg)) return RLX_EINVAL;
  return grid_for(n << *lg, grid) ? RLX_OK : RLX_EINVAL;
}

// After a generate launch without in-kernel write-back (records spanning
// several waves): advance every record by the `count` values the launch drew,
// `per_step` values per generator step, with a skip launch on the same
// stream, so the records are written only after every lane has read them.
// Records the generate kernel rejected are rejected here too (same checks,
// same error bits) and stay unchanged.
int advance_after(rlx_state* states, uint64_t n, uint64_t count, uint32_t per_step, int writeback, uint32_t p,
                  const uint32_t* W, uint32_t* err, hipStream_t s) {
  if (launch_status()) return RLX_EHIP;
  if (writeback) return RLX_OK;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  k_skip<<<grid, BLOCK, 0, s>>>(states, n, nullptr, count, p, W, err, 1, per_step);
  return launch_status();
}

// The tables of every level prepared on the current device, for the calls
// with p = RLX_P_RECORD; RLX_EINVAL beyond RLX_MAX_RECORD_LEVELS levels.
int level_set(LevelSet* L) {
  int dev;
  if (current_device(&dev)) return RLX_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  *L = LevelSet{};
  for (const auto& kv : g_tables) {
    if (kv.first.first != dev) continue;
    if (L->n == (uint32_t)MAX_RECORD_LEVELS) return RLX_EINVAL;
    L->p[L->n] = kv.first.second;
    L->C[L->n] = kv.second.C;
    L->M[L->n] = kv.second.M;
    L->W[L->n] = kv.second.W;
    ++L->n;
  }
  return RLX_OK;
}

template <Out K>
int generate_levels_impl(rlx_state* states, uint64_t n, uint64_t count, void* out, void* stream) {
  if (n == 0 || count == 0) return RLX_OK;
  uint32_t lg;
  dim3 grid;
  int rc = generate_args(states, n, count, out, RLX_P_RECORD, &lg, &grid, true);
  if (rc) return rc;
  hipStream_t s = as_stream(stream);
  LevelSet L;
  rc = level_set(&L);
  if (rc) return rc;
  uint32_t* err;
  rc = error_word(s, &err);
  if (rc) return rc;
  uint64_t* o = reinterpret_cast<uint64_t*>(out);
#define RLX_GENL(LG)                                                                                  \
  case LG:                                                                                            \
    k_generate_levels<K, LG><<<grid, BLOCK, 0, s>>>(states, (uint32_t)n, count, o, L, lg, err);       \
    break;
  switch (lg) {
    RLX_GENL(0) RLX_GENL(1) RLX_GENL(2) RLX_GENL(3) RLX_GENL(4) RLX_GENL(5) RLX_GENL(6)
    default: return RLX_EINVAL;
  }
#undef RLX_GENL
  return launch_status();
}

template <Out K, bool TRACE>
int generate_impl(rlx_state* states, uint64_t n, uint64_t count, void* out, uint64_t* trace,
                  uint64_t trace_steps, uint32_t p, void* stream, int force_general) {
  if (p == RLX_P_RECORD) {
    if (TRACE || force_general) return RLX_EINVAL;
    return generate_levels_impl<K>(states, n, count, out, stream);
  }
  if (n == 0 || count == 0) return RLX_OK;
  uint32_t lg;
  dim3 grid;
  int rc = generate_args(states, n, count, out, p, &lg, &grid);
  if (rc) return rc;
  if (TRACE) {
    if (!trace || !aligned(trace, 8)) return RLX_EINVAL;
    if (count > UINT64_MAX - 11) return RLX_EINVAL;
    const uint64_t need = (11 + count) / 12 + 1;
    if (trace_steps < need || trace_steps > UINT64_MAX / 72 / n) return RLX_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  Tables t;
  rc = tables(p, s, &t);
  if (rc) return rc;
  uint32_t* err;
  rc = error_word(s, &err);
  if (rc) return rc;
  uint64_t* o = reinterpret_cast<uint64_t*>(out);
  const uint32_t lgs = lg < 6 ? lg : 6;
  const int writeback = lg <= 6;
  const bool mf = g_step_kind.load(std::memory_order_relaxed) == RLX_STEP_MFMA;
#define RLX_GEN(L)                                                                                    \
  case L:                                                                                             \
    if (mf) {                                                                                         \
      k_generate<K, TRACE, L, true><<<grid, BLOCK, 0, s>>>(states, (uint32_t)n, count, o, trace, trace_steps, t.C, \
                                                            t.M, t.W, lg, p, err, force_general, writeback); \
    } else {                                                                                          \
      k_generate<K, TRACE, L, false><<<grid, BLOCK, 0, s>>>(states, (uint32_t)n, count, o, trace, trace_steps, t.C, \
                                                             t.M, t.W, lg, p, err, force_general, writeback); \
    }                                                                                                 \
    break;
  switch (lgs) {
    RLX_GEN(0) RLX_GEN(1) RLX_GEN(2) RLX_GEN(3) RLX_GEN(4) RLX_GEN(5) RLX_GEN(6)
  }
#undef RLX_GEN
  return advance_after(states, n, count, FIELDS, writeback, p, t.W, err, s);
}

int generate_lcg52_impl(rlx_state* states, uint64_t n, uint64_t count, double* out, uint32_t p, void* stream) {
  if (n == 0 || count == 0) return RLX_OK;
  uint32_t lg;
  dim3 grid;
  int rc = generate_args(states, n, count, out, p, &lg, &grid);
  if (rc) return rc;
  hipStream_t s = as_stream(stream);
  Tables t;
  rc = tables(p, s, &t);
  if (rc) return rc;
  uint32_t* err;
  rc = error_word(s, &err);
  if (rc) return rc;
  const uint32_t lgs = lg < 6 ? lg : 6;
  const int writeback = lg <= 6;
  const bool mf = g_step_kind.load(std::memory_order_relaxed) == RLX_STEP_MFMA;
#define RLX_GEN52(L)                                                                                        \
  case L:                                                                                                   \
    if (mf) {                                                                                               \
      k_generate_lcg52<L, true><<<grid, BLOCK, 0, s>>>(states, (uint32_t)n, count, out, t.C, t.M, t.W, lg, p, \
                                                       err, writeback);                                     \
    } else {                                                                                                \
      k_generate_lcg52<L, false><<<grid, BLOCK, 0, s>>>(states, (uint32_t)n, count, out, t.C, t.M, t.W, lg,  \
                                                        p, err, writeback);                                 \
    }                                                                                                       \
    break;
  switch (lgs) {
    RLX_GEN52(0) RLX_GEN52(1) RLX_GEN52(2) RLX_GEN52(3) RLX_GEN52(4) RLX_GEN52(5) RLX_GEN52(6)
  }
#undef RLX_GEN52
  return advance_after(states, n, count, LCG52_VALUES, writeback, p, t.W, err, s);
}

}  // namespace

extern "C" {

const char* rlx_strerror(int code) {
  switch (code) {
    case RLX_OK: return "ok";
    case RLX_EINVAL: return "invalid argument";
    case RLX_EHIP: return "HIP runtime or launch error";
    case RLX_ENOMEM: return "device allocation failed";
    case RLX_ESTATE: return "invalid stream record found on the device";
    case RLX_ECAPTURE:
      return "the stream is being captured and this luxury level's tables are not built yet: call "
             "rlx_prepare(p) before capturing";
    case RLX_ESCRATCH:
      return "the request needs more staging than the library's static device array holds "
             "(rlx_build_tables_static: rows <= RLX_FOLD_G)";
    default: return "unknown error";
  }
}

const char* rlx_version(void) { return "rlx 0.2 gfx950"; }

void rlx_constants(uint32_t m_words[18], uint32_t a_words[18]) {
  static const uint32_t a[18] = {0x00000001u, 0, 0, 0, 0, 0, 0x01000000u, 0xFFFF0000u,
                                 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu,
                                 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFEFFu};
  for (int k = 0; k < 18; ++k) {
    if (m_words) m_words[k] = m_word(k);
    if (a_words) a_words[k] = a[k];
  }
}

int rlx_prepare(uint32_t p, void* stream) {
  if (!valid_p(p)) return RLX_EINVAL;
  Tables t;
  int rc = tables(p, as_stream(stream), &t);
  if (rc) return rc;
  uint32_t* err;
  return error_word(as_stream(stream), &err);
}

int rlx_get_tables(uint32_t p, rlx_engine_tables* out, void* stream) {
  if (!out || !valid_p(p)) return RLX_EINVAL;
  Tables t;
  int rc = tables(p, as_stream(stream), &t);
  if (rc) return rc;
  out->windows = t.T;
  out->windows16 = t.W;
  out->folded = t.C;
  out->p = p;
  out->reserved = 0;
  out->mfma = t.M;
  return RLX_OK;
}

int rlx_build_tables_static(uint32_t p, uint32_t rows, uint32_t* windows, uint32_t* folded, uint32_t* windows16,
                            uint32_t* mfma, void* stream) {
  if (rows > (uint32_t)FOLD_G) return RLX_ESCRATCH;
  if (rows == 0 || !valid_p(p) || !windows || !folded || !windows16 || !mfma) return RLX_EINVAL;
  if (!aligned(windows, 4) || !aligned(folded, 4) || !aligned(windows16, 4) || !aligned(mfma, 16)) return RLX_EINVAL;
  uint8_t* sc;
  const int rc = scratch_ptr(&sc);
  if (rc) return rc;
  launch_table_build(p, (int)rows, windows, folded, windows16, mfma, reinterpret_cast<uint32_t*>(sc),
                     reinterpret_cast<int8_t*>(sc + SCRATCH_CW_BYTES), as_stream(stream));
  return launch_status();
}

int rlx_init_streams(rlx_state* states, uint64_t n, const uint64_t* ids, uint64_t id0, uint32_t p,
                     void* stream) {
  if (n == 0) return RLX_OK;
  if (!states || !valid_p(p) || !aligned(states, 16)) return RLX_EINVAL;
  if (ids && !aligned(ids, 8)) return RLX_EINVAL;
  if (!ids && id0 > UINT64_MAX - (n - 1)) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  Tables t;
  int rc = tables(p, s, &t);
  if (rc) return rc;
  k_init<<<grid, BLOCK, 0, s>>>(states, n, ids, id0, p, t.W);
  return launch_status();
}

int rlx_skip(rlx_state* states, uint64_t n, const uint64_t* steps, uint64_t steps0, uint32_t p,
             void* stream) {
  if (n == 0) return RLX_OK;
  if (!states || !(valid_p(p) || p == RLX_P_RECORD) || !aligned(states, 16)) return RLX_EINVAL;
  if (steps && !aligned(steps, 8)) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  uint32_t* err;
  if (p == RLX_P_RECORD) {
    LevelSet L;
    int rc = level_set(&L);
    if (rc) return rc;
    rc = error_word(s, &err);
    if (rc) return rc;
    k_skip_levels<<<grid, BLOCK, 0, s>>>(states, n, steps, steps0, L, err, 0, FIELDS);
    return launch_status();
  }
  Tables t;
  int rc = tables(p, s, &t);
  if (rc) return rc;
  rc = error_word(s, &err);
  if (rc) return rc;
  k_skip<<<grid, BLOCK, 0, s>>>(states, n, steps, steps0, p, t.W, err, 0, FIELDS);
  return launch_status();
}

int rlx_skip_values(rlx_state* states, uint64_t n, const uint64_t* values, uint64_t values0, uint32_t p,
                    void* stream) {
  if (n == 0) return RLX_OK;
  if (!states || !(valid_p(p) || p == RLX_P_RECORD) || !aligned(states, 16)) return RLX_EINVAL;
  if (values && !aligned(values, 8)) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  uint32_t* err;
  if (p == RLX_P_RECORD) {
    LevelSet L;
    int rc = level_set(&L);
    if (rc) return rc;
    rc = error_word(s, &err);
    if (rc) return rc;
    k_skip_levels<<<grid, BLOCK, 0, s>>>(states, n, values, values0, L, err, 1, FIELDS);
    return launch_status();
  }
  Tables t;
  int rc = tables(p, s, &t);
  if (rc) return rc;
  rc = error_word(s, &err);
  if (rc) return rc;
  k_skip<<<grid, BLOCK, 0, s>>>(states, n, values, values0, p, t.W, err, 1, FIELDS);
  return launch_status();
}

int rlx_export_ranlux(const rlx_state* states, uint64_t n, uint64_t* packed, uint32_t* carry, uint32_t* pos,
                      void* stream) {
  if (n == 0) return RLX_OK;
  if (!states || !packed || !carry || !aligned(states, 16) || !aligned(packed, 8)) return RLX_EINVAL;
  if (!aligned(carry, 4) || (pos && !aligned(pos, 4))) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  uint32_t* err;
  int rc = error_word(s, &err);
  if (rc) return rc;
  k_export<<<grid, BLOCK, 0, s>>>(states, n, packed, carry, pos, err);
  return launch_status();
}

int rlx_import_ranlux(rlx_state* states, uint64_t n, const uint64_t* packed, const uint32_t* carry,
                      const uint32_t* pos, uint32_t p, void* stream) {
  if (n == 0) return RLX_OK;
  if (!states || !packed || !carry || !valid_p(p) || !aligned(states, 16) || !aligned(packed, 8))
    return RLX_EINVAL;
  if (!aligned(carry, 4) || (pos && !aligned(pos, 4))) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  uint32_t* err;
  int rc = error_word(s, &err);
  if (rc) return rc;
  k_import<<<grid, BLOCK, 0, s>>>(states, n, packed, carry, pos, p, err);
  return launch_status();
}

int rlx_generate_f64(rlx_state* states, uint64_t n, uint64_t count, double* out, uint32_t p,
                     void* stream) {
  return generate_impl<Out::F64, false>(states, n, count, out, nullptr, 0, p, stream, 0);
}

int rlx_generate_u64(rlx_state* states, uint64_t n, uint64_t count, uint64_t* out, uint32_t p,
                     void* stream) {
  return generate_impl<Out::U64, false>(states, n, count, out, nullptr, 0, p, stream, 0);
}

int rlx_generate_normal_f64(rlx_state* states, uint64_t n, uint64_t count, double* out, uint32_t p,
                            void* stream) {
  return generate_impl<Out::NORMAL, false>(states, n, count, out, nullptr, 0, p, stream, 0);
}

int rlx_generate_f32(rlx_state* states, uint64_t n, uint64_t count, float* out, uint32_t p, void* stream) {
  if (count & 1) return RLX_EINVAL;
  return generate_impl<Out::F32, false>(states, n, count / 2, out, nullptr, 0, p, stream, 0);
}

int rlx_generate_f64_lcg52(rlx_state* states, uint64_t n, uint64_t count, double* out, uint32_t p,
                           void* stream) {
  return generate_lcg52_impl(states, n, count, out, p, stream);
}

int rlx_generate_f64_trace(rlx_state* states, uint64_t n, uint64_t count, double* out, uint64_t* trace,
                           uint64_t steps_per_stream, uint32_t p, void* stream) {
  if (n != 0 && count != 0 && !trace) return RLX_EINVAL;
  return generate_impl<Out::F64, true>(states, n, count, out, trace, steps_per_stream, p, stream, 0);
}

int rlx_test_generate_u64_general(rlx_state* states, uint64_t n, uint64_t count, uint64_t* out,
                                  uint32_t p, void* stream) {
  return generate_impl<Out::U64, false>(states, n, count, out, nullptr, 0, p, stream, 1);
}

int rlx_set_lanes_per_stream(uint32_t lanes) {
  if (lanes != 0 && (lanes > RLX_MAX_LANES || (lanes & (lanes - 1)) != 0)) return RLX_EINVAL;
  g_lanes_override.store(lanes, std::memory_order_relaxed);
  return RLX_OK;
}

uint32_t rlx_lanes_per_stream(uint64_t n, uint64_t count) { return lanes_for(n, count); }

int rlx_set_step_kernel(int kind) {
  if (kind != RLX_STEP_MFMA && kind != RLX_STEP_VALU) return RLX_EINVAL;
  g_step_kind.store(kind, std::memory_order_relaxed);
  return RLX_OK;
}

int rlx_step_kernel(void) { return g_step_kind.load(std::memory_order_relaxed); }

int rlx_check_errors(void* stream, uint32_t* flags) {
  hipStream_t s = as_stream(stream);
  uint32_t* err;
  int rc = error_word(s, &err);
  if (rc) return rc;
  if (hipStreamSynchronize(s) != hipSuccess) return RLX_EHIP;
  uint32_t h = 0;
  if (hipMemcpy(&h, err, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) return RLX_EHIP;
  if (h && hipMemset(err, 0, sizeof h) != hipSuccess) return RLX_EHIP;
  if (flags) *flags = h;
  return h ? RLX_ESTATE : RLX_OK;
}

int rlx_test_mulmod(const uint64_t* x, const uint64_t* y, uint64_t* out, uint64_t n, void* stream) {
  if (n == 0) return RLX_OK;
  if (!x || !y || !out) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  k_test_mulmod<<<grid, BLOCK, 0, as_stream(stream)>>>(x, y, out, n);
  return launch_status();
}

int rlx_test_pow(const uint64_t* base, const uint64_t* exps, uint64_t* out, uint64_t n, void* stream) {
  if (n == 0) return RLX_OK;
  if (!base || !exps || !out) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  k_test_pow<<<grid, BLOCK, 0, as_stream(stream)>>>(base, exps, out, n);
  return launch_status();
}

int rlx_test_step(const uint64_t* x, uint64_t* out, uint64_t n, uint32_t p, uint32_t g, int kind, int general,
                  void* stream) {
  if (n == 0) return RLX_OK;
  if (!x || !out || !valid_p(p) || g >= (uint32_t)FOLD_G) return RLX_EINVAL;
  if (kind != RLX_STEP_MFMA && kind != RLX_STEP_VALU) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  Tables t;
  int rc = tables(p, s, &t);
  if (rc) return rc;
  const uint32_t* ct = t.C + (size_t)g * FOLD_ROW_WORDS;
  const uint32_t* mt = t.M + (size_t)g * MF_LEVEL_WORDS;
  if (kind == RLX_STEP_MFMA) {
    k_test_step<true><<<grid, BLOCK, 0, s>>>(x, out, n, ct, mt, general);
  } else {
    k_test_step<false><<<grid, BLOCK, 0, s>>>(x, out, n, ct, mt, general);
  }
  return launch_status();
}

int rlx_test_to_ranlux(const uint64_t* x, uint64_t* d, uint32_t* carry, uint64_t n, void* stream) {
  if (n == 0) return RLX_OK;
  if (!x || !d || !carry) return RLX_EINVAL;
  dim3 grid;
  if (!grid_for(n, &grid)) return RLX_EINVAL;
  k_test_to_ranlux<<<grid, BLOCK, 0, as_stream(stream)>>>(x, d, carry, n);
  return launch_status();
}

}  // extern "C"
