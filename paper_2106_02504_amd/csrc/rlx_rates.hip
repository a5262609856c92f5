// rlx_rates.hip -- instruction-rate microbenchmarks of the units the
// generator's kernels use (test-only entry point rlx_test_rates): the
// measured issue rates are the denominators of the compute-side rooflines.
//
// Each kernel runs `iters` iterations of a fully unrolled body of
// independent dependency chains of one instruction kind, so that issue, not
// latency, sets the time:
//   kind 0  v_mad_u64_u32   64 per iteration (8 chains; each multiplies the
//                           low word of the next chain's accumulator, which
//                           keeps the compiler from merging them)
//   kind 1  v_add_co_u32 / v_addc_co_u32   64 per iteration (8 chains of
//                           8-word additions, the carry passed along)
//   kind 2  v_fma_f64       64 per iteration (8 chains)
//   kind 3  v_mfma_i32_32x32x32_i8         18 per iteration (6 accumulators
//                           of 3 operand pairs, as in a generator step)
// plus a few loop-control instructions per iteration.  Every lane writes one
// word of its results to out[i] so that nothing is dead.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rlx.h"
#include "rlx_arith.hpp"
#include "rlx_internal.hpp"
#include "rlx_mfma.hpp"

using namespace rlx;

namespace {

constexpr int RATE_BLOCK = 256;

__global__ __launch_bounds__(RATE_BLOCK) void k_rate_mad(uint32_t iters, uint32_t seed, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * RATE_BLOCK + threadIdx.x;
  uint64_t acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = (uint64_t)(i + k) * 0x9E3779B9u;
  const uint32_t m0 = seed | 1u, m1 = seed * 3u + 7u;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 64; ++k) acc[k & 7] = (uint64_t)(uint32_t)acc[(k + 1) & 7] * ((k & 1) ? m0 : m1) + acc[k & 7];
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= (uint32_t)acc[k] ^ (uint32_t)(acc[k] >> 32);
  out[i] = r;
}

__global__ __launch_bounds__(RATE_BLOCK) void k_rate_addc(uint32_t iters, uint32_t seed, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * RATE_BLOCK + threadIdx.x;
  uint32_t x[8][8], y[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    y[k] = seed * (k + 1) + i;
#pragma unroll
    for (int w = 0; w < 8; ++w) x[k][w] = i * (w + 3) + k;
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < 8; ++w) x[k][w] = addc(x[k][w], y[(k + w) & 7], c);
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int w = 0; w < 8; ++w) r ^= x[k][w];
  out[i] = r;
}

__global__ __launch_bounds__(RATE_BLOCK) void k_rate_fma(uint32_t iters, uint32_t seed, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * RATE_BLOCK + threadIdx.x;
  double d[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) d[k] = (double)(i + k) * 1e-9;
  const double m = 1.0 - 1e-12 * (double)(seed & 255u), c = 1e-15;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 64; ++k) d[k & 7] = __builtin_fma(d[k & 7], m, c);
  }
  double s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += d[k];
  out[i] = (uint32_t)(s * 1e6);
}

__global__ __launch_bounds__(RATE_BLOCK) void k_rate_mfma(uint32_t iters, uint32_t seed, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * RATE_BLOCK + threadIdx.x;
  mf_v4i a[3], b[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) a[k] = mf_v4i{(int)(i * 3 + k), (int)(i ^ k), (int)seed, (int)(i + k)};
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] = mf_v4i{(int)(i * 7 + k), (int)(seed ^ k), (int)i, (int)(i - k)};
  mf_v16i acc[6] = {};
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 18; ++k) acc[k % 6] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[k / 6], b[k & 1], acc[k % 6], 0, 0, 0);
  }
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int j = 0; j < 16; ++j) r ^= (uint32_t)acc[c][j];
  out[i] = r;
}

}  // namespace

extern "C" int rlx_test_rates(int kind, uint32_t iters, uint32_t* out, uint64_t n_threads, void* stream) {
  if (!out || n_threads == 0 || n_threads % RATE_BLOCK != 0 || n_threads / RATE_BLOCK > 0x7FFFFFFFull)
    return RLX_EINVAL;
  const dim3 grid((unsigned)(n_threads / RATE_BLOCK));
  hipStream_t s = rlx::host::as_stream(stream);
  switch (kind) {
    case 0: k_rate_mad<<<grid, RATE_BLOCK, 0, s>>>(iters, 12345u, out); break;
    case 1: k_rate_addc<<<grid, RATE_BLOCK, 0, s>>>(iters, 12345u, out); break;
    case 2: k_rate_fma<<<grid, RATE_BLOCK, 0, s>>>(iters, 12345u, out); break;
    case 3: k_rate_mfma<<<grid, RATE_BLOCK, 0, s>>>(iters, 12345u, out); break;
    default: return RLX_EINVAL;
  }
  return rlx::host::launch_status();
}
