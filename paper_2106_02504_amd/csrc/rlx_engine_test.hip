// rlx_engine_test.hip -- a kernel written as user code against the public
// device-side engine (rlx_engine.h), exported as rlx_test_engine for the
// tests and the benchmark.  It includes only the public headers, as a user
// kernel would.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rlx.h"
#include "rlx_engine.h"

namespace {

constexpr int ENGINE_BLOCK = 256;

// One thread per record; see rlx.h for the modes (one instantiation each,
// so every kernel holds only what its mode uses).  At most 3 waves per SIMD,
// as rlx_engine.h suggests: the matrix-core advance's accumulators then stay
// in ordinary registers (1.36 times the 5-wave vector-step kernel's speed on
// the paper's 1024 x 128 x 10^6 sum).
template <uint32_t mode>
__global__ __launch_bounds__(ENGINE_BLOCK) __attribute__((amdgpu_waves_per_eu(3))) void k_engine(
    rlx_state* __restrict__ st, uint64_t n, uint64_t count, double* __restrict__ out, rlx_engine_tables t) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rlx_engine e;
  if constexpr (mode == 1) {
    rlx_engine_seed(e, i, t);
  } else {
    if (!rlx_engine_load(e, st + i)) return;
  }
  if constexpr (mode == 2) rlx_engine_skip(e, i, t);
  if constexpr (mode == 5) {
    double sum = 0.0;
    for (uint64_t j = 0; j < count; ++j) sum += rlx_engine_next_f64(e, t);
    out[i] = sum;
  } else if constexpr (mode == 6) {
    // divergent calls: in each round, thread i draws (i mod 3) + 1 values
    // inside a branch of its own, so lanes of a wave call the engine at
    // different times and positions
    double* row = out + i * count;
    const uint32_t burst = (uint32_t)(i % 3) + 1;
    uint64_t j = 0;
    while (j < count) {
      if ((i & 1) == 0) {
        for (uint32_t b = 0; b < burst && j < count; ++b) row[j++] = rlx_engine_next_f64(e, t);
      } else {
        for (uint32_t b = 0; b < burst && j < count; ++b) row[j++] = rlx_engine_next_f64(e, t);
        __builtin_amdgcn_s_sleep(1);
      }
    }
  } else {
    double* row = out + i * count;
    for (uint64_t j = 0; j < count; ++j) {
      double v;
      if constexpr (mode == 3) {
        v = rlx_engine_next_normal(e, t);
      } else if constexpr (mode == 7) {
        const float2 f = rlx_engine_next_f32x2(e, t);
        __builtin_memcpy(&v, &f, 8);
      } else if constexpr (mode == 4) {
        const uint64_t u = rlx_engine_next_u48(e, t);
        __builtin_memcpy(&v, &u, 8);
      } else {
        v = rlx_engine_next_f64(e, t);
      }
      row[j] = v;
    }
  }
  rlx_engine_store(e, st + i, t.p);
}

}  // namespace

extern "C" int rlx_test_engine(rlx_state* states, uint64_t n, uint64_t count, double* out, uint32_t mode,
                               uint32_t p, void* stream) {
  if (n == 0) return RLX_OK;
  if (!states || !out || mode > 7) return RLX_EINVAL;
  if ((reinterpret_cast<uintptr_t>(states) & 15) != 0 || (reinterpret_cast<uintptr_t>(out) & 7) != 0)
    return RLX_EINVAL;
  if (n > RLX_MAX_STREAMS || (mode != 5 && count > UINT64_MAX / 8 / n)) return RLX_EINVAL;
  rlx_engine_tables t;
  const int rc = rlx_get_tables(p, &t, stream);
  if (rc) return rc;
  const uint64_t blocks = (n + ENGINE_BLOCK - 1) / ENGINE_BLOCK;
  if (blocks > 0x7FFFFFFFull) return RLX_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  switch (mode) {
#define RLX_ENGINE_MODE(M) \
  case M: k_engine<M><<<(unsigned)blocks, ENGINE_BLOCK, 0, s>>>(states, n, count, out, t); break;
    RLX_ENGINE_MODE(0) RLX_ENGINE_MODE(1) RLX_ENGINE_MODE(2) RLX_ENGINE_MODE(3) RLX_ENGINE_MODE(4)
    RLX_ENGINE_MODE(5) RLX_ENGINE_MODE(6) RLX_ENGINE_MODE(7)
#undef RLX_ENGINE_MODE
  }
  return hipGetLastError() == hipSuccess ? RLX_OK : RLX_EHIP;
}
