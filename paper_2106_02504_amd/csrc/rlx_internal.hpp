// rlx_internal.hpp -- host-side internals shared by the translation units of
// librlx.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlx.h"

namespace rlx {
namespace host {

// Device tables of one (device, luxury level): see rlx_device.hpp.
struct Tables {
  uint32_t* T = nullptr;  // TAB_WORDS words
  uint32_t* C = nullptr;  // FOLD_WORDS words
  uint32_t* W = nullptr;  // WIN_WORDS words
  uint32_t* M = nullptr;  // RLX_FOLD_G * MF_LEVEL_WORDS words: matrix-core step operands
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

inline bool valid_p(uint32_t p) { return p >= 24 && p < (1u << 31); }

inline int launch_status() { return hipGetLastError() == hipSuccess ? RLX_OK : RLX_EHIP; }

// Tables of luxury level p on the current device, built on `s` (and waited
// for) on first use.  Thread-safe.
int tables(uint32_t p, hipStream_t s, Tables* out);

// Device error word of the current device (created zeroed on first use).
int error_word(hipStream_t s, uint32_t** out);

}  // namespace host
}  // namespace rlx
