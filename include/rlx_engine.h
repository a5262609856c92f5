/* rlx_engine.h -- RANLUX++ inside user HIP kernels (gfx950): a per-thread
 * generator in registers.
 *
 * The paper's GPU use (section 4.2) gives every thread its own generator and
 * draws numbers one at a time inside the user's kernel.  This header is that
 * interface, header-only, on the same arithmetic as librlx.so:
 *
 *   __global__ void k(rlx_state* st, rlx_engine_tables t, ...) {
 *     rlx_engine e;
 *     rlx_engine_load(e, st + i);                 // or rlx_engine_seed(e, id, t)
 *     double u = rlx_engine_next_f64(e, t);       // ... as often as needed
 *     float2 f = rlx_engine_next_f32x2(e, t);     // or two 24-bit floats
 *     rlx_engine_store(e, st + i, t.p);
 *   }
 *
 * with `t` from rlx_get_tables() on the host, passed by value as a kernel
 * argument (so the table address is uniform and the step's multiplier is
 * read with scalar loads).  The values are exactly those of
 * rlx_generate_f64/u64 and rlx_generate_normal_f64 for the same record, and
 * records move freely between the two interfaces.
 *
 * Divergence.  The paper reports that threads which advance their
 * generators at different times stall their warp (more than 80 s against
 * 11.8 s, section 4.2): every advance is a 576-bit multiplication, and a
 * wave executes it once for each distinct group of lanes that needs it.  The
 * engine advances lazily and wave-synchronously: a lane's next state is
 * computed any time before its 12th value of the step is used, and as soon
 * as one lane of the wave reaches that point, every lane that has not yet
 * advanced does so in the same pass.  Lanes at staggered positions then
 * share one multiplication per 12 draws, as lanes in step do; only the
 * cheap conversion of the next state to RANLUX numbers stays per lane.
 * Calls may still be made under divergent control flow (each lane always
 * advances in time for itself); convergent calls are what make them cheap.
 *
 * Advance.  When the whole wave is active at an advance (the convergent
 * case) the step runs on the int8 matrix cores for all 64 lanes at once
 * (rlx_mfma.hpp, the library's step, with the operands of A_p from
 * t.mfma); otherwise, or with t.mfma == NULL, on the vector ALU.  Both give
 * the same state.
 *
 * Cost: about 40 VGPRs per engine (state, RANLUX numbers, position), plus
 * the matrix-core step's 32 accumulators at an advance.  Give the kernel
 * __attribute__((amdgpu_waves_per_eu(3))) (or a similar bound) so the
 * compiler keeps those in ordinary registers instead of spilling to the
 * accumulation registers.
 */
#ifndef RLX_ENGINE_H
#define RLX_ENGINE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlx.h"
#include "rlx_arith.hpp"
#include "rlx_gauss.hpp"
#include "rlx_mfma.hpp"

/* One generator: the step t being drawn from and its position. */
struct rlx_engine {
    uint32_t x[18];   /* LCG state X_t, or X_{t+1} once `ahead` is set */
    uint32_t d[18];   /* D of step t: its 24 RANLUX numbers, packed (section 2.3) */
    uint32_t pos;     /* values of step t already used, 0..11 */
    uint32_t carry;   /* RANLUX carry of step t: X_t = D - (D >> 336) + carry */
    uint32_t ahead;   /* x already holds X_{t+1} */
};

namespace rlx_engine_detail {

/* Start step t from its state X_t at position pos. */
__device__ __forceinline__ void set_state(rlx_engine& e, const uint32_t (&x)[rlx::NW], uint32_t pos) {
#pragma unroll
    for (int k = 0; k < rlx::NW; ++k) e.x[k] = x[k];
    rlx::to_ranlux(e.x, e.d, false);
    e.carry = rlx::ranlux_carry(e.x, e.d);
    e.pos = pos;
    e.ahead = 0;
}

/* X_t of the current step (from D and the carry once x has moved on). */
__device__ __forceinline__ void current_state(const rlx_engine& e, uint32_t (&x)[rlx::NW]) {
    if (e.ahead) {
        (void)rlx::from_ranlux(e.d, e.carry, x);
    } else {
#pragma unroll
        for (int k = 0; k < rlx::NW; ++k) x[k] = e.x[k];
    }
}

/* x <- A x for A = product of the 16-bit window entries selected by the
 * digits of the exponent k (rows row0, row0 + 1, ... of windows16:
 * A_p^(j 65536^i), or its seed rows).  With from_one, x is 1 on entry and
 * the first non-zero digit's entry is copied instead of multiplied. */
__device__ __forceinline__ void pow_windows16(uint32_t (&x)[rlx::NW], uint64_t k, const uint32_t* w16, int row0,
                                              bool from_one) {
    for (int d = 0; d < 4 && (k >> (16 * d)) != 0; ++d) {
        const uint32_t v = (uint32_t)(k >> (16 * d)) & 0xFFFFu;
        if (v == 0) continue;
        const uint32_t* w = w16 + ((size_t)(row0 + d) * RLX_WIN16_COLS + v) * rlx::NW;
        uint32_t y[rlx::NW];
#pragma unroll
        for (int i = 0; i < rlx::NW; ++i) y[i] = w[i];
        if (from_one) {
#pragma unroll
            for (int i = 0; i < rlx::NW; ++i) x[i] = y[i];
            from_one = false;
        } else {
            uint32_t r[rlx::NW];
            rlx::mulmod_generic(x, y, r);
#pragma unroll
            for (int i = 0; i < rlx::NW; ++i) x[i] = r[i];
        }
    }
}

/* The wave-synchronised lazy advance (see the header comment), then the
 * move to the next step once the current one is used up.  When every lane
 * of the wave is active (the usual, convergent call) the step runs on the
 * matrix cores for all 64 lanes (rlx_mfma.hpp, operands of A_p read through
 * the L1) and the lanes that have not advanced yet take the result; under
 * divergent control flow, or without matrix-core operands in the tables,
 * the lanes that need it take the vector step.  Both give the same X. */
__device__ __forceinline__ void before_draw(rlx_engine& e, const rlx_engine_tables& t) {
    if (__any(!e.ahead && e.pos == 11)) {
        if (t.mfma != nullptr && __builtin_amdgcn_read_exec() == ~0ull) {
            uint32_t y[rlx::NW];
#pragma unroll
            for (int k = 0; k < rlx::NW; ++k) y[k] = e.x[k];
            rlx::mfma_step(y, rlx::MfFromBuffer(t.mfma, __lane_id()), false);
            if (!e.ahead) {
#pragma unroll
                for (int k = 0; k < rlx::NW; ++k) e.x[k] = y[k];
                e.ahead = 1;
            }
        } else if (!e.ahead) {
            rlx::step(e.x, rlx::constant_table(t.folded), false, rlx::SgprBarrier());
            e.ahead = 1;
        }
    }
}

__device__ __forceinline__ void after_draw(rlx_engine& e) {
    if (++e.pos == 12) {
        rlx::to_ranlux(e.x, e.d, false);  /* x holds X_{t+1}: before_draw ran at pos 11 */
        e.carry = rlx::ranlux_carry(e.x, e.d);
        e.pos = 0;
        e.ahead = 0;
    }
}

/* Words 3i .. 3i + 2 of D hold fields 2i and 2i + 1; i is a per-lane value,
 * so the pair is picked with selects (5 per word) and D stays in registers. */
__device__ __forceinline__ void pair_words(const rlx_engine& e, uint32_t i, uint32_t& w0, uint32_t& w1,
                                           uint32_t& w2) {
    w0 = e.d[0];
    w1 = e.d[1];
    w2 = e.d[2];
#pragma unroll
    for (uint32_t k = 1; k < 6; ++k) {
        const bool hit = i == k;
        w0 = hit ? e.d[3 * k] : w0;
        w1 = hit ? e.d[3 * k + 1] : w1;
        w2 = hit ? e.d[3 * k + 2] : w2;
    }
}

}  // namespace rlx_engine_detail

/* Load a record written by librlx (or by rlx_engine_store).  Returns false,
 * leaving the engine unusable, if the record is not canonical (pos > 11 or
 * X >= m); the luxury level is the caller's to check. */
__device__ __forceinline__ bool rlx_engine_load(rlx_engine& e, const rlx_state* rec) {
    uint32_t x[rlx::NW];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        x[2 * k] = (uint32_t)rec->x[k];
        x[2 * k + 1] = (uint32_t)(rec->x[k] >> 32);
    }
    const uint32_t pos = rec->pos;
    if (pos > 11 || rlx::geq_m(x)) return false;
    rlx_engine_detail::set_state(e, x, pos);
    return true;
}

/* Write the engine back as a record of level p. */
__device__ __forceinline__ void rlx_engine_store(const rlx_engine& e, rlx_state* rec, uint32_t p) {
    uint32_t x[rlx::NW];
    rlx_engine_detail::current_state(e, x);
#pragma unroll
    for (int k = 0; k < 9; ++k) rec->x[k] = ((uint64_t)x[2 * k + 1] << 32) | x[2 * k];
    rec->pos = e.pos;
    rec->p = p;
}

/* Seed with stream id (section 2.4): X = A_p^(2^96 id), position 0 -- the
 * record rlx_init_streams writes for that id.  One table entry per non-zero
 * 16-bit digit of id: ids below 2^16 are a copy. */
__device__ __forceinline__ void rlx_engine_seed(rlx_engine& e, uint64_t id, const rlx_engine_tables& t) {
    uint32_t x[rlx::NW];
#pragma unroll
    for (int k = 0; k < rlx::NW; ++k) x[k] = k == 0 ? 1u : 0u;
    rlx_engine_detail::pow_windows16(x, id, t.windows16, RLX_WIN16_SEED_ROW0, true);
    rlx_engine_detail::set_state(e, x, 0);
}

/* Skip k generator steps (12 k values), position unchanged (section 2.4):
 * one multiplication per non-zero 16-bit digit of k. */
__device__ __forceinline__ void rlx_engine_skip(rlx_engine& e, uint64_t k, const rlx_engine_tables& t) {
    uint32_t x[rlx::NW];
    rlx_engine_detail::current_state(e, x);
    rlx_engine_detail::pow_windows16(x, k, t.windows16, 0, false);
    rlx_engine_detail::set_state(e, x, e.pos);
}

/* Next 48-bit value: field pos of step t, bits [48 pos, 48 pos + 48) of D. */
__device__ __forceinline__ uint64_t rlx_engine_next_u48(rlx_engine& e, const rlx_engine_tables& t) {
    rlx_engine_detail::before_draw(e, t);
    uint32_t w0, w1, w2;
    rlx_engine_detail::pair_words(e, e.pos >> 1, w0, w1, w2);
    const uint64_t v = (e.pos & 1u) ? (((uint64_t)(w2 >> 16) << 32) | __builtin_amdgcn_alignbit(w2, w1, 16))
                                    : (((uint64_t)(w1 & 0xFFFFu) << 32) | w0);
    rlx_engine_detail::after_draw(e);
    return v;
}

/* Next uniform double v 2^-48 in [0, 1) (exact). */
__device__ __forceinline__ double rlx_engine_next_f64(rlx_engine& e, const rlx_engine_tables& t) {
    return (double)rlx_engine_next_u48(e, t) * 0x1p-48;
}

/* Next position as two float32 values, its RANLUX numbers v 2^-24 (exact),
 * the older number in .x: the floats rlx_generate_f32 writes there. */
__device__ __forceinline__ float2 rlx_engine_next_f32x2(rlx_engine& e, const rlx_engine_tables& t) {
    const uint64_t v = rlx_engine_next_u48(e, t);
    return make_float2((float)(uint32_t)(v & 0xFFFFFFu) * 0x1p-24f, (float)(uint32_t)(v >> 24) * 0x1p-24f);
}

/* Next standard normal: Box-Muller on the field pair of the position, as
 * rlx_generate_normal_f64 (r = sqrt(-2 ln(1 - u1)) from the pair's even
 * field, r cos(2 pi u2) at even and r sin(2 pi u2) at odd positions). */
__device__ __forceinline__ double rlx_engine_next_normal(rlx_engine& e, const rlx_engine_tables& t) {
    rlx_engine_detail::before_draw(e, t);
    uint32_t w0, w1, w2;
    rlx_engine_detail::pair_words(e, e.pos >> 1, w0, w1, w2);
    double zc, zs;
    rlx::gauss::box_muller(w0, w1, w2, zc, zs);  /* the bulk kernels' evaluation, so the bits agree */
    const double z = (e.pos & 1u) ? zs : zc;
    rlx_engine_detail::after_draw(e);
    return z;
}

#endif /* RLX_ENGINE_H */
