/*
 * rlx.h -- RANLUX++ random numbers on an AMD Instinct MI355X (gfx950).
 *
 * C ABI of librlx.so.  The generator is RANLUX++ as described by Hahnfeld &
 * Moneta, "A Portable Implementation of RANLUX++" (arXiv 2106.02504):
 *
 *   - the state of a stream is the LCG state X in [0, m) with
 *     m = 2^576 - 2^240 + 1 (section 2.2), stored as nine 64-bit words
 *     (section 2), plus the position of the next 48-bit field (section 2);
 *   - one generator step is X <- A_p X mod m, A_p = a^p mod m, where a is the
 *     LCG multiplier equivalent to one subtract-with-borrow step of RANLUX
 *     and p the luxury level (section 1; the multiply and the reduction are
 *     sections 2.1 and 2.2);
 *   - the numbers of a step are obtained by converting X back to the 24
 *     RANLUX numbers (section 2.3) and taking 48 bits per value, 12 values
 *     per step (section 2.3);
 *   - seeding and skipping use exponentiation by squaring (section 2.4).
 *
 * Conventions shared by every entry point:
 *
 *   Memory     All array pointers are DEVICE pointers owned by the caller
 *              (e.g. PyTorch tensors).  The library never allocates, frees or
 *              retains caller memory.  It owns only per-(device, p) constant
 *              tables (about 38 MB per luxury level and device, kept until
 *              the process exits), the descriptors of batch plans
 *              (rlx_plan_create .. rlx_plan_destroy) and statically sized
 *              device variables (one error word per device).
 *   Streams    `stream` is a hipStream_t passed as void*; NULL is the default
 *              stream.  Work runs on the current HIP device and is enqueued
 *              asynchronously: calls return before the GPU has finished, and
 *              faults surface at the caller's next synchronisation.  The first
 *              call with a new luxury level p on a device builds that level's
 *              tables on `stream` and waits for them (about a millisecond);
 *              call rlx_prepare() first when the caller must not block.  On a
 *              stream under HIP graph capture that first call cannot allocate
 *              or wait: it returns RLX_ECAPTURE and enqueues nothing.  Once
 *              the level is prepared, the generate, seed and skip calls and
 *              rlx_plan_generate_* allocate, wait and clear nothing, so they
 *              can be captured.
 *   Errors     Functions return RLX_OK (0) or a positive error code; the
 *              library never aborts and never prints.  rlx_strerror() gives a
 *              message.  Invalid stream records found by a kernel (x >= m,
 *              pos > 11, or a luxury level different from `p`) are skipped --
 *              their outputs are left unwritten -- and flagged in the device
 *              error word, which rlx_check_errors() reads and clears.
 *   Sizes      n = 0 or count = 0 is a no-op returning RLX_OK.  One call of
 *              a generate entry point takes at most RLX_MAX_STREAMS records
 *              and RLX_MAX_COUNT values per record (RLX_EINVAL beyond).
 *   Threads    Entry points may be called from several host threads.
 *   Overlap    Output arrays must not overlap the state array or each other.
 */
#ifndef RLX_H
#define RLX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Stream record, 80 bytes, 16-byte aligned in arrays.
 *   x[9]  LCG state X, little-endian 64-bit words (x[0] least significant);
 *         must satisfy X < m.
 *   pos   number of 48-bit fields of the current step already used, 0..11.
 *         Records are kept in canonical form: the step is advanced as soon
 *         as its 12th field is used, so (x, pos) is a unique function of the
 *         number of values drawn since seeding.
 *   p     luxury level the record belongs to (>= 24). */
typedef struct rlx_state {
    uint64_t x[9];
    uint32_t pos;
    uint32_t p;
} rlx_state;

enum {
    RLX_OK = 0,
    RLX_EINVAL = 1,   /* bad argument: NULL with n > 0, p < 24, misalignment, overflow */
    RLX_EHIP = 2,     /* HIP runtime or launch error */
    RLX_ENOMEM = 3,   /* table allocation failed */
    RLX_ESTATE = 4,   /* a kernel found an invalid stream record */
    RLX_ECAPTURE = 5, /* tables of a new luxury level requested on a stream
                         under HIP graph capture (see rlx_prepare) */
    RLX_ESCRATCH = 6  /* request beyond the library's static device array
                         (rlx_build_tables_static) */
};

/* Size limits of one generate call (2^35 doubles are 256 GiB, more than
 * one device holds for a single record). */
#define RLX_MAX_STREAMS 0xFFFFFFFFull
#define RLX_MAX_COUNT   (1ull << 35)
#define RLX_MAX_LANES   65536u   /* lanes per record a generate call may use */
/* Largest segment length of a batch plan, in generator steps. */
#define RLX_MAX_SEG_BLOCKS (1ull << 26)

/* Error-word bits reported by rlx_check_errors(). */
#define RLX_ERR_BAD_P    0x1u   /* record's p differs from the call's p (or,
                                   with RLX_P_RECORD, is not prepared) */
#define RLX_ERR_BAD_POS  0x2u   /* record's pos > 11 */
#define RLX_ERR_BAD_X    0x4u   /* record's X >= m */
#define RLX_ERR_NOT_CANONICAL 0x8u  /* imported RANLUX state is not canonical */

/* Message for an error code (static string). */
const char *rlx_strerror(int code);

/* Library version, e.g. "rlx 0.2 gfx950". */
const char *rlx_version(void);

/* Build (if needed) the constant tables of luxury level p on the current
 * device, on `stream`, and wait for them.  p >= 24.  Tables: A_p folded for
 * the generator step; A_p^(j 16^i) for i < 40, j < 16 (4-bit windows, the
 * device-side engine's); and A_p^(j 65536^i) and A_p^(2^96 j 65536^i) for
 * i < 4, j < 65536 (16-bit windows, 37.7 MB per level, used by the library's
 * seeding, skipping and lane start-up; section 2.4: exponentiation by
 * windows). */
int rlx_prepare(uint32_t p, void *stream);

/* Layout of the device tables of one luxury level p (section 2.4; words are
 * 32-bit, 18 per 576-bit number, least significant first):
 *   windows[(i * RLX_TAB_COLS + j) * 18 .. + 17] = A_p^(j 16^i) mod m,
 *     i < RLX_TAB_ROWS, j < RLX_TAB_COLS.  Rows 0..15 are the 4-bit windows
 *     of a skip by k < 2^64 steps; rows RLX_SEED_ROW0.. those of a seed's
 *     exponent 2^96 id.
 *   folded[(g * 21 + j) * 18 .. + 17] = A_p^(2^g) 2^(o_j) mod m, g <
 *     RLX_FOLD_G, j < 21, o_j the limb offsets 0, 28, ..., 280, 307, ..., 550
 *     (ten 28-bit, ten 27-bit and one 26-bit limb): the folded multiplier of
 *     2^g generator steps, X <- A_p^(2^g) X = sum_j limb_j(X) C_g[j].
 *   windows16[(i * RLX_WIN16_COLS + j) * 18 .. + 17] = A_p^(j 65536^i) mod m
 *     for i < RLX_WIN16_SEED_ROW0 (16-bit windows of a skip by k < 2^64
 *     steps) and A_p^(2^96 j 65536^(i - RLX_WIN16_SEED_ROW0)) mod m for the
 *     rows from RLX_WIN16_SEED_ROW0 on (those of a seed's exponent 2^96 id,
 *     id < 2^64); i < RLX_WIN16_ROWS, j < RLX_WIN16_COLS (37.7 MB). */
#define RLX_TAB_ROWS 40
#define RLX_TAB_COLS 16
#define RLX_SEED_ROW0 24
#define RLX_FOLD_G 64
#define RLX_WIN16_ROWS 8
#define RLX_WIN16_COLS 65536
#define RLX_WIN16_SEED_ROW0 4

typedef struct rlx_engine_tables {
    const uint32_t *windows;    /* RLX_TAB_ROWS * RLX_TAB_COLS * 18 words */
    const uint32_t *folded;     /* RLX_FOLD_G * 21 * 18 words */
    const uint32_t *windows16;  /* RLX_WIN16_ROWS * RLX_WIN16_COLS * 18 words */
    uint32_t p;                 /* luxury level */
    uint32_t reserved;
    const uint32_t *mfma;       /* RLX_FOLD_G * RLX_MFMA_ROW_WORDS words: the
                                   matrix-core operands of a step by 2^g
                                   steps (row 0: the engine's step; NULL
                                   keeps the engine on the vector step) */
} rlx_engine_tables;

/* Words of one step size's matrix-core operands: nine A operands of
 * v_mfma_i32_32x32x32_i8 (three tiles of 32 output digits by three steps of
 * 32 input bytes), 64 lanes x 16 bytes each.  Lane l of operand 3 t + s
 * holds, in byte j, the balanced base-256 digit of row 32 t + (l mod 32) of
 * A_p^(2^g) 256^i mod m, where i is the input byte the generate kernels place
 * at (l div 32, j) of step s, or of K = 128 sum_i A_p^(2^g) 256^i for the
 * constant input, or 0. */
#define RLX_MFMA_ROW_WORDS (9u * 64u * 4u)

/* Size of the static device array behind rlx_build_tables_static: the
 * staging of every step size's matrix-core operands (RLX_FOLD_G x (72 x 72
 * bytes of words + 73 x 96 balanced digits)). */
#define RLX_STATIC_SCRATCH_BYTES 780288u

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): build the tables
 * of luxury level p that rlx_prepare and rlx_get_tables build, into device
 * buffers the caller owns, allocating nothing.  The staging of the
 * matrix-core operands (the library's own build allocates and frees it) lives
 * in a static device array of RLX_STATIC_SCRATCH_BYTES that each device holds
 * from the library's first use of it until the process exits.
 *   rows       number of step sizes 2^g built, g < rows, 1 <= rows <=
 *              RLX_FOLD_G (RLX_ESCRATCH beyond: more staging than the
 *              array holds; RLX_EINVAL for 0)
 *   windows    RLX_TAB_ROWS * RLX_TAB_COLS * 18 words, as rlx_engine_tables
 *   folded     rows * 21 * 18 words, as rlx_engine_tables (rows g < rows)
 *   windows16  RLX_WIN16_ROWS * RLX_WIN16_COLS * 18 words, as
 *              rlx_engine_tables
 *   mfma       rows * RLX_MFMA_ROW_WORDS words, 16-byte aligned, as
 *              rlx_engine_tables (rows g < rows)
 * The values equal those of rlx_get_tables for the same p.  The build is
 * enqueued on `stream` and the call returns without waiting, so it may be
 * captured.  Every call on one device stages through that device's one
 * array: calls that overlap on a device (other streams, or host threads)
 * race and must be ordered by the caller.  Words of folded and mfma past
 * `rows` are not written. */
int rlx_build_tables_static(uint32_t p, uint32_t rows, uint32_t *windows, uint32_t *folded,
                            uint32_t *windows16, uint32_t *mfma, void *stream);

/* Addresses of the tables of level p on the current device, for kernels
 * that run the device-side engine of rlx_engine.h (the paper's GPU use, one
 * generator per thread, section 4.2).  Builds them as rlx_prepare() does.
 * The memory is owned by the library, read-only for kernels, and valid until
 * the process ends.  RLX_EINVAL for p < 24 or out == NULL. */
int rlx_get_tables(uint32_t p, rlx_engine_tables *out, void *stream);

/* Seeding (section 2.4).  states[i] <- stream record of seed id
 * ids[i] (or id0 + i when ids == NULL) at luxury level p:
 *   x = A_p^(2^96 id) mod m applied to X = 1, pos = 0, p = p.
 * Seed ids are therefore 2^96 generator steps apart.  ids: device array of n
 * uint64 or NULL; id0 + n - 1 must not overflow 64 bits. */
int rlx_init_streams(rlx_state *states, uint64_t n, const uint64_t *ids,
                     uint64_t id0, uint32_t p, void *stream);

/* Records of several luxury levels in one call.  Passing p = RLX_P_RECORD
 * to rlx_skip, rlx_skip_values, rlx_generate_f64, rlx_generate_u64,
 * rlx_generate_normal_f64 or rlx_generate_f32 uses each record's own level
 * (its `p` field) instead of one level for all.  Every level that occurs
 * must already be prepared on the device (rlx_prepare, or an earlier call
 * with that p); records of any other level are flagged RLX_ERR_BAD_P and
 * left unchanged, their outputs unwritten.  With more than
 * RLX_MAX_RECORD_LEVELS levels prepared on the device such a call returns
 * RLX_EINVAL.  A generate call then uses at most 64 lanes per record.  The
 * step runs on the matrix cores with one multiplier per half-wave, so a
 * wave whose halves each hold records of one level (always the case with 32
 * or 64 lanes per record) runs at about the one-level speed; a half-wave
 * that mixes levels (fewer lanes per record, records not sorted by level)
 * multiplies lane by lane, at several times the vector work of a step.
 * rlx_init_streams, rlx_generate_f64_trace, rlx_generate_f64_lcg52 and
 * rlx_import_ranlux take one level (RLX_P_RECORD -> RLX_EINVAL); batch plans
 * mix levels per request (rlx_plan_create). */
#define RLX_P_RECORD 0u
#define RLX_MAX_RECORD_LEVELS 16

/* Skip-ahead (section 2.4).  For every record i with luxury level p:
 *   x <- A_p^k x mod m, pos unchanged,
 * with k = steps[i] (or steps0 when steps == NULL) GENERATOR STEPS; one step
 * is 12 values, so this advances the stream by 12 k values.  k < 2^64. */
int rlx_skip(rlx_state *states, uint64_t n, const uint64_t *steps,
             uint64_t steps0, uint32_t p, void *stream);

/* Uniform doubles (section 2.3).  For every record i (luxury level p), draw
 * `count` values into out[i * count + j], j < count, and advance the record.
 * When the lanes of one record span several waves (rlx_lanes_per_stream
 * above 64), the record is advanced by a second launch on `stream` after the
 * draws, as rlx_skip_values would, so no lane can read a record that another
 * has already advanced; this holds for every generate entry point below.
 * A value is a 48-bit field v of the step's RANLUX numbers, converted as
 * v * 2^-48 (exact; in [0, 1), 0 possible).  Field k of a step is bits
 * [48k, 48k + 48) of D = floor(X 2^576 / m), the 24 RANLUX numbers packed
 * with the oldest number in the least significant 24 bits.  out must be
 * 8-byte aligned; n * count must not overflow. */
int rlx_generate_f64(rlx_state *states, uint64_t n, uint64_t count,
                     double *out, uint32_t p, void *stream);

/* The same draws as rlx_generate_f64, as the 48-bit integers v,
 * zero-extended to 64 bits (section 2.4's integer draw). */
int rlx_generate_u64(rlx_state *states, uint64_t n, uint64_t count,
                     uint64_t *out, uint32_t p, void *stream);

/* Standard normal doubles: the value at stream position s is the
 * Box-Muller transform of the field pair of its step, positions s & ~1 and
 * s | 1 (u1, u2 their doubles): r cos(2 pi u2) for even s and r sin(2 pi u2)
 * for odd s, r = sqrt(-2 ln(1 - u1)).  So each value depends on its position
 * only, and count normals advance the record by count positions, as count
 * uniforms do.  The evaluation (rlx_gauss.hpp) uses only correctly rounded
 * binary64 operations: within 2 ulp of the exact transform in the host
 * build's checks, and the same bits on the host as on the device, but not
 * those of a CPU libm's log, sin and cos.  The paper leaves distributions to
 * the framework around the engine (section 2.4). */
int rlx_generate_normal_f64(rlx_state *states, uint64_t n, uint64_t count,
                            double *out, uint32_t p, void *stream);

/* Float32 draws, one RANLUX number each: v 2^-24 in [0, 1), exact in
 * binary32 (section 2.3 converts back to the 24-bit RANLUX numbers because
 * they are equally distributed).  A step gives 24 floats, its numbers in
 * the order the subtract-with-borrow recurrence produced them.  A record's
 * position counts 48-bit fields, which hold two numbers each, so `count`
 * (floats per record, row i at out + i * count) must be even and advances
 * the record by count / 2 positions: floats 2j and 2j + 1 of a row are the
 * low and high 24 bits of the value j that rlx_generate_u64 gives.  Odd
 * count (also with n = 0) or count / 2 > RLX_MAX_COUNT -> RLX_EINVAL.  out
 * must be 8-byte aligned. */
int rlx_generate_f32(rlx_state *states, uint64_t n, uint64_t count,
                     float *out, uint32_t p, void *stream);

/* Legacy doubles, for comparison only: the earlier conversion that section
 * 2.3 describes and rejects as biased (the top bits of X < m are 0 slightly
 * more often), 52 bits of the LCG state itself as the mantissa.  Value k of
 * a step is bits [52k, 52k + 52) of X, k = 0..10, as v 2^-52 (the top 4
 * bits of X are unused); 11 values per step, and the record's pos counts
 * these values: records with pos = 11 (or > 11) are flagged RLX_ERR_BAD_POS
 * and left unwritten.  A record moves between this call and the 48-bit
 * ones at pos = 0 only.  Layout and limits as rlx_generate_f64. */
int rlx_generate_f64_lcg52(rlx_state *states, uint64_t n, uint64_t count,
                           double *out, uint32_t p, void *stream);

/* rlx_generate_f64 that also writes the LCG state of every step it visits:
 * trace[(i * steps_per_stream + t) * 9 + w], t = 0 is the state on entry and
 * t = 1..A the states after each of the A = (pos + count) / 12 advances, so
 * steps_per_stream must be >= A + 1 for every record (all records must then
 * share one pos).  Returns RLX_EINVAL if steps_per_stream is too small for
 * pos = 11. */
int rlx_generate_f64_trace(rlx_state *states, uint64_t n, uint64_t count,
                           double *out, uint64_t *trace,
                           uint64_t steps_per_stream, uint32_t p, void *stream);

/* Skip-ahead counted in values: advance every record (luxury level p) by
 * v = values[i] (or values0 when values == NULL) draws, i.e. to position
 * pos + v: x <- A_p^((pos + v) / 12) x, pos <- (pos + v) mod 12. */
int rlx_skip_values(rlx_state *states, uint64_t n, const uint64_t *values,
                    uint64_t values0, uint32_t p, void *stream);

/* ---- RANLUX-form state (section 2: the final version stores the 24
 * RANLUX numbers packed in 576 bits plus the carry bit) ------------------ */

/* For every record: packed[9 i .. 9 i + 8] = D = floor(X 2^576 / m), the 24
 * RANLUX numbers of the current step (oldest in the least significant 24
 * bits), carry[i] = the RANLUX carry c = X - D + floor(D / 2^336) (0 or 1),
 * pos[i] = the record's pos (may be NULL).  Records with X >= m are flagged
 * RLX_ERR_BAD_X and their outputs left unwritten.  packed must be 8-byte,
 * carry and pos 4-byte aligned (RLX_EINVAL otherwise). */
int rlx_export_ranlux(const rlx_state *states, uint64_t n, uint64_t *packed,
                      uint32_t *carry, uint32_t *pos, void *stream);

/* The inverse: states[i] <- X = D - floor(D / 2^336) + c with D =
 * packed[9 i ..], c = carry[i], pos = pos[i] (or 0 when pos == NULL), p.
 * A state is imported only if it is a RANLUX state of this generator in
 * canonical form -- X < m (which excludes the degenerate state with every
 * number 2^24 - 1 and carry 1, X = m) and exporting X gives back (D, c);
 * otherwise the record is left unchanged and RLX_ERR_NOT_CANONICAL (or
 * RLX_ERR_BAD_POS for pos > 11) is flagged.  Any SWB state becomes canonical
 * after 24 steps of the subtract-with-borrow recurrence.  Alignment as for
 * rlx_export_ranlux. */
int rlx_import_ranlux(rlx_state *states, uint64_t n, const uint64_t *packed,
                      const uint32_t *carry, const uint32_t *pos, uint32_t p,
                      void *stream);

/* Lanes per stream record used by the generate calls.  G lanes of one
 * record interleave its generator steps (lane l takes steps l, l + G, ...,
 * advancing by the launch-uniform multiplier A_p^G), and their values are
 * staged through LDS so that stores write contiguous runs of the output row.
 * By default G is picked from n and count (rlx_lanes_per_stream reports the
 * pick); rlx_set_lanes_per_stream(G) forces a power of two G <=
 * RLX_MAX_LANES for all
 * later calls in the process (0 restores the automatic pick).  The values
 * produced never depend on G. */
int rlx_set_lanes_per_stream(uint32_t lanes);
uint32_t rlx_lanes_per_stream(uint64_t n, uint64_t count);

/* How the generate calls (rlx_generate_f64, _u64, _f32, _normal_f64,
 * _f64_trace and rlx_test_generate_u64_general) multiply the state by the
 * constant A_p^G in each generator step (sections 2.1, 2.2).  Both are exact
 * and give bit-identical values and records:
 *   RLX_STEP_MFMA  (default) the product as a contraction of the state's 72
 *                  bytes with the byte digits of A_p^G 256^i mod m on the
 *                  int8 matrix cores (v_mfma_i32_32x32x32_i8: exact 32-bit
 *                  sums of 8-bit products), then a carry chain and the
 *                  reduction mod m on the vector ALU;
 *   RLX_STEP_VALU  the product as 32-bit multiply-adds on the vector ALU
 *                  with the reduction folded into the multiplier.
 * rlx_set_step_kernel applies to all later calls in the process and returns
 * RLX_EINVAL for any other value; rlx_step_kernel reports the current one.
 * The batch plans (rlx_plan_generate_*) and the legacy 52-bit doubles
 * (rlx_generate_f64_lcg52) follow the same setting at launch. */
#define RLX_STEP_MFMA 0
#define RLX_STEP_VALU 1
int rlx_set_step_kernel(int kind);
int rlx_step_kernel(void);

/* ---- batched generation ---------------------------------------------------
 * Many requests, each a window of one stream, in ONE launch that
 * fuses skip-ahead, generation and conversion.  A request reads its stream
 * record without modifying it, so several requests may read the same record
 * (e.g. consecutive windows of one stream) and their results are exactly the
 * values a plain rlx_generate_f64 would produce at those positions. */

/* One request: values start, start + 1, ..., start + count - 1 of the stream
 * whose current position is record `state` (position 0 = the record's next
 * value), written to out[out_offset .. out_offset + count).  p must be the
 * record's luxury level.  The library does not know the length of the
 * states array a plan will run on: the caller guarantees that every
 * request's `state` indexes a record of it (the Python binding checks). */
typedef struct rlx_request {
    uint64_t state;       /* index into the states array */
    uint64_t start;       /* first value, counted from the record's position */
    uint64_t count;       /* number of values */
    uint64_t out_offset;  /* element offset in the output array */
    uint32_t p;           /* luxury level */
    uint32_t reserved;    /* must be 0 */
} rlx_request;

/* A plan holds the device descriptors of a batch (library-owned device
 * memory).  The planner splits every request into segments of at most
 * `seg_blocks` (1 .. RLX_MAX_SEG_BLOCKS) generator steps, gives each segment `lanes` (a power of two <=
 * 64) lanes that interleave its steps, and groups segments of one luxury
 * level into work items of 64 lanes.  At most 16 distinct luxury levels per
 * plan. */
typedef struct rlx_plan rlx_plan;

/* Create a plan for n host requests (capacity for later updates is sized
 * for `capacity_segments` segments, at most 2^32 - 1; 0 = exactly what these
 * requests need).  A plan belongs to the device current at creation: update
 * and generate calls made with another device current return RLX_EINVAL.
 * Builds the tables of every luxury level used (synchronising `stream`
 * once per new level) and uploads the descriptors on `stream`. */
int rlx_plan_create(rlx_plan **plan, const rlx_request *reqs, uint64_t n,
                    uint32_t lanes, uint64_t seg_blocks,
                    uint64_t capacity_segments, void *stream);

/* Re-plan new requests into an existing plan's device buffers (same lanes and
 * seg_blocks) with an asynchronous upload on `stream`; RLX_EINVAL if they
 * need more segments than the plan's capacity.  The buffers keep their
 * addresses, so a HIP graph that captured rlx_plan_generate_* replays the
 * new requests. */
int rlx_plan_update(rlx_plan *plan, const rlx_request *reqs, uint64_t n, void *stream);

/* Number of segments and work items of the plan's current requests. */
int rlx_plan_info(const rlx_plan *plan, uint64_t *segments, uint64_t *items,
                  uint64_t *total_values);

/* Run the plan: one kernel on `stream`, one wave per work item (no
 * allocation, no synchronisation, no memset: capturable).
 * The launch reads the work list, its length and the luxury tables from the
 * plan's device memory, so a captured launch runs whatever requests the plan
 * holds when it is replayed.  `states` are read only.  out must hold every
 * request's range. */
int rlx_plan_generate_f64(rlx_plan *plan, const rlx_state *states, double *out, void *stream);
int rlx_plan_generate_u64(rlx_plan *plan, const rlx_state *states, uint64_t *out, void *stream);
/* Float32 form of a plan (as rlx_generate_f32): each request's positions
 * give two floats each, so request value j goes to
 * out[2 (out_offset + j)] and out[2 (out_offset + j) + 1]; out must hold
 * 2 (out_offset + count) floats for every request. */
int rlx_plan_generate_f32(rlx_plan *plan, const rlx_state *states, float *out, void *stream);

/* Free the plan (synchronises the device first). */
int rlx_plan_destroy(rlx_plan *plan);

/* Host-only dry run of the planner (no GPU needed): validates the requests
 * exactly as rlx_plan_create does and reports what a plan would hold.  If
 * `segments` is not NULL it receives up to max_segments rows of six uint64
 * (state, first block, output index of field 0 of that block as int64,
 * lo, hi, nblocks | level slot << 32) in launch order: items in decreasing
 * cost, segments within an item consecutive. */
int rlx_plan_dry_run(const rlx_request *reqs, uint64_t n, uint32_t lanes,
                     uint64_t seg_blocks, uint64_t *n_segments, uint64_t *n_items,
                     uint64_t *total_values, uint64_t *segments, uint64_t max_segments);

/* Synchronise `stream`, then read and clear the device error word of the
 * current device: *flags receives the RLX_ERR_* bits set by kernels since
 * the last call.  Returns RLX_ESTATE if any bit was set. */
int rlx_check_errors(void *stream, uint32_t *flags);

/* ---- host-only introspection (no GPU needed) ---------------------------- */

/* The modulus m and the multiplier a (one SWB step) as eighteen 32-bit
 * words, least significant first. */
void rlx_constants(uint32_t m_words[18], uint32_t a_words[18]);

/* ---- test-only entry points ----------------------------------------------
 * These run the library's generic 576-bit arithmetic on arbitrary operands so
 * that tests can reach rare branches.  Arrays are device arrays of n records
 * of nine uint64 words. */

/* out[i] = x[i] * y[i] mod m (sections 2.1, 2.2): the full 1152-bit product
 * reduced to the canonical residue.  x[i], y[i] < 2^576 (need not be < m). */
int rlx_test_mulmod(const uint64_t *x, const uint64_t *y, uint64_t *out,
                    uint64_t n, void *stream);

/* out[i] = base[i]^e mod m with e = exps[3 i] + 2^64 exps[3 i + 1] +
 * 2^128 exps[3 i + 2] (square and multiply). base[i] < 2^576. */
int rlx_test_pow(const uint64_t *base, const uint64_t *exps, uint64_t *out,
                 uint64_t n, void *stream);

/* The conversion of section 2.3 on canonical X (< m): d[i] = the 24 RANLUX
 * numbers packed as D = floor(X 2^576 / m) (nine words), carry[i] = the
 * RANLUX carry bit c = X - D + floor(D / 2^336). */
int rlx_test_to_ranlux(const uint64_t *x, uint64_t *d, uint32_t *carry,
                       uint64_t n, void *stream);

/* Test-only: the device-side engine of rlx_engine.h driven from a kernel
 * written as user code, one thread per record:
 *   mode 0  load the record, draw `count` doubles into out[i * count + j]
 *           (rlx_engine_next_f64), store the record;
 *   mode 1  as 0 after seeding record i with id i (rlx_engine_seed);
 *   mode 2  as 0 after skipping i generator steps (rlx_engine_skip);
 *   mode 3  as 0 with rlx_engine_next_normal;
 *   mode 4  as 0 with rlx_engine_next_u48 (bits in out);
 *   mode 5  out[i] = the sum, in draw order, of `count` doubles (the
 *           paper's GPU benchmark, section 4.2); store the record;
 *   mode 6  as 0, but thread i draws in bursts of (i mod 3) + 1 values
 *           inside per-thread branches (divergent calls);
 *   mode 7  as 0 with rlx_engine_next_f32x2: slot j of the row holds the
 *           two floats of position j (the row as floats is what
 *           rlx_generate_f32 writes for 2 count floats). */
int rlx_test_engine(rlx_state *states, uint64_t n, uint64_t count,
                    double *out, uint32_t mode, uint32_t p, void *stream);

/* out[i] = A_p^(2^g) x[i] mod m: one generator step by 2^g steps (g <
 * RLX_FOLD_G) with the step kernel `kind` (RLX_STEP_MFMA or RLX_STEP_VALU)
 * that the generate calls use, on arbitrary x[i] < m (sections 2.1, 2.2).
 * general != 0 sends the final fold through its general branch.  Lanes past
 * n run on x = 1 and store nothing. */
int rlx_test_step(const uint64_t *x, uint64_t *out, uint64_t n, uint32_t p,
                  uint32_t g, int kind, int general, void *stream);

/* Instruction-rate microbenchmark of one unit the kernels use: n_threads
 * lanes (a multiple of 256) each run `iters` iterations of independent
 * chains of one instruction kind and write one word to out[i]:
 *   kind 0  v_mad_u64_u32 (32 x 32 + 64 -> 64 bits), 64 per iteration
 *   kind 1  add-with-carry chains (v_add_co_u32 / v_addc_co_u32), 80 vector
 *           instructions per iteration, 64 of them with carry in or out
 *   kind 2  v_fma_f64, 64 per iteration
 *   kind 3  v_mfma_i32_32x32x32_i8 (65536 int8 operations each), 18 per
 *           iteration per wave
 * Time the launch with events to get the issue rate; the values written are
 * meaningless. */
int rlx_test_rates(int kind, uint32_t iters, uint32_t *out, uint64_t n_threads, void *stream);

/* rlx_generate_u64 with every rare-case branch of the step and the
 * conversion taken by all lanes (the exact general code), so that the general
 * code can be compared with the fast path on ordinary inputs. */
int rlx_test_generate_u64_general(rlx_state *states, uint64_t n, uint64_t count,
                                  uint64_t *out, uint32_t p, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RLX_H */
