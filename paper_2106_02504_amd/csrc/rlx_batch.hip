// rlx_batch.hip -- batched generation: planner and one fused kernel.
//
// A batch is a list of requests, each a window [start, start + count) of one
// stream (values counted from field 0 of the record's current step).  The
// planner (host) cuts every request into segments of at most `seg_blocks`
// generator steps and groups segments of the same luxury level into work
// items of 64 lanes (64 / G segments of G lanes each).  One kernel then
// runs one wave per item; inside an item every segment is run by G lanes
// exactly as the plain kernel runs a record: lane l starts at the segment's
// block l (skip by 16-bit windows, section 2.4), then takes every G-th block
// with the multiplier A^G, converts (section 2.3) and stores through LDS.
// Records are only read.
//
// Segments are sorted by length (longest first) inside a level and items by
// cost, and the hardware dispatches waves in item order, so late waves get
// short items (longest-processing-time order); long requests are cut so
// that no item dominates the launch.  One wave per item, rather than
// persistent waves popping items from a counter, keeps the kernel's
// registers low: with the vector step it ran at 5 waves per SIMD against 4
// for the persistent form; with the matrix-core step it runs at 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "rlx.h"
#include "rlx_arith.hpp"
#include "rlx_device.hpp"
#include "rlx_internal.hpp"
#include "rlx_mfma.hpp"

using namespace rlx;
using namespace rlx::host;

namespace {

constexpr int MAX_LEVELS = 16;

// One segment: blocks block .. block + nblocks - 1 of record `state` (block 0
// is the record's current LCG state); field f of block block + t has output
// index jbase + 12 t + f and is written when that index is in [lo, hi).
struct Segment {
  uint64_t state;
  uint64_t block;
  int64_t jbase;
  int64_t lo;
  int64_t hi;
  uint32_t nblocks;
  uint32_t slot;  // luxury-level slot
};
static_assert(sizeof(Segment) == 48, "segment descriptor layout");

// Work item: segments seg0 .. seg0 + nseg - 1, all of level `slot`.
struct Item {
  uint32_t seg0;
  uint32_t nseg;
  uint32_t slot;
  uint32_t cost;  // longest segment, in blocks
};
static_assert(sizeof(Item) == 16, "item descriptor layout");

// Device-side header of a plan.  Everything a launch depends on that can
// change between updates lives here (not in kernel arguments), so a launch
// captured in a HIP graph replays whatever the plan holds at replay time.
struct Header {
  uint32_t reserved;
  uint32_t n_items;
  uint32_t pad[2];
  const uint32_t* C[MAX_LEVELS];  // folded multipliers A^(2^g) of each level
  const uint32_t* W[MAX_LEVELS];  // 16-bit window tables A^(j 65536^i) of each level
  const uint32_t* M[MAX_LEVELS];  // matrix-core step operands of each level
  uint32_t p[MAX_LEVELS];
};

template <Out K, int LGS, bool MF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MF ? 3 : 4))) void k_batch(const rlx_state* __restrict__ st,
                                                 const Segment* __restrict__ segs,
                                                 const Item* __restrict__ items, Header* __restrict__ hdr,
                                                 uint64_t* __restrict__ out, uint32_t* __restrict__ err) {
  constexpr uint32_t G = 1u << LGS;
  constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;
  __shared__ __align__(16) uint64_t stage[BLOCK * SLOT_VALUES];
  __shared__ mf_v4i af_lds[MF ? MF_FRAGS * 64 : 1];
  __shared__ uint32_t wave_slot[BLOCK / WAVE];
  const uint32_t tid_blk = threadIdx.x;
  const uint32_t lane = tid_blk & (WAVE - 1);
  const uint32_t team = lane >> LGS;
  const uint32_t l = lane & (G - 1);
  const uint32_t n_items = __builtin_amdgcn_readfirstlane(hdr->n_items);
  {
    // wave w of the grid runs item w; the grid covers the plan's capacity,
    // so waves past the current item count exit at once (after the block's
    // set-up below)
    const uint32_t it = __builtin_amdgcn_readfirstlane(blockIdx.x * (BLOCK / WAVE) + tid_blk / WAVE);
    // MF: when every item of the block has the same level (items are laid
    // out level by level, so nearly always), the block stages that level's
    // matrix-core operands for A^G in LDS once; otherwise each wave reads
    // its own level's operands from the table at every step
    bool lds_ok = false;
    if constexpr (MF) {
      if (lane == 0) wave_slot[tid_blk / WAVE] = it < n_items ? items[it].slot : NO_SLOT;
      __syncthreads();
      uint32_t s0 = NO_SLOT;
      bool same = true;
#pragma unroll
      for (uint32_t w = 0; w < BLOCK / WAVE; ++w) {
        const uint32_t v = __builtin_amdgcn_readfirstlane(wave_slot[w]);
        if (v != NO_SLOT) {
          same = same && (s0 == NO_SLOT || v == s0);
          s0 = s0 == NO_SLOT ? v : s0;
        }
      }
      lds_ok = same && s0 != NO_SLOT;
      if (lds_ok) mf_stage_operands(af_lds, hdr->M[s0] + (size_t)LGS * MF_LEVEL_WORDS, tid_blk, BLOCK);
      __syncthreads();
    }
    if (it >= n_items) return;
    const Item item = items[it];
    const uint32_t slot = __builtin_amdgcn_readfirstlane(item.slot);
    const uint32_t* __restrict__ ctabs = hdr->C[slot];
    const uint32_t* __restrict__ wtabs = hdr->W[slot];
    const uint32_t p = __builtin_amdgcn_readfirstlane(hdr->p[slot]);
    bool active = team < item.nseg;
    uint32_t si = item.seg0 + team;
    uint32_t nblocks = 0;
    uint32_t x[NW];
    uint64_t first = 0;  // this lane's first block: the segment's first + l
    if (active) {
      const Segment& sg = segs[si];
      uint32_t pos, sp;
      load_record(st, sg.state, x, pos, sp);
      uint32_t bad = 0;
      if (sp != p) bad |= RLX_ERR_BAD_P;
      if (geq_m(x)) bad |= RLX_ERR_BAD_X;
      if (bad) {
        if (l == 0) atomicOr(err, bad);
        active = false;
      } else {
        nblocks = sg.nblocks;
        first = sg.block + l;
      }
    }
    if (!active) set_one(x);
    skip_windows(x, first, wtabs);
    const uint32_t* __restrict__ ctab = ctabs + (size_t)LGS * FOLD_ROW_WORDS;
    // Output window of the segment: base[u] for u < span, with the
    // segment's first field at u = rel (rel >= -11; span < 2^30 because
    // segments hold at most 2^26 blocks).  Read after the lane set-up (the
    // index is made opaque so the load is not merged with the one above),
    // which keeps the window out of registers during it.
    asm volatile("" : "+v"(si));
    uint64_t* base = out;
    uint32_t span = 0;
    int32_t rel = 0;
    if (active) {
      const Segment& sg = segs[si];
      const int64_t lo = sg.lo > sg.jbase ? sg.lo : sg.jbase;
      const int64_t end = sg.jbase + (int64_t)FIELDS * nblocks;
      const int64_t hi = sg.hi < end ? sg.hi : end;
      base = out + lo;
      span = hi > lo ? (uint32_t)(hi - lo) : 0u;
      rel = (int32_t)(sg.jbase - lo);
    }
    // the loop, once per way of fetching the step's operands
    auto run = [&](const auto& fetch) {
      for (uint32_t k = 0;; ++k) {
        const uint32_t t = l + (k << LGS);
        const bool live = active && t < nblocks;
        if (!__any(live)) break;
        convert_to_lds<K>(x, stage + (size_t)tid_blk * SLOT_VALUES, false);
        const int32_t u0 = rel + (int32_t)(FIELDS * (t - l));
        group_store<LGS>(stage, tid_blk, l, u0, span, active, base);
        if (__any(live && t + G < nblocks)) {
          if constexpr (MF) {
            mfma_step(x, fetch, false);
          } else {
            step(x, constant_table(ctab), false, SgprBarrier());
          }
        }
      }
    };
    if constexpr (MF) {
      if (lds_ok) {
        run(MfFromArray{af_lds, lane});
      } else {
        run(MfFromBuffer(hdr->M[slot] + (size_t)LGS * MF_LEVEL_WORDS, lane));
      }
    } else {
      run(0);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host: the plan

struct rlx_plan {
  int device = 0;
  uint32_t lanes = 0, lg = 0;
  uint64_t seg_blocks = 0;
  uint64_t cap = 0;  // segments (and items) the device buffers hold
  Segment* d_segs = nullptr;
  Item* d_items = nullptr;
  Header* d_hdr = nullptr;
  Segment* h_segs = nullptr;  // pinned staging for uploads
  Item* h_items = nullptr;
  Header* h_hdr = nullptr;
  hipEvent_t uploaded = nullptr;
  uint64_t n_segs = 0, n_items = 0, total = 0;
};

namespace {

struct Planned {
  std::vector<Segment> segs;
  std::vector<Item> items;
  std::vector<uint32_t> ps;  // luxury level of each slot
  uint64_t total = 0;
};

// Segments are laid out level by level; inside a level, the full segments
// (seg_blocks steps) in request order, then the partial ones (at most one per
// request) by decreasing length.  Items take 64/G consecutive segments of one
// level and run longest first.  Only the partial segments and the items that
// hold them are sorted, so planning is linear in the number of segments.
int plan_requests(const rlx_request* reqs, uint64_t n, uint32_t lg, uint64_t seg_blocks, Planned* out) {
  Planned pl;
  std::vector<uint32_t> slot_of(n, 0);
  std::vector<uint64_t> full_n, part_n;  // per level
  for (uint64_t r = 0; r < n; ++r) {
    const rlx_request& q = reqs[r];
    if (q.reserved != 0 || !valid_p(q.p)) return RLX_EINVAL;
    if (q.count == 0) continue;
    if (q.start > UINT64_MAX - q.count) return RLX_EINVAL;
    if (q.out_offset > (uint64_t)INT64_MAX / 2 || q.count > (uint64_t)INT64_MAX / 2) return RLX_EINVAL;
    uint32_t slot = 0;
    while (slot < pl.ps.size() && pl.ps[slot] != q.p) ++slot;
    if (slot == pl.ps.size()) {
      if (pl.ps.size() == MAX_LEVELS) return RLX_EINVAL;
      pl.ps.push_back(q.p);
      full_n.push_back(0);
      part_n.push_back(0);
    }
    slot_of[r] = slot;
    const uint64_t nb = (q.start % FIELDS + q.count + FIELDS - 1) / FIELDS;
    full_n[slot] += nb / seg_blocks;
    part_n[slot] += (nb % seg_blocks) != 0;
    pl.total += q.count;
  }
  const size_t levels = pl.ps.size();
  std::vector<uint64_t> full_at(levels), part_at(levels), part_end(levels);
  uint64_t total_segs = 0;
  for (size_t k = 0; k < levels; ++k) {
    full_at[k] = total_segs;
    part_at[k] = total_segs + full_n[k];
    total_segs += full_n[k] + part_n[k];
    part_end[k] = total_segs;
  }
  if (total_segs > 0xFFFFFFFFull) return RLX_EINVAL;
  pl.segs.resize(total_segs);
  for (uint64_t r = 0; r < n; ++r) {
    const rlx_request& q = reqs[r];
    if (q.count == 0) continue;
    const uint32_t slot = slot_of[r];
    const uint64_t b0 = q.start / FIELDS;
    const uint64_t f0 = q.start % FIELDS;
    const uint64_t nb = (f0 + q.count + FIELDS - 1) / FIELDS;
    for (uint64_t k = 0; k * seg_blocks < nb; ++k) {
      const uint64_t len = std::min<uint64_t>(seg_blocks, nb - k * seg_blocks);
      Segment& sg = pl.segs[len == seg_blocks ? full_at[slot]++ : part_at[slot]++];
      sg.state = q.state;
      sg.block = b0 + k * seg_blocks;
      sg.jbase = (int64_t)q.out_offset + (int64_t)(FIELDS * k * seg_blocks) - (int64_t)f0;
      sg.lo = (int64_t)q.out_offset;
      sg.hi = (int64_t)(q.out_offset + q.count);
      sg.nblocks = (uint32_t)len;
      sg.slot = slot;
    }
  }
  for (size_t k = 0; k < levels; ++k) {
    std::stable_sort(pl.segs.begin() + (part_end[k] - part_n[k]), pl.segs.begin() + part_end[k],
                     [](const Segment& a, const Segment& b) { return a.nblocks > b.nblocks; });
  }
  // items: those that start with a full segment (cost seg_blocks) first, in
  // level order, then the rest by decreasing cost
  const uint32_t per_item = WAVE >> lg;  // segments per 64-lane item
  std::vector<Item> rest;
  pl.items.reserve(total_segs / per_item + 2 * levels);
  for (size_t k = 0, i = 0; k < levels; ++k) {
    const uint64_t end = part_end[k];
    while (i < end) {
      Item it;
      it.seg0 = (uint32_t)i;
      it.slot = (uint32_t)k;
      it.cost = pl.segs[i].nblocks;
      it.nseg = (uint32_t)std::min<uint64_t>(per_item, end - i);
      i += it.nseg;
      if (it.cost == seg_blocks) {
        pl.items.push_back(it);
      } else {
        rest.push_back(it);
      }
    }
  }
  std::stable_sort(rest.begin(), rest.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
  pl.items.insert(pl.items.end(), rest.begin(), rest.end());
  *out = std::move(pl);
  return RLX_OK;
}

int upload(rlx_plan* plan, const Planned& pl, hipStream_t s) {
  if (pl.segs.size() > plan->cap || pl.items.size() > plan->cap) return RLX_EINVAL;
  if (pl.ps.size() > MAX_LEVELS) return RLX_EINVAL;
  Header hd{};
  hd.n_items = (uint32_t)pl.items.size();
  for (size_t k = 0; k < pl.ps.size(); ++k) {
    Tables t;
    const int rc = tables(pl.ps[k], s, &t);
    if (rc) return rc;
    hd.C[k] = t.C;
    hd.W[k] = t.W;
    hd.M[k] = t.M;
    hd.p[k] = pl.ps[k];
  }
  // the previous upload must have left the staging buffers
  if (hipEventSynchronize(plan->uploaded) != hipSuccess) return RLX_EHIP;
  *plan->h_hdr = hd;
  if (hipMemcpyAsync(plan->d_hdr, plan->h_hdr, sizeof(Header), hipMemcpyHostToDevice, s) != hipSuccess)
    return RLX_EHIP;
  if (!pl.segs.empty()) std::memcpy(plan->h_segs, pl.segs.data(), pl.segs.size() * sizeof(Segment));
  if (!pl.items.empty()) std::memcpy(plan->h_items, pl.items.data(), pl.items.size() * sizeof(Item));
  if (!pl.segs.empty() &&
      hipMemcpyAsync(plan->d_segs, plan->h_segs, pl.segs.size() * sizeof(Segment), hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return RLX_EHIP;
  if (!pl.items.empty() &&
      hipMemcpyAsync(plan->d_items, plan->h_items, pl.items.size() * sizeof(Item), hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return RLX_EHIP;
  if (hipEventRecord(plan->uploaded, s) != hipSuccess) return RLX_EHIP;
  plan->n_segs = pl.segs.size();
  plan->n_items = pl.items.size();
  plan->total = pl.total;
  return RLX_OK;
}

void free_plan(rlx_plan* p) {
  if (!p) return;
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_hdr) (void)hipFree(p->d_hdr);
  if (p->h_hdr) (void)hipHostFree(p->h_hdr);
  if (p->h_segs) (void)hipHostFree(p->h_segs);
  if (p->h_items) (void)hipHostFree(p->h_items);
  if (p->uploaded) (void)hipEventDestroy(p->uploaded);
  delete p;
}

// The plan's tables and descriptors live on the device it was created on.
bool on_plan_device(const rlx_plan* plan) {
  int dev;
  return hipGetDevice(&dev) == hipSuccess && dev == plan->device;
}

template <Out K>
int plan_launch(rlx_plan* plan, const rlx_state* states, void* out, void* stream) {
  if (!plan) return RLX_EINVAL;
  if (!on_plan_device(plan)) return RLX_EINVAL;
  if (!states || !out || !aligned(states, 16) || !aligned(out, 8)) return RLX_EINVAL;
  hipStream_t s = as_stream(stream);
  uint32_t* err;
  int rc = error_word(s, &err);
  if (rc) return rc;
  // One wave per item of a full plan (items never outnumber the segment
  // capacity).  The grid depends only on the capacity, so a captured launch
  // stays valid after updates; waves past the current item count exit.
  const uint64_t blocks = (plan->cap + (BLOCK / WAVE) - 1) / (BLOCK / WAVE);
  if (blocks == 0 || blocks > 0x7FFFFFFFull) return RLX_EINVAL;
  uint64_t* o = reinterpret_cast<uint64_t*>(out);
  const bool mf = rlx_step_kernel() == RLX_STEP_MFMA;
#define RLX_BATCH(L)                                                                                      \
  case L:                                                                                                 \
    if (mf) {                                                                                             \
      k_batch<K, L, true><<<(unsigned)blocks, BLOCK, 0, s>>>(states, plan->d_segs, plan->d_items, plan->d_hdr, \
                                                              o, err);                                    \
    } else {                                                                                              \
      k_batch<K, L, false><<<(unsigned)blocks, BLOCK, 0, s>>>(states, plan->d_segs, plan->d_items,       \
                                                               plan->d_hdr, o, err);                      \
    }                                                                                                     \
    break;
  switch (plan->lg) {
    RLX_BATCH(0) RLX_BATCH(1) RLX_BATCH(2) RLX_BATCH(3) RLX_BATCH(4) RLX_BATCH(5) RLX_BATCH(6)
    default: return RLX_EINVAL;
  }
#undef RLX_BATCH
  return launch_status();
}

}  // namespace

extern "C" {

int rlx_plan_create(rlx_plan** plan, const rlx_request* reqs, uint64_t n, uint32_t lanes, uint64_t seg_blocks,
                    uint64_t capacity_segments, void* stream) try {
  if (!plan) return RLX_EINVAL;
  *plan = nullptr;
  if (n > 0 && !reqs) return RLX_EINVAL;
  if (lanes == 0 || lanes > (uint32_t)WAVE || (lanes & (lanes - 1)) != 0) return RLX_EINVAL;
  if (seg_blocks == 0 || seg_blocks > RLX_MAX_SEG_BLOCKS) return RLX_EINVAL;
  // a plan never holds more than 2^32 - 1 segments (the planner's limit)
  if (capacity_segments > 0xFFFFFFFFull) return RLX_EINVAL;
  const uint32_t lg = (uint32_t)__builtin_ctz(lanes);
  Planned pl;
  int rc = plan_requests(reqs, n, lg, seg_blocks, &pl);
  if (rc) return rc;
  rlx_plan* p = new (std::nothrow) rlx_plan();
  if (!p) return RLX_ENOMEM;
  if (hipGetDevice(&p->device) != hipSuccess) {
    free_plan(p);
    return RLX_EHIP;
  }
  p->lanes = lanes;
  p->lg = lg;
  p->seg_blocks = seg_blocks;
  p->cap = std::max<uint64_t>({capacity_segments, (uint64_t)pl.segs.size(), 1});
  if (hipMalloc(&p->d_segs, p->cap * sizeof(Segment)) != hipSuccess ||
      hipMalloc(&p->d_items, p->cap * sizeof(Item)) != hipSuccess ||
      hipMalloc(&p->d_hdr, sizeof(Header)) != hipSuccess ||
      hipHostMalloc(&p->h_hdr, sizeof(Header), 0) != hipSuccess ||
      hipHostMalloc(&p->h_segs, p->cap * sizeof(Segment), 0) != hipSuccess ||
      hipHostMalloc(&p->h_items, p->cap * sizeof(Item), 0) != hipSuccess) {
    free_plan(p);
    return RLX_ENOMEM;
  }
  if (hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(p->uploaded, as_stream(stream)) != hipSuccess) {
    free_plan(p);
    return RLX_EHIP;
  }
  rc = upload(p, pl, as_stream(stream));
  if (rc) {
    free_plan(p);
    return rc;
  }
  *plan = p;
  return RLX_OK;
} catch (const std::bad_alloc&) {
  return RLX_ENOMEM;
}

int rlx_plan_update(rlx_plan* plan, const rlx_request* reqs, uint64_t n, void* stream) try {
  if (!plan || (n > 0 && !reqs)) return RLX_EINVAL;
  if (!on_plan_device(plan)) return RLX_EINVAL;
  Planned pl;
  int rc = plan_requests(reqs, n, plan->lg, plan->seg_blocks, &pl);
  if (rc) return rc;
  return upload(plan, pl, as_stream(stream));
} catch (const std::bad_alloc&) {
  return RLX_ENOMEM;
}

int rlx_plan_info(const rlx_plan* plan, uint64_t* segments, uint64_t* items, uint64_t* total_values) {
  if (!plan) return RLX_EINVAL;
  if (segments) *segments = plan->n_segs;
  if (items) *items = plan->n_items;
  if (total_values) *total_values = plan->total;
  return RLX_OK;
}

int rlx_plan_generate_f64(rlx_plan* plan, const rlx_state* states, double* out, void* stream) {
  return plan_launch<Out::F64>(plan, states, out, stream);
}

int rlx_plan_generate_u64(rlx_plan* plan, const rlx_state* states, uint64_t* out, void* stream) {
  return plan_launch<Out::U64>(plan, states, out, stream);
}

int rlx_plan_generate_f32(rlx_plan* plan, const rlx_state* states, float* out, void* stream) {
  return plan_launch<Out::F32>(plan, states, out, stream);
}

int rlx_plan_dry_run(const rlx_request* reqs, uint64_t n, uint32_t lanes, uint64_t seg_blocks,
                     uint64_t* n_segments, uint64_t* n_items, uint64_t* total_values, uint64_t* segments,
                     uint64_t max_segments) try {
  if (n > 0 && !reqs) return RLX_EINVAL;
  if (lanes == 0 || lanes > (uint32_t)WAVE || (lanes & (lanes - 1)) != 0) return RLX_EINVAL;
  if (seg_blocks == 0 || seg_blocks > RLX_MAX_SEG_BLOCKS) return RLX_EINVAL;
  Planned pl;
  const int rc = plan_requests(reqs, n, (uint32_t)__builtin_ctz(lanes), seg_blocks, &pl);
  if (rc) return rc;
  if (n_segments) *n_segments = pl.segs.size();
  if (n_items) *n_items = pl.items.size();
  if (total_values) *total_values = pl.total;
  if (segments) {
    uint64_t row = 0;
    for (const Item& it : pl.items) {
      for (uint32_t k = 0; k < it.nseg && row < max_segments; ++k, ++row) {
        const Segment& sg = pl.segs[it.seg0 + k];
        uint64_t* r = segments + 6 * row;
        r[0] = sg.state;
        r[1] = sg.block;
        r[2] = (uint64_t)sg.jbase;
        r[3] = (uint64_t)sg.lo;
        r[4] = (uint64_t)sg.hi;
        r[5] = (uint64_t)sg.nblocks | ((uint64_t)sg.slot << 32);
      }
    }
  }
  return RLX_OK;
} catch (const std::bad_alloc&) {
  return RLX_ENOMEM;
}

int rlx_plan_destroy(rlx_plan* plan) {
  if (!plan) return RLX_OK;
  const bool ok = hipDeviceSynchronize() == hipSuccess;
  free_plan(plan);
  return ok ? RLX_OK : RLX_EHIP;
}

}  // extern "C"
