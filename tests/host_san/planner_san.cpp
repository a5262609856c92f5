// Host-only driver of the batch planner (rlx_plan_dry_run), built with the
// address and undefined-behaviour sanitizers on the host side: random and
// edge-case request sets, every lanes / segment-length combination, output
// rows truncated to fewer than the plan holds, and the refusals.  Prints
// "ok" and exits 0 when every call behaved; any sanitizer report aborts.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rlx.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {  // splitmix64
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int fail(const char* what) {
  std::fprintf(stderr, "planner_san: %s\n", what);
  return 1;
}

int main() {
  const uint32_t levels[5] = {24, 218, 404, 794, 2048};
  const uint32_t lanes_set[7] = {1, 2, 4, 8, 16, 32, 64};
  const uint64_t seg_set[4] = {1, 7, 512, 8192};
  for (int round = 0; round < 12; ++round) {
    const uint64_t n = next_u64() % 200;
    std::vector<rlx_request> reqs(n);
    uint64_t off = 0;
    for (uint64_t i = 0; i < n; ++i) {
      const uint64_t kind = next_u64() % 4;
      uint64_t count = kind == 0 ? 0 : kind == 1 ? 1 + next_u64() % 12 : 1 + next_u64() % (1u << 16);
      reqs[i].state = next_u64() % 64;
      reqs[i].start = next_u64() % 3 == 0 ? 0 : next_u64() % (1ull << 40);
      reqs[i].count = count;
      reqs[i].out_offset = off;
      reqs[i].p = levels[next_u64() % 5];
      reqs[i].reserved = 0;
      off += count;
    }
    for (uint32_t lanes : lanes_set) {
      for (uint64_t seg : seg_set) {
        uint64_t ns = 0, ni = 0, tv = 0;
        if (rlx_plan_dry_run(reqs.data(), n, lanes, seg, &ns, &ni, &tv, nullptr, 0) != 0)
          return fail("dry run refused valid requests");
        if (tv != off) return fail("total values differ from the request counts");
        std::vector<uint64_t> rows(6 * ns + 6);
        uint64_t ns2 = 0, ni2 = 0, tv2 = 0;
        if (rlx_plan_dry_run(reqs.data(), n, lanes, seg, &ns2, &ni2, &tv2, rows.data(), ns) != 0 ||
            ns2 != ns || ni2 != ni || tv2 != tv)
          return fail("second dry run differs");
        const uint64_t part = ns / 2;  // fewer rows than the plan holds
        std::vector<uint64_t> few(6 * part + 1);
        if (rlx_plan_dry_run(reqs.data(), n, lanes, seg, &ns2, &ni2, &tv2, few.data(), part) != 0)
          return fail("truncated dry run refused");
      }
    }
  }
  // one request far beyond 2^32 values at an output offset beyond 2^32
  {
    rlx_request big = {3, (1ull << 40) + 5, (1ull << 34) + 7, (1ull << 33) + 1, 2048, 0};
    uint64_t ns = 0, ni = 0, tv = 0;
    if (rlx_plan_dry_run(&big, 1, 64, 8192, &ns, &ni, &tv, nullptr, 0) != 0 || tv != big.count)
      return fail("large request");
    std::vector<uint64_t> rows(6 * ns);
    if (rlx_plan_dry_run(&big, 1, 64, 8192, &ns, &ni, &tv, rows.data(), ns) != 0) return fail("large rows");
  }
  // refusals: lanes not a power of two, zero segment length, 17 levels,
  // a non-zero reserved field, a level below 24
  rlx_request r = {0, 0, 10, 0, 24, 0};
  uint64_t a = 0, b = 0, c = 0;
  if (rlx_plan_dry_run(&r, 1, 3, 64, &a, &b, &c, nullptr, 0) == 0) return fail("lanes 3 accepted");
  if (rlx_plan_dry_run(&r, 1, 8, 0, &a, &b, &c, nullptr, 0) == 0) return fail("segment length 0 accepted");
  std::vector<rlx_request> many(17, r);
  for (int k = 0; k < 17; ++k) many[k].p = 24 + k;
  if (rlx_plan_dry_run(many.data(), 17, 8, 64, &a, &b, &c, nullptr, 0) == 0) return fail("17 levels accepted");
  r.reserved = 1;
  if (rlx_plan_dry_run(&r, 1, 8, 64, &a, &b, &c, nullptr, 0) == 0) return fail("reserved field accepted");
  r.reserved = 0;
  r.p = 10;
  if (rlx_plan_dry_run(&r, 1, 8, 64, &a, &b, &c, nullptr, 0) == 0) return fail("level 10 accepted");
  if (rlx_plan_dry_run(nullptr, 0, 8, 64, &a, &b, &c, nullptr, 0) != 0 || a != 0 || b != 0 || c != 0)
    return fail("empty request set");
  std::printf("ok\n");
  return 0;
}
