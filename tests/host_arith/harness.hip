// Host build of the library's 576-bit arithmetic (rlx_arith.hpp), for the CPU
// test-suite: reads operands (hex words) and writes, for each case, the
// generic mulmod, the constant-multiplier step on its fast and general
// paths, the conversion to RANLUX numbers on both paths, the carry and the
// 12 fields as u64 and as doubles.
#include "rlx_arith.hpp"
#include <cstdio>
#include <cstring>
#include <vector>
using namespace rlx;
static void rd(FILE* f, uint32_t (&w)[NW]) { for (int k = 0; k < NW; ++k) fscanf(f, "%x", &w[k]); }
static void wr(FILE* f, const uint32_t (&w)[NW]) { for (int k = 0; k < NW; ++k) fprintf(f, "%08x ", w[k]); fprintf(f, "\n"); }
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "r"); FILE* o = fopen(argv[2], "w");
  std::vector<uint32_t> tab(NL * NW);
  for (auto& v : tab) fscanf(f, "%x", &v);
  int n; fscanf(f, "%d", &n);
  for (int i = 0; i < n; ++i) {
    uint32_t x[NW], y[NW], r[NW], s1[NW], s2[NW], d1[NW], d2[NW];
    rd(f, x); rd(f, y);
    mulmod_generic(x, y, r); wr(o, r);
    memcpy(s1, x, sizeof x); step(s1, tab.data(), false); wr(o, s1);
    memcpy(s2, x, sizeof x); step(s2, tab.data(), true); wr(o, s2);
    to_ranlux(x, d1, false); wr(o, d1);
    to_ranlux(x, d2, true); wr(o, d2);
    fprintf(o, "%u\n", ranlux_carry(x, d1));
    for (int k = 0; k < 12; ++k) { double v = field_f64(d1, k); unsigned long long u = field_u64(d1, k);
      fprintf(o, "%llx %a ", u, v); }
    fprintf(o, "\n");
  }
  fclose(o);
  return 0;
}
