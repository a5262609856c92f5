// Host build of the Box-Muller evaluation (rlx_gauss.hpp), for the CPU
// test-suite: reads field pairs as three hex words each and writes, per
// pair, ln(1 - u1), cos(2 pi u2), sin(2 pi u2) and the two normals as hex
// floats.
#include "rlx_gauss.hpp"
#include <cstdio>
using namespace rlx::gauss;
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "r"); FILE* o = fopen(argv[2], "w");
  if (!f || !o) return 1;
  int n; if (fscanf(f, "%d", &n) != 1) return 1;
  for (int i = 0; i < n; ++i) {
    unsigned w0, w1, w2;
    if (fscanf(f, "%x %x %x", &w0, &w1, &w2) != 3) return 1;
    const double u1 = from_bits(w0, (w1 & 0xFFFFu) | 0x40300000u) - 16.0;
    const double t = from_bits((w1 >> 16) | (w2 << 16), (w2 >> 16) | 0x40500000u) - 64.0;
    double c, s, zc, zs;
    cos_sin_quarter_turns(t, c, s);
    box_muller(w0, w1, w2, zc, zs);
    fprintf(o, "%a %a %a %a %a\n", log_unit(1.0 - u1), c, s, zc, zs);
  }
  fclose(o);
  return 0;
}
