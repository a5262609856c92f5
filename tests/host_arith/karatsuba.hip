// A one-level Karatsuba form of the generic 576 x 576-bit product, kept as
// the measured alternative to the library's schoolbook product (mul576 in
// rlx_arith.hpp); it is not part of the library.
//
// With the 21 digits of 28 bits (B = 2^28) split as X = X0 + X1 B^11 (11 and
// 10 digits), X Y = P0 + (P1 - P0 - P2) B^11 + P2 B^22 for P0 = X0 Y0,
// P2 = X1 Y1 and P1 = (X0 + X1)(Y0 + Y1): 121 + 100 + 121 digit products
// instead of 441 (the digit sums have 29 bits, so a column of P1 stays below
// 11 2^58).  The column sums of the three products are combined raw, with a
// signed carry between columns.
//
// Built two ways by the CPU test-suite: for the host (main reads operand
// pairs as hex words and writes the 36-word products) and as gfx950 device
// assembly, where the two kernels below are counted instruction by
// instruction.
#include "rlx_arith.hpp"
#include <cstdio>

namespace {

using namespace rlx;

__host__ __device__ __forceinline__ void mul576_karatsuba(const uint32_t (&x)[NW], const uint32_t (&y)[NW],
                                                          uint32_t (&p)[2 * NW]) {
  uint32_t a[GD], b[GD];
  digits28(x, a);
  digits28(y, b);
  uint32_t sa[11], sb[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    sa[i] = a[i] + (i < 10 ? a[i + 11] : 0u);
    sb[i] = b[i] + (i < 10 ? b[i + 11] : 0u);
  }
  uint64_t c0[21], c1[21], c2[19];
#pragma unroll
  for (int c = 0; c < 21; ++c) {
    uint64_t s0 = 0, s1 = 0;
#pragma unroll
    for (int i = (c < 11 ? 0 : c - 10); i <= (c < 11 ? c : 10); ++i) {
      s0 += (uint64_t)a[i] * b[c - i];
      s1 += (uint64_t)sa[i] * sb[c - i];
    }
    c0[c] = s0;
    c1[c] = s1;
  }
#pragma unroll
  for (int c = 0; c < 19; ++c) {
    uint64_t s2 = 0;
#pragma unroll
    for (int i = (c < 10 ? 0 : c - 9); i <= (c < 10 ? c : 9); ++i) s2 += (uint64_t)a[11 + i] * b[11 + c - i];
    c2[c] = s2;
  }
  uint32_t d[2 * GD];
  int64_t carry = 0;
#pragma unroll
  for (int c = 0; c < 2 * GD - 1; ++c) {
    uint64_t t = (uint64_t)carry;
    if (c < 21) t += c0[c];
    if (c >= 11 && c - 11 < 21) t += c1[c - 11] - c0[c - 11];
    if (c >= 11 && c - 11 < 19) t -= c2[c - 11];
    if (c >= 22 && c - 22 < 19) t += c2[c - 22];
    d[c] = (uint32_t)t & 0x0FFFFFFFu;
    carry = (int64_t)t >> 28;
  }
  d[2 * GD - 1] = (uint32_t)carry;
#pragma unroll
  for (int k = 0; k < 2 * NW; ++k) {
    const int c = (32 * k) / 28;
    const int s = (32 * k) % 28;
    uint32_t v = d[c] >> s;
    if (c + 1 < 2 * GD) v |= d[c + 1] << (28 - s);
    if (c + 2 < 2 * GD && 56 - s < 32) v |= d[c + 2] << (56 - s);
    p[k] = v;
  }
}

}  // namespace

// one product per lane, operands and products as words in global memory
extern "C" __global__ void k_product_schoolbook(const uint32_t* x, const uint32_t* y, uint32_t* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[NW], b[NW], p[2 * NW];
  for (int k = 0; k < NW; ++k) { a[k] = x[t * NW + k]; b[k] = y[t * NW + k]; }
  mul576(a, b, p);
  for (int k = 0; k < 2 * NW; ++k) out[t * 2 * NW + k] = p[k];
}

extern "C" __global__ void k_product_karatsuba(const uint32_t* x, const uint32_t* y, uint32_t* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[NW], b[NW], p[2 * NW];
  for (int k = 0; k < NW; ++k) { a[k] = x[t * NW + k]; b[k] = y[t * NW + k]; }
  mul576_karatsuba(a, b, p);
  for (int k = 0; k < 2 * NW; ++k) out[t * 2 * NW + k] = p[k];
}

int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "r");
  FILE* o = fopen(argv[2], "w");
  if (!f || !o) return 1;
  int n;
  if (fscanf(f, "%d", &n) != 1) return 1;
  for (int i = 0; i < n; ++i) {
    uint32_t x[NW], y[NW], p[2 * NW];
    for (int k = 0; k < NW; ++k) if (fscanf(f, "%x", &x[k]) != 1) return 1;
    for (int k = 0; k < NW; ++k) if (fscanf(f, "%x", &y[k]) != 1) return 1;
    mul576_karatsuba(x, y, p);
    for (int k = 0; k < 2 * NW; ++k) fprintf(o, "%08x ", p[k]);
    fprintf(o, "\n");
  }
  fclose(o);
  return 0;
}
