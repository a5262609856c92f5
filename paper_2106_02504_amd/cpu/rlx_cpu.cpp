// rlx_cpu.cpp -- RANLUX++ on the host CPU: the paper's portable form
// (section 3: nine 64-bit words, products with unsigned __int128), one
// std::thread per hardware thread.  This is the CPU baseline the GPU path is
// compared with; it shares no code with the GPU arithmetic.
//
//   m = 2^576 - 2^240 + 1 (section 2.2), a = 2^-24 mod m (one subtract-with-
//   borrow step), A_p = a^p, one generator step X <- A_p X mod m;
//   the numbers of a step are the 24 base-2^24 digits of D = floor(X 2^576 /
//   m) (section 2.3), and value k of a step is bits [48k, 48k + 48) of D as
//   v 2^-48; seeding X = A_p^(2^96 id), skipping X <- A_p^k X.
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

typedef unsigned __int128 u128;
constexpr int W = 9;  // 64-bit words of a number below 2^576

struct Num {
  uint64_t w[W];
};

// m = 2^576 - 2^240 + 1: words 0 = 1, 3 = 0xFFFF000000000000, 4..8 all ones
const Num M = {{1ull, 0ull, 0ull, 0xFFFF000000000000ull, ~0ull, ~0ull, ~0ull, ~0ull, ~0ull}};

bool geq(const uint64_t* x, const Num& y) {
  for (int k = W - 1; k >= 0; --k) {
    if (x[k] != y.w[k]) return x[k] > y.w[k];
  }
  return true;
}

// x (nx words) -= y (ny <= nx words), the borrow carried through all of x
void sub_in_place(uint64_t* x, const uint64_t* y, int nx, int ny) {
  uint64_t br = 0;
  for (int k = 0; k < nx; ++k) {
    const u128 d = (u128)x[k] - (k < ny ? y[k] : 0) - br;
    x[k] = (uint64_t)d;
    br = (uint64_t)(d >> 64) & 1u;
  }
}

// t += (h << 240) over nt words, h given as nh words (240 = 3 words + 48
// bits), then t -= h with the borrow carried through all nt words; t stays
// non-negative because h 2^240 >= h.
template <int NT, int NH>
inline void add_shift240_sub(uint64_t (&t)[NT], const uint64_t* h) {
  u128 c = 0;
  for (int k = 3; k < NT; ++k) {
    const int j = k - 3;
    uint64_t part = 0;
    if (j < NH) part |= h[j] << 48;
    if (j >= 1 && j - 1 < NH) part |= h[j - 1] >> 16;
    c += (u128)t[k] + part;
    t[k] = (uint64_t)c;
    c >>= 64;
  }
  uint64_t br = 0;
  for (int k = 0; k < NT; ++k) {
    const u128 d = (u128)t[k] - (k < NH ? h[k] : 0) - br;
    t[k] = (uint64_t)d;
    br = (uint64_t)(d >> 64) & 1u;
  }
}

// r = p mod m for the 1152-bit product p (18 words), with
// 2^576 = 2^240 - 1 (mod m) applied twice (section 2.2: only additions,
// subtractions and shifts): p = L + H 2^576 gives T = L + H 2^240 - H below
// 2^817; T = T0 + T1 2^576 gives T0 + T1 2^240 - T1 below 2^577; a last bit
// above 2^576 folds once more without overflow, and one comparison with m
// makes the result canonical.
void reduce(const uint64_t* p, Num& r) {
  uint64_t t[13] = {};
  for (int k = 0; k < W; ++k) t[k] = p[k];
  add_shift240_sub<13, W>(t, p + W);
  uint64_t u[10] = {};
  for (int k = 0; k < W; ++k) u[k] = t[k];
  add_shift240_sub<10, 4>(u, t + W);
  const uint64_t top = u[W];
  u[W] = 0;
  if (top) {
    const uint64_t h[1] = {top};
    add_shift240_sub<10, 1>(u, h);
  }
  for (int k = 0; k < W; ++k) r.w[k] = u[k];
  if (geq(r.w, M)) sub_in_place(r.w, M.w, W, W);
}

// x y mod m: the 1152-bit product column by column (section 2.1: the 81
// 64 x 64 -> 128-bit partial products of a column go into a three-word
// accumulator, so the products of a column do not wait on each other's
// carries), then the reduction.
Num mulmod(const Num& a, const Num& b) {
  uint64_t p[2 * W];
  uint64_t lo = 0, hi = 0, top = 0;
#pragma GCC unroll 17
  for (int k = 0; k < 2 * W - 1; ++k) {
    const int i0 = k < W ? 0 : k - W + 1, i1 = k < W ? k : W - 1;
#pragma GCC unroll 9
    for (int i = i0; i <= i1; ++i) {
      const u128 t = (u128)a.w[i] * b.w[k - i];
      const u128 s0 = (u128)lo + (uint64_t)t;
      const u128 s1 = (u128)hi + (uint64_t)(t >> 64) + (uint64_t)(s0 >> 64);
      lo = (uint64_t)s0;
      hi = (uint64_t)s1;
      top += (uint64_t)(s1 >> 64);
    }
    p[k] = lo;
    lo = hi;
    hi = top;
    top = 0;
  }
  p[2 * W - 1] = lo;
  Num r;
  reduce(p, r);
  return r;
}

Num one() {
  Num r = {};
  r.w[0] = 1;
  return r;
}

// a = m - (m - 1) / 2^24 = 2^576 - 2^552 - 2^240 + 2^216 + 1
Num multiplier_a() {
  Num mm1 = M;
  mm1.w[0] -= 1;  // m - 1 = 2^576 - 2^240, divisible by 2^24
  Num q;
  for (int k = 0; k < W; ++k) q.w[k] = (mm1.w[k] >> 24) | (k + 1 < W ? mm1.w[k + 1] << 40 : 0);
  Num a = M;
  sub_in_place(a.w, q.w, W, W);
  return a;
}

// base^e by square-and-multiply from the top bit of e (words of e least
// significant first)
Num power(Num base, const uint64_t* e, int words) {
  Num r = one();
  bool started = false;
  for (int k = words - 1; k >= 0; --k) {
    for (int b = 63; b >= 0; --b) {
      if (started) r = mulmod(r, r);
      if ((e[k] >> b) & 1u) {
        r = started ? mulmod(r, base) : base;
        started = true;
      }
    }
  }
  return r;
}

struct Level {
  Num A;  // A_p
  Num B;  // A_p^(2^96), the seed spacing
};

Level level(uint32_t p) {
  Level L;
  const uint64_t ep[1] = {p};
  L.A = power(multiplier_a(), ep, 1);
  Num b = L.A;
  for (int i = 0; i < 96; ++i) b = mulmod(b, b);
  L.B = b;
  return L;
}

// D = floor(X 2^576 / m): with q0 = X >> 336 and D' = X + q0, D = D' - 1
// exactly when D' m > X 2^576, i.e. when q0 2^576 > D' (2^240 - 1)
// (both sides below 2^817, compared as 13-word numbers), else D = D'.
Num to_ranlux(const Num& x) {
  uint64_t q0[W] = {};
  for (int k = 0; k < W; ++k) {
    const int src = k + 5;  // 336 = 5 words + 16 bits
    uint64_t v = src < W ? x.w[src] >> 16 : 0;
    if (src + 1 < W) v |= x.w[src + 1] << 48;
    q0[k] = v;
  }
  uint64_t d[W + 1] = {};
  u128 c = 0;
  for (int k = 0; k < W; ++k) {
    c += (u128)x.w[k] + q0[k];
    d[k] = (uint64_t)c;
    c >>= 64;
  }
  d[W] = (uint64_t)c;
  // lhs = q0 << 576 (words 9..12), rhs = (d << 240) - d
  uint64_t lhs[13] = {}, rhs[13] = {};
  for (int k = 0; k < 4; ++k) lhs[W + k] = q0[k];
  u128 cc = 0;
  for (int k = 0; k < 13; ++k) {
    const int j = k - 3;  // 240 = 3 words + 48 bits
    uint64_t part = 0;
    if (j >= 0 && j <= W) part |= d[j] << 48;
    if (j - 1 >= 0 && j - 1 <= W) part |= d[j - 1] >> 16;
    cc += part;
    rhs[k] = (uint64_t)cc;
    cc >>= 64;
  }
  sub_in_place(rhs, d, 13, W + 1);
  bool greater = false;
  for (int k = 12; k >= 0; --k) {
    if (lhs[k] != rhs[k]) {
      greater = lhs[k] > rhs[k];
      break;
    }
  }
  if (greater) {
    const uint64_t one_w[1] = {1};
    sub_in_place(d, one_w, W + 1, 1);
  }
  Num r;
  std::memcpy(r.w, d, sizeof r.w);  // D < 2^576
  return r;
}

uint64_t field(const Num& d, int k) {
  const int bit = 48 * k, w = bit >> 6, s = bit & 63;
  uint64_t v = d.w[w] >> s;
  if (s > 16 && w + 1 < W) v |= d.w[w + 1] << (64 - s);
  return v & ((1ull << 48) - 1);
}

template <class F>
void parallel(uint64_t n, int threads, F f) {
  if (threads <= 1 || n < 2) {
    f(0, n);
    return;
  }
  std::vector<std::thread> pool;
  const uint64_t per = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const uint64_t lo = t * per, hi = lo + per < n ? lo + per : n;
    if (lo >= hi) break;
    pool.emplace_back([=]() { f(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

int threads_or_all(int threads) {
  if (threads > 0) return threads;
  const unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

// 4-bit windows of a base for 64-bit exponents: T[i][j] = base^(j 16^i),
// i < 16, j < 16 (built with 256 multiplications), so that base^e costs one
// multiplication per non-zero hexadecimal digit of e.
struct Windows {
  Num t[16][16];
  explicit Windows(const Num& base) {
    Num b = base;
    for (int i = 0; i < 16; ++i) {
      t[i][0] = one();
      t[i][1] = b;
      for (int j = 2; j < 16; ++j) t[i][j] = mulmod(t[i][j - 1], b);
      b = mulmod(t[i][15], b);  // base^(16^(i+1))
    }
  }
  // x base^e
  Num apply(Num x, uint64_t e) const {
    for (int i = 0; i < 16 && e; ++i, e >>= 4) {
      const unsigned d = (unsigned)(e & 15u);
      if (d) x = mulmod(x, t[i][d]);
    }
    return x;
  }
};

// X <- A^k X for a 64-bit k
Num skip(const Num& x, const Num& A, uint64_t k) {
  const uint64_t e[1] = {k};
  return mulmod(power(A, e, 1), x);
}

// count values of the stream at X (position 0): value j is field j mod 12 of
// step j / 12; out[j] = v 2^-48 (or the 48-bit v when u48 is set)
void draw(Num x, const Num& A, uint64_t count, double* out, uint64_t* out_u) {
  uint64_t j = 0;
  while (j < count) {
    const Num d = to_ranlux(x);
    for (int k = 0; k < 12 && j < count; ++k, ++j) {
      const uint64_t v = field(d, k);
      if (out) out[j] = (double)v * 0x1p-48;
      if (out_u) out_u[j] = v;
    }
    if (j < count) x = mulmod(x, A);
  }
}

void store(uint64_t* dst, const Num& x) { std::memcpy(dst, x.w, sizeof x.w); }
Num load(const uint64_t* src) {
  Num x;
  std::memcpy(x.w, src, sizeof x.w);
  return x;
}

}  // namespace

extern "C" {

// Seeds X = A_p^(2^96 id) for id = id0 + i, i < n, into x[9 i .. 9 i + 8].
void rlx_cpu_seed(uint64_t* x, uint64_t n, uint64_t id0, uint32_t p, int threads) {
  const Level L = level(p);
  const Windows B(L.B);
  parallel(n, threads_or_all(threads), [&](uint64_t lo, uint64_t hi) {
    for (uint64_t i = lo; i < hi; ++i) store(x + 9 * i, B.apply(one(), id0 + i));
  });
}

// x[i] <- A_p^(k[i]) x[i] for i < n.
void rlx_cpu_skip(uint64_t* x, uint64_t n, const uint64_t* k, uint32_t p, int threads) {
  const Level L = level(p);
  const Windows A(L.A);
  parallel(n, threads_or_all(threads), [&](uint64_t lo, uint64_t hi) {
    for (uint64_t i = lo; i < hi; ++i) store(x + 9 * i, A.apply(load(x + 9 * i), k[i]));
  });
}

// Streams seeded with ids id0 + i (i < n), `count` doubles each from position
// 0 into out[i * count + j] (out_u, when not null, gets the 48-bit values).
void rlx_cpu_generate(uint64_t n, uint64_t id0, uint64_t count, uint32_t p, double* out, uint64_t* out_u,
                      int threads) {
  const Level L = level(p);
  const Windows B(L.B);
  parallel(n, threads_or_all(threads), [&](uint64_t lo, uint64_t hi) {
    for (uint64_t i = lo; i < hi; ++i)
      draw(B.apply(one(), id0 + i), L.A, count, out ? out + i * count : nullptr, out_u ? out_u + i * count : nullptr);
  });
}

// One stream (id) of `count` doubles split over the threads in blocks of
// whole steps, each thread starting from its own skip (block-split).
void rlx_cpu_generate_split(uint64_t id, uint64_t count, uint32_t p, double* out, int threads) {
  const Level L = level(p);
  const uint64_t e[1] = {id};
  const Num x0 = power(L.B, e, 1);
  const uint64_t steps = (count + 11) / 12;
  const int t = threads_or_all(threads);
  parallel(steps, t, [&](uint64_t lo, uint64_t hi) {
    const uint64_t j0 = lo * 12, j1 = hi * 12 < count ? hi * 12 : count;
    draw(skip(x0, L.A, lo), L.A, j1 - j0, out + j0, nullptr);
  });
}

// Batched requests: request r draws count[r] values from position start[r]
// of the stream seeded with id[r] at level p[r], into out + offset[r].
void rlx_cpu_generate_requests(uint64_t n, const uint64_t* id, const uint64_t* start, const uint64_t* count,
                               const uint32_t* p, const uint64_t* offset, double* out, int threads) {
  // levels present (a few), built once
  std::vector<uint32_t> ps;
  std::vector<Level> levels;
  for (uint64_t r = 0; r < n; ++r) {
    bool have = false;
    for (uint32_t q : ps) have |= q == p[r];
    if (!have) {
      ps.push_back(p[r]);
      levels.push_back(level(p[r]));
    }
  }
  parallel(n, threads_or_all(threads), [&](uint64_t lo, uint64_t hi) {
    std::vector<double> tmp;
    for (uint64_t r = lo; r < hi; ++r) {
      size_t li = 0;
      while (ps[li] != p[r]) ++li;
      const Level& L = levels[li];
      const uint64_t e[1] = {id[r]};
      const Num x = skip(power(L.B, e, 1), L.A, start[r] / 12);
      const uint64_t f0 = start[r] % 12;
      tmp.resize(f0 + count[r]);
      draw(x, L.A, f0 + count[r], tmp.data(), nullptr);
      std::memcpy(out + offset[r], tmp.data() + f0, sizeof(double) * count[r]);
    }
  });
}

// test hooks: out = x y mod m, and D = floor(X 2^576 / m)
void rlx_cpu_mulmod(const uint64_t* x, const uint64_t* y, uint64_t* out) {
  store(out, mulmod(load(x), load(y)));
}

void rlx_cpu_to_ranlux(const uint64_t* x, uint64_t* d) { store(d, to_ranlux(load(x))); }

int rlx_cpu_threads(void) { return threads_or_all(0); }

}  // extern "C"
