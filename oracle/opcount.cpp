// opcount.cpp -- algorithmic operation count of one stage of the oracle.
//
// TEST INFRASTRUCTURE ONLY.  Compiles the oracle's C source with `double`
// replaced by a type that counts every floating-point add/subtract, multiply,
// divide and square root, then applies one stage to a seeded input read from a
// raw file and prints the counts per cell.  The counts are the algorithmic
// operations of the method as the oracle writes it (every face solved once,
// each slope evaluated where the oracle evaluates it); comparisons, fabs and
// selects are not counted.  "repeated" counts the operations the oracle spends
// re-forming, for a cell's lower face, the one-sided differences and limited
// slope that its upper face already formed (each face difference serves two
// cells); "method_flops" is the count without them: every difference, slope,
// face state, Riemann solve and update formed once.
//
// Build: g++ -O1 -std=c++17 -o opcount oracle/opcount.cpp
// Run:   ./opcount state.bin nx ny nz   (8 float64 fields, [nz][ny][nx] each)
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>

typedef double real_t;
static long long g_add = 0, g_mul = 0, g_div = 0, g_sqrt = 0;
// operations inside a scope the oracle marks as repeated work (the lower-face
// reconstruction, whose differences and slope the upper face already formed)
static int g_rep_depth = 0;
static long long g_rep = 0;
struct RepeatedScope {
  RepeatedScope() { ++g_rep_depth; }
  ~RepeatedScope() { --g_rep_depth; }
};
static inline void tick(long long& c) {
  ++c;
  if (g_rep_depth) ++g_rep;
}

struct CD {
  real_t v;
  CD() = default;
  constexpr CD(real_t x) : v(x) {}
  explicit operator real_t() const { return v; }
};
static inline CD operator+(CD a, CD b) { tick(g_add); return CD(a.v + b.v); }
static inline CD operator-(CD a, CD b) { tick(g_add); return CD(a.v - b.v); }
static inline CD operator-(CD a) { return CD(-a.v); }
static inline CD operator*(CD a, CD b) { tick(g_mul); return CD(a.v * b.v); }
static inline CD operator/(CD a, CD b) { tick(g_div); return CD(a.v / b.v); }
static inline CD& operator+=(CD& a, CD b) { a = a + b; return a; }
static inline bool operator>(CD a, CD b) { return a.v > b.v; }
static inline bool operator<(CD a, CD b) { return a.v < b.v; }
static inline bool operator>=(CD a, CD b) { return a.v >= b.v; }
static inline bool operator<=(CD a, CD b) { return a.v <= b.v; }
static inline bool operator==(CD a, CD b) { return a.v == b.v; }
static inline bool operator!=(CD a, CD b) { return a.v != b.v; }
static inline CD sqrt_c(CD a) { tick(g_sqrt); return CD(std::sqrt(a.v)); }
static inline CD fabs_c(CD a) { return CD(std::fabs(a.v)); }
static inline bool isfinite_c(CD a) { return std::isfinite(a.v); }

// the oracle's headers, included before the renaming below
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>
// single-threaded: OpenMP pragmas are ignored without -fopenmp
extern "C" int omp_get_max_threads(void) { return 1; }
extern "C" void omp_set_num_threads(int) {}

#define ORC_OPCOUNT_REPEATED RepeatedScope repeated_scope_;
#define double CD
#define sqrt sqrt_c
#define fabs fabs_c
#define isfinite isfinite_c
#include "mhd_oracle.c"
#undef double

int main(int argc, char** argv) {
  if (argc < 5) {
    std::fprintf(stderr, "usage: opcount state.bin nx ny nz [hll]\n");
    return 2;
  }
  int nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  long n = (long)nx * ny * nz;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  std::vector<real_t> raw(8 * n);
  if (std::fread(raw.data(), sizeof(real_t), 8 * n, f) != (size_t)(8 * n)) return 2;
  std::fclose(f);
  std::vector<CD> st(8 * n), out(8 * n);
  for (long i = 0; i < 8 * n; ++i) st[i] = CD(raw[i]);
  orc_params p = {nx, ny, nz, 1.0, 1.0, 1.0, CD(5.0 / 3.0), CD(0.3),
                  argc > 5 ? ORC_HLL : ORC_HLLD, ORC_RK2};
  p.lx = CD((real_t)nx / std::max(nx, std::max(ny, nz)));
  p.ly = CD((real_t)ny / std::max(nx, std::max(ny, nz)));
  p.lz = CD((real_t)nz / std::max(nx, std::max(ny, nz)));
  orc_state s, d;
  CD* a[8];
  CD* b[8];
  for (int q = 0; q < 8; ++q) { a[q] = st.data() + q * n; b[q] = out.data() + q * n; }
  s = {a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7]};
  d = {b[0], b[1], b[2], b[3], b[4], b[5], b[6], b[7]};
  grid_t g;
  grid_init(&g, &p);
  work_t w;
  work_alloc(&w, g.n);
  CD mi;
  g_add = g_mul = g_div = g_sqrt = g_rep = 0;
  stage(&g, &s, nullptr, CD(1), CD(0), &d, CD(1e-4), &mi, &w, nullptr, nullptr, nullptr);
  real_t c = (real_t)n;
  std::printf("{\"cells\": %ld, \"add_sub\": %.2f, \"mul\": %.2f, \"div\": %.2f, \"sqrt\": %.2f, "
              "\"flops\": %.2f, \"repeated\": %.2f, \"method_flops\": %.2f}\n", n, g_add / c,
              g_mul / c, g_div / c, g_sqrt / c, (g_add + g_mul + g_div + g_sqrt) / c, g_rep / c,
              (g_add + g_mul + g_div + g_sqrt - g_rep) / c);
  return 0;
}
