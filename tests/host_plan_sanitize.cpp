// Host planner under AddressSanitizer / UndefinedBehaviorSanitizer (a CPU
// build with g++, no GPU code): reads meshes from a binary file and prints,
// per mesh, the plan's sizes and digests of its integer decisions, or the
// error status it raised. Driven by tests/test_host_sanitize.py.
//
// File: repeated records of  int64 nv, nv*3 double, int64 nt, nt*3 int32,
// double freq_hz, double h_lambda, int32 order, double near_radius_lambda.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "aim_internal.h"

template <typename T>
static bool rd(FILE *f, T *p, size_t n) {
  return fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  for (;;) {
    int64_t nv = 0, nt = 0;
    if (!rd(f, &nv, 1)) break;
    std::vector<double> v((size_t)(nv > 0 ? nv : 0) * 3);
    if (!rd(f, v.data(), v.size()) || !rd(f, &nt, 1)) return 3;
    std::vector<int32_t> t((size_t)(nt > 0 ? nt : 0) * 3);
    double freq = 0, h = 0, rn = 0;
    int32_t order = 0;
    if (!rd(f, t.data(), t.size()) || !rd(f, &freq, 1) || !rd(f, &h, 1) || !rd(f, &order, 1) ||
        !rd(f, &rn, 1))
      return 3;
    aim_mesh m{nv, v.empty() ? nullptr : v.data(), nt, t.empty() ? nullptr : t.data(), freq};
    aim_params p{};
    p.h_lambda = h;
    p.order = order;
    p.near_radius_lambda = rn;
    aim::HostPlan hp;
    try {
      aim::host_plan_build(m, p, &hp);
    } catch (const aim::Error &e) {
      printf("error %d\n", (int)e.status);
      continue;
    }
    long long sa = 0, sc = 0, se = 0;
    for (size_t i = 0; i < hp.anchor.size(); ++i) sa += (long long)(i % 7 + 1) * hp.anchor[i];
    for (size_t i = 0; i < hp.cols.size(); ++i) sc += (long long)(i % 13 + 1) * hp.cols[i];
    for (int64_t i = 0; i < hp.n; ++i)
      se += (long long)(i % 5 + 1) * (hp.e_lo[i] + 3LL * hp.e_hi[i] + 5LL * hp.tp[i] + 7LL * hp.tm[i]);
    printf("ok %lld %lld %d %d %d %d %d %d %lld %lld %lld\n", (long long)hp.n, (long long)hp.nnz,
           hp.grid[0], hp.grid[1], hp.grid[2], hp.pad[0], hp.pad[1], hp.pad[2], sa, sc, se);
  }
  fclose(f);
  return 0;
}
