// Host-only check of the domain-decomposition planner (plan.cpp), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_native_sanitizers.py.
// For many lattice shapes, leaf edges, partitions and periodic flags it builds
// the plan and checks its invariants; invalid inputs must be refused with a
// message (no crash, no out-of-bounds access).
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1102_3137_amd/csrc/plan.h"

using namespace dyson;

static int fails = 0;
#define CHECK(c, ...)                                       \
  do {                                                      \
    if (!(c)) {                                             \
      std::fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                    \
      std::fprintf(stderr, "\n");                           \
      ++fails;                                              \
      return;                                               \
    }                                                       \
  } while (0)

static void check_plan(int dim, int lx, int ly, int lz, int s, int part, int px, int py, int pz) {
  dyson_lattice lat{};
  lat.dim = dim;
  lat.L[0] = lx;
  lat.L[1] = dim > 1 ? ly : 1;
  lat.L[2] = dim > 2 ? lz : 1;
  lat.periodic[0] = px;
  lat.periodic[1] = dim > 1 ? py : 0;
  lat.periodic[2] = dim > 2 ? pz : 0;
  lat.t = -1.0;
  lat.mu = 0.5;
  dyson_opts o = default_opts();
  o.leaf_edge = s;
  o.partition = part;
  HostPlan P;
  const std::string e = build_plan(lat, o, P);
  if (!e.empty()) return;  // refused shapes (e.g. a periodic extent not a multiple of s)
  const int N = P.N;
  CHECK(N == lat.L[0] * lat.L[1] * lat.L[2], "N");
  CHECK((int)P.pos_of.size() == N && (int)P.site_of.size() == P.T * P.S, "map sizes");
  std::vector<int> seen(P.T * P.S, 0);
  for (int i = 0; i < N; ++i) {
    const int p = P.pos_of[i];
    CHECK(p >= 0 && p < P.T * P.S, "pos_of range");
    CHECK(P.site_of[p] == i, "site_of(pos_of(i)) = i");
    CHECK(P.kind[p] == KIND_LEAF || P.kind[p] == KIND_SEP, "kind of a site");
    ++seen[p];
  }
  for (int p = 0; p < P.T * P.S; ++p) {
    CHECK(seen[p] <= 1, "position used twice");
    CHECK((P.site_of[p] < 0) == (P.kind[p] == KIND_PAD), "padding");
  }
  for (int t = 0; t < P.T; ++t)
    for (int d = 0; d < 6; ++d) {
      const int u = P.nbr[t * 6 + d];
      CHECK(u >= -1 && u < P.T, "neighbour range");
      if (u >= 0) CHECK(P.nbr[u * 6 + (d ^ 1)] == t, "neighbour table symmetric");
    }
  for (size_t l = 0; l < P.levels.size(); ++l) {
    const LevelTable& L = P.levels[l];
    CHECK((int)L.tile_node.size() == P.T && (int)L.m.size() == L.n_nodes, "level sizes");
    int prev_hi = 0;
    for (int n = 0; n < L.n_nodes; ++n) {
      CHECK(L.tile_lo[n] >= prev_hi && L.tile_lo[n] < L.tile_hi[n] && L.tile_hi[n] <= P.T,
            "tile ranges ordered and disjoint");
      prev_hi = L.tile_hi[n];
      int m = 0;
      for (int t = L.tile_lo[n]; t < L.tile_hi[n]; ++t) {
        CHECK(L.tile_node[t] == n, "tile_node");
        for (int q = 0; q < P.S; ++q) {
          const int p = t * P.S + q;
          m += (P.kind[p] == KIND_SEP && P.depth[p] == (int)l);
        }
      }
      CHECK(m == L.m[n], "interface size of a domain");
    }
  }
}

int main() {
  int n = 0;
  for (int part = 0; part < 2; ++part) {
    for (int s : {2, 3, 5, 8, 16})
      for (int L : {1, 2, 7, 16, 33, 64})
        for (int p = 0; p < 2; ++p) check_plan(1, L, 1, 1, s, part, p, 0, 0), ++n;
    for (int s : {2, 3, 4, 8, 12, 16})
      for (int lx : {1, 5, 16, 29, 48})
        for (int ly : {3, 16, 37})
          for (int p = 0; p < 4; ++p) check_plan(2, lx, ly, 1, s, part, p & 1, p >> 1, 0), ++n;
    for (int s : {2, 3, 4, 5, 6})
      for (int lx : {4, 9, 12})
        for (int ly : {5, 12})
          for (int lz : {6, 13})
            for (int p = 0; p < 8; ++p)
              check_plan(3, lx, ly, lz, s, part, p & 1, (p >> 1) & 1, p >> 2), ++n;
  }
  // invalid input: refused with a message
  dyson_lattice bad{};
  bad.dim = 4;
  bad.L[0] = bad.L[1] = bad.L[2] = 4;
  HostPlan P;
  dyson_opts o = default_opts();
  if (build_plan(bad, o, P).empty()) ++fails;
  bad.dim = 2;
  bad.L[0] = 0;
  if (build_plan(bad, o, P).empty()) ++fails;
  bad.L[0] = 8;
  bad.L[2] = 1;
  o.leaf_edge = 1;
  if (build_plan(bad, o, P).empty()) ++fails;
  o.leaf_edge = 16;
  o.level_streams = 99;
  if (build_plan(bad, o, P).empty()) ++fails;
  std::printf("%d plans checked, %d failures\n", n, fails);
  return fails ? 1 : 0;
}
