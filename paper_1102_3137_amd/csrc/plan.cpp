// Domain decomposition planner: Fig. 1 / eq. (4) (one level, every separator
// at once) and the recursive variant at the end of Sec. II.C (one separator
// plane per domain, through the longest axis, nearest its middle, which
// alternates (d_x, d_y) = (2,1), (1,2), ... on square domains; on cubes it
// cycles x, y, z).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <functional>

namespace dyson {

dyson_opts default_opts() {
  dyson_opts o{};
  o.leaf_edge = 16;
  o.partition = DYSON_PART_NESTED;
  o.precision = DYSON_PREC_FP64;
  o.max_rank = 0;
  o.extra_steps = 10;
  o.max_inner_iters = 2000;
  o.inner_tol = 1e-14;
  o.lanczos_tol = 1e-11;
  o.seed = 0x5eedULL;
  o.profile = 0;
  o.level_streams = 4;
  o.check_sites = 2;
  o.breakdown_tol = 1e-4;
  return o;
}

dyson_opts merge_opts(const dyson_opts* u) {
  dyson_opts o = default_opts();
  if (!u) return o;
  if (u->leaf_edge) o.leaf_edge = u->leaf_edge;
  o.partition = u->partition;
  o.precision = u->precision;
  o.max_rank = u->max_rank;
  if (u->extra_steps) o.extra_steps = u->extra_steps;
  if (u->max_inner_iters) o.max_inner_iters = u->max_inner_iters;
  if (u->inner_tol > 0) o.inner_tol = u->inner_tol;
  if (u->lanczos_tol > 0) o.lanczos_tol = u->lanczos_tol;
  if (u->seed) o.seed = u->seed;
  o.profile = u->profile;
  if (u->level_streams) o.level_streams = u->level_streams;
  if (u->check_sites) o.check_sites = u->check_sites < 0 ? 0 : u->check_sites;
  o.fault_step = u->fault_step;
  o.fault_attempts = u->fault_attempts;
  if (u->breakdown_tol > 0) o.breakdown_tol = u->breakdown_tol;
  o.interface_lanczos = u->interface_lanczos;
  o.inner_graphs = u->inner_graphs;
  return o;
}

namespace {

struct Box {  // tile box [lo[a], hi[a]) per axis
  int lo[3], hi[3];
};

}  // namespace

std::string build_plan(const dyson_lattice& lat, const dyson_opts& opts, HostPlan& P) {
  if (lat.dim < 1 || lat.dim > 3) return "dim must be 1, 2 or 3";
  for (int a = 0; a < 3; ++a) {
    if (lat.L[a] < 1) return "lattice extents must be >= 1";
    if (a >= lat.dim && lat.L[a] != 1) return "unused lattice axes must have extent 1";
    if (lat.periodic[a] != 0 && lat.periodic[a] != 1) return "periodic flags must be 0 or 1";
    if (a >= lat.dim && lat.periodic[a]) return "unused lattice axes cannot be periodic";
  }
  if (!std::isfinite(lat.t) || !std::isfinite(lat.mu)) return "t and mu must be finite";
  const int smax = (lat.dim == 3) ? 6 : 16;
  if (opts.leaf_edge < 2 || opts.leaf_edge > smax)
    return lat.dim == 3 ? "leaf_edge must be in [2, 6] for cubic lattices"
                        : "leaf_edge must be in [2, 16]";
  if (opts.partition != DYSON_PART_NESTED && opts.partition != DYSON_PART_SINGLE)
    return "unknown partition";
  if (opts.precision != DYSON_PREC_FP64 && opts.precision != DYSON_PREC_MIXED &&
      opts.precision != DYSON_PREC_MIXED16)
    return "unknown precision";
  if (opts.max_rank < 0 || opts.extra_steps < 0) return "max_rank and extra_steps must be >= 0";
  if (opts.max_inner_iters < 1 || opts.max_inner_iters > 1000000)
    return "max_inner_iters must be in [1, 1000000] (0 selects the default)";
  if (opts.level_streams < 1 || opts.level_streams > 8) return "level_streams must be in [1, 8]";
  if (opts.check_sites < 0 || opts.check_sites > 2) return "check_sites must be in [-1, 2]";
  if (opts.fault_step < 0 || opts.fault_attempts < 0 || opts.fault_attempts > 3)
    return "fault_step must be >= 0 and fault_attempts in [0, 3]";
  if (!(opts.breakdown_tol > 0.0 && opts.breakdown_tol < 1.0))
    return "breakdown_tol must be in (0, 1)";
  if (opts.interface_lanczos != 0 && opts.interface_lanczos != 1)
    return "interface_lanczos must be 0 or 1";
  if (opts.inner_graphs < -1 || opts.inner_graphs > 1) return "inner_graphs must be -1, 0 or 1";
  if (opts.interface_lanczos && opts.max_rank > 0)
    return "the interface form runs to full rank (max_rank must be 0)";
  long long n = (long long)lat.L[0] * lat.L[1] * lat.L[2];
  if (n > (1LL << 28)) return "lattice too large";

  for (int a = 0; a < lat.dim; ++a)
    if (lat.periodic[a] && (lat.L[a] < 3 || lat.L[a] % opts.leaf_edge != 0))
      return "a periodic axis needs L >= 3 and L a multiple of leaf_edge";
  P = HostPlan{};
  P.dim = lat.dim;
  for (int a = 0; a < 3; ++a) P.L[a] = lat.L[a], P.periodic[a] = lat.periodic[a];
  P.t = lat.t;
  P.mu = lat.mu;
  P.opts = opts;
  P.s = opts.leaf_edge;
  const int s = P.s, D = lat.dim;
  // block rows of the tile factorization: rows of s sites (chain, square) or
  // planes of s^2 sites (cubic), stacked along the slowest axis
  P.sx = (D == 3) ? s * s : s;
  P.sy = (D == 1) ? 1 : s;
  P.S = P.sx * P.sy;
  int TT[3] = {1, 1, 1};
  for (int a = 0; a < D; ++a) TT[a] = (P.L[a] + s - 1) / s;
  P.Tx = TT[0];
  P.Ty = TT[1];
  P.Tz = TT[2];
  P.T = TT[0] * TT[1] * TT[2];
  P.N = (int)n;

  // site coordinate range of a tile box along axis a; the high fringe belongs
  // to an ancestor separator unless the box reaches an open lattice edge (on
  // a periodic axis the last plane is the top level's wrap separator)
  auto range = [&](const Box& b, int a, int& lo, int& hi) {
    if (a >= D) { lo = 0; hi = 1; return; }
    lo = s * b.lo[a];
    hi = (b.hi[a] < TT[a] || P.periodic[a]) ? s * b.hi[a] - 1 : P.L[a];
  };

  struct Node {
    Box box;
    int level;
    std::vector<int> split[3];  // tile boundaries i: separator plane at s*i-1
    bool wrap[3] = {false, false, false};  // top level: plane L-1 of a periodic axis
    std::vector<int> children;
  };
  std::vector<Node> nodes;
  std::function<int(Box, int)> rec = [&](Box b, int level) -> int {
    int id = (int)nodes.size();
    nodes.push_back(Node{b, level, {}, {false, false, false}, {}});
    std::vector<int> cand[3];
    bool any = false, wrap = false;
    for (int a = 0; a < 3; ++a) {
      for (int i = b.lo[a] + 1; i < b.hi[a]; ++i) cand[a].push_back(i);
      any |= !cand[a].empty();
      if (level == 0 && a < D && P.periodic[a]) nodes[id].wrap[a] = wrap = true;
    }
    if (!any && !wrap) return id;
    std::vector<int> sp[3];
    if (!any) {
      // only wrap planes: the one child is the same tile box, now open
    } else if (opts.partition == DYSON_PART_SINGLE) {
      for (int a = 0; a < 3; ++a) sp[a] = cand[a];
    } else {
      int best_axis = -1, best_ext = -1;
      for (int a = 0; a < 3; ++a) {
        if (cand[a].empty()) continue;
        int lo, hi;
        range(b, a, lo, hi);
        if (hi - lo > best_ext) { best_ext = hi - lo; best_axis = a; }  // first longest axis
      }
      int lo, hi;
      range(b, best_axis, lo, hi);
      const double mid = 0.5 * (lo + hi - 1);
      int best = cand[best_axis][0];
      double bd = std::fabs((s * best - 1) - mid);
      for (int i : cand[best_axis]) {
        double dd = std::fabs((s * i - 1) - mid);
        if (dd < bd) { bd = dd; best = i; }  // ties keep the lower plane
      }
      sp[best_axis].push_back(best);
    }
    for (int a = 0; a < 3; ++a) nodes[id].split[a] = sp[a];
    std::vector<int> edges[3];
    for (int a = 0; a < 3; ++a) {
      edges[a].push_back(b.lo[a]);
      for (int i : sp[a]) edges[a].push_back(i);
      edges[a].push_back(b.hi[a]);
    }
    std::vector<int> ch;
    for (size_t zi = 0; zi + 1 < edges[2].size(); ++zi)
      for (size_t yi = 0; yi + 1 < edges[1].size(); ++yi)
        for (size_t xi = 0; xi + 1 < edges[0].size(); ++xi)
          ch.push_back(rec(Box{{edges[0][xi], edges[1][yi], edges[2][zi]},
                               {edges[0][xi + 1], edges[1][yi + 1], edges[2][zi + 1]}},
                           level + 1));
    nodes[id].children = ch;
    return id;
  };
  rec(Box{{0, 0, 0}, {TT[0], TT[1], TT[2]}}, 0);

  // depth-first tile order
  auto gidx = [&](int gx, int gy, int gz) { return (gz * TT[1] + gy) * TT[0] + gx; };
  std::vector<int> tile_of_grid(P.T, -1);
  P.tile_gx.clear();
  P.tile_gy.clear();
  P.tile_gz.clear();
  std::vector<int> first(nodes.size()), last(nodes.size());
  std::function<void(int)> dfs = [&](int id) {
    first[id] = (int)P.tile_gx.size();
    const Node& nd = nodes[id];
    if (nd.children.empty()) {
      tile_of_grid[gidx(nd.box.lo[0], nd.box.lo[1], nd.box.lo[2])] = (int)P.tile_gx.size();
      P.tile_gx.push_back(nd.box.lo[0]);
      P.tile_gy.push_back(nd.box.lo[1]);
      P.tile_gz.push_back(nd.box.lo[2]);
    } else {
      for (int c : nd.children) dfs(c);
    }
    last[id] = (int)P.tile_gx.size();
  };
  dfs(0);
  if ((int)P.tile_gx.size() != P.T) return "internal: tile count mismatch";

  P.nbr.assign(P.T * 6, -1);
  for (int t = 0; t < P.T; ++t) {
    const int g[3] = {P.tile_gx[t], P.tile_gy[t], P.tile_gz[t]};
    for (int a = 0; a < 3; ++a)
      for (int sgn = 0; sgn < 2; ++sgn) {
        int h[3] = {g[0], g[1], g[2]};
        h[a] += sgn ? 1 : -1;
        if (a < D && P.periodic[a]) h[a] = (h[a] + TT[a]) % TT[a];  // wrap bond
        if (h[a] < 0 || h[a] >= TT[a]) continue;
        P.nbr[t * 6 + 2 * a + sgn] = tile_of_grid[gidx(h[0], h[1], h[2])];
      }
  }

  // site maps
  P.kind.assign((size_t)P.T * P.S, KIND_PAD);
  P.depth.assign((size_t)P.T * P.S, 0);
  P.site_of.assign((size_t)P.T * P.S, -1);
  P.pos_of.assign(P.N, -1);
  const int Lx = P.L[0], Ly = P.L[1], Lz = P.L[2];
  auto pos = [&](int x, int y, int z) {
    const int t = tile_of_grid[gidx(x / s, y / s, z / s)];
    int l = x % s;
    if (D >= 2) l += s * (y % s);
    if (D == 3) l += s * s * (z % s);
    return (size_t)t * P.S + l;
  };
  for (int z = 0; z < Lz; ++z)
    for (int y = 0; y < Ly; ++y)
      for (int x = 0; x < Lx; ++x) {
        const size_t p = pos(x, y, z);
        const int i = x + Lx * (y + Ly * z);
        P.site_of[p] = i;
        P.pos_of[i] = (int)p;
      }

  // separators top-down (a site takes the level of the first plane through
  // it), leaf sites take the depth of their leaf
  int max_level = -1;
  for (const Node& nd : nodes)
    if (!nd.children.empty()) max_level = std::max(max_level, nd.level);
  P.levels.assign(max_level + 1, LevelTable{});
  for (auto& lv : P.levels) lv.tile_node.assign(P.T, -1);
  std::vector<int> order(nodes.size());
  for (size_t i = 0; i < nodes.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return nodes[a].level < nodes[b].level; });
  std::vector<char> claimed(P.N, 0);
  for (int id : order) {
    const Node& nd = nodes[id];
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      range(nd.box, a, lo[a], hi[a]);
      if (nd.wrap[a]) hi[a] = P.L[a];  // the top level owns the wrap plane
    }
    const bool leaf = nd.children.empty();
    int m = 0;
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) {
          const int c[3] = {x, y, z};
          bool on = false;
          for (int a = 0; a < 3 && !leaf; ++a) {
            for (int i : nd.split[a]) on |= (c[a] == s * i - 1);
            on |= nd.wrap[a] && c[a] == P.L[a] - 1;
          }
          const int i = x + Lx * (y + Ly * z);
          if ((!leaf && !on) || claimed[i]) continue;
          claimed[i] = 1;
          const size_t p = P.pos_of[i];
          P.kind[p] = leaf ? KIND_LEAF : KIND_SEP;
          P.depth[p] = (uint8_t)nd.level;
          ++m;
        }
    if (leaf) continue;
    LevelTable& lv = P.levels[nd.level];
    const int idx = lv.n_nodes++;
    lv.tile_lo.push_back(first[id]);
    lv.tile_hi.push_back(last[id]);
    lv.m.push_back(m);
    for (int tt = first[id]; tt < last[id]; ++tt) lv.tile_node[tt] = idx;
    P.max_m = std::max(P.max_m, m);
  }
  for (int i = 0; i < P.N; ++i)
    if (!claimed[i]) return "internal: unclaimed site";
  if ((int)P.levels.size() > 31) return "too many levels";
  return "";
}

}  // namespace dyson
