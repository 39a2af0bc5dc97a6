// Domain decomposition planner: Fig. 1 / eq. (4) (one level, every separator
// at once) and the recursive variant at the end of Sec. II.C (one separator
// plane per domain, through the longest axis, nearest its middle, which
// alternates (d_x, d_y) = (2,1), (1,2), ... on square domains).
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
  return o;
}

namespace {

struct Box {  // tile box [x0,x1) x [y0,y1)
  int x0, x1, y0, y1;
};

}  // namespace

std::string build_plan(const dyson_lattice& lat, const dyson_opts& opts, HostPlan& P) {
  if (lat.dim != 1 && lat.dim != 2)
    return "dim must be 1 or 2 (3-D lattices are not built in this library yet)";
  for (int a = 0; a < 3; ++a) {
    if (lat.L[a] < 1) return "lattice extents must be >= 1";
    if (a >= lat.dim && lat.L[a] != 1) return "unused lattice axes must have extent 1";
  }
  if (!std::isfinite(lat.t) || !std::isfinite(lat.mu)) return "t and mu must be finite";
  if (opts.leaf_edge < 2 || opts.leaf_edge > 16) return "leaf_edge must be in [2, 16]";
  if (opts.partition != DYSON_PART_NESTED && opts.partition != DYSON_PART_SINGLE)
    return "unknown partition";
  if (opts.precision != DYSON_PREC_FP64 && opts.precision != DYSON_PREC_MIXED)
    return "unknown precision";
  if (opts.max_rank < 0 || opts.extra_steps < 0) return "max_rank and extra_steps must be >= 0";
  long long n = (long long)lat.L[0] * lat.L[1] * lat.L[2];
  if (n > (1LL << 28)) return "lattice too large";

  P = HostPlan{};
  P.dim = lat.dim;
  for (int a = 0; a < 3; ++a) P.L[a] = lat.L[a];
  P.t = lat.t;
  P.mu = lat.mu;
  P.opts = opts;
  P.s = opts.leaf_edge;
  P.sx = P.s;
  P.sy = (lat.dim == 2) ? P.s : 1;
  P.S = P.sx * P.sy;
  P.Tx = (P.L[0] + P.s - 1) / P.s;
  P.Ty = (lat.dim == 2) ? (P.L[1] + P.s - 1) / P.s : 1;
  P.T = P.Tx * P.Ty;
  P.N = (int)n;
  const int s = P.s, Lx = P.L[0], Ly = P.L[1];

  // site coordinate ranges of a tile box; the high fringe belongs to an
  // ancestor separator unless the box reaches the lattice edge
  auto xr = [&](const Box& b, int& lo, int& hi) {
    lo = s * b.x0;
    hi = (b.x1 < P.Tx) ? s * b.x1 - 1 : Lx;
  };
  auto yr = [&](const Box& b, int& lo, int& hi) {
    if (P.dim == 1) { lo = 0; hi = 1; return; }
    lo = s * b.y0;
    hi = (b.y1 < P.Ty) ? s * b.y1 - 1 : Ly;
  };

  struct Node {
    Box box;
    int level;
    std::vector<int> split_x, split_y;  // tile boundaries i: separator line at s*i-1
    std::vector<int> children;
  };
  std::vector<Node> nodes;
  std::function<int(Box, int)> rec = [&](Box b, int level) -> int {
    int id = (int)nodes.size();
    nodes.push_back(Node{b, level, {}, {}, {}});
    std::vector<int> cx, cy;
    for (int i = b.x0 + 1; i < b.x1; ++i) cx.push_back(i);
    for (int i = b.y0 + 1; i < b.y1; ++i) cy.push_back(i);
    if (cx.empty() && cy.empty()) return id;
    std::vector<int> sxs, sys;
    if (opts.partition == DYSON_PART_SINGLE) {
      sxs = cx;
      sys = cy;
    } else {
      int xlo, xhi, ylo, yhi;
      xr(b, xlo, xhi);
      yr(b, ylo, yhi);
      int ex = cx.empty() ? -1 : xhi - xlo, ey = cy.empty() ? -1 : yhi - ylo;
      bool along_x = ex >= ey;  // first longest axis
      const std::vector<int>& c = along_x ? cx : cy;
      double mid = along_x ? 0.5 * (xlo + xhi - 1) : 0.5 * (ylo + yhi - 1);
      int best = c[0];
      double bd = std::fabs((s * best - 1) - mid);
      for (int i : c) {
        double dd = std::fabs((s * i - 1) - mid);
        if (dd < bd) { bd = dd; best = i; }  // ties keep the lower plane
      }
      (along_x ? sxs : sys).push_back(best);
    }
    nodes[id].split_x = sxs;
    nodes[id].split_y = sys;
    std::vector<int> bx{b.x0}, by{b.y0};
    for (int i : sxs) bx.push_back(i);
    bx.push_back(b.x1);
    for (int i : sys) by.push_back(i);
    by.push_back(b.y1);
    std::vector<int> ch;
    for (size_t yi = 0; yi + 1 < by.size(); ++yi)
      for (size_t xi = 0; xi + 1 < bx.size(); ++xi)
        ch.push_back(rec(Box{bx[xi], bx[xi + 1], by[yi], by[yi + 1]}, level + 1));
    nodes[id].children = ch;
    return id;
  };
  rec(Box{0, P.Tx, 0, P.Ty}, 0);

  // depth-first tile order
  std::vector<int> tile_of_grid(P.T, -1);
  P.tile_gx.clear();
  P.tile_gy.clear();
  std::vector<int> first(nodes.size()), last(nodes.size());
  std::function<void(int)> dfs = [&](int id) {
    first[id] = (int)P.tile_gx.size();
    const Node& nd = nodes[id];
    if (nd.children.empty()) {
      tile_of_grid[nd.box.y0 * P.Tx + nd.box.x0] = (int)P.tile_gx.size();
      P.tile_gx.push_back(nd.box.x0);
      P.tile_gy.push_back(nd.box.y0);
    } else {
      for (int c : nd.children) dfs(c);
    }
    last[id] = (int)P.tile_gx.size();
  };
  dfs(0);
  if ((int)P.tile_gx.size() != P.T) return "internal: tile count mismatch";

  P.nbr.assign(P.T * 4, -1);
  for (int t = 0; t < P.T; ++t) {
    int gx = P.tile_gx[t], gy = P.tile_gy[t];
    if (gx > 0) P.nbr[t * 4 + 0] = tile_of_grid[gy * P.Tx + gx - 1];
    if (gx + 1 < P.Tx) P.nbr[t * 4 + 1] = tile_of_grid[gy * P.Tx + gx + 1];
    if (gy > 0) P.nbr[t * 4 + 2] = tile_of_grid[(gy - 1) * P.Tx + gx];
    if (gy + 1 < P.Ty) P.nbr[t * 4 + 3] = tile_of_grid[(gy + 1) * P.Tx + gx];
  }

  // site maps
  P.kind.assign((size_t)P.T * P.S, KIND_PAD);
  P.depth.assign((size_t)P.T * P.S, 0);
  P.site_of.assign((size_t)P.T * P.S, -1);
  P.pos_of.assign(P.N, -1);
  auto pos = [&](int x, int y) {
    int t = tile_of_grid[(y / s) * P.Tx + (x / s)];
    return (size_t)t * P.S + (x % s) + P.sx * (P.dim == 2 ? (y % s) : 0);
  };
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x < Lx; ++x) {
      size_t p = pos(x, y);
      P.site_of[p] = x + Lx * y;
      P.pos_of[x + Lx * y] = (int)p;
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
    int xlo, xhi, ylo, yhi;
    xr(nd.box, xlo, xhi);
    yr(nd.box, ylo, yhi);
    if (nd.children.empty()) {
      for (int y = ylo; y < yhi; ++y)
        for (int x = xlo; x < xhi; ++x) {
          int i = x + Lx * y;
          if (claimed[i]) continue;
          claimed[i] = 1;
          size_t p = P.pos_of[i];
          P.kind[p] = KIND_LEAF;
          P.depth[p] = (uint8_t)nd.level;
        }
      continue;
    }
    int m = 0;
    for (int y = ylo; y < yhi; ++y)
      for (int x = xlo; x < xhi; ++x) {
        bool on = false;
        for (int i : nd.split_x) on |= (x == s * i - 1);
        for (int i : nd.split_y) on |= (y == s * i - 1);
        int i = x + Lx * y;
        if (!on || claimed[i]) continue;
        claimed[i] = 1;
        size_t p = P.pos_of[i];
        P.kind[p] = KIND_SEP;
        P.depth[p] = (uint8_t)nd.level;
        ++m;
      }
    LevelTable& lv = P.levels[nd.level];
    int idx = lv.n_nodes++;
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
