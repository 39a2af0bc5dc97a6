// Host-side domain decomposition plan (integer work only).
//
// The lattice is cut by one-site-wide separator lines at p with (p+1) % s == 0,
// p < L-1 (the Fig. 1 layout generalised to any size), so every subdomain
// ("leaf") spans at most s-1 sites per axis (s at the last tile).  A tile is
// the s x s block of the lattice holding one leaf plus the separator sites
// on its high-x / high-y fringe.  On a periodic axis the plane at L-1 (one
// end of the wrap bonds) is a separator of the top level as well.  Tiles are
// numbered in depth-first order of the domain tree, so every domain of every
// level owns a contiguous range of tiles.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dyson.h"

namespace dyson {

enum : uint8_t { KIND_PAD = 0, KIND_LEAF = 1, KIND_SEP = 2 };

struct LevelTable {
  int n_nodes = 0;
  std::vector<int> tile_lo, tile_hi;  // [n_nodes] contiguous tile ranges
  std::vector<int> m;                 // [n_nodes] interface (separator) sites
  std::vector<int> tile_node;         // [T] node at this level or -1
};

struct HostPlan {
  int dim = 2;
  int L[3] = {1, 1, 1};
  int periodic[3] = {0, 0, 0};
  double t = -1.0, mu = 0.0;
  dyson_opts opts{};
  int s = 16;         // leaf edge
  int sx = 16, sy = 16;  // block rows of a tile: sy slices of sx sites
                         // (rows of s sites; planes of s*s sites on cubes)
  int S = 256;        // padded sites per tile (sx*sy = s^dim)
  int Tx = 1, Ty = 1, Tz = 1, T = 1;
  int N = 1;
  std::vector<int> tile_gx, tile_gy, tile_gz;  // grid coordinates of tile t
  std::vector<int> nbr;  // [T*6]: -x, +x, -y, +y, -z, +z neighbour tile or -1
  std::vector<uint8_t> kind, depth;   // [T*S] tile-major
  std::vector<int> site_of;           // [T*S] natural site index or -1 (padding)
  std::vector<int> pos_of;            // [N] tile-major position of natural site
  std::vector<LevelTable> levels;     // correction levels 0..levels-1
  int max_m = 0;
};

// Builds the plan; returns an empty string on success, else a message.
std::string build_plan(const dyson_lattice& lat, const dyson_opts& opts, HostPlan& out);

dyson_opts default_opts();
dyson_opts merge_opts(const dyson_opts* user);

}  // namespace dyson
