// Inner solves of the X-matvec (eqs. (10)-(11)): preconditioned COCG, the
// conjugate-gradient variant for complex-symmetric matrices in which every
// inner product is the bilinear form of Sec. II.A (no conjugation).
//
// A_g is the lattice restricted to the sites active in graph g; M is the
// block diagonal of A_g over tiles (a tile = one leaf subdomain plus its
// high-side separator fringe), factored by k_factor as a block LDL^T over
// the tile's rows of sx sites.
//
// Work unit = one (tile, frequency).  Slices of at most 16 sites (rows of
// square tiles, planes of 4^3 cubic tiles): ONE wavefront per unit, four
// units per workgroup, and nothing synchronises across waves: the tile solve
// passes its row vectors through the wave's own LDS slice.  Plane slices of
// 25 or 36 sites (cubic tiles of edge 5, 6): one workgroup per unit.  No data crosses
// workgroups inside a launch (the eight XCDs keep separate L2 caches): each
// unit writes its partial sums, and the NEXT launch's waves re-reduce the
// partials of their item in a fixed order (so every wave derives the same
// scalars, deterministically); the wave on the item's first tile records
// the item state.  An iteration is two launches (stencil, update); the host
// polls convergence through a check kernel (one wave per item).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devcommon.h"
#include "kernels.h"

namespace dyson {
namespace {
using namespace dev;

constexpr int WAVES = 4;  // units per workgroup

struct Unit {
  int k, t, node, item, lane, wave;
  bool ok;
};

// Units of a launch: (frequency slot, tile) pairs, the slot taken through
// the compacted list of open frequencies when there is one.
// The list length, the list entry and the tile's domain are read together
// (the entry and the tile through a clamped, always valid unit index), so a
// unit's first memory round trip yields all three.
__device__ __forceinline__ Unit decode_id(const CocgLaunch& a, int id) {
  Unit u;
  u.wave = threadIdx.x >> 6;
  u.lane = threadIdx.x & 63;
  const int kt = a.K * a.G.T;
  const int idc = id < kt ? id : kt - 1;
  const int ks = idc / a.G.T;
  u.t = idc - ks * a.G.T;
  const int nk = a.klist ? *a.kcount : a.K;
  const int kk = a.klist ? a.klist[ks] : ks;
  const int node = a.tile_node[u.t];
  u.ok = id < nk * a.G.T && node >= 0;
  u.k = u.ok ? kk : 0;
  u.node = u.ok ? node : -1;
  u.item = u.k * a.n_nodes + u.node;
  return u;
}
// The stencil and update launches: workgroup b goes to XCD b mod 8, so the
// 4-tile groups of one frequency are dealt out so that each XCD takes a
// contiguous range of tiles (tile rows, whose neighbours in the lattice share
// its L2), while every frequency still spreads over all eight XCDs (the open
// frequencies come first in the list).  Any tile count that is not a multiple
// of 32 keeps the plain order.
// A workgroup whose frequency slot lies past the list's end leaves after the
// one scalar load of the list length, before any vector load: in the late
// launches of a solve most of the grid is such workgroups.
__device__ __forceinline__ Unit decode_xcd(const CocgLaunch& a) {
  const int T = a.G.T;
  if ((T & 31) != 0) return decode_id(a, blockIdx.x * WAVES + (threadIdx.x >> 6));
  const int nW = T / WAVES;  // workgroups per frequency, a multiple of 8
  const int b = blockIdx.x, ks = b / nW, j = b - ks * nW;
  if (a.klist && ks >= *a.kcount) {
    return Unit{0, 0, -1, -1, (int)(threadIdx.x & 63), (int)(threadIdx.x >> 6), false};
  }
  const int g = (j & 7) * (nW >> 3) + (j >> 3);
  return decode_id(a, ks * T + g * WAVES + (threadIdx.x >> 6));
}

// every unit, one per wave (the initialisation: no list)
__device__ __forceinline__ Unit decode(const CocgLaunch& a) {
  CocgLaunch b = a;
  b.klist = nullptr;
  return decode_id(b, blockIdx.x * WAVES + (threadIdx.x >> 6));
}

// Sum over the item's tiles of `per` complex partials per unit, fixed order:
// lane L adds tiles lo+L, lo+L+64, ... in turn, then the wave reduces.  The
// loads of a chunk of CH tiles per lane go out together (addresses clamped to
// the range, so every load is valid) and are added in order afterwards: one
// memory round trip per chunk instead of one per tile.
template <int CH = 2>
__device__ __forceinline__ void item_sum_of(const double* part, int per, const CocgLaunch& a,
                                            int k, int lo, int hi, int lane, cd& s0, cd& s1) {
  s0 = cmk(0.0, 0.0);
  s1 = cmk(0.0, 0.0);
  const size_t kb = (size_t)k * a.G.T;
  for (int t0 = lo + lane; t0 < hi; t0 += 64 * CH) {
    cd v0[CH], v1[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int tt = t0 + 64 * q;
      const size_t qq = (kb + (tt < hi ? tt : hi - 1)) * per;
      v0[q] = ld(part, qq);
      v1[q] = per == 2 ? ld(part, qq + 1) : cmk(0.0, 0.0);
    }
    // a select, not a branch: a load used only under a branch would be sunk
    // into it and cost a round trip of its own
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const bool in = t0 + 64 * q < hi;
      s0 = cadd(s0, in ? v0[q] : cmk(0.0, 0.0));
      if (per == 2) s1 = cadd(s1, in ? v1[q] : cmk(0.0, 0.0));
    }
  }
  s0 = wave_sum(s0);
  if (per == 2) s1 = wave_sum(s1);
}
// The item's state and the tile range of its domain, read together: the
// three loads depend only on the unit, so they share one memory round trip.
// The callers pin the range above their state test (an empty asm that uses
// it): a load used only past a branch is otherwise sunk below it and costs a
// round trip of its own.
struct ItemHead {
  int state, lo, hi;
};
__device__ __forceinline__ ItemHead item_head(const CocgLaunch& a, const Unit& u) {
  const int node = u.ok ? u.node : 0;  // clamped: always a valid index
  const int item = u.ok ? u.item : 0;
  return ItemHead{a.st.done[item], a.tlo[node], a.thi[node]};
}
template <int CH = 2>
__device__ __forceinline__ void item_sum(const double* part, int per, const CocgLaunch& a,
                                         const Unit& u, const ItemHead& h, cd& s0, cd& s1) {
  item_sum_of<CH>(part, per, a, u.k, h.lo, h.hi, u.lane, s0, s1);
}

// ---------------------------------------------------------- tile solve
// Lane L owns row i = L>>2 and columns 4c..4c+3 (c = L&3) of every slice
// inverse S_y^{-1}.  complex64 factors stay in registers (64 complex per
// lane, loaded once); FP64 factors are streamed per slice in both sweeps.
// Arithmetic is FP64 either way.
template <typename F, bool REG>
struct WaveFactor;

// complex64 factors held in registers for the whole solve (raw bits, so the
// compiler keeps 64 complex64 values = 128 VGPRs instead of widening them)
template <>
struct WaveFactor<float, true> {
  uint32_t gr[16][4], gi[16][4];
  __device__ __forceinline__ void load(const float* fac, size_t fbase, int sx, int sy, int lane) {
    const int i = lane >> 2, c = lane & 3;
    if (sx == 16) {
      // full tiles: lane L reads complex64 entries 4L..4L+3 of each slice,
      // 32 contiguous bytes, the wave 2 KB per slice
      const float4* f4 = reinterpret_cast<const float4*>(fac + 2 * fbase);
#pragma unroll
      for (int y = 0; y < 16; ++y) {  // slices y >= sy re-read slice sy-1 (unused)
        const size_t yy = (size_t)(y < sy ? y : sy - 1);
        const float4 a = f4[yy * 128 + 2 * lane];
        const float4 b = f4[yy * 128 + 2 * lane + 1];
        gr[y][0] = __float_as_uint(a.x); gi[y][0] = __float_as_uint(a.y);
        gr[y][1] = __float_as_uint(a.z); gi[y][1] = __float_as_uint(a.w);
        gr[y][2] = __float_as_uint(b.x); gi[y][2] = __float_as_uint(b.y);
        gr[y][3] = __float_as_uint(b.z); gi[y][3] = __float_as_uint(b.w);
      }
      return;
    }
#pragma unroll
    for (int y = 0; y < 16; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * c + e;
        float2 v = (y < sy && i < sx && j < sx)
                       ? reinterpret_cast<const float2*>(fac)[fbase + (size_t)y * sx * sx + i * sx + j]
                       : make_float2(0.f, 0.f);
        gr[y][e] = __float_as_uint(v.x);
        gi[y][e] = __float_as_uint(v.y);
      }
  }
  __device__ __forceinline__ cd get(int y, int e, const float*, size_t, int, int) const {
    uint32_t a = gr[y][e], b = gi[y][e];
    asm volatile("" : "+v"(a), "+v"(b));
    return cmk((double)__uint_as_float(a), (double)__uint_as_float(b));
  }
};

// complex32 factors (two FP16 halves per entry) held in registers: 64 VGPRs
template <>
struct WaveFactor<__half, true> {
  uint32_t g[16][4];
  __device__ __forceinline__ void load(const __half* fac, size_t fbase, int sx, int sy, int lane) {
    const int i = lane >> 2, c = lane & 3;
    if (sx == 16) {
      // slices y >= sy are never used by the sweep: they re-read slice sy-1,
      // so all sixteen loads are unconditional and go out back to back
      const uint4* f4 = reinterpret_cast<const uint4*>(fac + 2 * fbase);
#pragma unroll
      for (int y = 0; y < 16; ++y) {
        const uint4 a = f4[(size_t)(y < sy ? y : sy - 1) * 64 + lane];
        g[y][0] = a.x;
        g[y][1] = a.y;
        g[y][2] = a.z;
        g[y][3] = a.w;
      }
      return;
    }
    const uint32_t* f1 = reinterpret_cast<const uint32_t*>(fac + 2 * fbase);
#pragma unroll
    for (int y = 0; y < 16; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * c + e;
        g[y][e] = (y < sy && i < sx && j < sx) ? f1[(size_t)y * sx * sx + i * sx + j] : 0u;
      }
  }
  __device__ __forceinline__ cd get(int y, int e, const __half*, size_t, int, int) const {
    uint32_t a = g[y][e];
    asm volatile("" : "+v"(a));
    const __half2 h = *reinterpret_cast<const __half2*>(&a);
    return cmk((double)__low2float(h), (double)__high2float(h));
  }
};

// factors streamed from memory slice by slice (read in both sweeps)
template <typename F>
struct WaveFactor<F, false> {
  __device__ __forceinline__ void load(const F*, size_t, int, int, int) {}
  __device__ __forceinline__ cd get(int y, int e, const F* fac, size_t fbase, int sx,
                                    int lane) const {
    const int i = lane >> 2, j = 4 * (lane & 3) + e;
    return (i < sx && j < sx) ? ldf<F>(fac, fbase + (size_t)y * sx * sx + i * sx + j)
                              : cmk(0.0, 0.0);
  }
};

// In place: zl holds r on entry and z = M^{-1} r on exit (tile-local index
// l = x + sx*y).  Block forward z_y = r_y - T_y S_{y-1}^{-1} z_{y-1}, block
// backward v_y = S_y^{-1}(z_y - T_{y+1} v_{y+1}), T_y = t diag(active bonds).
// The bond mask of T_y costs no test inside the sweeps: an inactive site has
// the row and column of the identity in every S_y^{-1} (k_factor) and its
// entry of zl is held at exactly zero (r is zero there and the sweeps write
// zero there), so a bond to it adds an exact zero.  The reads of a step do
// not depend on the lane's columns being inside the slice (a column j >= sx
// meets zero factor entries), so they go out together and the step waits on
// LDS once.  Lane L owns row i = L>>2: its bits of `am` (bit y: site i + sx*y
// is active) decide which sites it writes.  SX = 16 fixes the slice width at
// compile time (full rows of 16x16 tiles, planes of 4^3 tiles): every LDS
// address of the sweeps is then the lane's base plus an immediate offset,
// instead of one register per slice; SX = 0 takes the width from sx.
template <typename F, bool REG, int SX>
__device__ __forceinline__ void wave_tile_solve(const WaveFactor<F, REG>& f, const F* fac, size_t fbase,
                                                cd* zl, const uint8_t* act, int sx_rt, int sy,
                                                double tt, int lane) {
  const int sx = SX ? SX : sx_rt;
  const int i = lane >> 2, c = lane & 3;
  wave_sync();
  unsigned am = 0;
#pragma unroll
  for (int y = 0; y < 16; ++y) am |= (act[i + sx * y] ? 1u : 0u) << y;  // i + sx*y <= 255
  asm volatile("" : "+v"(am));  // one mask register, formed before the sweeps
  const bool row_lane = c == 0 && i < sx;
#pragma unroll
  for (int y = 1; y < 16; ++y) {
    if (y < sy) {
      cd zv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) zv[e] = zl[4 * c + e + sx * (y - 1)];
      const cd zo = zl[i + sx * y];
      cd acc = cmk(0.0, 0.0);
#pragma unroll
      for (int e = 0; e < 4; ++e) acc = cfma(f.get(y - 1, e, fac, fbase, sx, lane), zv[e], acc);
      acc = quad_sum(acc);
      if (row_lane && ((am >> y) & 1u)) zl[i + sx * y] = csub(zo, cscale(acc, tt));
      wave_sync();
    }
  }
  // backward: the lane that writes v_y(i) also folds it into the slice below,
  // z_{y-1}(i) - t v_y(i), which is all that slice's step reads of z_{y-1}
#pragma unroll
  for (int y = 15; y >= 0; --y) {
    if (y < sy) {
      cd rw[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) rw[e] = zl[4 * c + e + sx * y];
      const cd zb = zl[i + sx * (y > 0 ? y - 1 : 0)];
      cd acc = cmk(0.0, 0.0);
#pragma unroll
      for (int e = 0; e < 4; ++e) acc = cfma(f.get(y, e, fac, fbase, sx, lane), rw[e], acc);
      acc = quad_sum(acc);
      const cd v = ((am >> y) & 1u) ? acc : cmk(0.0, 0.0);
      wave_sync();
      if (row_lane) {
        zl[i + sx * y] = v;
        if (y > 0) zl[i + sx * (y - 1)] = csub(zb, cscale(v, tt));
      }
      wave_sync();
    }
  }
}

template <typename F, bool REG, int SX>
__device__ __forceinline__ void tile_solve_any(const WaveFactor<F, REG>& f, const F* fac,
                                               size_t fbase, cd* zl, const uint8_t* act,
                                               const TileGeom& G, int lane) {
  wave_tile_solve<F, REG, SX>(f, fac, fbase, zl, act, G.sx, G.sy, G.t, lane);
}

// One lane's complex value (16 bytes) copied from global memory into LDS
// without passing through registers: the wave's 64 lanes fill 64 consecutive
// slots from `row` (lane i writes row[i]).
__device__ __forceinline__ void lds_copy16(const double* g, cd* row) {
  __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g),
                                   (__attribute__((address_space(3))) void*)(row), 16, 0, 0);
}
// Waits for every outstanding vector memory access of the wave (vmcnt = 0),
// which includes the LDS copies; the empty asm keeps the compiler from moving
// LDS reads above it.
__device__ __forceinline__ void wait_vm_all() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt not waited on
  __asm__ volatile("" ::: "memory");
}

// Item state: 0 open; 1 closed at the start (zero right-hand side or a
// stopped Lanczos item); otherwise the mark of the launch that closed it.  A
// unit that reads its own launch's mark was closed by a sibling unit of the
// same item during this launch: it still applies its tile's share of the
// closing work (the pending x update), as the sibling did.
__device__ __forceinline__ int stencil_mark(int it) { return 4 * it + 3; }
__device__ __forceinline__ int update_mark(int it) { return 4 * it + 4; }
__device__ __forceinline__ bool open_here(int state, int mark) {
  return state == 0 || state == mark;
}

// ------------------------------------------------------------- kernels
// r = b (masked to graph g), x = 0, p = 0, z = M^{-1} r;
// item totals: rho = r^T z, bn2 = |b|^2
template <typename F, bool REG, int SX>
__global__ __launch_bounds__(256) void k_cocg_init(CocgLaunch a, const double* __restrict__ b) {
  const Unit u = decode(a);
  if (!u.ok) return;
  if (a.item_skip && a.item_skip[u.item]) return;
  const TileGeom& G = a.G;
  __shared__ cd zsh[WAVES][256];
  __shared__ uint8_t ash[WAVES][256];
  cd* zl = zsh[u.wave];
  uint8_t* act = ash[u.wave];
  const size_t base = (size_t)u.k * G.T * G.S + (size_t)u.t * G.S;
  // factors, activity bytes and b all go out before anything waits
  const F* fac = (const F*)a.fac;
  const size_t fbase = ((size_t)u.k * G.T + u.t) * (size_t)G.sy * G.sx * G.sx;
  WaveFactor<F, REG> f;
  f.load(fac, fbase, SX ? SX : G.sx, G.sy, u.lane);
  cd rv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    const int lc = l < G.S ? l : G.S - 1;  // clamped: always a valid site
    const size_t p = (size_t)u.t * G.S + lc;
    const bool ac = active(G.kind[p], G.depth[p], a.g) && l < G.S;
    const cd bv = ld(b, base + lc);
    rv[e] = ac ? bv : cmk(0.0, 0.0);
    act[l] = ac ? 1 : 0;
    zl[l] = rv[e];
  }
  tile_solve_any<F, REG, SX>(f, fac, fbase, zl, act, G, u.lane);
  cd rz = cmk(0.0, 0.0), rr = cmk(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    if (l < G.S) {
      const cd zv = act[l] ? zl[l] : cmk(0.0, 0.0);
      st(a.r, base + l, rv[e]);
      st(a.z, base + l, zv);
      st(a.x, base + l, cmk(0.0, 0.0));
      st(a.p_old, base + l, cmk(0.0, 0.0));
      rz = cfma(rv[e], zv, rz);
      rr.x += cabs2(rv[e]);
    }
  }
  rz = wave_sum(rz);
  rr = wave_sum(rr);
  if (u.lane == 0) {
    const size_t q = ((size_t)u.k * G.T + u.t) * 2;
    st(a.partU, q, rz);
    st(a.partU, q + 1, rr);
  }
}

// Halo of a tile: the sites of the adjacent tiles that its face sites bond
// to.  Slot h = dir * F + pos, F = s^(D-1) sites per face, pos = the face
// site's coordinates other than the axis of dir (x fastest).  At most 2*D*F
// = 96 slots (D = 3, s = 4), so two per lane.
__device__ __forceinline__ int halo_pos(const TileGeom& G, int a, int x, int y, int z) {
  const int s = G.edge;
  if (G.dim == 1) return 0;
  if (G.dim == 2) return a == 0 ? y : x;
  return a == 0 ? y + s * z : (a == 1 ? x + s * z : x + s * y);
}
// the face site (tile-local index) of slot h, and the direction it faces
__device__ __forceinline__ int halo_site(const TileGeom& G, int h, int& dir) {
  const int s = G.edge;
  const int F = G.dim == 1 ? 1 : (G.dim == 2 ? s : s * s);
  dir = G.dim == 1 ? h : (G.dim == 2 ? div_edge(G, h) : div_edge(G, div_edge(G, h)));
  const int pos = h - dir * F;
  const int a = dir >> 1, c = (dir & 1) ? s - 1 : 0;
  if (G.dim == 1) return c;
  if (G.dim == 2) return a == 0 ? c + s * pos : pos + s * c;
  const int p1 = div_edge(G, pos), p0 = pos - s * p1;
  const int x = a == 0 ? c : p0, y = a == 0 ? p0 : (a == 1 ? c : p1), z = a == 2 ? c : p1;
  return x + s * y + s * s * z;
}

// Convergence test of the previous update, beta = rho_i / rho_{i-1};
// p_new = z + beta p_old ; s = A_g p_new ; partial mu = p^T s.
// Every load that does not depend on beta goes out before the item
// reduction: the tile's own p_old, z, d and activity bytes, and the halo
// (p_old, z and activity of the neighbouring tiles' sites next to this
// tile), whose p_new = z + beta p_old is formed here as for the own sites
// (the neighbour tile, when active, belongs to the same domain and so to
// the same item and beta).
__device__ __forceinline__ void stencil_unit(const CocgLaunch& a, int it, const Unit& u) {
  if (!u.ok) return;
  const ItemHead h = item_head(a, u);
  const TileGeom& G = a.G;
  const int s = G.edge;
  const int H = 2 * G.dim * (G.dim == 1 ? 1 : (G.dim == 2 ? s : s * s));
  // The tile's neighbours in the halo directions (slots lane, lane + 64) and
  // the activity of its own sites depend on the tile alone: a few bytes, read
  // with the item head so that they share its round trip, and the halo loads
  // below are not one round trip further back.
  int hn[2], hown[2], hnl[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int hs = u.lane + 64 * j;
    int dir = 0;
    hown[j] = halo_site(G, hs < H ? hs : 0, dir);
    const int stride = (dir >> 1) == 0 ? 1 : ((dir >> 1) == 1 ? s : s * s);
    hn[j] = hs < H ? G.nbr[u.t * 6 + dir] : -1;
    // the neighbour's site (the own face site is a valid stand-in when there is none)
    hnl[j] = (dir & 1) ? hown[j] - (s - 1) * stride : hown[j] + (s - 1) * stride;
  }
  unsigned acm = 0;  // bit e: site lane + 64 e is active in graph g
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    const size_t p = (size_t)u.t * G.S + (l < G.S ? l : G.S - 1);  // clamped: always valid
    acm |= (active(G.kind[p], G.depth[p], a.g) && l < G.S) ? (1u << e) : 0u;
  }
  asm volatile("" : : "v"(hn[0]), "v"(hn[1]), "v"(acm), "v"(h.lo), "v"(h.hi));  // above the test
  if (!open_here(h.state, stencil_mark(it))) return;
  const size_t NP = (size_t)G.T * G.S;
  const size_t kb = (size_t)u.k * NP;
  const size_t base = kb + (size_t)u.t * G.S;
  const bool lead = u.t == h.lo;  // records the item state
  size_t hi_[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
    hi_[j] = hn[j] >= 0 ? (size_t)hn[j] * G.S + hnl[j] : (size_t)u.t * G.S + hown[j];
  bool ac[4];
  cd po[4], zo[4], dv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    const size_t p = (size_t)u.t * G.S + (l < G.S ? l : G.S - 1);  // clamped: always valid
    ac[e] = (acm >> e) & 1u;
    po[e] = ld(a.p_old, kb + p);
    zo[e] = ld(a.z, kb + p);
    dv[e] = ld(a.d, kb + p);
  }
  // the halo slots' loads are unconditional (hi_ is always a valid site), so
  // they go out with the own sites' loads instead of each waiting on a branch
  bool hac[2];
  uint8_t hk[2], hd[2];
  cd hpo[2], hz[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    hk[j] = G.kind[hi_[j]];
    hd[j] = G.depth[hi_[j]];
    hpo[j] = ld(a.p_old, kb + hi_[j]);
    hz[j] = ld(a.z, kb + hi_[j]);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) hac[j] = (hn[j] >= 0) & active(hk[j], hd[j], a.g);
  cd beta = cmk(0.0, 0.0);
  if (it > 0) {
    const double bn2 = a.st.bn2[u.item];
    const cd rho_prev = ld(a.rho2 + (size_t)((it - 1) & 1) * a.n_items * 2, u.item);
    cd rho, rr;
    item_sum<4>(a.partU, 2, a, u, h, rho, rr);
    if (a.flush || rr.x <= a.tol2 * bn2) {
      if (it & 1) {  // the last update was even: x still lacks alpha_{i-1} p_{i-1}
        const cd ap = ld(a.alph, u.item);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int l = u.lane + 64 * e;
          if (ac[e]) st(a.x, base + l, cfma(ap, po[e], ld(a.x, base + l)));
        }
      }
      if (lead && u.lane == 0) {
        a.st.done[u.item] = stencil_mark(it);
        a.st.iters[u.item] = it;
      }
      return;
    }
    beta = cdiv(rho, rho_prev);
    if (lead && u.lane == 0) st(a.rho2 + (size_t)(it & 1) * a.n_items * 2, u.item, rho);
  }
  if (lead && u.lane == 0) a.kalive[u.k] = it + 2;  // the item stays open
  // profiling: the item's lead wave books the algorithmic bytes of all the
  // item's units; an atomic add that returns nothing, so the wave does not
  // wait for it (a read-modify-write would add a round trip to the unit)
  if (a.wctr && lead && u.lane == 0)
    atomicAdd(&a.wctr[(size_t)1 * a.n_items + u.item],
              (unsigned long long)(h.hi - h.lo) *
                  ((unsigned long long)(G.S * (5 * 16 + 2)) + 2ull * 2 * (G.sx + G.sy) * 16));
  __shared__ cd psh[WAVES][256];
  __shared__ cd hsh[WAVES][128];
  cd* pl = psh[u.wave];
  cd* hl = hsh[u.wave];
  cd pn[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    pn[e] = ac[e] ? cfma(beta, po[e], zo[e]) : cmk(0.0, 0.0);
    if (l < G.S) st(a.p_new, base + l, pn[e]);
    pl[l] = pn[e];
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) hl[u.lane + 64 * j] = hac[j] ? cfma(beta, hpo[j], hz[j]) : cmk(0.0, 0.0);
  wave_sync();
  cd mu = cmk(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    if (l >= G.S) continue;
    if (!ac[e]) {
      st(a.s, base + l, cmk(0.0, 0.0));
      continue;
    }
    const int q1 = div_edge(G, l), q2 = div_edge(G, q1);
    const int x = l - s * q1, y = q1 - s * q2, z = q2;
    cd nb = cmk(0.0, 0.0);
    for (int dir = 0; dir < 2 * G.dim; ++dir) {
      const int ax = dir >> 1, up = dir & 1;
      const int c = ax == 0 ? x : (ax == 1 ? y : z);
      const int stride = ax == 0 ? 1 : (ax == 1 ? s : s * s);
      if (up ? (c < s - 1) : (c > 0)) {
        nb = cadd(nb, pl[up ? l + stride : l - stride]);  // inactive sites hold 0 in pl
      } else {
        const int F = G.dim == 1 ? 1 : (G.dim == 2 ? s : s * s);
        nb = cadd(nb, hl[dir * F + halo_pos(G, ax, x, y, z)]);  // 0 without a neighbour
      }
    }
    const cd sv = cfma(dv[e], pn[e], cscale(nb, G.t));
    st(a.s, base + l, sv);
    mu = cfma(pn[e], sv, mu);
  }
  mu = wave_sum(mu);
  if (u.lane == 0) st(a.partS, (size_t)u.k * G.T + u.t, mu);
}

// Wave w of workgroup b takes unit b * WAVES + w of the launch's list; the
// grid covers every unit, and the waves past the list's end leave at once.
__global__ __launch_bounds__(256) void k_cocg_stencil(CocgLaunch a, int it) {
  stencil_unit(a, it, decode_xcd(a));
}

// r -= alpha s ; z = M^{-1} r ; item totals rho' = r^T z, |r|^2 ; converged
// when |r|^2 <= tol^2 |b|^2, else beta = rho'/rho.  x += alpha p is applied
// every other iteration: on odd iterations x += alpha_{i-1} p_{i-1} + alpha_i
// p_i (both directions are still resident), on even ones alpha_i is kept for
// the next; the stencil launch that finds an item converged after an even
// iteration applies the pending alpha_{i-1} p_{i-1}.
template <typename F, bool REG, int SX>
__device__ __forceinline__ void cocg_update_unit(const CocgLaunch& a, int it, const Unit& u) {
  if (!u.ok) return;
  const ItemHead h = item_head(a, u);
  asm volatile("" : : "v"(h.lo), "v"(h.hi));  // the range is read above the state test
  if (!open_here(h.state, update_mark(it))) return;
  const TileGeom& G = a.G;
  const size_t base = (size_t)u.k * G.T * G.S + (size_t)u.t * G.S;
  const F* fac = (const F*)a.fac;
  const size_t fbase = ((size_t)u.k * G.T + u.t) * (size_t)G.sy * G.sx * G.sx;
  __shared__ cd zsh[WAVES][256];
  __shared__ cd rsh[WAVES][256];
  __shared__ uint8_t ash[WAVES][256];
  cd* zl = zsh[u.wave];
  cd* rl = rsh[u.wave];
  uint8_t* act = ash[u.wave];
  // r and s of the tile go straight into the wave's LDS slices (no registers
  // held), then the factors: both are in flight during the item reduction
  // instead of r and s waiting for alpha
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    if (l < G.S) {
      lds_copy16(a.r + 2 * (base + l), rl + 64 * e);
      lds_copy16(a.s + 2 * (base + l), zl + 64 * e);
    }
  }
  // the activity bytes of the lane's sites and the item's rho, loaded with
  // the factors; complex64 register factors take 128 VGPRs, so there they
  // are loaded after the reduction instead of being held across it
  constexpr bool kEarly = !(REG && sizeof(F) == 4);
  unsigned acm = 0;  // bit e: site lane + 64 e is active in graph g
  cd rho;
  auto load_item_state = [&]() {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int l = u.lane + 64 * e;
      const size_t p = (size_t)u.t * G.S + (l < G.S ? l : G.S - 1);  // clamped: always valid
      const bool on = active(G.kind[p], G.depth[p], a.g);
      acm |= (on && l < G.S) ? (1u << e) : 0u;
    }
    rho = ld(a.rho2 + (size_t)(it & 1) * a.n_items * 2, u.item);
  };
  if constexpr (kEarly) load_item_state();
  WaveFactor<F, REG> f;
  f.load(fac, fbase, SX ? SX : G.sx, G.sy, u.lane);
  cd mu, unused;
  item_sum(a.partS, 1, a, u, h, mu, unused);
  if constexpr (!kEarly) load_item_state();
  const bool odd = it & 1;
  if (cabs2(mu) == 0.0) {  // breakdown of the bilinear form in the inner solve
    wait_vm_all();  // the LDS copies land before the wave leaves
    if (odd) {  // apply the pending alpha_{i-1} p_{i-1} before closing the item
      const cd ap = ld(a.alph, u.item);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if ((acm >> e) & 1u) {
          const size_t i = base + u.lane + 64 * e;
          st(a.x, i, cfma(ap, ld(a.p_old, i), ld(a.x, i)));
        }
    }
    if (u.t == h.lo && u.lane == 0) a.st.done[u.item] = update_mark(it);
    return;
  }
  const cd alpha = cdiv(rho, mu);
  if (u.t == h.lo && u.lane == 0) {
    if (!odd) st(a.alph, u.item, alpha);
    // algorithmic bytes: r, s read and r, z written every iteration; x read and
    // written and p_{i-1}, p_i read on odd ones; the factors (booked as in
    // the stencil, by an atomic add the wave does not wait for)
    if (a.wctr)
      atomicAdd(&a.wctr[u.item], (unsigned long long)(h.hi - h.lo) *
                                     ((unsigned long long)(G.S * ((odd ? 8 : 4) * 16 + 2)) +
                                      (unsigned long long)G.sy * G.sx * G.sx * (2 * sizeof(F))));
  }
  // complex64 register factors: the deferred x update in this loop (alpha
  // is then dead during the sweep); otherwise after the sweep, below
  const cd aprev_in_loop = (!kEarly && odd) ? ld(a.alph, u.item) : cmk(0.0, 0.0);
  wait_vm_all();  // r and s are in LDS
  cd rr = cmk(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    const uint8_t ac = (acm >> e) & 1u;
    cd rv = cmk(0.0, 0.0);
    if (l < G.S) {
      if (!kEarly && odd && ac)
        st(a.x, base + l,
           cfma(alpha, ld(a.p_new, base + l), cfma(aprev_in_loop, ld(a.p_old, base + l), ld(a.x, base + l))));
      if (ac) rv = csub(rl[l], cmul(alpha, zl[l]));
      st(a.r, base + l, rv);
      rr.x += cabs2(rv);
    }
    act[l] = ac;
    zl[l] = rv;
    rl[l] = rv;
  }
  tile_solve_any<F, REG, SX>(f, fac, fbase, zl, act, G, u.lane);
  cd rz = cmk(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = u.lane + 64 * e;
    if (l < G.S) {
      const cd zv = act[l] ? zl[l] : cmk(0.0, 0.0);
      st(a.z, base + l, zv);
      rz = cfma(rl[l], zv, rz);
    }
  }
  rz = wave_sum(rz);
  rr = wave_sum(rr);
  if (u.lane == 0) {
    const size_t q = ((size_t)u.k * G.T + u.t) * 2;
    st(a.partU, q, rz);
    st(a.partU, q + 1, rr);
  }
  // the deferred solution update x += alpha_{i-1} p_{i-1} + alpha_i p_i,
  // after the sweep (nothing in it reads x); the loads of the four sites go
  // out together (clamped addresses, always valid)
  if (kEarly && odd) {
    __asm__ volatile("" ::: "memory");  // keeps these loads below the sweep
    const cd aprev = ld(a.alph, u.item);
    cd xv[4], pn[4], po[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int l = u.lane + 64 * e;
      const size_t i = base + (l < G.S ? l : G.S - 1);
      xv[e] = ld(a.x, i);
      pn[e] = ld(a.p_new, i);
      po[e] = ld(a.p_old, i);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if ((acm >> e) & 1u)
        st(a.x, base + u.lane + 64 * e, cfma(alpha, pn[e], cfma(aprev, po[e], xv[e])));
  }
}

template <typename F, bool REG, int SX>
__device__ __forceinline__ void cocg_update_body(const CocgLaunch& a, int it) {
  cocg_update_unit<F, REG, SX>(a, it, decode_xcd(a));
}

template <typename F, bool REG, int SX>
__global__ __launch_bounds__(256) void k_cocg_update(CocgLaunch a, int it) {
  cocg_update_body<F, REG, SX>(a, it);
}
// complex64 register factors: 168 VGPRs, capped for 3 waves per SIMD (the
// latency of the 2 x 16 slice sweep is what this kernel must hide)
template <typename F, bool REG, int SX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_cocg_update_occ3(CocgLaunch a, int it) {
  cocg_update_body<F, REG, SX>(a, it);
}

// ------------------------------------------- plane slices: a workgroup per unit
// Cubic tiles of edge 5 or 6 have slices of n = 25 or 36 sites (planes).  One
// workgroup (256 threads) handles one (tile, frequency) unit: one thread per
// site for the vector work, and for the slice sweeps thread (i = tid>>2,
// c = tid&3) owns columns c*PW .. c*PW+PW-1 of row i of every S_y^{-1}.
// complex32 / complex64 factors are loaded into registers in one burst at
// the start, so the 2*ns-1 dependent slice steps wait only on LDS and
// workgroup barriers; FP64 factors are read per step.
constexpr int PW = 9;   // columns per thread: 4*PW >= 36
constexpr int PNS = 6;  // most slices per tile

template <typename F>
struct PlaneFactor;

template <>
struct PlaneFactor<__half> {
  uint32_t g[PNS][PW];
  __device__ __forceinline__ void load(const __half* fac, size_t fbase, int n, int ns, int i,
                                       int c) {
    const uint32_t* f1 = reinterpret_cast<const uint32_t*>(fac) + fbase;
#pragma unroll
    for (int y = 0; y < PNS; ++y)
#pragma unroll
      for (int e = 0; e < PW; ++e) {
        const int j = c * PW + e;
        g[y][e] = (y < ns && i < n && j < n) ? f1[(size_t)y * n * n + i * n + j] : 0u;
      }
  }
  __device__ __forceinline__ cd get(int y, int e, const __half*, size_t, int, int, int) const {
    uint32_t a = g[y][e];
    asm volatile("" : "+v"(a));
    const __half2 h = *reinterpret_cast<const __half2*>(&a);
    return cmk((double)__low2float(h), (double)__high2float(h));
  }
};

template <>
struct PlaneFactor<float> {
  uint32_t gr[PNS][PW], gi[PNS][PW];
  __device__ __forceinline__ void load(const float* fac, size_t fbase, int n, int ns, int i,
                                       int c) {
    const float2* f2 = reinterpret_cast<const float2*>(fac) + fbase;
#pragma unroll
    for (int y = 0; y < PNS; ++y)
#pragma unroll
      for (int e = 0; e < PW; ++e) {
        const int j = c * PW + e;
        const float2 v =
            (y < ns && i < n && j < n) ? f2[(size_t)y * n * n + i * n + j] : make_float2(0.f, 0.f);
        gr[y][e] = __float_as_uint(v.x);
        gi[y][e] = __float_as_uint(v.y);
      }
  }
  __device__ __forceinline__ cd get(int y, int e, const float*, size_t, int, int, int) const {
    uint32_t a = gr[y][e], b = gi[y][e];
    asm volatile("" : "+v"(a), "+v"(b));
    return cmk((double)__uint_as_float(a), (double)__uint_as_float(b));
  }
};

template <>
struct PlaneFactor<double> {
  __device__ __forceinline__ void load(const double*, size_t, int, int, int, int) {}
  __device__ __forceinline__ cd get(int y, int e, const double* fac, size_t fbase, int n, int i,
                                    int c) const {
    const int j = c * PW + e;
    return (i < n && j < n) ? ld(fac, fbase + (size_t)y * n * n + i * n + j) : cmk(0.0, 0.0);
  }
};

// In place over the workgroup: zl = r on entry, z = M^{-1} r on exit; the
// same block forward / backward sweeps as wave_tile_solve, with the same
// test-free treatment of inactive sites (identity rows and columns of
// S_y^{-1}, zeros in zl) and unconditional reads per step.
template <typename F>
__device__ __forceinline__ void plane_tile_solve(const PlaneFactor<F>& f, const F* fac,
                                                 size_t fbase, cd* zl, const uint8_t* act, int n,
                                                 int ns, double tt) {
  const int i = threadIdx.x >> 2, c = threadIdx.x & 3;
  __syncthreads();
  unsigned am = 0;  // bit y: site i + n*y is active
#pragma unroll
  for (int y = 0; y < PNS; ++y) am |= (act[i + n * y] ? 1u : 0u) << y;  // i + n*y <= 243
  asm volatile("" : "+v"(am));  // one mask register, formed before the sweeps
  const bool row_thread = c == 0 && i < n;
#pragma unroll
  for (int y = 1; y < PNS; ++y) {
    if (y < ns) {
      cd acc = cmk(0.0, 0.0);
#pragma unroll
      for (int e = 0; e < PW; ++e)
        acc = cfma(f.get(y - 1, e, fac, fbase, n, i, c), zl[c * PW + e + n * (y - 1)], acc);
      const cd zo = zl[i + n * y];
      acc = quad_sum(acc);
      if (row_thread && ((am >> y) & 1u)) zl[i + n * y] = csub(zo, cscale(acc, tt));
      __syncthreads();
    }
  }
#pragma unroll
  for (int y = PNS - 1; y >= 0; --y) {
    if (y < ns) {
      cd acc = cmk(0.0, 0.0);
#pragma unroll
      for (int e = 0; e < PW; ++e)
        acc = cfma(f.get(y, e, fac, fbase, n, i, c), zl[c * PW + e + n * y], acc);
      const cd zb = zl[i + n * (y > 0 ? y - 1 : 0)];
      acc = quad_sum(acc);
      const cd v = ((am >> y) & 1u) ? acc : cmk(0.0, 0.0);
      __syncthreads();
      if (row_thread) {  // v_y(i), and z_{y-1}(i) - t v_y(i) for the next step
        zl[i + n * y] = v;
        if (y > 0) zl[i + n * (y - 1)] = csub(zb, cscale(v, tt));
      }
      __syncthreads();
    }
  }
}

// Unit of a workgroup-per-unit launch (uniform over the workgroup).
__device__ __forceinline__ Unit decode_wg(const CocgLaunch& a) {
  CocgLaunch b = a;
  b.klist = nullptr;
  return decode_id(b, blockIdx.x);
}

template <typename F>
__global__ __launch_bounds__(256) void k_cocg_init_planes(CocgLaunch a,
                                                          const double* __restrict__ b) {
  const Unit u = decode_wg(a);
  if (!u.ok) return;
  if (a.item_skip && a.item_skip[u.item]) return;
  const TileGeom& G = a.G;
  __shared__ cd zl[256];
  __shared__ uint8_t act[256];
  const size_t base = (size_t)u.k * G.T * G.S + (size_t)u.t * G.S;
  const F* fac = (const F*)a.fac;
  const size_t fbase = ((size_t)u.k * G.T + u.t) * (size_t)G.sy * G.sx * G.sx;
  PlaneFactor<F> f;
  f.load(fac, fbase, G.sx, G.sy, threadIdx.x >> 2, threadIdx.x & 3);
  const int l = threadIdx.x;
  cd rv = cmk(0.0, 0.0);
  uint8_t ac = 0;
  if (l < G.S) {
    const size_t p = (size_t)u.t * G.S + l;
    ac = active(G.kind[p], G.depth[p], a.g) ? 1 : 0;
    if (ac) rv = ld(b, base + l);
  }
  act[l] = ac;
  zl[l] = rv;
  plane_tile_solve<F>(f, fac, fbase, zl, act, G.sx, G.sy, G.t);
  cd rz = cmk(0.0, 0.0), rr = cmk(0.0, 0.0);
  if (l < G.S) {
    const cd zv = ac ? zl[l] : cmk(0.0, 0.0);
    st(a.r, base + l, rv);
    st(a.z, base + l, zv);
    st(a.x, base + l, cmk(0.0, 0.0));
    st(a.p_old, base + l, cmk(0.0, 0.0));
    rz = cmul(rv, zv);
    rr.x = cabs2(rv);
  }
  block_sum2(rz, rr);
  if (threadIdx.x == 0) {
    const size_t q = ((size_t)u.k * G.T + u.t) * 2;
    st(a.partU, q, rz);
    st(a.partU, q + 1, rr);
  }
}

// The stencil launch of k_cocg_stencil, one thread per site and one halo
// slot per thread (6 s^2 <= 216 slots).
__device__ __forceinline__ void stencil_planes_unit(const CocgLaunch& a, int it, const Unit& u) {
  if (!u.ok) return;
  const ItemHead h = item_head(a, u);
  const TileGeom& G = a.G;
  const int s = G.edge;
  const int F = G.dim == 1 ? 1 : (G.dim == 2 ? s : s * s);
  const int H = 2 * G.dim * F;  // <= 216 halo slots (s = 6): one per thread
  const int l = threadIdx.x;
  // as in k_cocg_stencil: the thread's halo neighbour and its site's activity
  // are read with the item head; the own site's p_old, z, d and the halo slot
  // go out before the item reduction
  const size_t p = (size_t)u.t * G.S + (l < G.S ? l : G.S - 1);  // clamped: always valid
  const bool ac = active(G.kind[p], G.depth[p], a.g) && l < G.S;
  int hdir = 0;
  const int hsite = halo_site(G, l < H ? l : 0, hdir);
  const int hstride = (hdir >> 1) == 0 ? 1 : ((hdir >> 1) == 1 ? s : s * s);
  const int hn = l < H ? G.nbr[u.t * 6 + hdir] : -1;
  asm volatile("" : : "v"(hn), "v"((int)ac), "v"(h.lo), "v"(h.hi));  // above the state test
  if (!open_here(h.state, stencil_mark(it))) return;
  const size_t NP = (size_t)G.T * G.S;
  const size_t kb = (size_t)u.k * NP;
  const size_t base = kb + (size_t)u.t * G.S;
  const bool lead = u.t == h.lo;
  const cd po = ld(a.p_old, kb + p), zo = ld(a.z, kb + p), dv = ld(a.d, kb + p);
  const size_t hp = hn >= 0 ? (size_t)hn * G.S + ((hdir & 1) ? hsite - (s - 1) * hstride
                                                               : hsite + (s - 1) * hstride)
                            : (size_t)u.t * G.S + hsite;
  const bool hac = hn >= 0 && active(G.kind[hp], G.depth[hp], a.g);
  const cd hpo = ld(a.p_old, kb + hp), hz = ld(a.z, kb + hp);
  cd beta = cmk(0.0, 0.0);
  if (it > 0) {
    const double bn2 = a.st.bn2[u.item];
    const cd rho_prev = ld(a.rho2 + (size_t)((it - 1) & 1) * a.n_items * 2, u.item);
    cd rho, rr;
    item_sum(a.partU, 2, a, u, h, rho, rr);
    if (a.flush || rr.x <= a.tol2 * bn2) {
      if ((it & 1) && ac)  // pending alpha_{i-1} p_{i-1} of the deferred x update
        st(a.x, base + l, cfma(ld(a.alph, u.item), po, ld(a.x, base + l)));
      if (lead && threadIdx.x == 0) {
        a.st.done[u.item] = stencil_mark(it);
        a.st.iters[u.item] = it;
      }
      return;
    }
    beta = cdiv(rho, rho_prev);
    if (lead && threadIdx.x == 0) st(a.rho2 + (size_t)(it & 1) * a.n_items * 2, u.item, rho);
  }
  if (lead && threadIdx.x == 0) a.kalive[u.k] = it + 2;  // the item stays open
  if (a.wctr && lead && threadIdx.x == 0)
    atomicAdd(&a.wctr[(size_t)1 * a.n_items + u.item],
              (unsigned long long)(h.hi - h.lo) *
                  ((unsigned long long)(G.S * (5 * 16 + 2)) + 2ull * 2 * (G.sx + G.sy) * 16));
  __shared__ cd pl[256];
  __shared__ cd hl[256];
  const cd pn = ac ? cfma(beta, po, zo) : cmk(0.0, 0.0);
  if (l < G.S) st(a.p_new, base + l, pn);
  pl[l] = pn;
  hl[l] = hac ? cfma(beta, hpo, hz) : cmk(0.0, 0.0);
  __syncthreads();
  cd mu = cmk(0.0, 0.0);
  if (l < G.S) {
    if (!ac) {
      st(a.s, base + l, cmk(0.0, 0.0));
    } else {
      const int q1 = div_edge(G, l), q2 = div_edge(G, q1);
      const int x = l - s * q1, y = q1 - s * q2, z = q2;
      cd nb = cmk(0.0, 0.0);
      for (int dir = 0; dir < 2 * G.dim; ++dir) {
        const int ax = dir >> 1, up = dir & 1;
        const int c = ax == 0 ? x : (ax == 1 ? y : z);
        const int stride = ax == 0 ? 1 : (ax == 1 ? s : s * s);
        if (up ? (c < s - 1) : (c > 0)) nb = cadd(nb, pl[up ? l + stride : l - stride]);
        else nb = cadd(nb, hl[dir * F + halo_pos(G, ax, x, y, z)]);
      }
      const cd sv = cfma(dv, pn, cscale(nb, G.t));
      st(a.s, base + l, sv);
      mu = cmul(pn, sv);
    }
  }
  cd unused = cmk(0.0, 0.0);
  block_sum2(mu, unused);
  if (threadIdx.x == 0) st(a.partS, (size_t)u.k * G.T + u.t, mu);
}

// A workgroup per unit of the launch's list (the grid covers every unit).
__global__ __launch_bounds__(256) void k_cocg_stencil_planes(CocgLaunch a, int it) {
  stencil_planes_unit(a, it, decode_id(a, blockIdx.x));
}

template <typename F>
__device__ __forceinline__ void update_planes_unit(const CocgLaunch& a, int it, const Unit& u) {
  if (!u.ok) return;
  const ItemHead h = item_head(a, u);
  asm volatile("" : : "v"(h.lo), "v"(h.hi));  // the range is read above the state test
  if (!open_here(h.state, update_mark(it))) return;
  const TileGeom& G = a.G;
  const size_t base = (size_t)u.k * G.T * G.S + (size_t)u.t * G.S;
  // as in the wave kernel: everything that does not depend on alpha (the
  // site's r, s and activity, the item's rho, the factors) goes out before
  // the item reduction; the deferred x update follows the sweep
  const int l = threadIdx.x;
  const int lc = l < G.S ? l : G.S - 1;  // clamped: always a valid site
  const size_t p = (size_t)u.t * G.S + lc;
  const uint8_t ac = (active(G.kind[p], G.depth[p], a.g) && l < G.S) ? 1 : 0;
  const cd r0 = ld(a.r, base + lc), s0 = ld(a.s, base + lc);
  const cd rho = ld(a.rho2 + (size_t)(it & 1) * a.n_items * 2, u.item);
  const F* fac = (const F*)a.fac;
  const size_t fbase = ((size_t)u.k * G.T + u.t) * (size_t)G.sy * G.sx * G.sx;
  PlaneFactor<F> f;
  f.load(fac, fbase, G.sx, G.sy, threadIdx.x >> 2, threadIdx.x & 3);
  cd mu, unused;
  item_sum(a.partS, 1, a, u, h, mu, unused);
  const bool odd = it & 1;
  if (cabs2(mu) == 0.0) {
    if (odd && ac)
      st(a.x, base + l, cfma(ld(a.alph, u.item), ld(a.p_old, base + l), ld(a.x, base + l)));
    if (u.t == h.lo && threadIdx.x == 0) a.st.done[u.item] = update_mark(it);
    return;
  }
  const cd alpha = cdiv(rho, mu);
  if (u.t == h.lo && threadIdx.x == 0) {
    if (!odd) st(a.alph, u.item, alpha);
    if (a.wctr)
      atomicAdd(&a.wctr[u.item], (unsigned long long)(h.hi - h.lo) *
                                     ((unsigned long long)(G.S * ((odd ? 8 : 4) * 16 + 2)) +
                                      (unsigned long long)G.sy * G.sx * G.sx * (2 * sizeof(F))));
  }
  __shared__ cd zl[256];
  __shared__ uint8_t act[256];
  cd rv = cmk(0.0, 0.0), rr = cmk(0.0, 0.0);
  if (l < G.S) {
    if (ac) rv = csub(r0, cmul(alpha, s0));
    st(a.r, base + l, rv);
    rr.x = cabs2(rv);
  }
  act[l] = ac;
  zl[l] = rv;
  plane_tile_solve<F>(f, fac, fbase, zl, act, G.sx, G.sy, G.t);
  cd rz = cmk(0.0, 0.0);
  if (l < G.S) {
    const cd zv = ac ? zl[l] : cmk(0.0, 0.0);
    st(a.z, base + l, zv);
    rz = cmul(rv, zv);
  }
  block_sum2(rz, rr);
  if (threadIdx.x == 0) {
    const size_t q = ((size_t)u.k * G.T + u.t) * 2;
    st(a.partU, q, rz);
    st(a.partU, q + 1, rr);
  }
  if (odd && ac)  // x += alpha_{i-1} p_{i-1} + alpha_i p_i
    st(a.x, base + l,
       cfma(alpha, ld(a.p_new, base + l), cfma(ld(a.alph, u.item), ld(a.p_old, base + l), ld(a.x, base + l))));
}

template <typename F>
__global__ __launch_bounds__(256) void k_cocg_update_planes(CocgLaunch a, int it) {
  update_planes_unit<F>(a, it, decode_id(a, blockIdx.x));
}

// Convergence bookkeeping after launch `it` (it = 0 follows the
// initialisation) and the number of items still open, added into *open
// (zeroed by the launcher).  One wave per item, reducing the item's partials
// in the same order as item_sum in the other kernels, so its convergence
// test agrees with the stencil's bit for bit.
__global__ __launch_bounds__(256) void k_cocg_check(CocgLaunch a, int it, int* __restrict__ open) {
  __shared__ int cnt[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + wave;
  int mine = 0;
  if (item < a.n_items) {
    const int k = item / a.n_nodes, node = item % a.n_nodes;
    if (a.item_skip && a.item_skip[item]) {
      if (lane == 0) a.st.done[item] = 1;
    } else if (it == 0 || !a.st.done[item]) {
      cd s0, s1;
      item_sum_of(a.partU, 2, a, k, a.tlo[node], a.thi[node], lane, s0, s1);
      if (it == 0) {
        if (lane == 0) {
          a.st.bn2[item] = s1.x;
          st(a.rho2, item, s0);
          a.st.iters[item] = 0;
          a.st.done[item] = (s1.x > 0.0) ? 0 : 1;
          if (s1.x > 0.0) a.kalive[k] = 1;
        }
        mine = s1.x > 0.0;
      } else {
        // converged items are marked (and their deferred x update applied)
        // by the next stencil launch; here they only stop counting as open
        mine = !(s1.x <= a.tol2 * a.st.bn2[item]);
      }
    }
  }
  if (lane == 0) cnt[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int c = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    if (c) atomicAdd(open, c);
  }
}

// The frequencies whose stamp says they still have an open item, in
// increasing order, and their number: the unit list of the following
// stencil and update launches.  One workgroup; a block-wide prefix count.
__global__ __launch_bounds__(1024) void k_cocg_compact(CocgLaunch a, int stamp,
                                                       int* __restrict__ klist,
                                                       int* __restrict__ kcount) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int k0 = 0; k0 < a.K; k0 += 1024) {
    const int k = k0 + threadIdx.x;
    const bool live = k < a.K && a.kalive[k] == stamp;
    const unsigned long long m = __ballot(live);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int i = 0; i < w; ++i) off += wsum[i];
    if (live) klist[off + before] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int i = 0; i < 16; ++i) tot += wsum[i];
      base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *kcount = base;
}

// profiling: fold per-item byte counts [classes][n] into tot[class], zeroing them
__global__ __launch_bounds__(256) void k_prof_collect(unsigned long long* __restrict__ per_item,
                                                      int n, int classes, int first_class,
                                                      unsigned long long* __restrict__ tot) {
  __shared__ unsigned long long red[256];
  for (int c = 0; c < classes; ++c) {
    unsigned long long mine = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      mine += per_item[(size_t)c * n + i];
      per_item[(size_t)c * n + i] = 0;
    }
    red[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[first_class + c] += red[0];
    __syncthreads();
  }
}

}  // namespace

static inline unsigned cocg_blocks(const CocgLaunch& L) {
  return (unsigned)(((size_t)L.K * L.G.T + WAVES - 1) / WAVES);
}

static inline unsigned planes_blocks(const CocgLaunch& L) {
  return (unsigned)((size_t)L.K * L.G.T);
}


void launch_cocg_init(const CocgLaunch& L, const double* b, hipStream_t s) {
  if (L.G.sx > 16) {  // plane slices: a workgroup per unit
    if (L.fp16) k_cocg_init_planes<__half><<<planes_blocks(L), 256, 0, s>>>(L, b);
    else if (L.fp32) k_cocg_init_planes<float><<<planes_blocks(L), 256, 0, s>>>(L, b);
    else k_cocg_init_planes<double><<<planes_blocks(L), 256, 0, s>>>(L, b);
    return;
  }
  // slices of at most 16 sites: a wave per unit, low-precision factors in
  // registers; slices of exactly 16 sites take the fixed-width instance
  const unsigned nb = cocg_blocks(L);
  const bool w16 = L.G.sx == 16;
  if (L.fp16) {
    if (w16) k_cocg_init<__half, true, 16><<<nb, 64 * WAVES, 0, s>>>(L, b);
    else k_cocg_init<__half, true, 0><<<nb, 64 * WAVES, 0, s>>>(L, b);
  } else if (L.fp32) {
    if (w16) k_cocg_init<float, true, 16><<<nb, 64 * WAVES, 0, s>>>(L, b);
    else k_cocg_init<float, true, 0><<<nb, 64 * WAVES, 0, s>>>(L, b);
  } else {
    if (w16) k_cocg_init<double, false, 16><<<nb, 64 * WAVES, 0, s>>>(L, b);
    else k_cocg_init<double, false, 0><<<nb, 64 * WAVES, 0, s>>>(L, b);
  }
}
void launch_cocg_stencil(const CocgLaunch& L, int it, hipStream_t s) {
  if (L.G.sx > 16) k_cocg_stencil_planes<<<planes_blocks(L), 256, 0, s>>>(L, it);
  else k_cocg_stencil<<<cocg_blocks(L), 64 * WAVES, 0, s>>>(L, it);
}
void launch_cocg_compact(const CocgLaunch& L, int stamp, int* klist, int* kcount, hipStream_t s) {
  k_cocg_compact<<<1, 1024, 0, s>>>(L, stamp, klist, kcount);
}
void launch_prof_collect(unsigned long long* per_item, int n, int classes, int first_class,
                         unsigned long long* tot, hipStream_t s) {
  k_prof_collect<<<1, 256, 0, s>>>(per_item, n, classes, first_class, tot);
}
void launch_cocg_check(const CocgLaunch& L, int it, int* open, hipStream_t s) {
  launch_zero(open, sizeof(int), s);
  if (L.n_items > 0) k_cocg_check<<<(unsigned)((L.n_items + 3) / 4), 256, 0, s>>>(L, it, open);
}
void launch_cocg_update(const CocgLaunch& L, int it, hipStream_t s) {
  if (L.G.sx > 16) {
    const unsigned nb = planes_blocks(L);
    if (L.fp16) k_cocg_update_planes<__half><<<nb, 256, 0, s>>>(L, it);
    else if (L.fp32) k_cocg_update_planes<float><<<nb, 256, 0, s>>>(L, it);
    else k_cocg_update_planes<double><<<nb, 256, 0, s>>>(L, it);
    return;
  }
  const unsigned nb = cocg_blocks(L);
  const bool w16 = L.G.sx == 16;
  if (L.fp16) {
    if (w16) k_cocg_update<__half, true, 16><<<nb, 64 * WAVES, 0, s>>>(L, it);
    else k_cocg_update<__half, true, 0><<<nb, 64 * WAVES, 0, s>>>(L, it);
  } else if (L.fp32) {
    if (w16) k_cocg_update_occ3<float, true, 16><<<nb, 64 * WAVES, 0, s>>>(L, it);
    else k_cocg_update_occ3<float, true, 0><<<nb, 64 * WAVES, 0, s>>>(L, it);
  } else {
    if (w16) k_cocg_update<double, false, 16><<<nb, 64 * WAVES, 0, s>>>(L, it);
    else k_cocg_update<double, false, 0><<<nb, 64 * WAVES, 0, s>>>(L, it);
  }
}

}  // namespace dyson
