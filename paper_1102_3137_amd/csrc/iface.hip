// Lanczos on the Schur complement (the interface-space form of the
// correction, derived from eqs. (5)-(7)): for a correction domain with
// interface C and subdomains B, eq. (6) gives X = H^{-1} - blkdiag(B^{-1}, 0) =
// [W; -I] S^{-1} [W^T, -I] with W = B^{-1} E and S = C - E^T B^{-1} E.  Bilinear
// Lanczos on S, run for exactly m steps (m = interface size), yields a basis
// P of the whole interface space with P^T P = I and S P = P H (H the projected
// Hessenberg matrix: the tridiagonal recurrence plus the re-orthogonalization
// coefficients), so S^{-1} = P H^{-1} P^T and
//   diag(X) = diag(V H^{-1} V^T),  V = [W P; P] (subdomain sites; interface),
// whose columns are the step vectors v_j = p_j + u_j, u_j = B^{-1} E p_j.
// One subdomain solve per step (the X form needs two), then one dense
// inversion of H per (domain, frequency) and one product for the diagonal.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devcommon.h"
#include "kernels.h"

namespace dyson {
namespace {
using namespace dev;

#define IF_ITEM()                                   \
  const int t = blockIdx.x, k = blockIdx.y;         \
  const int node = a.tile_node[t];                  \
  if (node < 0) return;                             \
  const int item = k * a.n_nodes + node;            \
  if (a.stopped[item]) return;                      \
  const size_t NP = (size_t)a.G.T * a.G.S;          \
  const size_t kb = (size_t)k * NP;                 \
  const size_t base = kb + (size_t)t * a.G.S;

__device__ __forceinline__ bool on_iface(const TileGeom& G, size_t p, int level) {
  return G.kind[p] == 2 && G.depth[p] == level;
}

// Index of site l of tile t in a basis vector of frequency k: compact storage
// keeps the tiles that hold interface sites only (t must be one of them).
__device__ __forceinline__ size_t p_at(const LzArgs& a, int k, int t, int l) {
  return a.qcompact ? ((size_t)k * a.n_tlist + a.tpos[t]) * a.G.S + l
                    : ((size_t)k * a.G.T + t) * a.G.S + l;
}

// rhs = E p: on the subdomain sites (graph level + 1) the hopping from the
// level's interface sites (p vanishes elsewhere).
__global__ __launch_bounds__(256) void k_f1_rhs(LzArgs a, const double* __restrict__ p,
                                                double* __restrict__ rhs) {
  IF_ITEM();
  const TileGeom& G = a.G;
  const int tid = threadIdx.x;
  if (tid >= G.S) return;
  const size_t pp = (size_t)t * G.S + tid;
  cd out = cmk(0.0, 0.0);
  if (active(G.kind[pp], G.depth[pp], a.level + 1)) {
    cd acc = cmk(0.0, 0.0);
    for (int dir = 0; dir < 6; ++dir) {
      int nt, nl;
      if (!site_nbr(G, t, tid, dir, nt, nl)) continue;
      const size_t np = (size_t)nt * G.S + nl;
      if (on_iface(G, np, a.level)) acc = cadd(acc, ld(p, p_at(a, k, nt, nl)));
    }
    out = cscale(acc, G.t);
  }
  st(rhs, base + tid, out);
}

// s = S p = (H (p - u))|_C with u = B^{-1} E p (zero on C): on the interface
// sites d p + t (sum of the neighbours' p - u, p on interface neighbours and
// u on subdomain ones); zero elsewhere.  Also v = p + u.
__global__ __launch_bounds__(256) void k_f1_smat(LzArgs a, const double* __restrict__ d,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ u,
                                                 double* __restrict__ s, double* __restrict__ v) {
  IF_ITEM();
  const TileGeom& G = a.G;
  const int tid = threadIdx.x;
  if (tid >= G.S) return;
  const size_t pp = (size_t)t * G.S + tid;
  cd out = cmk(0.0, 0.0);
  // p is read on interface sites only: the vector kernels keep it on the
  // interface tiles, and other tiles of the buffer hold stale values
  const bool mine = on_iface(G, pp, a.level);
  const cd pv = mine ? ld(p, p_at(a, k, t, tid)) : cmk(0.0, 0.0);
  if (mine) {
    cd acc = cmk(0.0, 0.0);
    for (int dir = 0; dir < 6; ++dir) {
      int nt, nl;
      if (!site_nbr(G, t, tid, dir, nt, nl)) continue;
      const size_t np = (size_t)nt * G.S + nl;
      if (on_iface(G, np, a.level)) acc = cadd(acc, ld(p, p_at(a, k, nt, nl)));
      else if (active(G.kind[np], G.depth[np], a.level)) acc = csub(acc, ld(u, kb + np));
    }
    out = cfma(ld(d, base + tid), pv, cscale(acc, G.t));
  }
  st(s, base + tid, out);
  st(v, base + tid, cadd(pv, ld(u, base + tid)));
}

// Column j of H for every open item:
//   op 0: alpha_j on the diagonal, beta_j above it, plus the first
//         re-orthogonalization pass's coefficients h_i (i <= j);
//   op 1: the second pass's coefficients (items whose second pass ran);
//   op 2: beta_{j+1} below the diagonal (items still open after the step).
__global__ void k_f1_hcol(LzArgs a, double* __restrict__ Hm, int mm, int j, int op) {
  const int item = blockIdx.x;
  if (item >= a.n_items || a.stopped[item]) return;
  if (op == 1 && !a.reorth[item]) return;
  double* H = Hm + (size_t)item * mm * mm * 2;
  if (op == 2) {
    // zero below the diagonal where the basis met an invariant subspace
    if (threadIdx.x == 0 && j + 1 < mm)
      st(H, (size_t)(j + 1) * mm + j, a.armed[item] == 2 ? cmk(0.0, 0.0) : ld(a.beta, item));
    return;
  }
  const double* h = a.h + (size_t)item * a.hstride * 2;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    cd v = cadd(ld(H, (size_t)i * mm + j), ld(h, i));
    if (op == 0 && i == j) v = cadd(v, ld(a.alpha, item));
    if (op == 0 && i == j - 1) v = cadd(v, ld(a.beta, item));
    st(H, (size_t)i * mm + j, v);
  }
}

// mask[item] = 0 for the open items that continue from a fresh direction
// (armed == 2), 1 otherwise: the skip array of the continuation's kernels.
__global__ void k_f1_mask(LzArgs a, int* __restrict__ mask) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= a.n_items) return;
  mask[item] = (a.stopped[item] == 0 && a.armed[item] == 2) ? 0 : 1;
}

// After the continuation: a fresh direction with a vanishing bilinear norm
// (armed == 3) redoes the item; every flag is cleared.
__global__ void k_f1_settle(LzArgs a) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= a.n_items) return;
  if (a.armed[item] == 3 && a.stopped[item] == 0) a.stopped[item] = 3;
  a.armed[item] = 0;
}

// Before an attempt: clear H of the items that (re)start.
__global__ void k_f1_hzero(LzArgs a, double* __restrict__ Hm, int mm) {
  const int item = blockIdx.y;
  if (item >= a.n_items || a.stopped[item]) return;
  double* H = Hm + (size_t)item * mm * mm * 2;
  const size_t n = (size_t)mm * mm;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    st(H, e, cmk(0.0, 0.0));
}

// Identity beyond an item's own steps, so the padded block inverts to
// blkdiag(H^{-1}, I) in the batched inversion.
__global__ void k_f1_hpad(LzArgs a, double* __restrict__ Hm, int mm) {
  const int item = blockIdx.x;
  if (item >= a.n_items) return;
  double* H = Hm + (size_t)item * mm * mm * 2;
  for (int i = a.steps[item] + threadIdx.x; i < mm; i += blockDim.x)
    st(H, (size_t)i * mm + i, cmk(1.0, 0.0));
}

// D = diag(V M V^T), M = H^{-1} of the tile's item: one workgroup per (tile,
// 64-site chunk, frequency), Y = V M formed in 64-column blocks (operands
// staged in LDS, 4 x 4 outputs per thread) and folded into the diagonal
// against V before the next block.
constexpr int FA = 32;  // inner chunk
__global__ __launch_bounds__(256) void k_f1_diag(LzArgs a, const double* __restrict__ Vb,
                                                 size_t qstride, const double* __restrict__ Minv,
                                                 int mm, double* __restrict__ D) {
  const int t = blockIdx.x, c0 = blockIdx.y * 64, k = blockIdx.z;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const TileGeom& G = a.G;
  const int item = k * a.n_nodes + node;
  const int kk = a.steps[item];
  const size_t base = (size_t)k * G.T * G.S + (size_t)t * G.S;
  const double* M = Minv + (size_t)item * mm * mm * 2;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ cd As[64][FA];
  __shared__ cd Bs[FA][64];
  cd dsum[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) dsum[u] = cmk(0.0, 0.0);
  for (int b0 = 0; b0 < kk; b0 += 64) {
    cd acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[u][w] = cmk(0.0, 0.0);
    for (int a0 = 0; a0 < kk; a0 += FA) {
      __syncthreads();
      for (int e = threadIdx.x; e < 64 * FA; e += 256) {
        const int r = e % 64, c = e / 64, l = c0 + r, av = a0 + c;
        As[r][c] = (l < G.S && av < kk) ? ld(Vb + (size_t)av * qstride, base + l) : cmk(0.0, 0.0);
      }
      for (int e = threadIdx.x; e < FA * 64; e += 256) {
        const int c = e / 64, r = e % 64, av = a0 + c, bv = b0 + r;
        Bs[c][r] = (av < kk && bv < kk) ? ld(M, (size_t)av * mm + bv) : cmk(0.0, 0.0);
      }
      __syncthreads();
      for (int c = 0; c < FA; ++c) {
        cd x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = As[ty + 16 * u][c];
#pragma unroll
        for (int w = 0; w < 4; ++w) y[w] = Bs[c][tx + 16 * w];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w) acc[u][w] = cfma(x[u], y[w], acc[u][w]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int l = c0 + ty + 16 * u;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int bv = b0 + tx + 16 * w;
        if (l < G.S && bv < kk)
          dsum[u] = cfma(acc[u][w], ld(Vb + (size_t)bv * qstride, base + l), dsum[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const cd v = row16_sum(dsum[u]);
    const int l = c0 + ty + 16 * u;
    if (tx == 0 && l < G.S) st(D, base + l, v);
  }
}

}  // namespace

static inline dim3 f1_grid(const LzArgs& a, int K) { return dim3(a.G.T, K); }

void launch_f1_rhs(const LzArgs& a, int K, const double* p, double* rhs, hipStream_t s) {
  k_f1_rhs<<<f1_grid(a, K), 256, 0, s>>>(a, p, rhs);
}
void launch_f1_smat(const LzArgs& a, int K, const double* d, const double* p, const double* u,
                    double* sv, double* v, hipStream_t s) {
  k_f1_smat<<<f1_grid(a, K), 256, 0, s>>>(a, d, p, u, sv, v);
}
void launch_f1_hcol(const LzArgs& a, double* Hm, int mm, int j, int op, hipStream_t s) {
  if (a.n_items > 0) k_f1_hcol<<<(unsigned)a.n_items, 256, 0, s>>>(a, Hm, mm, j, op);
}
void launch_f1_mask(const LzArgs& a, int* mask, hipStream_t s) {
  if (a.n_items > 0) k_f1_mask<<<(unsigned)((a.n_items + 127) / 128), 128, 0, s>>>(a, mask);
}
void launch_f1_settle(const LzArgs& a, hipStream_t s) {
  if (a.n_items > 0) k_f1_settle<<<(unsigned)((a.n_items + 127) / 128), 128, 0, s>>>(a);
}
void launch_f1_hzero(const LzArgs& a, double* Hm, int mm, hipStream_t s) {
  const size_t n = (size_t)mm * mm;
  const unsigned bx = (unsigned)std::min<size_t>((n + 255) / 256, 64);
  if (a.n_items > 0) k_f1_hzero<<<dim3(bx, (unsigned)a.n_items), 256, 0, s>>>(a, Hm, mm);
}
void launch_f1_hpad(const LzArgs& a, double* Hm, int mm, hipStream_t s) {
  if (a.n_items > 0) k_f1_hpad<<<(unsigned)a.n_items, 256, 0, s>>>(a, Hm, mm);
}
void launch_f1_diag(const LzArgs& a, int K, const double* Vb, size_t qstride, const double* Minv,
                    int mm, double* D, hipStream_t s) {
  dim3 grid((unsigned)a.G.T, (unsigned)((a.G.S + 63) / 64), (unsigned)K);
  k_f1_diag<<<grid, 256, 0, s>>>(a, Vb, qstride, Minv, mm, D);
}

}  // namespace dyson
