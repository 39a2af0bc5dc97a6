// HIP kernels for gfx950 (CDNA4, wave64).  Every kernel works on the
// tile-major layout of the plan: one workgroup of 256 threads per
// (tile, frequency), one lattice site per thread.  Complex numbers are
// interleaved (re, im) pairs; all products are bilinear (no conjugation):
// H is complex symmetric (Sec. I), and so are its blocks and inverses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "devcommon.h"
#include "kernels.h"

namespace dyson {
namespace {
using namespace dev;

// ----------------------------------------------------------------- layout
__global__ void k_to_tile(TileGeom G, int K, const double* __restrict__ nat,
                          double* __restrict__ tile, cd fill) {
  const size_t NP = (size_t)G.T * G.S;
  size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (p >= NP) return;
  int i = G.site_of[p];
  cd v = (i >= 0) ? ld(nat, (size_t)k * G.N + i) : fill;
  st(tile, (size_t)k * NP + p, v);
}

__global__ void k_from_tile(TileGeom G, int K, const double* __restrict__ tile,
                            double* __restrict__ nat) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (i >= (size_t)G.N) return;
  st(nat, (size_t)k * G.N + i, ld(tile, (size_t)k * G.T * G.S + G.pos_of[i]));
}

// Frequency k's energy: z_k = i w_k (Matsubara, zmode 0: omega holds w_k)
// or any z_k with Im z_k > 0 (zmode 1: omega holds complex z_k).
__device__ __forceinline__ cd energy(const double* omega, int k, int zmode) {
  return zmode ? ld(omega, k) : cmk(0.0, omega[k]);
}

// eq. (1): d_i(k) = z_k + mu - V_i - Sigma_i(z_k), z_k = i w_k on the
// Matsubara axis; padding sites get 1.
__global__ void k_assemble(TileGeom G, int K, double mu, const double* __restrict__ V,
                           const double* __restrict__ omega, int zmode,
                           const double* __restrict__ sigma, double* __restrict__ d) {
  const size_t NP = (size_t)G.T * G.S;
  size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (p >= NP) return;
  int i = G.site_of[p];
  cd v = cmk(1.0, 0.0);
  if (i >= 0) {
    const cd sg = ld(sigma, (size_t)k * G.N + i), z = energy(omega, k, zmode);
    v = cmk(z.x + mu - V[i] - sg.x, z.y - sg.y);
  }
  st(d, (size_t)k * NP + p, v);
}

// Input checks of eq. (1); Im(i w_k - Sigma_i) > 0 keeps Im H positive
// definite, which the pivot-free factorizations rely on.
__global__ void k_validate(int N, const double* __restrict__ V, const double* __restrict__ omega,
                           int zmode, const double* __restrict__ sigma, double min_im,
                           int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= N) return;
  int f = 0;
  const cd z = energy(omega, k, zmode);
  if (!isfinite(z.x) || !isfinite(z.y) || !(z.y > 0.0)) f |= 2;
  if (k == 0 && !isfinite(V[i])) f |= 1;
  const cd sg = ld(sigma, (size_t)k * N + i);
  if (!isfinite(sg.x) || !isfinite(sg.y)) f |= 4;
  else if (!(z.y - sg.y > 0.0)) f |= 8;
  else if (z.y - sg.y < min_im) f |= 16;
  if (f) atomicOr(flag, f);
}

// ------------------------------------------------------ tile factorization
// Block LDL^T of the tile block restricted to the sites active in graph g,
// block rows = slices of n sites (a row of a square tile, a plane of a cubic
// one): S_0 = A_0, S_y = A_y - T_y S_{y-1}^{-1} T_y with T_y = t diag(c_y)
// the bonds between slices y-1 and y.  The dense inverses S_y^{-1} (n x n,
// complex symmetric, pivot-free because Im > 0) are stored per slice,
// symmetrized so that lower-precision copies stay exactly symmetric.
// NM = widest slice the instance handles (16: rows of square tiles and planes
// of 4^3 tiles; 36: planes of 5^3 and 6^3 tiles).  256 threads per block; each
// owns PER entries of the slice matrix, kept in registers across a pivot step.
template <int NM>
struct FactorSmem {
  static constexpr int PER = (NM * NM + 255) / 256;
  cd dl[256];
  uint8_t act[256];
  cd A[NM][NM + 1];
  cd Gp[NM][NM + 1];
  cd tmp[NM][NM + 1];
};

template <int NM>
__device__ __forceinline__ void factor_load(FactorSmem<NM>& sm, const TileGeom& G, int g, int t,
                                            int k, const double* __restrict__ d) {
  const size_t NP = (size_t)G.T * G.S;
  for (int l = threadIdx.x; l < G.S; l += 256) {
    const size_t p = (size_t)t * G.S + l;
    sm.dl[l] = ld(d, (size_t)k * NP + p);
    sm.act[l] = active(G.kind[p], G.depth[p], g) ? 1 : 0;
  }
  __syncthreads();
}

// Forms S_y (into A) and inverts it in place (Gauss-Jordan, no pivoting).
template <int NM>
__device__ __forceinline__ void factor_slice(FactorSmem<NM>& sm, const TileGeom& G, int y) {
  constexpr int PER = FactorSmem<NM>::PER;
  const int n = G.sx, nn = n * n;
  const double tt = G.t;
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int e = threadIdx.x + 256 * c;
    if (e >= nn) break;
    const int i = e / n, j = e % n;
    const int li = i + n * y, lj = j + n * y;
    const bool ai = sm.act[li], aj = sm.act[lj];
    cd v = cmk(0.0, 0.0);
    if (i == j) v = ai ? sm.dl[li] : cmk(1.0, 0.0);  // identity rows for inactive sites
    else if (ai && aj && slice_adj(G, i, j)) v = cmk(tt, 0.0);
    if (y > 0 && ai && aj && sm.act[li - n] && sm.act[lj - n])
      v = csub(v, cscale(sm.Gp[i][j], tt * tt));
    sm.A[i][j] = v;
  }
  __syncthreads();
  for (int q = 0; q < n; ++q) {
    const cd pinv = cdiv(cmk(1.0, 0.0), sm.A[q][q]);
    cd nv[PER];
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int e = threadIdx.x + 256 * c;
      nv[c] = cmk(0.0, 0.0);
      if (e < nn) {
        const int i = e / n, j = e % n;
        if (i == q && j == q) nv[c] = pinv;
        else if (i == q) nv[c] = cmul(sm.A[q][j], pinv);
        else if (j == q) nv[c] = cscale(cmul(sm.A[i][q], pinv), -1.0);
        else nv[c] = csub(sm.A[i][j], cmul(cmul(sm.A[i][q], sm.A[q][j]), pinv));
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int e = threadIdx.x + 256 * c;
      if (e < nn) sm.A[e / n][e % n] = nv[c];
    }
    __syncthreads();
  }
}

template <typename F, int NM>
__global__ __launch_bounds__(256) void k_factor(TileGeom G, int g, const int* __restrict__ tile_node,
                                                const double* __restrict__ d, F* __restrict__ fac) {
  const int t = blockIdx.x, k = blockIdx.y;
  if (tile_node && tile_node[t] < 0) return;
  __shared__ FactorSmem<NM> sm;
  factor_load(sm, G, g, t, k, d);
  const int n = G.sx, nn = n * n;
  const size_t fbase = ((size_t)k * G.T + t) * (size_t)G.sy * nn;
  for (int y = 0; y < G.sy; ++y) {
    factor_slice(sm, G, y);
    for (int e = threadIdx.x; e < nn; e += 256) {
      const int i = e / n, j = e % n;
      stf<F>(fac, fbase + (size_t)y * nn + e, cscale(cadd(sm.A[i][j], sm.A[j][i]), 0.5));
      sm.Gp[i][j] = sm.A[i][j];
    }
    __syncthreads();
  }
}

// Leaf graph (every separator inactive): factors in complex128 and the exact
// diagonal of each leaf block's inverse (eq. (13), first term) by the backward
// recursion G_yy = S_y^{-1} + S_y^{-1} T_{y+1} G_{y+1,y+1} T_{y+1} S_y^{-1}.
template <int NM>
__global__ __launch_bounds__(256) void k_factor_diag(TileGeom G, const double* __restrict__ d,
                                                     double* __restrict__ fac,
                                                     double* __restrict__ gdiag) {
  constexpr int PER = FactorSmem<NM>::PER;
  const int t = blockIdx.x, k = blockIdx.y;
  __shared__ FactorSmem<NM> sm;
  factor_load(sm, G, 255, t, k, d);
  const int n = G.sx, nn = n * n, ns = G.sy;
  const double tt = G.t;
  const size_t NP = (size_t)G.T * G.S;
  const size_t fbase = ((size_t)k * G.T + t) * (size_t)ns * nn;
  for (int y = 0; y < ns; ++y) {
    factor_slice(sm, G, y);
    for (int e = threadIdx.x; e < nn; e += 256) {
      const int i = e / n, j = e % n;
      st(fac, fbase + (size_t)y * nn + e, cscale(cadd(sm.A[i][j], sm.A[j][i]), 0.5));
      sm.Gp[i][j] = sm.A[i][j];
    }
    __syncthreads();
  }
  // Gp = G_{ns-1,ns-1}
  auto write_diag = [&](int y) {
    for (int i = threadIdx.x; i < n; i += 256) {
      const size_t p = (size_t)t * G.S + i + n * y;
      if (G.kind[p] == 1) st(gdiag, (size_t)k * NP + p, sm.Gp[i][i]);
    }
  };
  write_diag(ns - 1);
  for (int y = ns - 2; y >= 0; --y) {
    for (int e = threadIdx.x; e < nn; e += 256)
      sm.A[e / n][e % n] = ld(fac, fbase + (size_t)y * nn + e);  // S_y^{-1}
    __syncthreads();
    // tmp = C M C S_y^{-1}, C = diag(bonds between slices y and y+1)
    for (int e = threadIdx.x; e < nn; e += 256) {
      const int i = e / n, j = e % n;
      cd acc = cmk(0.0, 0.0);
      if (sm.act[i + n * (y + 1)] && sm.act[i + n * y])
        for (int l = 0; l < n; ++l)
          if (sm.act[l + n * (y + 1)] && sm.act[l + n * y]) acc = cfma(sm.Gp[i][l], sm.A[l][j], acc);
      sm.tmp[i][j] = acc;
    }
    __syncthreads();
    cd nv[PER];
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int e = threadIdx.x + 256 * c;
      nv[c] = cmk(0.0, 0.0);
      if (e < nn) {
        const int i = e / n, j = e % n;
        cd acc = cmk(0.0, 0.0);
        for (int l = 0; l < n; ++l) acc = cfma(sm.A[i][l], sm.tmp[l][j], acc);
        nv[c] = cadd(sm.A[i][j], cscale(acc, tt * tt));
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int e = threadIdx.x + 256 * c;
      if (e < nn) sm.Gp[e / n][e % n] = nv[c];
    }
    __syncthreads();
    write_diag(y);
    __syncthreads();
  }
}

__global__ void k_count_open(const int* __restrict__ done, int n, int* __restrict__ out) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) mine += (done[i] == 0);
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) *out = c;
}

// -------------------------------------------------------------- Lanczos
// Items are (domain, frequency) pairs of one level; stopped[item] != 0 makes
// every kernel skip the item (1 exhausted, 2 step cap, 3 breakdown, 4 done
// in an earlier attempt).

// A tile of the Lanczos vectors: through the level's tile list when it is set.
__device__ __forceinline__ int lz_tile(const LzArgs& a, int i) { return a.tlist ? a.tlist[i] : i; }

#define LZ_ITEM()                                   \
  const int ti = blockIdx.x, k = blockIdx.y;        \
  const int t = lz_tile(a, ti);                     \
  const int node = a.tile_node[t];                  \
  if (node < 0) return;                             \
  const int item = k * a.n_nodes + node;            \
  if (a.stopped[item]) return;                      \
  const size_t NP = (size_t)a.G.T * a.G.S;          \
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S; \
  const size_t qb = a.qcompact ? ((size_t)k * a.n_tlist + ti) * a.G.S : base; \
  (void)qb;

// Start vector: seeded random complex entries (real ones if real_only) on
// the level's separator sites (the interface C of eq. (4)) of every
// correction domain, zero elsewhere; partial q^T q.
__global__ __launch_bounds__(256) void k_lz_random(LzArgs a, double* __restrict__ q, uint64_t salt,
                                                   int real_only) {
  LZ_ITEM();
  const TileGeom& G = a.G;
  const int tid = threadIdx.x;
  cd qq = cmk(0.0, 0.0), un = cmk(0.0, 0.0);
  if (tid < G.S) {
    const size_t p = (size_t)t * G.S + tid;
    cd v = cmk(0.0, 0.0);
    if (G.kind[p] == 2 && G.depth[p] == a.level) {
      // keyed by the frequency itself (not its batch slot), the level, the
      // site and the attempt, so a result does not depend on the batch
      const uint64_t key = splitmix64(a.seed ^ (salt * 0xD1B54A32D192ED03ULL) ^ a.fkey[k]) ^
                           (((uint64_t)a.level << 40) + (uint64_t)G.site_of[p]);
      const uint64_t h1 = splitmix64(key), h2 = splitmix64(h1 ^ 0xA5A5A5A5A5A5A5A5ULL);
      v = cmk(2.0 * u01(h1) - 1.0, real_only ? 0.0 : 2.0 * u01(h2) - 1.0);
    }
    st(q, qb + tid, v);
    qq = cmul(v, v);
  }
  block_sum2(qq, un);
  if (tid == 0) st(a.partial, (size_t)k * G.T + t, qq);
}

// Identity of frequency k for the start vectors: the bits of Im z_k, mixed
// with those of Re z_k when it is not zero, so z_k = i w_k keys exactly as
// the Matsubara frequency w_k.
__global__ void k_freq_keys(const double* __restrict__ omega, int zmode, int K,
                            uint64_t* __restrict__ fkey) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  if (!omega) {
    fkey[k] = (uint64_t)k;
    return;
  }
  const cd z = energy(omega, k, zmode);
  uint64_t key = (uint64_t)__double_as_longlong(z.y);
  if (z.x != 0.0) key ^= splitmix64((uint64_t)__double_as_longlong(z.x));
  fkey[k] = key;
}

// q *= scal[item] (the inverse principal root of q^T q)
__global__ void k_lz_scale(LzArgs a, double* __restrict__ q) {
  LZ_ITEM();
  const cd inv = ld(a.scal, item);
  if (threadIdx.x < a.G.S) st(q, qb + threadIdx.x, cmul(ld(q, qb + threadIdx.x), inv));
}

// Defect of the block solve (eqs. (10)-(12) with the solve of (10) started
// from w = blkdiag(B^{-1},0) q): b = q - H w, which vanishes on the subdomain
// sites and equals q_C - E^T w on the level's interface sites.
__global__ __launch_bounds__(256) void k_lz_defect(LzArgs a, const double* __restrict__ q,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ b) {
  LZ_ITEM();
  const TileGeom& G = a.G;
  const size_t kb = (size_t)k * NP;
  const int tid = threadIdx.x;
  if (tid >= G.S) return;
  const size_t p = (size_t)t * G.S + tid;
  cd out = cmk(0.0, 0.0);
  if (G.kind[p] == 2 && G.depth[p] == a.level) {
    const int gB = a.level + 1;
    cd acc = cmk(0.0, 0.0);
    for (int dir = 0; dir < 6; ++dir) {
      int nt, nl;
      if (!site_nbr(G, t, tid, dir, nt, nl)) continue;
      const size_t np = (size_t)nt * G.S + nl;
      if (active(G.kind[np], G.depth[np], gB)) acc = cadd(acc, ld(w, kb + np));
    }
    out = csub(ld(q, kb + p), cscale(acc, G.t));
  }
  st(b, kb + p, out);
}

// alpha partials: q^T u and |u|^2
__global__ __launch_bounds__(256) void k_lz_alpha(LzArgs a, const double* __restrict__ q,
                                                  const double* __restrict__ u) {
  LZ_ITEM();
  const int tid = threadIdx.x;
  cd qu = cmk(0.0, 0.0), uu = cmk(0.0, 0.0);
  if (tid < a.G.S) {
    const cd uv = ld(u, base + tid);
    qu = cmul(ld(q, qb + tid), uv);
    uu = cmk(cabs2(uv), 0.0);
  }
  block_sum2(qu, uu);
  if (tid == 0) {
    st(a.partial, ((size_t)k * a.G.T + t) * 2, qu);
    st(a.partial, ((size_t)k * a.G.T + t) * 2 + 1, uu);
  }
}

// Three-term recurrence and the streaming diagonal (after eq. (13)):
// D += alpha_j q_j*q_j + 2 beta_j q_{j-1}*q_j ; r = u - alpha_j q_j - beta_j q_{j-1}
__global__ __launch_bounds__(256) void k_lz_recur(LzArgs a, const double* __restrict__ q,
                                                  const double* __restrict__ qprev,
                                                  const double* __restrict__ u,
                                                  double* __restrict__ r, double* __restrict__ D) {
  LZ_ITEM();
  const int tid = threadIdx.x;
  if (tid >= a.G.S) return;
  const cd al = ld(a.alpha, item), be = ld(a.beta, item);
  const cd qv = ld(q, qb + tid);
  const cd qp = qprev ? ld(qprev, qb + tid) : cmk(0.0, 0.0);
  if (D) {  // the X form's streamed diagonal (the interface form takes it at the end)
    cd gv = ld(D, base + tid);
    gv = cadd(gv, cmul(al, cmul(qv, qv)));
    gv = cadd(gv, cscale(cmul(be, cmul(qp, qv)), 2.0));
    st(D, base + tid, gv);
  }
  cd rv = csub(ld(u, base + tid), cmul(al, qv));
  rv = csub(rv, cmul(be, qp));
  st(r, qb + tid, rv);
}

// Classical Gram-Schmidt, bilinear: h_i = Q_i^T r for i < nvec.  Each wave
// takes every fourth basis vector of the tile; lanes cover 4 sites each.
// Pass 0 also records the partial |r|^2 (slot nvec); pass 1 runs only for
// the items the selective test flagged.
__global__ __launch_bounds__(256) void k_cgs_dot(LzArgs a, const double* __restrict__ Q,
                                                 size_t qstride, int nvec,
                                                 const double* __restrict__ r, int pass) {
  LZ_ITEM();
  if (pass == 1 && !a.reorth[item]) return;
  const TileGeom& G = a.G;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (a.wctr && threadIdx.x == 0 && ti == a.tlo[node])  // non-returning: nothing waits on it
    atomicAdd(&a.wctr[(size_t)1 * a.n_items + item],
              (unsigned long long)(a.thi[node] - a.tlo[node]) *
                  ((unsigned long long)(nvec + 1) * G.S * 16 + 16ull * nvec));
  cd rl[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int l = lane + 64 * c;
    rl[c] = (l < G.S) ? ld(r, qb + l) : cmk(0.0, 0.0);
  }
  double* out = a.hpart + ((size_t)k * G.T + t) * (size_t)a.hstride * 2;
  if (pass == 0 && wv == 0) {
    double rr = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) rr += cabs2(rl[c]);
    const cd s2 = wave_sum(cmk(rr, 0.0));
    if (lane == 0) st(out, nvec, s2);
  }
  for (int i = wv; i < nvec; i += 4) {
    const double* qi = Q + (size_t)i * qstride;
    cd acc = cmk(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int l = lane + 64 * c;
      if (l < G.S) acc = cfma(ld(qi, qb + l), rl[c], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) st(out, i, acc);
  }
}

// Sums over a domain's tiles [lo, hi) in increasing tile order, the loads of
// TB consecutive tiles issued together (addresses clamped into the range, so
// every load is valid) and added in order afterwards: one memory round trip
// per TB tiles instead of one per tile, with the same result bit for bit.
constexpr int TB = 8;

// h[item][i] = sum over the domain's tiles of the partials (fixed order);
// pass 0 also sums |r|^2 into h[item][nvec].  One block per item.
__global__ void k_cgs_reduce(LzArgs a, int K, const int* __restrict__ tlo,
                             const int* __restrict__ thi, int nvec, int pass) {
  const int item = blockIdx.x;
  const int k = item / a.n_nodes, node = item % a.n_nodes;
  if (a.stopped[item]) return;
  if (pass == 1 && !a.reorth[item]) return;
  const int n = (pass == 0) ? nvec + 1 : nvec;
  const int lo = tlo[node], hi = thi[node];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    cd s = cmk(0.0, 0.0);
    for (int t0 = lo; t0 < hi; t0 += TB) {
      cd v[TB];
#pragma unroll
      for (int q = 0; q < TB; ++q) {
        const int t = lz_tile(a, t0 + q < hi ? t0 + q : hi - 1);
        v[q] = ld(a.hpart + ((size_t)k * a.G.T + t) * (size_t)a.hstride * 2, i);
      }
#pragma unroll
      for (int q = 0; q < TB; ++q)
        if (t0 + q < hi) s = cadd(s, v[q]);
    }
    st(a.h, (size_t)item * a.hstride + i, s);
  }
}

// r -= sum_i h_i Q_i, and D += (sum_i h_i Q_i) * q_j: with full
// re-orthogonalization the matrix of X in the computed basis is the
// Hessenberg H = T + (re-orthogonalization coefficients); its column j
// above the tridiagonal band is added here so that diag(Q H Q^T) is formed.
// Pass 0 records the partial |r'|^2 of the updated r for the selective test.
__global__ __launch_bounds__(256) void k_cgs_update(LzArgs a, const double* __restrict__ Q,
                                                    size_t qstride, int nvec,
                                                    double* __restrict__ r, double* __restrict__ D,
                                                    int pass) {
  LZ_ITEM();
  if (pass == 1 && !a.reorth[item]) return;
  const TileGeom& G = a.G;
  if (a.wctr && threadIdx.x == 0 && ti == a.tlo[node])  // non-returning: nothing waits on it
    atomicAdd(&a.wctr[item], (unsigned long long)(a.thi[node] - a.tlo[node]) *
                                 ((unsigned long long)(nvec + 4) * G.S * 16 + 16ull * nvec));
  __shared__ cd hl[1024];
  const double* hs = a.h + (size_t)item * a.hstride * 2;
  for (int i = threadIdx.x; i < nvec && i < 1024; i += blockDim.x) hl[i] = ld(hs, i);
  __syncthreads();
  const int tid = threadIdx.x;
  double rr = 0.0;
  if (tid < G.S) {
    cd acc = cmk(0.0, 0.0);
    for (int i = 0; i < nvec; ++i) {
      const cd hv = (i < 1024) ? hl[i] : ld(hs, i);
      acc = cfma(hv, ld(Q + (size_t)i * qstride, qb + tid), acc);
    }
    const cd rn = csub(ld(r, qb + tid), acc);
    st(r, qb + tid, rn);
    rr = cabs2(rn);
    if (D) {
      const cd qj = ld(Q + (size_t)(nvec - 1) * qstride, qb + tid);
      st(D, base + tid, cfma(acc, qj, ld(D, base + tid)));
    }
  }
  if (pass == 0) {
    cd s0 = cmk(rr, 0.0), s1 = cmk(0.0, 0.0);
    block_sum2(s0, s1);
    if (tid == 0) st(a.partial, ((size_t)k * G.T + t) * 2, s0);
  }
}

// Selective second pass (Daniel, Gragg, Kaufman and Stewart, 1976): repeat
// the projection only when the first one removed most of r.
__global__ void k_cgs_decide(LzArgs a, int K, const int* __restrict__ tlo,
                             const int* __restrict__ thi, int nvec, double eta2) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= K * a.n_nodes) return;
  if (a.stopped[item]) return;
  const int k = item / a.n_nodes, node = item % a.n_nodes;
  double r1 = 0.0;
  const int lo = tlo[node], hi = thi[node];
  for (int t0 = lo; t0 < hi; t0 += TB) {
    double v[TB];
#pragma unroll
    for (int q = 0; q < TB; ++q)
      v[q] = a.partial[((size_t)k * a.G.T + lz_tile(a, t0 + q < hi ? t0 + q : hi - 1)) * 4];
#pragma unroll
    for (int q = 0; q < TB; ++q)
      if (t0 + q < hi) r1 += v[q];
  }
  const double r0 = a.h[((size_t)item * a.hstride + nvec) * 2];
  a.reorth[item] = (r1 < eta2 * r0) ? 1 : 0;
}

// partials |r|^2 and r^T r
__global__ __launch_bounds__(256) void k_lz_norms(LzArgs a, const double* __restrict__ r) {
  LZ_ITEM();
  const int tid = threadIdx.x;
  cd rr = cmk(0.0, 0.0), rtr = cmk(0.0, 0.0);
  if (tid < a.G.S) {
    const cd v = ld(r, qb + tid);
    rr = cmk(cabs2(v), 0.0);
    rtr = cmul(v, v);
  }
  block_sum2(rr, rtr);
  if (tid == 0) {
    st(a.partial, ((size_t)k * a.G.T + t) * 2, rr);
    st(a.partial, ((size_t)k * a.G.T + t) * 2 + 1, rtr);
  }
}

// q_{j+1} = r / beta_{j+1}
__global__ void k_lz_next(LzArgs a, const double* __restrict__ r, double* __restrict__ qn) {
  LZ_ITEM();
  if (threadIdx.x >= a.G.S) return;
  const cd inv = cdiv(cmk(1.0, 0.0), ld(a.beta, item));
  st(qn, qb + threadIdx.x, cmul(ld(r, qb + threadIdx.x), inv));
}

// Per-item scalar steps of the Lanczos recurrence.
//   op 0: start   scal = 1/sqrt(q^T q)
//   op 1: alpha   alpha = q^T u, unorm2 = |u|^2; an armed item whose new
//                 |u| = |X q_j| is at the noise level stops here (exhausted)
//   op 2: norms   stop test, beta_{j+1} = principal sqrt(r^T r)
//   op 3: (interface form) beta of a fresh direction after an invariant
//         subspace
//
// Stopping (Sec. II.C: the coefficients vanish once the Krylov space of X is
// exhausted).  A residual that passes the L2 test |r| <= tol |u| may also be
// a transient dip; the item is then armed and runs one more step: at
// exhaustion q_{j+1} is bilinear-orthogonal to a basis that spans the range
// of X, so |X q_{j+1}| is at the noise level of the inner solves, while a
// dip leaves a direction with |X q_{j+1}| comparable to |X|.  The step count
// and the diagonal keep only the steps before the confirming one.
__global__ void k_lz_scalars(LzArgs a, int K, const int* __restrict__ tlo,
                             const int* __restrict__ thi, const int* __restrict__ mcap, int op,
                             int j, double tol, double brk, int force) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= K * a.n_nodes) return;
  const int k = item / a.n_nodes, node = item % a.n_nodes;
  if (a.stopped[item]) return;
  const int per = (op == 0) ? 1 : 2;
  cd s0 = cmk(0.0, 0.0), s1 = cmk(0.0, 0.0);
  const int lo = tlo[node], hi = thi[node];
  for (int t0 = lo; t0 < hi; t0 += TB) {
    cd v0[TB], v1[TB];
#pragma unroll
    for (int q = 0; q < TB; ++q) {
      const size_t qq = ((size_t)k * a.G.T + lz_tile(a, t0 + q < hi ? t0 + q : hi - 1)) * per;
      v0[q] = ld(a.partial, qq);
      v1[q] = per == 2 ? ld(a.partial, qq + 1) : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < TB; ++q)
      if (t0 + q < hi) {
        s0 = cadd(s0, v0[q]);
        if (per == 2) s1 = cadd(s1, v1[q]);
      }
  }
  if (op == 0) {
    if (cabs2(s0) == 0.0) {  // degenerate draw
      a.stopped[item] = 3;
      return;
    }
    st(a.scal, item, cdiv(cmk(1.0, 0.0), csqrt_p(s0)));
    st(a.beta, item, cmk(0.0, 0.0));
    a.steps[item] = 0;
    a.umax2[item] = 0.0;
    a.armed[item] = 0;
    return;
  }
  if (op == 1) {
    if (!a.iface && a.armed[item]) {
      // the confirming step: |u|^2 <= tol |X|^2 (|u| <= sqrt(tol) max|u|)
      if (s1.x <= tol * a.umax2[item]) {
        a.stopped[item] = 1;  // exhausted; this step contributes nothing
        return;
      }
      a.armed[item] = 0;  // a transient dip: carry on
    }
    st(a.alpha, item, s0);
    a.unorm2[item] = s1.x;
    a.umax2[item] = fmax(a.umax2[item], s1.x);
    return;
  }
  if (op == 3) {
    // interface form, fresh direction after an invariant subspace (armed ==
    // 2): its normalization, or armed = 3 when its bilinear norm vanishes
    if (s0.x == 0.0 || sqrt(cabs2(s1)) <= brk * s0.x) {
      a.armed[item] = 3;
      return;
    }
    st(a.beta, item, csqrt_p(s1));
    return;
  }
  const int steps = j + 1;
  a.steps[item] = steps;
  if (force) {
    a.stopped[item] = 3;  // test hook: breakdown declared at this step
    return;
  }
  if (a.iface) {
    // Lanczos on the Schur complement S (m x m, non-singular): after m steps
    // the basis spans the whole interface space and S^{-1} = P H^{-1} P^T
    // exactly; a residual that vanishes earlier means the start vector lay
    // in an invariant subspace, so the item is redone from a fresh vector
    const double rn = sqrt(s0.x), un = sqrt(a.unorm2[item]);
    if (steps >= mcap[node]) {
      a.stopped[item] = 1;
      return;
    }
    if (un == 0.0) {
      a.stopped[item] = 3;
      return;
    }
    if (rn <= tol * un) {
      // the basis spans an invariant subspace of S (a repeated eigenvalue
      // limits the Krylov space): the subdiagonal entry is zero and the
      // basis continues from a fresh direction orthogonal to it
      a.armed[item] = 2;
      st(a.beta, item, cmk(1.0, 0.0));
      return;
    }
    if (sqrt(cabs2(s1)) <= brk * s0.x) {
      a.stopped[item] = 3;
      return;
    }
    st(a.beta, item, csqrt_p(s1));
    return;
  }
  // the residual far below the largest |u| seen (an estimate of |X|), or a
  // zero X-matvec: exhausted without doubt; the L2 test arms the item
  const double rn = sqrt(s0.x), un = sqrt(a.unorm2[item]);
  if (rn <= 1e-3 * tol * sqrt(a.umax2[item]) || un == 0.0) {
    a.stopped[item] = 1;  // the Krylov space of X is exhausted: T_j is complete
    return;
  }
  const bool l2 = rn <= tol * un;
  const bool broken = sqrt(cabs2(s1)) <= brk * s0.x;
  if (l2 && (steps >= mcap[node] || broken)) {
    a.stopped[item] = 1;  // no room (or no usable vector) to confirm: the L2 test decides
    return;
  }
  if (steps >= mcap[node]) {
    a.stopped[item] = 2;  // step cap (rank cap or m + extra)
    return;
  }
  if (broken) {
    a.stopped[item] = 3;  // serious breakdown of the bilinear form: redo the item
    return;
  }
  if (l2) a.armed[item] = 1;
  st(a.beta, item, csqrt_p(s1));
}

// Between attempts: clear D on the tiles of items that broke down (stopped
// == 3) ...
__global__ void k_lz_clear_bad(LzArgs a, double* __restrict__ D) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item] != 3) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  if (threadIdx.x < a.G.S) st(D, base + threadIdx.x, cmk(0.0, 0.0));
}
// ... then reopen those items and park the finished ones
__global__ void k_lz_reopen(LzArgs a, int n_items) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= n_items) return;
  a.stopped[item] = (a.stopped[item] == 3) ? 0 : 4;
}

// Zero fill of n 4-byte words (vector stores; takes the place of a
// runtime memset, so a stream of this library's work holds kernels only).
__global__ void k_zero(uint32_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// b = e_pos in every frequency row (tile layout)
__global__ void k_unit_vector(TileGeom G, int pos, double* __restrict__ b) {
  const size_t NP = (size_t)G.T * G.S;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (p >= NP) return;
  st(b, (size_t)k * NP + p, cmk(p == (size_t)pos ? 1.0 : 0.0, 0.0));
}

// err = max(err, max_k |x_k - g_k| / |x_k|) at tile position pos; one thread
__global__ void k_sample_err(TileGeom G, int K, int pos, const double* __restrict__ x,
                             const double* __restrict__ g, double* __restrict__ err) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const size_t NP = (size_t)G.T * G.S;
  double e = err[0];
  for (int k = 0; k < K; ++k) {
    const cd xv = ld(x, (size_t)k * NP + pos), gv = ld(g, (size_t)k * NP + pos);
    const double r = sqrt(cabs2(csub(xv, gv)) / cabs2(xv));
    e = (r > e || r != r) ? r : e;
  }
  err[0] = e;
}

// G += D over the level's domains
__global__ void k_add_into(LzArgs a, const double* __restrict__ D, double* __restrict__ G) {
  const int t = blockIdx.x, k = blockIdx.y;
  if (a.tile_node[t] < 0) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  if (threadIdx.x < a.G.S) st(G, base + threadIdx.x, cadd(ld(G, base + threadIdx.x), ld(D, base + threadIdx.x)));
}

}  // namespace

// ----------------------------------------------------------------- launchers
static inline dim3 tiles_grid(const TileGeom& G, int K) { return dim3(G.T, K); }
static inline dim3 lz_grid(const LzArgs& a, int K) {
  return dim3(a.tlist ? (unsigned)a.n_tlist : (unsigned)a.G.T, K);
}

void launch_to_tile(const TileGeom& G, int K, const double* nat, double* tile, double fre,
                    hipStream_t s) {
  size_t NP = (size_t)G.T * G.S;
  dim3 grid((unsigned)((NP + 255) / 256), K);
  k_to_tile<<<grid, 256, 0, s>>>(G, K, nat, tile, cd{fre, 0.0});
}
void launch_from_tile(const TileGeom& G, int K, const double* tile, double* nat, hipStream_t s) {
  dim3 grid((unsigned)((G.N + 255) / 256), K);
  k_from_tile<<<grid, 256, 0, s>>>(G, K, tile, nat);
}
void launch_assemble(const TileGeom& G, int K, double mu, const double* V, const double* omega,
                     int zmode, const double* sigma, double* d, hipStream_t s) {
  size_t NP = (size_t)G.T * G.S;
  dim3 grid((unsigned)((NP + 255) / 256), K);
  k_assemble<<<grid, 256, 0, s>>>(G, K, mu, V, omega, zmode, sigma, d);
}
void launch_validate(int N, int K, const double* V, const double* omega, int zmode,
                     const double* sigma, double min_im, int* flag, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), K);
  k_validate<<<grid, 256, 0, s>>>(N, V, omega, zmode, sigma, min_im, flag);
}
void launch_factor(const TileGeom& G, int K, int g, const int* tile_node, const double* d,
                   void* fac, bool fp32, bool fp16, hipStream_t s) {
  dim3 grid = tiles_grid(G, K);
  if (G.sx <= 16) {
    if (fp16) k_factor<__half, 16><<<grid, 256, 0, s>>>(G, g, tile_node, d, (__half*)fac);
    else if (fp32) k_factor<float, 16><<<grid, 256, 0, s>>>(G, g, tile_node, d, (float*)fac);
    else k_factor<double, 16><<<grid, 256, 0, s>>>(G, g, tile_node, d, (double*)fac);
  } else {
    if (fp16) k_factor<__half, 36><<<grid, 256, 0, s>>>(G, g, tile_node, d, (__half*)fac);
    else if (fp32) k_factor<float, 36><<<grid, 256, 0, s>>>(G, g, tile_node, d, (float*)fac);
    else k_factor<double, 36><<<grid, 256, 0, s>>>(G, g, tile_node, d, (double*)fac);
  }
}
void launch_factor_diag(const TileGeom& G, int K, const double* d, double* fac64, double* gdiag,
                        hipStream_t s) {
  if (G.sx <= 16) k_factor_diag<16><<<tiles_grid(G, K), 256, 0, s>>>(G, d, fac64, gdiag);
  else k_factor_diag<36><<<tiles_grid(G, K), 256, 0, s>>>(G, d, fac64, gdiag);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;  // every buffer cleared here is a multiple of 4 bytes
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  k_zero<<<(unsigned)blocks, 256, 0, s>>>(reinterpret_cast<uint32_t*>(p), n);
}
void launch_count_open(const int* done, int n, int* out, hipStream_t s) {
  k_count_open<<<1, 256, 0, s>>>(done, n, out);
}
void launch_freq_keys(const double* omega, int zmode, int K, uint64_t* fkey, hipStream_t s) {
  k_freq_keys<<<(K + 63) / 64, 64, 0, s>>>(omega, zmode, K, fkey);
}
void launch_lz_random(const LzArgs& a, int K, double* q, uint64_t salt, hipStream_t s,
                      int real_only) {
  k_lz_random<<<lz_grid(a, K), 256, 0, s>>>(a, q, salt, real_only);
}
void launch_lz_scale(const LzArgs& a, int K, double* q, hipStream_t s) {
  k_lz_scale<<<lz_grid(a, K), 256, 0, s>>>(a, q);
}
void launch_lz_defect(const LzArgs& a, int K, const double* q, const double* w, double* b,
                      hipStream_t s) {
  k_lz_defect<<<lz_grid(a, K), 256, 0, s>>>(a, q, w, b);
}
void launch_lz_alpha(const LzArgs& a, int K, const double* q, const double* u, hipStream_t s) {
  k_lz_alpha<<<lz_grid(a, K), 256, 0, s>>>(a, q, u);
}
void launch_lz_recur(const LzArgs& a, int K, const double* q, const double* qprev, const double* u,
                     double* r, double* D, hipStream_t s) {
  k_lz_recur<<<lz_grid(a, K), 256, 0, s>>>(a, q, qprev, u, r, D);
}
void launch_cgs_dot(const LzArgs& a, int K, const double* Q, size_t qstride, int nvec,
                    const double* r, int pass, hipStream_t s) {
  k_cgs_dot<<<lz_grid(a, K), 256, 0, s>>>(a, Q, qstride, nvec, r, pass);
}
void launch_cgs_reduce(const LzArgs& a, int K, const int* tlo, const int* thi, int nvec, int pass,
                       hipStream_t s) {
  k_cgs_reduce<<<(unsigned)(K * a.n_nodes), 256, 0, s>>>(a, K, tlo, thi, nvec, pass);
}
void launch_cgs_update(const LzArgs& a, int K, const double* Q, size_t qstride, int nvec, double* r,
                       double* D, int pass, hipStream_t s) {
  k_cgs_update<<<lz_grid(a, K), 256, 0, s>>>(a, Q, qstride, nvec, r, D, pass);
}
void launch_cgs_decide(const LzArgs& a, int K, const int* tlo, const int* thi, int nvec,
                       double eta2, hipStream_t s) {
  const int n = K * a.n_nodes;
  k_cgs_decide<<<(n + 127) / 128, 128, 0, s>>>(a, K, tlo, thi, nvec, eta2);
}
void launch_lz_norms(const LzArgs& a, int K, const double* r, hipStream_t s) {
  k_lz_norms<<<lz_grid(a, K), 256, 0, s>>>(a, r);
}
void launch_lz_next(const LzArgs& a, int K, const double* r, double* qn, hipStream_t s) {
  k_lz_next<<<lz_grid(a, K), 256, 0, s>>>(a, r, qn);
}
void launch_lz_scalars(const LzArgs& a, int K, const int* tlo, const int* thi, const int* mcap,
                       int op, int j, double tol, double brk, int force, hipStream_t s) {
  int n = K * a.n_nodes;
  k_lz_scalars<<<(n + 127) / 128, 128, 0, s>>>(a, K, tlo, thi, mcap, op, j, tol, brk, force);
}
void launch_lz_reopen(const LzArgs& a, int K, double* D, hipStream_t s) {
  k_lz_clear_bad<<<tiles_grid(a.G, K), 256, 0, s>>>(a, D);
  const int n = K * a.n_nodes;
  k_lz_reopen<<<(n + 127) / 128, 128, 0, s>>>(a, n);
}
void launch_unit_vector(const TileGeom& G, int K, int pos, double* b, hipStream_t s) {
  const size_t NP = (size_t)G.T * G.S;
  k_unit_vector<<<dim3((unsigned)((NP + 255) / 256), K), 256, 0, s>>>(G, pos, b);
}
void launch_sample_err(const TileGeom& G, int K, int pos, const double* x, const double* g,
                       double* err, hipStream_t s) {
  k_sample_err<<<1, 64, 0, s>>>(G, K, pos, x, g, err);
}
void launch_add_into(const LzArgs& a, int K, const double* D, double* G, hipStream_t s) {
  k_add_into<<<tiles_grid(a.G, K), 256, 0, s>>>(a, D, G);
}

}  // namespace dyson
