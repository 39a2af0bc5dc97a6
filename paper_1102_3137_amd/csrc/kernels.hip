// HIP kernels for gfx950 (CDNA4, wave64).  Every kernel works on the
// tile-major layout of the plan: one workgroup of 256 threads per
// (tile, frequency), one lattice site per thread.  Complex numbers are
// interleaved (re, im) pairs; all products are bilinear (no conjugation):
// H is complex symmetric (Sec. I), and so are its blocks and inverses.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dyson {
namespace {

struct cd {
  double x, y;
};
__device__ __forceinline__ cd cmk(double a, double b) { return cd{a, b}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.x * s, a.y * s}; }
__device__ __forceinline__ cd cfma(cd a, cd b, cd c) {  // a*b + c
  return cd{fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
__device__ __forceinline__ cd cdiv(cd a, cd b) {
  double den = b.x * b.x + b.y * b.y;
  return cd{(a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den};
}
__device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
// principal square root of a complex number
__device__ __forceinline__ cd csqrt_p(cd a) {
  double r = sqrt(sqrt(a.x * a.x + a.y * a.y));
  double th = 0.5 * atan2(a.y, a.x);
  return cd{r * cos(th), r * sin(th)};
}

__device__ __forceinline__ cd ld(const double* p, size_t i) {
  const double2 v = reinterpret_cast<const double2*>(p)[i];
  return cd{v.x, v.y};
}
__device__ __forceinline__ void st(double* p, size_t i, cd v) {
  reinterpret_cast<double2*>(p)[i] = make_double2(v.x, v.y);
}
template <typename F>
__device__ __forceinline__ cd ldf(const F* p, size_t i);
template <>
__device__ __forceinline__ cd ldf<double>(const double* p, size_t i) {
  return ld(p, i);
}
template <>
__device__ __forceinline__ cd ldf<float>(const float* p, size_t i) {
  const float2 v = reinterpret_cast<const float2*>(p)[i];
  return cd{(double)v.x, (double)v.y};
}
template <typename F>
__device__ __forceinline__ void stf(F* p, size_t i, cd v);
template <>
__device__ __forceinline__ void stf<double>(double* p, size_t i, cd v) {
  st(p, i, v);
}
template <>
__device__ __forceinline__ void stf<float>(float* p, size_t i, cd v) {
  reinterpret_cast<float2*>(p)[i] = make_float2((float)v.x, (float)v.y);
}

__device__ __forceinline__ bool active(uint8_t kind, uint8_t depth, int g) {
  return kind == 1 || (kind == 2 && (int)depth >= g);
}

// wave64 sum of a complex value
__device__ __forceinline__ cd wave_sum(cd v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}
// sum over the 16-lane row group (lanes with equal tid>>4)
__device__ __forceinline__ cd row16_sum(cd v) {
  for (int o = 8; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 16);
    v.y += __shfl_xor(v.y, o, 16);
  }
  return v;
}
// block (256 threads) sum of up to two complex values; result valid in thread 0
__device__ __forceinline__ void block_sum2(cd& a, cd& b) {
  __shared__ cd red[2][4];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = cadd(cadd(red[0][0], red[0][1]), cadd(red[0][2], red[0][3]));
    b = cadd(cadd(red[1][0], red[1][1]), cadd(red[1][2], red[1][3]));
  }
}

// SplitMix64 (Steele, Lea & Flood 2014): counter-based 64-bit mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(uint64_t z) {  // [0,1)
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

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

// eq. (1): d_i(k) = i w_k + mu - V_i - Sigma_i(i w_k); padding sites get 1.
__global__ void k_assemble(TileGeom G, int K, double mu, const double* __restrict__ V,
                           const double* __restrict__ omega,
                           const double* __restrict__ sigma, double* __restrict__ d) {
  const size_t NP = (size_t)G.T * G.S;
  size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int k = blockIdx.y;
  if (p >= NP) return;
  int i = G.site_of[p];
  cd v = cmk(1.0, 0.0);
  if (i >= 0) {
    cd sg = ld(sigma, (size_t)k * G.N + i);
    v = cmk(mu - V[i] - sg.x, omega[k] - sg.y);
  }
  st(d, (size_t)k * NP + p, v);
}

// ------------------------------------------------------ tile factorization
// Block LDL^T of the tile block restricted to the sites active in graph g,
// slices = rows of sx sites: S_0 = A_0, S_y = A_y - T_y S_{y-1}^{-1} T_y with
// T_y = t diag(c_y) the bonds between rows y-1 and y.  The dense inverses
// S_y^{-1} (sx x sx, complex symmetric, pivot-free because Im > 0) are
// stored per slice.  With DIAG, the exact diagonal of the tile block's
// inverse follows from the backward recursion
// G_yy = S_y^{-1} + S_y^{-1} T_{y+1} G_{y+1,y+1} T_{y+1} S_y^{-1}.
template <typename F, bool DIAG>
__global__ __launch_bounds__(256) void k_factor(TileGeom G, int g, const int* __restrict__ tile_node,
                                                const double* __restrict__ d, F* __restrict__ fac,
                                                double* __restrict__ gdiag) {
  const int t = blockIdx.x, k = blockIdx.y;
  if (tile_node && tile_node[t] < 0) return;
  const int sx = G.sx, sy = G.sy, S = G.S;
  const size_t NP = (size_t)G.T * G.S;
  const int tid = threadIdx.x, i = tid >> 4, j = tid & 15;
  __shared__ cd dl[256];
  __shared__ uint8_t act[256];
  __shared__ cd A[16][17];
  __shared__ cd Gp[16][17];
  __shared__ cd Gall[DIAG ? 16 : 1][16][17];
  __shared__ cd tmp[16][17];
  const double tt = G.t;
  if (tid < S) {
    size_t p = (size_t)t * S + tid;
    dl[tid] = ld(d, (size_t)k * NP + p);
    act[tid] = active(G.kind[p], G.depth[p], g) ? 1 : 0;
  }
  __syncthreads();
  const size_t fbase = ((size_t)k * G.T + t) * (size_t)sy * sx * sx;
  for (int y = 0; y < sy; ++y) {
    // assemble the slice block (identity rows for inactive or padded sites)
    if (i < 16 && j < 16) {
      cd v = cmk(i == j ? 1.0 : 0.0, 0.0);
      if (i < sx && j < sx) {
        const int li = i + sx * y, lj = j + sx * y;
        const bool ai = act[li], aj = act[lj];
        v = cmk(0.0, 0.0);
        if (i == j) v = ai ? dl[li] : cmk(1.0, 0.0);
        else if ((i - j == 1 || j - i == 1) && ai && aj) v = cmk(tt, 0.0);
        if (y > 0 && ai && aj && act[i + sx * (y - 1)] && act[j + sx * (y - 1)])
          v = csub(v, cscale(Gp[i][j], tt * tt));
      }
      A[i][j] = v;
    }
    __syncthreads();
    // in-place Gauss-Jordan inversion, no pivoting
    for (int q = 0; q < sx; ++q) {
      cd piv = A[q][q], aiq = A[i][q], aqj = A[q][j], aij = A[i][j];
      __syncthreads();
      cd pinv = cdiv(cmk(1.0, 0.0), piv);
      cd nv;
      if (i == q && j == q) nv = pinv;
      else if (i == q) nv = cmul(aqj, pinv);
      else if (j == q) nv = cscale(cmul(aiq, pinv), -1.0);
      else nv = csub(aij, cmul(cmul(aiq, aqj), pinv));
      if (i < sx && j < sx) A[i][j] = nv;
      __syncthreads();
    }
    if (i < sx && j < sx) {
      if (fac) stf<F>(fac, fbase + (size_t)y * sx * sx + i * sx + j, A[i][j]);
      Gp[i][j] = A[i][j];
      if (DIAG) Gall[y][i][j] = A[i][j];
    }
    __syncthreads();
  }
  if (!DIAG) return;
  // backward selected inversion: Gc holds G_{y+1,y+1} in Gp
  if (i < sx && j < sx) Gp[i][j] = Gall[sy - 1][i][j];
  __syncthreads();
  if (tid < sx) {
    const int l = tid + sx * (sy - 1);
    size_t p = (size_t)t * S + l;
    if (G.kind[p] == 1) st(gdiag, (size_t)k * NP + p, Gp[tid][tid]);
  }
  for (int y = sy - 2; y >= 0; --y) {
    // tmp = C M C G_y, C = diag(c_{y+1})
    if (i < sx && j < sx) {
      cd acc = cmk(0.0, 0.0);
      const bool ci = act[i + sx * (y + 1)] && act[i + sx * y];
      if (ci)
        for (int l = 0; l < sx; ++l)
          if (act[l + sx * (y + 1)] && act[l + sx * y]) acc = cfma(Gp[i][l], Gall[y][l][j], acc);
      tmp[i][j] = acc;
    }
    __syncthreads();
    cd nv = cmk(0.0, 0.0);
    if (i < sx && j < sx) {
      cd acc = cmk(0.0, 0.0);
      for (int l = 0; l < sx; ++l) acc = cfma(Gall[y][i][l], tmp[l][j], acc);
      nv = cadd(Gall[y][i][j], cscale(acc, tt * tt));
    }
    __syncthreads();
    if (i < sx && j < sx) Gp[i][j] = nv;
    __syncthreads();
    if (tid < sx) {
      const int l = tid + sx * y;
      size_t p = (size_t)t * S + l;
      if (G.kind[p] == 1) st(gdiag, (size_t)k * NP + p, Gp[tid][tid]);
    }
  }
}

// ------------------------------------------------------ tile block solve
// z = M^{-1} r on one tile: forward z_y = r_y - T_y S_{y-1}^{-1} z_{y-1},
// backward v_y = S_y^{-1} (z_y - T_{y+1} v_{y+1}).  Thread (i, j) holds
// S_y^{-1}[i][j] for every slice y in registers; rows are reduced over the
// 16-lane groups.  rl (input) and zl (output, may alias nothing) live in LDS.
template <typename F>
struct TileFactor {
  cd g[16];
  __device__ __forceinline__ void load(const F* __restrict__ fac, size_t fbase, int sx, int sy) {
    const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
#pragma unroll
    for (int y = 0; y < 16; ++y)
      g[y] = (y < sy && i < sx && j < sx) ? ldf<F>(fac, fbase + (size_t)y * sx * sx + i * sx + j)
                                          : cmk(0.0, 0.0);
  }
};

template <typename F>
__device__ __forceinline__ void tile_solve(const TileFactor<F>& f, const cd* rl, cd* zl,
                                           const uint8_t* act, int sx, int sy, double tt) {
  const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
  __shared__ cd row[16];
  // forward
  if (threadIdx.x < sx) zl[threadIdx.x] = rl[threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int y = 1; y < 16; ++y) {
    if (y < sy) {
      cd prod = (j < sx) ? cmul(f.g[y - 1], zl[j + sx * (y - 1)]) : cmk(0.0, 0.0);
      prod = row16_sum(prod);
      if (j == 0 && i < sx) {
        const int l = i + sx * y;
        const bool c = act[l] && act[l - sx];
        zl[l] = c ? csub(rl[l], cscale(prod, tt)) : rl[l];
      }
    }
    __syncthreads();
  }
  // backward (in place over zl)
#pragma unroll
  for (int y = 15; y >= 0; --y) {
    if (y < sy) {
      if (y < sy - 1) {
        if (threadIdx.x < sx) {
          const int l = threadIdx.x + sx * y;
          const bool c = act[l + sx] && act[l];
          if (c) row[threadIdx.x] = csub(zl[l], cscale(zl[l + sx], tt));
          else row[threadIdx.x] = zl[l];
        }
      } else {
        if (threadIdx.x < sx) row[threadIdx.x] = zl[threadIdx.x + sx * y];
      }
      __syncthreads();
      cd prod = (j < sx) ? cmul(f.g[y], row[j]) : cmk(0.0, 0.0);
      prod = row16_sum(prod);
      if (j == 0 && i < sx) zl[i + sx * y] = prod;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- COCG
// Preconditioned conjugate orthogonal conjugate gradient (the complex-
// symmetric CG: every inner product bilinear) for A_g x = b, A_g the lattice
// restricted to the sites active in graph g, M the tile blocks of A_g.
// Items (domain, frequency) iterate in lock step; converged ones are skipped.
struct CocgArgs {
  TileGeom G;
  int g;
  const int* tile_node;
  int n_nodes;
  const int* item_skip;   // Lanczos-level "stopped" flags (may be null)
  CocgState st;           // per-item scalars
  const double* d;
  double *x, *r, *z, *p_old, *p_new, *s;
  double* partial;        // [K*T*2] complex
  unsigned long long* wctr;
};

template <typename F>
__global__ __launch_bounds__(256) void k_cocg_init(CocgArgs a, const double* __restrict__ b,
                                                   const F* __restrict__ fac) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  const TileGeom& G = a.G;
  if (a.item_skip && a.item_skip[item]) return;
  const size_t NP = (size_t)G.T * G.S;
  const size_t base = (size_t)k * NP + (size_t)t * G.S;
  __shared__ cd rl[256], zl[256];
  __shared__ uint8_t act[256];
  const int tid = threadIdx.x;
  cd rv = cmk(0.0, 0.0);
  if (tid < G.S) {
    const size_t p = (size_t)t * G.S + tid;
    const bool ac = active(G.kind[p], G.depth[p], a.g);
    act[tid] = ac;
    rv = ac ? ld(b, base + tid) : cmk(0.0, 0.0);
    rl[tid] = rv;
  } else if (tid < 256) {
    act[tid] = 0;
  }
  TileFactor<F> f;
  f.load(fac, ((size_t)k * G.T + t) * (size_t)G.sy * G.sx * G.sx, G.sx, G.sy);
  __syncthreads();
  tile_solve<F>(f, rl, zl, act, G.sx, G.sy, G.t);
  cd rz = cmk(0.0, 0.0), rr = cmk(0.0, 0.0);
  if (tid < G.S) {
    cd zv = act[tid] ? zl[tid] : cmk(0.0, 0.0);
    st(a.r, base + tid, rv);
    st(a.z, base + tid, zv);
    st(a.x, base + tid, cmk(0.0, 0.0));
    st(a.p_old, base + tid, cmk(0.0, 0.0));
    rz = cmul(rv, zv);
    rr = cmk(cabs2(rv), 0.0);
  }
  block_sum2(rz, rr);
  if (tid == 0) {
    const size_t q = ((size_t)k * G.T + t) * 2;
    st(a.partial, q, rz);
    st(a.partial, q + 1, rr);
  }
}

// p_new = z + beta p_old ; s = A_g p_new ; partial mu = p_new^T s
__global__ __launch_bounds__(256) void k_cocg_stencil(CocgArgs a) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.st.done[item]) return;
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  const size_t kb = (size_t)k * NP;
  const size_t base = kb + (size_t)t * G.S;
  const cd beta = ld(a.st.beta, item);
  if (a.wctr && threadIdx.x == 0)
    atomicAdd(&a.wctr[1], (unsigned long long)(G.S * (5 * 16 + 2)) + 2ull * 2 * (G.sx + G.sy) * 16);
  __shared__ cd pl[256];
  const int tid = threadIdx.x;
  const int sx = G.sx;
  bool ac = false;
  cd pn = cmk(0.0, 0.0);
  if (tid < G.S) {
    const size_t p = (size_t)t * G.S + tid;
    ac = active(G.kind[p], G.depth[p], a.g);
    if (ac) pn = cadd(ld(a.z, base + tid), cmul(beta, ld(a.p_old, base + tid)));
    pl[tid] = pn;
    st(a.p_new, base + tid, pn);
  }
  __syncthreads();
  cd mu = cmk(0.0, 0.0), unused = cmk(0.0, 0.0);
  if (tid < G.S && ac) {
    const int lx = tid % sx, ly = tid / sx;
    cd acc = cmul(ld(a.d, base + tid), pn);
    cd nb = cmk(0.0, 0.0);
    // -x
    if (lx > 0) nb = cadd(nb, pl[tid - 1]);
    else if (G.nbr[t * 4 + 0] >= 0) {
      const int nt = G.nbr[t * 4 + 0], nl = tid + sx - 1;
      const size_t np = (size_t)nt * G.S + nl;
      if (active(G.kind[np], G.depth[np], a.g))
        nb = cadd(nb, cadd(ld(a.z, kb + np), cmul(beta, ld(a.p_old, kb + np))));
    }
    // +x
    if (lx < sx - 1) nb = cadd(nb, pl[tid + 1]);
    else if (G.nbr[t * 4 + 1] >= 0) {
      const int nt = G.nbr[t * 4 + 1], nl = tid - (sx - 1);
      const size_t np = (size_t)nt * G.S + nl;
      if (active(G.kind[np], G.depth[np], a.g))
        nb = cadd(nb, cadd(ld(a.z, kb + np), cmul(beta, ld(a.p_old, kb + np))));
    }
    if (G.sy > 1) {
      // -y
      if (ly > 0) nb = cadd(nb, pl[tid - sx]);
      else if (G.nbr[t * 4 + 2] >= 0) {
        const int nt = G.nbr[t * 4 + 2], nl = tid + sx * (G.sy - 1);
        const size_t np = (size_t)nt * G.S + nl;
        if (active(G.kind[np], G.depth[np], a.g))
          nb = cadd(nb, cadd(ld(a.z, kb + np), cmul(beta, ld(a.p_old, kb + np))));
      }
      // +y
      if (ly < G.sy - 1) nb = cadd(nb, pl[tid + sx]);
      else if (G.nbr[t * 4 + 3] >= 0) {
        const int nt = G.nbr[t * 4 + 3], nl = tid - sx * (G.sy - 1);
        const size_t np = (size_t)nt * G.S + nl;
        if (active(G.kind[np], G.depth[np], a.g))
          nb = cadd(nb, cadd(ld(a.z, kb + np), cmul(beta, ld(a.p_old, kb + np))));
      }
    }
    acc = cadd(acc, cscale(nb, G.t));
    st(a.s, base + tid, acc);
    mu = cmul(pn, acc);
  } else if (tid < G.S) {
    st(a.s, base + tid, cmk(0.0, 0.0));
  }
  block_sum2(mu, unused);
  if (tid == 0) st(a.partial, ((size_t)k * G.T + t) * 2, mu);
}

// x += alpha p ; r -= alpha s ; z = M^{-1} r ; partials r^T z, |r|^2
template <typename F>
__global__ __launch_bounds__(256) void k_cocg_update(CocgArgs a, const F* __restrict__ fac) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.st.done[item]) return;
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  const size_t base = (size_t)k * NP + (size_t)t * G.S;
  const cd alpha = ld(a.st.alpha, item);
  if (a.wctr && threadIdx.x == 0)
    atomicAdd(&a.wctr[0], (unsigned long long)(G.S * (7 * 16 + 2)) +
                              (unsigned long long)G.sy * G.sx * G.sx * (2 * sizeof(F)));
  __shared__ cd rl[256], zl[256];
  __shared__ uint8_t act[256];
  const int tid = threadIdx.x;
  cd rv = cmk(0.0, 0.0);
  if (tid < G.S) {
    const size_t p = (size_t)t * G.S + tid;
    const bool ac = active(G.kind[p], G.depth[p], a.g);
    act[tid] = ac;
    if (ac) {
      const cd pv = ld(a.p_new, base + tid);
      cd xv = ld(a.x, base + tid);
      xv = cfma(alpha, pv, xv);
      st(a.x, base + tid, xv);
      rv = csub(ld(a.r, base + tid), cmul(alpha, ld(a.s, base + tid)));
    }
    rl[tid] = rv;
  } else {
    act[tid] = 0;
  }
  TileFactor<F> f;
  f.load(fac, ((size_t)k * G.T + t) * (size_t)G.sy * G.sx * G.sx, G.sx, G.sy);
  __syncthreads();
  tile_solve<F>(f, rl, zl, act, G.sx, G.sy, G.t);
  cd rz = cmk(0.0, 0.0), rr = cmk(0.0, 0.0);
  if (tid < G.S) {
    cd zv = act[tid] ? zl[tid] : cmk(0.0, 0.0);
    st(a.r, base + tid, rv);
    st(a.z, base + tid, zv);
    rz = cmul(rv, zv);
    rr = cmk(cabs2(rv), 0.0);
  }
  block_sum2(rz, rr);
  if (tid == 0) {
    const size_t q = ((size_t)k * G.T + t) * 2;
    st(a.partial, q, rz);
    st(a.partial, q + 1, rr);
  }
}

// Per-item reduction of the tile partials and the scalar recurrences.
// op 0: after init   rho = r^T z, bn2 = |b|^2, beta = 0, done = (bn2 == 0)
// op 1: after stencil alpha = rho / mu
// op 2: after update  converged if |r|^2 <= tol^2 bn2, else beta = rho'/rho
__global__ void k_cocg_scalars(CocgArgs a, int K, const int* __restrict__ tlo,
                               const int* __restrict__ thi, int op, double tol2, int it) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= K * a.n_nodes) return;
  const int k = item / a.n_nodes, node = item % a.n_nodes;
  if (a.item_skip && a.item_skip[item]) {
    if (op == 0) a.st.done[item] = 1;
    return;
  }
  if (op != 0 && a.st.done[item]) return;
  cd s0 = cmk(0.0, 0.0), s1 = cmk(0.0, 0.0);
  for (int t = tlo[node]; t < thi[node]; ++t) {
    const size_t q = ((size_t)k * a.G.T + t) * 2;
    s0 = cadd(s0, ld(a.partial, q));
    if (op != 1) s1 = cadd(s1, ld(a.partial, q + 1));
  }
  if (op == 0) {
    st(a.st.rho, item, s0);
    a.st.bn2[item] = s1.x;
    st(a.st.beta, item, cmk(0.0, 0.0));
    a.st.iters[item] = 0;
    a.st.done[item] = (s1.x == 0.0) ? 1 : 0;
  } else if (op == 1) {
    if (cabs2(s0) == 0.0) {  // breakdown of the bilinear form: give up on this item
      a.st.done[item] = 2;
      return;
    }
    st(a.st.alpha, item, cdiv(ld(a.st.rho, item), s0));
  } else {
    a.st.iters[item] = it + 1;
    if (s1.x <= tol2 * a.st.bn2[item]) {
      a.st.done[item] = 1;
      return;
    }
    const cd rho = ld(a.st.rho, item);
    st(a.st.beta, item, cdiv(s0, rho));
    st(a.st.rho, item, s0);
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
// Start vector: seeded random complex entries on the level's separator
// sites (the interface C of eq. (4)) of every correction domain, zero
// elsewhere; partial q^T q.
__global__ __launch_bounds__(256) void k_lz_random(LzArgs a, double* __restrict__ q, int only_flag,
                                                   uint64_t salt) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  if (only_flag && !a.restart[item]) return;
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  const size_t base = (size_t)k * NP + (size_t)t * G.S;
  const int tid = threadIdx.x;
  cd qq = cmk(0.0, 0.0), un = cmk(0.0, 0.0);
  if (tid < G.S) {
    const size_t p = (size_t)t * G.S + tid;
    cd v = cmk(0.0, 0.0);
    if (G.kind[p] == 2 && G.depth[p] == a.level) {
      // keyed by the frequency itself (not its batch slot), the level, the
      // site and the restart count, so a result does not depend on the batch
      const uint64_t key = splitmix64(a.seed ^ (salt * 0xD1B54A32D192ED03ULL) ^ a.fkey[k]) ^
                           (((uint64_t)a.level << 40) + (uint64_t)G.site_of[p]);
      const uint64_t h1 = splitmix64(key), h2 = splitmix64(h1 ^ 0xA5A5A5A5A5A5A5A5ULL);
      v = cmk(2.0 * u01(h1) - 1.0, 2.0 * u01(h2) - 1.0);
    }
    st(q, base + tid, v);
    qq = cmul(v, v);
  }
  block_sum2(qq, un);
  if (tid == 0) st(a.partial, (size_t)k * G.T + t, qq);
}

__global__ void k_freq_keys(const double* __restrict__ omega, int K, uint64_t* __restrict__ fkey) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  fkey[k] = omega ? (uint64_t)__double_as_longlong(omega[k]) : (uint64_t)k;
}

// dst = src / sqrt(src^T src) (principal root, precomputed in scal) for the
// flagged items (only_flag) or all open ones
__global__ void k_lz_scale(LzArgs a, const double* src, double* dst, int only_flag) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  if (only_flag && !a.restart[item]) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  const cd inv = ld(a.scal, item);
  if (threadIdx.x < a.G.S) st(dst, base + threadIdx.x, cmul(ld(src, base + threadIdx.x), inv));
}

// Defect of the block solve (eqs. (10)-(12) with the solve of (10) started
// from w = blkdiag(B^{-1},0) q): b = q - H w, which vanishes on the subdomain
// sites and equals q_C - E^T w on the level's interface sites.
__global__ __launch_bounds__(256) void k_lz_defect(LzArgs a, const double* __restrict__ q,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ b) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  const size_t kb = (size_t)k * NP;
  const int tid = threadIdx.x, sx = G.sx;
  if (tid >= G.S) return;
  const size_t p = (size_t)t * G.S + tid;
  cd out = cmk(0.0, 0.0);
  if (G.kind[p] == 2 && G.depth[p] == a.level) {
    const int gB = a.level + 1;
    const int lx = tid % sx, ly = tid / sx;
    cd acc = cmk(0.0, 0.0);
    auto add = [&](int nt, int nl) {
      const size_t np = (size_t)nt * G.S + nl;
      if (active(G.kind[np], G.depth[np], gB)) acc = cadd(acc, ld(w, kb + np));
    };
    if (lx > 0) add(t, tid - 1);
    else if (G.nbr[t * 4 + 0] >= 0) add(G.nbr[t * 4 + 0], tid + sx - 1);
    if (lx < sx - 1) add(t, tid + 1);
    else if (G.nbr[t * 4 + 1] >= 0) add(G.nbr[t * 4 + 1], tid - (sx - 1));
    if (G.sy > 1) {
      if (ly > 0) add(t, tid - sx);
      else if (G.nbr[t * 4 + 2] >= 0) add(G.nbr[t * 4 + 2], tid + sx * (G.sy - 1));
      if (ly < G.sy - 1) add(t, tid + sx);
      else if (G.nbr[t * 4 + 3] >= 0) add(G.nbr[t * 4 + 3], tid - sx * (G.sy - 1));
    }
    out = csub(ld(q, kb + p), cscale(acc, G.t));
  }
  st(b, kb + p, out);
}

// alpha partials: q^T u and |u|^2
__global__ __launch_bounds__(256) void k_lz_alpha(LzArgs a, const double* __restrict__ q,
                                                  const double* __restrict__ u) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  const int tid = threadIdx.x;
  cd qu = cmk(0.0, 0.0), uu = cmk(0.0, 0.0);
  if (tid < a.G.S) {
    const cd uv = ld(u, base + tid);
    qu = cmul(ld(q, base + tid), uv);
    uu = cmk(cabs2(uv), 0.0);
  }
  block_sum2(qu, uu);
  if (tid == 0) {
    st(a.partial, ((size_t)k * a.G.T + t) * 2, qu);
    st(a.partial, ((size_t)k * a.G.T + t) * 2 + 1, uu);
  }
}

// Three-term recurrence and the streaming diagonal (after eq. (13)):
// Gacc += alpha_j q_j*q_j + 2 beta_j q_{j-1}*q_j ; r = u - alpha_j q_j - beta_j q_{j-1}
__global__ __launch_bounds__(256) void k_lz_recur(LzArgs a, const double* __restrict__ q,
                                                  const double* __restrict__ qprev,
                                                  const double* __restrict__ u,
                                                  double* __restrict__ r, double* __restrict__ gacc) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  const int tid = threadIdx.x;
  if (tid >= a.G.S) return;
  const cd al = ld(a.alpha, item), be = ld(a.beta, item);
  const cd qv = ld(q, base + tid);
  const cd qp = qprev ? ld(qprev, base + tid) : cmk(0.0, 0.0);
  cd gv = ld(gacc, base + tid);
  gv = cadd(gv, cmul(al, cmul(qv, qv)));
  gv = cadd(gv, cscale(cmul(be, cmul(qp, qv)), 2.0));
  st(gacc, base + tid, gv);
  cd rv = csub(ld(u, base + tid), cmul(al, qv));
  rv = csub(rv, cmul(be, qp));
  st(r, base + tid, rv);
}

// Classical Gram-Schmidt, bilinear: h_i = Q_i^T r for i <= j.  Each wave
// takes every fourth basis vector of the tile; lanes cover 4 sites each.
__global__ __launch_bounds__(256) void k_cgs_dot(LzArgs a, const double* __restrict__ Q,
                                                 size_t qstride, int nvec,
                                                 const double* __restrict__ r, int only_flag) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  if (only_flag && !a.restart[item]) return;
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  const size_t base = (size_t)k * NP + (size_t)t * G.S;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (a.wctr && threadIdx.x == 0)
    atomicAdd(&a.wctr[3], (unsigned long long)(nvec + 1) * G.S * 16 + 16ull * nvec);
  cd rl[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int l = lane + 64 * c;
    rl[c] = (l < G.S) ? ld(r, base + l) : cmk(0.0, 0.0);
  }
  double* out = a.hpart + ((size_t)k * G.T + t) * (size_t)a.hstride * 2;
  for (int i = wv; i < nvec; i += 4) {
    const double* qi = Q + (size_t)i * qstride;
    cd acc = cmk(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int l = lane + 64 * c;
      if (l < G.S) acc = cfma(ld(qi, base + l), rl[c], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) st(out, i, acc);
  }
}

// h[item][i] = sum over the domain's tiles of the partials
__global__ void k_cgs_reduce(LzArgs a, int K, const int* __restrict__ tlo,
                             const int* __restrict__ thi, int nvec, int only_flag) {
  const int item = blockIdx.y;
  const int k = item / a.n_nodes, node = item % a.n_nodes;
  if (a.stopped[item]) return;
  if (only_flag && !a.restart[item]) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += gridDim.x * blockDim.x) {
    cd s = cmk(0.0, 0.0);
    for (int t = tlo[node]; t < thi[node]; ++t)
      s = cadd(s, ld(a.hpart + ((size_t)k * a.G.T + t) * (size_t)a.hstride * 2, i));
    st(a.h, (size_t)item * a.hstride + i, s);
  }
}

// r -= sum_i h_i Q_i
__global__ __launch_bounds__(256) void k_cgs_update(LzArgs a, const double* __restrict__ Q,
                                                    size_t qstride, int nvec,
                                                    double* __restrict__ r, int only_flag) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  if (only_flag && !a.restart[item]) return;
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  const size_t base = (size_t)k * NP + (size_t)t * G.S;
  if (a.wctr && threadIdx.x == 0)
    atomicAdd(&a.wctr[2], (unsigned long long)(nvec + 2) * G.S * 16 + 16ull * nvec);
  __shared__ cd hl[1024];
  const double* hs = a.h + (size_t)item * a.hstride * 2;
  for (int i = threadIdx.x; i < nvec && i < 1024; i += blockDim.x) hl[i] = ld(hs, i);
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid >= G.S) return;
  cd acc = cmk(0.0, 0.0);
  for (int i = 0; i < nvec; ++i) {
    const cd hv = (i < 1024) ? hl[i] : ld(hs, i);
    acc = cfma(hv, ld(Q + (size_t)i * qstride, base + tid), acc);
  }
  st(r, base + tid, csub(ld(r, base + tid), acc));
}

// partials |r|^2 and r^T r
__global__ __launch_bounds__(256) void k_lz_norms(LzArgs a, const double* __restrict__ r,
                                                  int only_flag) {
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item]) return;
  if (only_flag && !a.restart[item]) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  const int tid = threadIdx.x;
  cd rr = cmk(0.0, 0.0), rtr = cmk(0.0, 0.0);
  if (tid < a.G.S) {
    const cd v = ld(r, base + tid);
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
  const int t = blockIdx.x, k = blockIdx.y;
  const int node = a.tile_node[t];
  if (node < 0) return;
  const int item = k * a.n_nodes + node;
  if (a.stopped[item] || a.restart[item]) return;
  const size_t NP = (size_t)a.G.T * a.G.S;
  const size_t base = (size_t)k * NP + (size_t)t * a.G.S;
  if (threadIdx.x >= a.G.S) return;
  const cd inv = cdiv(cmk(1.0, 0.0), ld(a.beta, item));
  st(qn, base + threadIdx.x, cmul(ld(r, base + threadIdx.x), inv));
}

// Per-item scalar steps of the Lanczos recurrence.
//   op 0: start      scal = 1/sqrt(q^T q)
//   op 1: alpha      alpha = q^T u, unorm2 = |u|^2
//   op 2: norms      stop / restart decision, beta_{j+1} = sqrt(r^T r)
//   op 3: restart    scal = 1/sqrt(r^T r) of the fresh re-orthogonalized
//                    vector, beta_{j+1} = 0 (T splits into blocks)
__global__ void k_lz_scalars(LzArgs a, int K, const int* __restrict__ tlo,
                             const int* __restrict__ thi, const int* __restrict__ mcap, int op,
                             int j, double tol, double brk, int max_restarts) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= K * a.n_nodes) return;
  const int k = item / a.n_nodes, node = item % a.n_nodes;
  if (a.stopped[item]) return;
  if (op == 3 && !a.restart[item]) return;
  const int per = (op == 0) ? 1 : 2;
  cd s0 = cmk(0.0, 0.0), s1 = cmk(0.0, 0.0);
  for (int t = tlo[node]; t < thi[node]; ++t) {
    const size_t q = ((size_t)k * a.G.T + t) * per;
    s0 = cadd(s0, ld(a.partial, q));
    if (per == 2) s1 = cadd(s1, ld(a.partial, q + 1));
  }
  if (op == 0 || op == 3) {
    const cd qq = (op == 0) ? s0 : s1;  // q^T q of the new start vector
    if (cabs2(qq) == 0.0) {             // empty interface or a degenerate draw
      a.stopped[item] = (op == 0) ? 1 : 3;
      return;
    }
    st(a.scal, item, cdiv(cmk(1.0, 0.0), csqrt_p(qq)));
    if (op == 3) st(a.beta, item, cmk(0.0, 0.0));
    return;
  }
  if (op == 1) {
    st(a.alpha, item, s0);
    a.unorm2[item] = s1.x;
    return;
  }
  // op 2
  const int steps = j + 1;
  a.steps[item] = steps;
  a.restart[item] = 0;
  const double rn = sqrt(s0.x), un = sqrt(a.unorm2[item]);
  if (rn <= tol * un || un == 0.0) {
    a.stopped[item] = 1;  // the Krylov space of X is exhausted: T_j is complete
    return;
  }
  if (steps >= mcap[node]) {
    a.stopped[item] = 2;  // step cap (rank cap or m + extra)
    return;
  }
  if (sqrt(cabs2(s1)) <= brk * s0.x) {
    // serious breakdown of the bilinear form: restart from a fresh vector
    if (a.nrestart[item] >= max_restarts) {
      a.stopped[item] = 3;
      return;
    }
    a.nrestart[item] += 1;
    a.restart[item] = 1;
    return;
  }
  st(a.beta, item, csqrt_p(s1));
}

}  // namespace

// ----------------------------------------------------------------- launchers
static inline dim3 tiles_grid(const TileGeom& G, int K) { return dim3(G.T, K); }

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
                     const double* sigma, double* d, hipStream_t s) {
  size_t NP = (size_t)G.T * G.S;
  dim3 grid((unsigned)((NP + 255) / 256), K);
  k_assemble<<<grid, 256, 0, s>>>(G, K, mu, V, omega, sigma, d);
}
void launch_factor(const TileGeom& G, int K, int g, const int* tile_node, const double* d,
                   void* fac, bool fp32, double* gdiag, hipStream_t s) {
  dim3 grid = tiles_grid(G, K);
  if (gdiag) {
    k_factor<double, true><<<grid, 256, 0, s>>>(G, g, tile_node, d, (double*)fac, gdiag);
  } else if (fp32) {
    k_factor<float, false><<<grid, 256, 0, s>>>(G, g, tile_node, d, (float*)fac, nullptr);
  } else {
    k_factor<double, false><<<grid, 256, 0, s>>>(G, g, tile_node, d, (double*)fac, nullptr);
  }
}

void launch_cocg_init(const CocgLaunch& L, const double* b, hipStream_t s) {
  CocgArgs a{L.G, L.g, L.tile_node, L.n_nodes, L.item_skip, L.st, L.d,
             L.x, L.r, L.z, L.p_old, L.p_new, L.s, L.partial, L.wctr};
  dim3 grid = tiles_grid(L.G, L.K);
  if (L.fp32) k_cocg_init<float><<<grid, 256, 0, s>>>(a, b, (const float*)L.fac);
  else k_cocg_init<double><<<grid, 256, 0, s>>>(a, b, (const double*)L.fac);
}
void launch_cocg_stencil(const CocgLaunch& L, hipStream_t s) {
  CocgArgs a{L.G, L.g, L.tile_node, L.n_nodes, L.item_skip, L.st, L.d,
             L.x, L.r, L.z, L.p_old, L.p_new, L.s, L.partial, L.wctr};
  k_cocg_stencil<<<tiles_grid(L.G, L.K), 256, 0, s>>>(a);
}
void launch_cocg_update(const CocgLaunch& L, hipStream_t s) {
  CocgArgs a{L.G, L.g, L.tile_node, L.n_nodes, L.item_skip, L.st, L.d,
             L.x, L.r, L.z, L.p_old, L.p_new, L.s, L.partial, L.wctr};
  dim3 grid = tiles_grid(L.G, L.K);
  if (L.fp32) k_cocg_update<float><<<grid, 256, 0, s>>>(a, (const float*)L.fac);
  else k_cocg_update<double><<<grid, 256, 0, s>>>(a, (const double*)L.fac);
}
void launch_cocg_scalars(const CocgLaunch& L, const int* tlo, const int* thi, int op, double tol2,
                         int it, hipStream_t s) {
  CocgArgs a{L.G, L.g, L.tile_node, L.n_nodes, L.item_skip, L.st, L.d,
             L.x, L.r, L.z, L.p_old, L.p_new, L.s, L.partial, L.wctr};
  int n = L.K * L.n_nodes;
  k_cocg_scalars<<<(n + 127) / 128, 128, 0, s>>>(a, L.K, tlo, thi, op, tol2, it);
}
void launch_count_open(const int* done, int n, int* out, hipStream_t s) {
  k_count_open<<<1, 256, 0, s>>>(done, n, out);
}

void launch_freq_keys(const double* omega, int K, uint64_t* fkey, hipStream_t s) {
  k_freq_keys<<<(K + 63) / 64, 64, 0, s>>>(omega, K, fkey);
}
void launch_lz_random(const LzArgs& a, int K, double* q, int only_flag, uint64_t salt,
                      hipStream_t s) {
  k_lz_random<<<tiles_grid(a.G, K), 256, 0, s>>>(a, q, only_flag, salt);
}
void launch_lz_scale(const LzArgs& a, int K, const double* src, double* dst, int only_flag,
                     hipStream_t s) {
  k_lz_scale<<<tiles_grid(a.G, K), 256, 0, s>>>(a, src, dst, only_flag);
}
void launch_lz_defect(const LzArgs& a, int K, const double* q, const double* w, double* b,
                      hipStream_t s) {
  k_lz_defect<<<tiles_grid(a.G, K), 256, 0, s>>>(a, q, w, b);
}
void launch_lz_alpha(const LzArgs& a, int K, const double* q, const double* u, hipStream_t s) {
  k_lz_alpha<<<tiles_grid(a.G, K), 256, 0, s>>>(a, q, u);
}
void launch_lz_recur(const LzArgs& a, int K, const double* q, const double* qprev, const double* u,
                     double* r, double* gacc, hipStream_t s) {
  k_lz_recur<<<tiles_grid(a.G, K), 256, 0, s>>>(a, q, qprev, u, r, gacc);
}
void launch_cgs_dot(const LzArgs& a, int K, const double* Q, size_t qstride, int nvec,
                    const double* r, int only_flag, hipStream_t s) {
  k_cgs_dot<<<tiles_grid(a.G, K), 256, 0, s>>>(a, Q, qstride, nvec, r, only_flag);
}
void launch_cgs_reduce(const LzArgs& a, int K, const int* tlo, const int* thi, int nvec,
                       int only_flag, hipStream_t s) {
  dim3 grid((nvec + 255) / 256, K * a.n_nodes);
  k_cgs_reduce<<<grid, 256, 0, s>>>(a, K, tlo, thi, nvec, only_flag);
}
void launch_cgs_update(const LzArgs& a, int K, const double* Q, size_t qstride, int nvec, double* r,
                       int only_flag, hipStream_t s) {
  k_cgs_update<<<tiles_grid(a.G, K), 256, 0, s>>>(a, Q, qstride, nvec, r, only_flag);
}
void launch_lz_norms(const LzArgs& a, int K, const double* r, int only_flag, hipStream_t s) {
  k_lz_norms<<<tiles_grid(a.G, K), 256, 0, s>>>(a, r, only_flag);
}
void launch_lz_next(const LzArgs& a, int K, const double* r, double* qn, hipStream_t s) {
  k_lz_next<<<tiles_grid(a.G, K), 256, 0, s>>>(a, r, qn);
}
void launch_lz_scalars(const LzArgs& a, int K, const int* tlo, const int* thi, const int* mcap,
                       int op, int j, double tol, double brk, int max_restarts, hipStream_t s) {
  int n = K * a.n_nodes;
  k_lz_scalars<<<(n + 127) / 128, 128, 0, s>>>(a, K, tlo, thi, mcap, op, j, tol, brk, max_restarts);
}

}  // namespace dyson
