// Explicit Schur-complement domain decomposition (Sec. II.B, eqs. (4)-(6)):
// the standard method the paper contrasts with the low-rank correction.  For
// a one-level decomposition (every separator in one interface C, the
// subdomains B block diagonal over the leaves),
//   H^{-1} = blkdiag(B^{-1}, 0) + [B^{-1}E; -I] S^{-1} [E^T B^{-1}, -I],
//   S = C - E^T B^{-1} E,
// so diag(H^{-1}) is diag(S^{-1}) on the interface and
// diag(B^{-1}) + diag(W S^{-1} W^T), W = B^{-1} E, inside the subdomains.
//
// Steps, all frequencies of a call at once:
//   1. leaf factors and diag(B^{-1}) (the same kernel as the low-rank path);
//   2. W_t = B_t^{-1} E_t per tile, one wave per interface site next to the
//      tile's leaf (a right-hand side of at most two entries), by the block
//      forward / backward sweeps over the complex128 slice inverses;
//   3. S assembled densely, one thread per entry, each entry summing its
//      tiles in a fixed order (no atomics: the result does not depend on
//      scheduling);
//   4. S^{-1} in place by blocked Gauss-Jordan without pivoting (Im S is
//      positive definite: S^{-1} is a principal block of H^{-1}, whose
//      imaginary part is negative definite, so every pivot block is
//      non-singular), 32-wide pivot blocks, the trailing update an LDS-tiled
//      complex FP64 product;
//   5. the diagonal, a workgroup per (tile, frequency).
// Memory: K m^2 complex128 for S (m interface sites), so it serves lattices
// whose interface fits; larger ones get DYSON_ENOMEM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dyson.h"
#include "devcommon.h"
#include "engine.h"

namespace dyson {

// Interface lists of a one-level plan (host-built, device copies).
struct SchurData {
  int m = 0;        // interface sites
  int nI = 1;       // most interface sites next to one leaf
  int D2 = 2;       // 2 * dim: neighbour slots per site
  int* a_pos = nullptr;   // [m] tile position of interface site a
  int* a_leaf = nullptr;  // [m][D2] tile positions of a's leaf neighbours, -1 padded
  int* a_ifc = nullptr;   // [m][D2] a's interface neighbours, -1 padded
  int* t_I = nullptr;     // [T][nI] interface sites next to the tile's leaf, ascending, -1 padded
  int* t_nI = nullptr;    // [T]
  int* t_rhs = nullptr;   // [T][nI][2] tile-local leaf sites bonded to t_I[T][q], -1 padded
  int* pos_a = nullptr;   // [T*S] interface index of a tile position, -1 elsewhere
  ~SchurData() {
    for (int* q : {a_pos, a_leaf, a_ifc, t_I, t_nI, t_rhs, pos_a})
      if (q) (void)hipFree(q);
  }
};

namespace {
using namespace dev;

constexpr int NB = 32;  // Gauss-Jordan pivot block

struct SchurArgs {
  TileGeom G;
  int K, m, nI, D2;
  const int *a_pos, *a_leaf, *a_ifc, *t_I, *t_nI, *t_rhs, *pos_a;
  const double* d;      // [K][T][S] assembled diagonal
  const double* fac;    // complex128 leaf factors
  double* W;            // [K][T][nI][S]
  double* Sm;           // [K][m][m]
};

__device__ __forceinline__ bool leaf_site(const TileGeom& G, size_t p) { return G.kind[p] == 1; }

// W_t[:, q] = B_t^{-1} E_t[:, q]: E_t[:, q] = t at the leaf sites bonded to
// interface site t_I[t][q].  Block forward z_y = r_y - T_y S_{y-1}^{-1} z_{y-1},
// backward x_y = S_y^{-1}(z_y - T_{y+1} x_{y+1}), T_y = t diag(bonds of leaf
// sites between slices y-1 and y); lane i owns row i of a slice (n <= 36).
__global__ __launch_bounds__(64) void k_schur_w(SchurArgs a) {
  const int q = blockIdx.x, t = blockIdx.y, k = blockIdx.z;
  const TileGeom& G = a.G;
  if (q >= a.t_nI[t]) return;
  const int lane = threadIdx.x, n = G.sx, ns = G.sy;
  __shared__ cd z[256];
  __shared__ cd x[256];
  __shared__ uint8_t act[256];
  for (int l = lane; l < 256; l += 64) {
    z[l] = cmk(0.0, 0.0);
    x[l] = cmk(0.0, 0.0);
    act[l] = (l < G.S && leaf_site(G, (size_t)t * G.S + l)) ? 1 : 0;
  }
  wave_sync();
  if (lane < 2) {
    const int l = a.t_rhs[((size_t)t * a.nI + q) * 2 + lane];
    if (l >= 0) z[l] = cmk(G.t, 0.0);
  }
  wave_sync();
  const size_t fb = ((size_t)k * G.T + t) * (size_t)ns * n * n;
  const double tt = G.t;
  for (int y = 1; y < ns; ++y) {
    cd acc = cmk(0.0, 0.0);
    if (lane < n)
      for (int j = 0; j < n; ++j) acc = cfma(ld(a.fac, fb + (size_t)(y - 1) * n * n + lane * n + j), z[j + n * (y - 1)], acc);
    wave_sync();
    if (lane < n) {
      const int l = lane + n * y;
      if (act[l] && act[l - n]) z[l] = csub(z[l], cscale(acc, tt));
    }
    wave_sync();
  }
  for (int y = ns - 1; y >= 0; --y) {
    cd acc = cmk(0.0, 0.0);
    if (lane < n)
      for (int j = 0; j < n; ++j) {
        const int l = j + n * y;
        cd row = z[l];
        if (y < ns - 1 && act[l] && act[l + n]) row = csub(row, cscale(x[l + n], tt));
        acc = cfma(ld(a.fac, fb + (size_t)y * n * n + lane * n + j), row, acc);
      }
    if (lane < n) x[lane + n * y] = act[lane + n * y] ? acc : cmk(0.0, 0.0);
    wave_sync();
  }
  double* out = a.W + (((size_t)k * G.T + t) * a.nI + q) * (size_t)G.S * 2;
  for (int l = lane; l < G.S; l += 64) st(out, l, x[l]);
}

// index of b among the ascending t_I[t][0 .. cnt), or -1
__device__ __forceinline__ int find_iface(const int* lst, int cnt, int b) {
  int lo = 0, hi = cnt - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1, v = lst[mid];
    if (v == b) return mid;
    if (v < b) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// S_ab = C_ab - sum over the tiles next to a (fixed order) of
// t * W_t[b][leaf neighbour of a in t]; C = diag(d) + t on interface bonds.
__global__ __launch_bounds__(256) void k_schur_s(SchurArgs a) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const size_t mm = (size_t)a.m * a.m;
  if (e >= mm) return;
  const int ia = (int)(e / a.m), b = (int)(e - (size_t)ia * a.m);
  const TileGeom& G = a.G;
  const size_t NP = (size_t)G.T * G.S;
  cd acc = cmk(0.0, 0.0);
  if (ia == b) acc = ld(a.d, (size_t)k * NP + a.a_pos[ia]);
  for (int q = 0; q < a.D2; ++q)
    if (a.a_ifc[(size_t)ia * a.D2 + q] == b) acc.x += G.t;
  for (int q = 0; q < a.D2; ++q) {
    const int p = a.a_leaf[(size_t)ia * a.D2 + q];
    if (p < 0) continue;
    const int t = p / G.S, l = p - t * G.S;
    const int bl = find_iface(a.t_I + (size_t)t * a.nI, a.t_nI[t], b);
    if (bl < 0) continue;
    const cd wv = ld(a.W, (((size_t)k * G.T + t) * a.nI + bl) * (size_t)G.S + l);
    acc = csub(acc, cscale(wv, G.t));
  }
  st(a.Sm, (size_t)k * mm + e, acc);
}

// ---------------------------------------------- blocked Gauss-Jordan, in place
// Pivot block [p0, p0 + nbp): Q = A_pp^{-1} (one workgroup per frequency).
__global__ __launch_bounds__(256) void k_gj_pivot(double* __restrict__ A, int m, int p0, int nbp,
                                                  double* __restrict__ Qb) {
  const int k = blockIdx.x;
  __shared__ cd P[NB][NB + 1];
  const double* Ak = A + (size_t)k * m * m * 2;
  for (int e = threadIdx.x; e < nbp * nbp; e += 256) {
    const int i = e / nbp, j = e % nbp;
    P[i][j] = ld(Ak, (size_t)(p0 + i) * m + p0 + j);
  }
  __syncthreads();
  for (int q = 0; q < nbp; ++q) {
    const cd pinv = cdiv(cmk(1.0, 0.0), P[q][q]);
    cd nv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = threadIdx.x + 256 * c;
      nv[c] = cmk(0.0, 0.0);
      if (e < nbp * nbp) {
        const int i = e / nbp, j = e % nbp;
        if (i == q && j == q) nv[c] = pinv;
        else if (i == q) nv[c] = cmul(P[q][j], pinv);
        else if (j == q) nv[c] = cscale(cmul(P[i][q], pinv), -1.0);
        else nv[c] = csub(P[i][j], cmul(cmul(P[i][q], P[q][j]), pinv));
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = threadIdx.x + 256 * c;
      if (e < nbp * nbp) P[e / nbp][e % nbp] = nv[c];
    }
    __syncthreads();
  }
  double* Qk = Qb + (size_t)k * NB * NB * 2;
  for (int e = threadIdx.x; e < nbp * nbp; e += 256) st(Qk, e, P[e / nbp][e % nbp]);
}

// Panels of step p, 64 columns / rows per workgroup:
//   Rx[r][j] = (Q A_{p,j})_r for j outside the pivot block, Q[r][j - p0] inside;
//   Cb[i][c] = A[i][p0 + c] (the old pivot columns).
__global__ __launch_bounds__(256) void k_gj_panels(const double* __restrict__ A, int m, int p0,
                                                   int nbp, const double* __restrict__ Qb,
                                                   double* __restrict__ Rx, double* __restrict__ Cb) {
  const int k = blockIdx.y, c0 = blockIdx.x * 64;
  __shared__ cd Q[NB][NB + 1];
  __shared__ cd Ap[NB][65];
  const double* Ak = A + (size_t)k * m * m * 2;
  const double* Qk = Qb + (size_t)k * NB * NB * 2;
  for (int e = threadIdx.x; e < nbp * nbp; e += 256) Q[e / nbp][e % nbp] = ld(Qk, e);
  for (int e = threadIdx.x; e < nbp * 64; e += 256) {
    const int r = e / 64, c = e % 64, j = c0 + c;
    Ap[r][c] = j < m ? ld(Ak, (size_t)(p0 + r) * m + j) : cmk(0.0, 0.0);
  }
  __syncthreads();
  double* Rk = Rx + (size_t)k * NB * m * 2;
  for (int e = threadIdx.x; e < nbp * 64; e += 256) {
    const int r = e / 64, c = e % 64, j = c0 + c;
    if (j >= m) continue;
    cd v;
    if (j >= p0 && j < p0 + nbp) {
      v = Q[r][j - p0];
    } else {
      v = cmk(0.0, 0.0);
      for (int q = 0; q < nbp; ++q) v = cfma(Q[r][q], Ap[q][c], v);
    }
    st(Rk, (size_t)r * m + j, v);
  }
  double* Ck = Cb + (size_t)k * m * NB * 2;
  for (int e = threadIdx.x; e < 64 * nbp; e += 256) {
    const int i = c0 + e / nbp, c = e % nbp;
    if (i < m) st(Ck, (size_t)i * NB + c, ld(Ak, (size_t)i * m + p0 + c));
  }
}

// A_ij <- (j in pivot block ? 0 : A_ij) - sum_c Cb[i][c] Rx[c][j] outside the
// pivot rows; A_pj <- Rx[p - p0][j] on them.  64 x 64 outputs per workgroup,
// 4 x 4 per thread (rows ty + 16 u, columns tx + 16 v), operands staged in LDS.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int m, int p0, int nbp,
                                                   const double* __restrict__ Rx,
                                                   const double* __restrict__ Cb) {
  const int k = blockIdx.z, i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ cd Cs[64][NB];
  __shared__ cd Rs[NB][64];
  const double* Ck = Cb + (size_t)k * m * NB * 2;
  const double* Rk = Rx + (size_t)k * NB * m * 2;
  for (int e = threadIdx.x; e < 64 * NB; e += 256) {
    const int r = e / NB, c = e % NB, i = i0 + r;
    Cs[r][c] = (i < m && c < nbp) ? ld(Ck, (size_t)i * NB + c) : cmk(0.0, 0.0);
  }
  for (int e = threadIdx.x; e < NB * 64; e += 256) {
    const int c = e / 64, r = e % 64, j = j0 + r;
    Rs[c][r] = (j < m && c < nbp) ? ld(Rk, (size_t)c * m + j) : cmk(0.0, 0.0);
  }
  __syncthreads();
  cd acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = cmk(0.0, 0.0);
  for (int c = 0; c < nbp; ++c) {
    cd av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) av[u] = Cs[ty + 16 * u][c];
#pragma unroll
    for (int v = 0; v < 4; ++v) bv[v] = Rs[c][tx + 16 * v];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = cfma(av[u], bv[v], acc[u][v]);
  }
  double* Ak = A + (size_t)k * m * m * 2;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ty + 16 * u;
    if (i >= m) continue;
    const bool prow = i >= p0 && i < p0 + nbp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + tx + 16 * v;
      if (j >= m) continue;
      const size_t ij = (size_t)i * m + j;
      cd out;
      if (prow) {
        out = Rs[i - p0][tx + 16 * v];
      } else {
        const bool pcol = j >= p0 && j < p0 + nbp;
        out = csub(pcol ? cmk(0.0, 0.0) : ld(Ak, ij), acc[u][v]);
      }
      st(Ak, ij, out);
    }
  }
}

// G on the tile layout: S^{-1}_aa on interface sites; diag(B^{-1}) (already in
// g) plus sum_{a,b} W[a][l] S^{-1}_{I_a I_b} W[b][l] on leaf sites.
__global__ __launch_bounds__(256) void k_schur_diag(SchurArgs a, double* __restrict__ g) {
  const int t = blockIdx.x, k = blockIdx.y, l = threadIdx.x;
  const TileGeom& G = a.G;
  if (l >= G.S) return;
  const size_t NP = (size_t)G.T * G.S, p = (size_t)t * G.S + l;
  const size_t mm = (size_t)a.m * a.m;
  const double* Sk = a.Sm + (size_t)k * mm * 2;
  if (G.kind[p] == 2) {
    const int ia = a.pos_a[p];
    if (ia >= 0) st(g, (size_t)k * NP + p, ld(Sk, (size_t)ia * a.m + ia));
    return;
  }
  if (G.kind[p] != 1) return;
  const int cnt = a.t_nI[t];
  const int* I = a.t_I + (size_t)t * a.nI;
  const double* Wt = a.W + ((size_t)k * G.T + t) * a.nI * (size_t)G.S * 2;
  cd corr = cmk(0.0, 0.0);
  constexpr int CH = 8;
  for (int q0 = 0; q0 < cnt; q0 += CH) {
    cd wa[CH], acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      wa[c] = q0 + c < cnt ? ld(Wt, (size_t)(q0 + c) * G.S + l) : cmk(0.0, 0.0);
      acc[c] = cmk(0.0, 0.0);
    }
    for (int r = 0; r < cnt; ++r) {
      const cd wb = ld(Wt, (size_t)r * G.S + l);
      const int ib = I[r];
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (q0 + c < cnt) acc[c] = cfma(ld(Sk, (size_t)I[q0 + c] * a.m + ib), wb, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) corr = cfma(wa[c], acc[c], corr);
  }
  st(g, (size_t)k * NP + p, cadd(ld(g, (size_t)k * NP + p), corr));
}

// ------------------------------------------------------------- host side
template <typename T>
dyson_status upload(T** dst, const std::vector<T>& v) {
  if (hipMalloc((void**)dst, std::max<size_t>(1, v.size()) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    set_error("device allocation of the interface lists failed");
    return DYSON_ENOMEM;
  }
  if (!v.empty() &&
      hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("copy of the interface lists failed");
    return DYSON_EDEVICE;
  }
  return DYSON_OK;
}

// Interface sites, their leaf and interface neighbours, and each tile's
// adjacent interface sites, from the plan's site maps (natural coordinates,
// wrap bonds on periodic axes).
dyson_status build_schur(const dyson_plan* pl, std::shared_ptr<SchurData>* out) {
  const HostPlan& P = pl->hp;
  auto sd = std::make_shared<SchurData>();
  const int N = P.N, D = P.dim, D2 = 2 * D;
  sd->D2 = D2;
  std::vector<int> aidx(N, -1), a_pos;
  for (int i = 0; i < N; ++i)
    if (P.kind[P.pos_of[i]] == KIND_SEP) {
      aidx[i] = (int)a_pos.size();
      a_pos.push_back(P.pos_of[i]);
    }
  const int m = (int)a_pos.size();
  sd->m = m;
  auto nbrs = [&](int i, int* o) {  // natural neighbours, -1 where there is none
    int c[3] = {i % P.L[0], (i / P.L[0]) % P.L[1], i / (P.L[0] * P.L[1])};
    const int st[3] = {1, P.L[0], P.L[0] * P.L[1]};
    for (int ax = 0; ax < D; ++ax)
      for (int sg = 0; sg < 2; ++sg) {
        int cc = c[ax] + (sg ? 1 : -1), j = -1;
        if (cc >= 0 && cc < P.L[ax]) j = i + (sg ? st[ax] : -st[ax]);
        else if (P.periodic[ax] && P.L[ax] > 2) {
          cc = (cc + P.L[ax]) % P.L[ax];
          j = i + (cc - c[ax]) * st[ax];
        }
        o[2 * ax + sg] = j;
      }
  };
  std::vector<int> a_leaf((size_t)m * D2, -1), a_ifc((size_t)m * D2, -1);
  std::vector<std::vector<int>> tI(P.T);
  std::vector<std::vector<std::pair<int, int>>> tb(P.T);  // (interface a, leaf tile-local l)
  int o[6];
  for (int i = 0; i < N; ++i) {
    nbrs(i, o);
    const int pi = P.pos_of[i];
    if (aidx[i] >= 0) {
      const int ia = aidx[i];
      for (int q = 0; q < D2; ++q) {
        if (o[q] < 0) continue;
        const int pj = P.pos_of[o[q]];
        if (P.kind[pj] == KIND_LEAF) a_leaf[(size_t)ia * D2 + q] = pj;
        else if (aidx[o[q]] >= 0) a_ifc[(size_t)ia * D2 + q] = aidx[o[q]];
      }
    } else if (P.kind[pi] == KIND_LEAF) {
      const int t = pi / P.S, l = pi % P.S;
      for (int q = 0; q < D2; ++q)
        if (o[q] >= 0 && aidx[o[q]] >= 0) {
          tI[t].push_back(aidx[o[q]]);
          tb[t].push_back({aidx[o[q]], l});
        }
    }
  }
  int nI = 1;
  for (auto& v : tI) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    nI = std::max(nI, (int)v.size());
  }
  sd->nI = nI;
  std::vector<int> t_I((size_t)P.T * nI, -1), t_nI(P.T, 0), t_rhs((size_t)P.T * nI * 2, -1);
  for (int t = 0; t < P.T; ++t) {
    t_nI[t] = (int)tI[t].size();
    for (int q = 0; q < t_nI[t]; ++q) t_I[(size_t)t * nI + q] = tI[t][q];
    for (auto& bl : tb[t]) {
      const int q = (int)(std::lower_bound(tI[t].begin(), tI[t].end(), bl.first) - tI[t].begin());
      int* slot = &t_rhs[((size_t)t * nI + q) * 2];
      if (slot[0] < 0) slot[0] = bl.second;
      else if (slot[1] < 0 && slot[0] != bl.second) slot[1] = bl.second;
      else if (slot[0] != bl.second && slot[1] != bl.second) {
        set_error("an interface site bonds to more than two sites of one leaf");
        return DYSON_EUNSUPPORTED;
      }
    }
  }
  std::vector<int> pos_a((size_t)P.T * P.S, -1);
  for (int ia = 0; ia < m; ++ia) pos_a[a_pos[ia]] = ia;
  dyson_status s;
  if ((s = upload(&sd->a_pos, a_pos)) != DYSON_OK) return s;
  if ((s = upload(&sd->a_leaf, a_leaf)) != DYSON_OK) return s;
  if ((s = upload(&sd->a_ifc, a_ifc)) != DYSON_OK) return s;
  if ((s = upload(&sd->t_I, t_I)) != DYSON_OK) return s;
  if ((s = upload(&sd->t_nI, t_nI)) != DYSON_OK) return s;
  if ((s = upload(&sd->t_rhs, t_rhs)) != DYSON_OK) return s;
  if ((s = upload(&sd->pos_a, pos_a)) != DYSON_OK) return s;
  *out = sd;
  return DYSON_OK;
}

}  // namespace

// In-place inverse of `batch` m x m complex matrices (contiguous, row-major),
// blocked Gauss-Jordan without pivoting; Cb [batch][m][32], Rx [batch][32][m]
// and Qb [batch][32][32] complex are scratch.
void launch_gj_invert(double* A, int m, int batch, double* Cb, double* Rx, double* Qb,
                      hipStream_t s) {
  const unsigned nt = (unsigned)((m + 63) / 64);
  for (int p0 = 0; p0 < m; p0 += NB) {
    const int nbp = std::min<int>(NB, m - p0);
    k_gj_pivot<<<(unsigned)batch, 256, 0, s>>>(A, m, p0, nbp, Qb);
    k_gj_panels<<<dim3(nt, (unsigned)batch), 256, 0, s>>>(A, m, p0, nbp, Qb, Rx, Cb);
    k_gj_update<<<dim3(nt, nt, (unsigned)batch), 256, 0, s>>>(A, m, p0, nbp, Rx, Cb);
  }
}

size_t schur_bytes(const dyson_plan* p, int K, const SchurData& sd) {
  const size_t m = (size_t)sd.m;
  return (size_t)K * (m * m + 2 * m * NB + NB * NB + (size_t)p->hp.T * sd.nI * p->hp.S) * 16;
}

}  // namespace dyson

using namespace dyson;

extern "C" dyson_status dyson_solve_schur(dyson_plan* p, int K, const double* d_V,
                                          const double* d_omega, const double* d_sigma,
                                          double* d_G, void* stream, dyson_report* rep) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p || !p->ctx) {
    set_error("plan has no device context");
    return DYSON_EINVAL;
  }
  if (K < 1 || K > 65535) {
    set_error("K must be in [1, 65535]");
    return DYSON_EINVAL;
  }
  const HostPlan& P = p->hp;
  if (P.levels.size() > 1) {
    set_error("the explicit Schur-complement path takes a one-level decomposition "
              "(DYSON_PART_SINGLE, eq. (4))");
    return DYSON_EUNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(p->ctx->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return DYSON_EDEVICE;
  }
  dyson_status st;
  if (!p->schur) {
    std::shared_ptr<SchurData> sd;
    if ((st = build_schur(p, &sd)) != DYSON_OK) return st;
    p->schur = sd;
  }
  const SchurData& sd = *p->schur;
  Work* w = &p->main;
  if ((st = ensure_work(p, w, K, s)) != DYSON_OK) return st;
  Slice sl{K, d_V, d_omega, d_sigma, d_G, 0};
  if ((st = validate_slices(p, w, &sl, 1, s)) != DYSON_OK) return st;
  const size_t NP = (size_t)P.T * P.S;
  launch_assemble(p->geom, K, P.mu, d_V, d_omega, 0, d_sigma, w->d, s);
  launch_zero(w->gacc, (size_t)K * NP * 16, s);
  launch_factor_diag(p->geom, K, w->d, w->fac64, w->gacc, s);
  const size_t m = (size_t)sd.m;
  char* buf = nullptr;
  const size_t need = schur_bytes(p, K, sd);
  hipEvent_t ev[2] = {nullptr, nullptr};
  long long gj_launches = 0;
  if (m > 0) {
    buf = (char*)ctx_alloc(p->ctx, need + 2048, s);
    if (!buf) {
      set_error("the explicit Schur complement needs " + std::to_string(need) +
                " bytes of device memory");
      return DYSON_ENOMEM;
    }
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    double* Sm = (double*)buf;
    double* Cb = (double*)(buf + al((size_t)K * m * m * 16));
    double* Rx = (double*)((char*)Cb + al((size_t)K * m * NB * 16));
    double* Qb = (double*)((char*)Rx + al((size_t)K * m * NB * 16));
    double* W = (double*)((char*)Qb + al((size_t)K * NB * NB * 16));
    SchurArgs a{p->geom, K, sd.m, sd.nI, sd.D2, sd.a_pos, sd.a_leaf, sd.a_ifc, sd.t_I,
                sd.t_nI, sd.t_rhs, sd.pos_a, w->d, w->fac64, W, Sm};
    k_schur_w<<<dim3((unsigned)sd.nI, (unsigned)P.T, (unsigned)K), 64, 0, s>>>(a);
    k_schur_s<<<dim3((unsigned)((m * m + 255) / 256), (unsigned)K), 256, 0, s>>>(a);
    const unsigned nt = (unsigned)((m + 63) / 64);
    if (P.opts.profile && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)) {
      (void)hipGetLastError();
      ev[0] = ev[1] = nullptr;
    }
    if (ev[0]) (void)hipEventRecord(ev[0], s);
    for (int p0 = 0; p0 < (int)m; p0 += NB) {
      const int nbp = std::min<int>(NB, (int)m - p0);
      k_gj_pivot<<<(unsigned)K, 256, 0, s>>>(Sm, (int)m, p0, nbp, Qb);
      k_gj_panels<<<dim3(nt, (unsigned)K), 256, 0, s>>>(Sm, (int)m, p0, nbp, Qb, Rx, Cb);
      k_gj_update<<<dim3(nt, nt, (unsigned)K), 256, 0, s>>>(Sm, (int)m, p0, nbp, Rx, Cb);
      gj_launches += 3;
    }
    if (ev[1]) (void)hipEventRecord(ev[1], s);
    k_schur_diag<<<dim3((unsigned)P.T, (unsigned)K), 256, 0, s>>>(a, w->gacc);
  }
  launch_from_tile(p->geom, K, w->gacc, d_G, s);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamSynchronize(s);
  if (buf) ctx_free(p->ctx, buf, s);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error(std::string("explicit Schur path: ") +
              hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return DYSON_EDEVICE;
  }
  float gj_ms = 0.f;
  if (ev[0] && ev[1] && hipEventElapsedTime(&gj_ms, ev[0], ev[1]) != hipSuccess) gj_ms = 0.f;
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    // profile: class 0 is the Gauss-Jordan inversion of S (HIP events on the
    // call's stream), its bytes field the algorithmic flops, 8 m^3 per frequency
    rep->kern_ms[0] = gj_ms;
    rep->kern_launches[0] = gj_launches;
    rep->kern_bytes[0] = 8.0 * (double)m * (double)m * (double)m * K;
    rep->levels = (int)P.levels.size();
    rep->max_rank_used = (int)m;
    rep->batches = 1;
    rep->hbm_bytes = w->bytes + (m > 0 ? need : 0);
    rep->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return DYSON_OK;
}
