// Device helpers shared by the HIP sources: complex FP64 arithmetic on
// interleaved pairs, loads/stores, wave and block reductions, the
// activity rule of a graph level and a counter-based random generator.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dyson {
namespace dev {

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
template <>
__device__ __forceinline__ cd ldf<__half>(const __half* p, size_t i) {
  const __half2 v = reinterpret_cast<const __half2*>(p)[i];
  return cd{(double)__low2float(v), (double)__high2float(v)};
}
template <typename F>
__device__ __forceinline__ void stf(F* p, size_t i, cd v);
template <>
__device__ __forceinline__ void stf<__half>(__half* p, size_t i, cd v) {
  reinterpret_cast<__half2*>(p)[i] = __floats2half2_rn((float)v.x, (float)v.y);
}
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


// v / s for the tile edge s and 0 <= v < 2^16: one multiply-high by the
// precomputed floor(2^32/s) + 1 (exact: the rounding error stays below 1/s)
__device__ __forceinline__ int div_edge(const TileGeom& G, int v) {
  return (int)__umulhi((unsigned)v, G.edge_magic);
}

// Neighbour of tile-local site l in direction dir (0..5 = -x,+x,-y,+y,-z,+z):
// the same tile or the adjacent one; false at the lattice edge.
__device__ __forceinline__ bool site_nbr(const TileGeom& G, int t, int l, int dir, int& nt,
                                         int& nl) {
  const int s = G.edge, a = dir >> 1, up = dir & 1;
  if (a >= G.dim) return false;
  const int stride = (a == 0) ? 1 : (a == 1 ? s : s * s);
  const int q1 = div_edge(G, l), q2 = div_edge(G, q1);
  const int c = (a == 0) ? l - s * q1 : (a == 1 ? q1 - s * q2 : q2);
  if (up ? (c < s - 1) : (c > 0)) {
    nt = t;
    nl = up ? l + stride : l - stride;
    return true;
  }
  nt = G.nbr[t * 6 + dir];
  if (nt < 0) return false;
  nl = up ? l - (s - 1) * stride : l + (s - 1) * stride;
  return true;
}

// Bond between slice-local sites i and j (a row of a square tile, or a
// plane of a cubic one).
__device__ __forceinline__ bool slice_adj(const TileGeom& G, int i, int j) {
  if (G.dim < 3) return i - j == 1 || j - i == 1;
  const int s = G.edge;
  const int xi = i % s, yi = i / s, xj = j % s, yj = j / s;
  return (yi == yj && (xi - xj == 1 || xj - xi == 1)) ||
         (xi == xj && (yi - yj == 1 || yj - yi == 1));
}

// wave-scope fence + barrier: orders LDS traffic between the lanes of one wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP quad permutations of a double (lane i of each quad reads lane i^1 or
// i^2 of the same quad); quad_perm selectors [1,0,3,2] and [2,3,0,1]
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the 4 lanes of a quad (lanes 4q..4q+3), every lane gets the sum
__device__ __forceinline__ cd quad_sum(cd v) {
  v.x += dpp_quad<0xB1>(v.x);
  v.y += dpp_quad<0xB1>(v.y);
  v.x += dpp_quad<0x4E>(v.x);
  v.y += dpp_quad<0x4E>(v.y);
  return v;
}

}  // namespace dev
}  // namespace dyson
