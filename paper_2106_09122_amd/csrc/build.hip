// Library build: gather, interpolate and rotate (Sec. 2; Eqs. (4)-(5)).
// This file holds the gather form (PSFs too large to stage in LDS) and the
// cubic-spline rotation (any size), which gathers 4 x 4 coefficient pairs.
//
// Column j of A is the datacube interpolated to the field point's offset,
// Q = (1-w) P_k + w P_{k+1}, rotated about the array centre to the field
// point's position angle and sampled bilinearly with zero padding.  One
// workgroup builds one group of 8 adjacent columns; each thread produces row i
// of all 8 columns, so every store is coalesced: the FP32 form writes 8
// contiguous 256-byte runs per wave (one per column), the 16-bit forms one
// 16-byte group per thread (1 KiB per wave).  Coordinates are float64
// (bit-for-bit the oracle's operation order, no contraction); the fractional
// offsets are rounded once to float32, and the weights, the radial blend and
// the weighted sum run in float32, in the LDS-staged builds' order.  Column sums are
// accumulated in float64 and reduced in a fixed order.
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

struct ColumnParams {
  const float2* src;  // pairs (P_k, P_{k+1}) of this column's bracket
  double ct, st;
  float wk0, wk1;     // (1-w), w rounded to float32
  int32_t e;          // 16-bit exponent
  bool live;          // false: identically zero (ZERO mode, or padding)
};

// One radially blended tap; zero outside the n x n frame.
__device__ __forceinline__ float tap(const float2* __restrict__ P, int n, int r, int c, float wk0,
                                     float wk1) {
  if ((unsigned)r < (unsigned)n && (unsigned)c < (unsigned)n) {
    const float2 v = P[r * n + c];
    return fmaf(wk1, v.y, wk0 * v.x);
  }
  return 0.0f;
}

// Source coordinates of output pixel offset (ux, uy) under R(-theta) (float64,
// no contraction, in the oracle's order) and the fractional offsets and their
// complements, each rounded once to float32; the bilinear weights are their
// float32 products, as in the LDS-staged builds, so both forms give identical
// values.
struct Bilinear {
  int r0, c0;
  float fx, gx, fy, gy;
};

__device__ __forceinline__ Bilinear bilinear_weights(double ct, double st, double c, double ux,
                                                     double uy) {
#pragma clang fp contract(off)
  const double sx = ct * ux + st * uy;
  const double sy = (-st) * ux + ct * uy;
  const double colf = c + sx;
  const double rowf = c + sy;
  const double c0f = floor(colf);
  const double r0f = floor(rowf);
  const double fx = colf - c0f;
  const double fy = rowf - r0f;
  Bilinear b;
  b.fx = (float)fx;
  b.gx = (float)(1.0 - fx);
  b.fy = (float)fy;
  b.gy = (float)(1.0 - fy);
  b.c0 = (int)c0f;
  b.r0 = (int)r0f;
  return b;
}

__device__ __forceinline__ float column_value(const ColumnParams& cp, int n, double c, double ux,
                                              double uy) {
  const Bilinear b = bilinear_weights(cp.ct, cp.st, c, ux, uy);
  const float q00 = tap(cp.src, n, b.r0, b.c0, cp.wk0, cp.wk1);
  const float q01 = tap(cp.src, n, b.r0, b.c0 + 1, cp.wk0, cp.wk1);
  const float q10 = tap(cp.src, n, b.r0 + 1, b.c0, cp.wk0, cp.wk1);
  const float q11 = tap(cp.src, n, b.r0 + 1, b.c0 + 1, cp.wk0, cp.wk1);
  float v = (b.gy * b.gx) * q00;
  v = fmaf(b.gy * b.fx, q01, v);
  v = fmaf(b.fy * b.gx, q10, v);
  v = fmaf(b.fy * b.fx, q11, v);
  return v;
}

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // finite inputs: round to nearest, ties to even
  return u >> 16;
}

__device__ __forceinline__ uint32_t f32_to_f16_rne(float f) {
  const _Float16 h = (_Float16)f;  // v_cvt_f16_f32, round to nearest even
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

// Coefficient pair at (r, c) of the padded array, zero outside it.
__device__ __forceinline__ float2 tap_pair(const float2* __restrict__ P, int Np, int r, int c) {
  if ((unsigned)r < (unsigned)Np && (unsigned)c < (unsigned)Np) return P[r * Np + c];
  return make_float2(0.0f, 0.0f);
}

// Cubic-spline rotation: the same source point as the bilinear form, in the
// coordinates of the spline coefficients (padded by kSplinePad), sampled with
// the 4 x 4 B-spline weights, taps outside the padded array zero.  Each tap
// is the radial blend (1-w) C_k + w C_{k+1} of its coefficient pair; the taps
// are summed separably (each row's weighted sum, then those rows weighted) in
// the order the LDS-staged cubic orbit build uses, so both forms give
// identical values.
__device__ __forceinline__ float column_value_cubic(const ColumnParams& cp, int Np, double c,
                                                    double ux, double uy) {
#pragma clang fp contract(off)
  const double sx = cp.ct * ux + cp.st * uy;
  const double sy = (-cp.st) * ux + cp.ct * uy;
  const double colf = c + sx + (double)kSplinePad;
  const double rowf = c + sy + (double)kSplinePad;
  const double c0f = floor(colf), r0f = floor(rowf);
  const int c0 = (int)c0f;
  const int r0 = (int)r0f;
  float wy[4], wx[4];
  cubic_weights(rowf - r0f, wy);
  cubic_weights(colf - c0f, wx);
  float V = 0.0f;
#pragma unroll
  for (int dr = 0; dr < 4; ++dr) {
    const int r = r0 + dr - 1;
    float q[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float2 p = tap_pair(cp.src, Np, r, c0 - 1 + e);
      q[e] = fmaf(cp.wk1, p.y, cp.wk0 * p.x);
    }
    float v = wx[0] * q[0];
    v = fmaf(wx[1], q[1], v);
    v = fmaf(wx[2], q[2], v);
    v = fmaf(wx[3], q[3], v);
    V = fmaf(wy[dr], v, V);
  }
  return V;
}

template <int STORE, bool CUBIC>
__global__ __launch_bounds__(kBuildThreads) void build_kernel(const float2* __restrict__ pairs,
                                                              const ColGeom* __restrict__ geo,
                                                              int n, int64_t M, int64_t ncols,
                                                              int64_t ncols_pad,
                                                              void* __restrict__ lib,
                                                              double* __restrict__ tau) {
  __shared__ double red[8][kBuildThreads];
  const int64_t grp = blockIdx.x;
  const int64_t j0 = grp * 8;
  const int tid = threadIdx.x;

  ColumnParams cp[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t j = j0 + u;
    cp[u].live = false;
    cp[u].src = pairs;
    cp[u].ct = 1.0; cp[u].st = 0.0; cp[u].wk0 = 1.0f; cp[u].wk1 = 0.0f; cp[u].e = 0;
    if (j < ncols_pad) {
      const ColGeom g = geo[j];
      if (g.k >= 0 && j < ncols) {
        cp[u].live = true;
        cp[u].src = pairs + (int64_t)g.k * (CUBIC ? (int64_t)(n + 2 * kSplinePad) * (n + 2 * kSplinePad) : M);
        cp[u].ct = g.ct;
        cp[u].st = g.st;
        cp[u].wk0 = (float)(1.0 - g.w);
        cp[u].wk1 = (float)g.w;
        cp[u].e = g.e;
      }
    }
  }

  const double c = (double)(n - 1) * 0.5;
  double tacc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) tacc[u] = 0.0;

  int a = tid / n, b = tid % n;
  const int da = kBuildThreads / n, db = kBuildThreads % n;
  for (int64_t i = tid; i < M; i += kBuildThreads) {
    const double ux = (double)b - c;
    const double uy = (double)a - c;
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if constexpr (CUBIC)
        v[u] = cp[u].live ? column_value_cubic(cp[u], n + 2 * kSplinePad, c, ux, uy) : 0.0f;
      else
        v[u] = cp[u].live ? column_value(cp[u], n, c, ux, uy) : 0.0f;
      tacc[u] += (double)v[u];
    }
    if constexpr (STORE == PSFLIB_FP32) {
      float* A = reinterpret_cast<float*>(lib);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < ncols) __builtin_nontemporal_store(v[u], A + (j0 + u) * M + i);
    } else {
      uint32_t h[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float s = ldexpf(v[u], -cp[u].e);  // exact power-of-two scaling
        h[u] = (STORE == PSFLIB_BF16_POW2) ? f32_to_bf16_rne(s) : f32_to_f16_rne(s);
      }
      u32x4 pk;
      pk.x = h[0] | (h[1] << 16);
      pk.y = h[2] | (h[3] << 16);
      pk.z = h[4] | (h[5] << 16);
      pk.w = h[6] | (h[7] << 16);
      u32x4* Mp = reinterpret_cast<u32x4*>(lib);
      __builtin_nontemporal_store(pk, Mp + grp * M + i);
    }
    b += db;
    a += da;
    if (b >= n) {
      b -= n;
      a += 1;
    }
  }

  // Column sums: fixed-order tree over the workgroup.
#pragma unroll
  for (int u = 0; u < 8; ++u) red[u][tid] = tacc[u];
  __syncthreads();
  for (int w = kBuildThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int u = 0; u < 8; ++u) red[u][tid] += red[u][tid + w];
    }
    __syncthreads();
  }
  if (tid < 8 && j0 + tid < ncols) tau[j0 + tid] = red[tid][0];
}

template <bool CUBIC>
static hipError_t launch_build_t(int storage, const float* pairs, const ColGeom* geo, int n,
                                 int64_t M, int64_t ncols, int64_t ncols_pad, void* lib,
                                 double* tau, hipStream_t s) {
  const int64_t groups = (ncols_pad + 7) / 8;
  const float2* P = reinterpret_cast<const float2*>(pairs);
  // gridDim.x is limited to 2^31-1 groups: far above any library that fits in memory.
  const dim3 grid((unsigned)groups);
  switch (storage) {
    case PSFLIB_FP32:
      build_kernel<PSFLIB_FP32, CUBIC><<<grid, kBuildThreads, 0, s>>>(P, geo, n, M, ncols, ncols_pad, lib, tau);
      break;
    case PSFLIB_BF16_POW2:
      build_kernel<PSFLIB_BF16_POW2, CUBIC><<<grid, kBuildThreads, 0, s>>>(P, geo, n, M, ncols, ncols_pad, lib, tau);
      break;
    default:
      build_kernel<PSFLIB_FP16_POW2, CUBIC><<<grid, kBuildThreads, 0, s>>>(P, geo, n, M, ncols, ncols_pad, lib, tau);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_build(int storage, const float* pairs, const ColGeom* geo, int n, int64_t M,
                        int64_t ncols, int64_t ncols_pad, void* lib, double* tau, hipStream_t s) {
  return launch_build_t<false>(storage, pairs, geo, n, M, ncols, ncols_pad, lib, tau, s);
}

hipError_t launch_build_cubic(int storage, const float* pairs, const ColGeom* geo, int n, int64_t M,
                              int64_t ncols, int64_t ncols_pad, void* lib, double* tau,
                              hipStream_t s) {
  return launch_build_t<true>(storage, pairs, geo, n, M, ncols, ncols_pad, lib, tau, s);
}

}  // namespace psflib
