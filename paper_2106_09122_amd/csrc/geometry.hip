// Scene geometry and radial brackets of every library column, plus the two
// small preparations of the PSF datacube used by the build.
//
// Paper: Sec. 2, Eqs. (2)-(3) (half-pixel-shifted meshgrid scaled by the
// scene pixel scale, flattened row-major), the polar conversion of each field
// point, and the radial interpolation of the datacube (linear or nearest).
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

// Largest value of each sampled PSF (exact float32 max); used for the 16-bit
// column exponents.  One workgroup per PSF, four independent loads in flight
// per thread.
__global__ __launch_bounds__(1024) void cube_max_kernel(const float* __restrict__ cube, int64_t M,
                                                        float* __restrict__ pmax) {
  __shared__ float red[16];
  const float* P = cube + (int64_t)blockIdx.x * M;
  float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
  int64_t i = threadIdx.x;
  for (; i + 3 * 1024 < M; i += 4 * 1024) {
    m0 = fmaxf(m0, P[i]);
    m1 = fmaxf(m1, P[i + 1024]);
    m2 = fmaxf(m2, P[i + 2 * 1024]);
    m3 = fmaxf(m3, P[i + 3 * 1024]);
  }
  for (; i < M; i += 1024) m0 = fmaxf(m0, P[i]);
  float m = fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x < 64) {
    m = threadIdx.x < 16 ? red[threadIdx.x] : 0.0f;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if (threadIdx.x == 0) pmax[blockIdx.x] = m;
  }
}

// pairs[k][p] = (P_k[p], P_{k+1}[p]) for k < max(K-1, 1), so one 8-byte load
// fetches both radial neighbours of a tap (P_1 reads as 0 when K == 1).
__global__ __launch_bounds__(256) void pair_cube_kernel(const float* __restrict__ cube, int K,
                                                        int64_t M, float2* __restrict__ pairs) {
  const int64_t npairs = (K > 1) ? (int64_t)(K - 1) : 1;
  const int64_t total = npairs * M;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t k = t / M, p = t - k * M;
    float2 v;
    v.x = cube[k * M + p];
    v.y = (K > 1) ? cube[(k + 1) * M + p] : 0.0f;
    pairs[t] = v;
  }
}

// Power-of-two exponent e with m * 2^-e in [2^14, 2^15); kZeroColumnExp for
// m == 0 (a zero column has no scale: with this exponent every scene value
// at the column scales to exactly 0, so it can neither set a scene's
// exponent nor overflow the 16-bit format).
__device__ inline int32_t scale_exponent(double m) {
  if (m == 0.0) return kZeroColumnExp;
  int E;
  (void)frexp(m, &E);  // m = f * 2^E, f in [0.5, 1)
  return E - 15;
}

// One thread per column j (and per padding column up to ncols_pad).
__global__ __launch_bounds__(256) void geometry_kernel(int N, double S,
                                                       const double* __restrict__ radii, int K,
                                                       int interp, int oob,
                                                       const float* __restrict__ pmax,
                                                       int want_exp, ColGeom* __restrict__ geo,
                                                       int64_t ncols_pad,
                                                       int32_t* __restrict__ exps) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ncols = (int64_t)N * N;
  if (j >= ncols_pad) return;
  ColGeom g;
  g.pad[0] = g.pad[1] = 0;
  if (j >= ncols) {  // padding column of the 16-bit layout: identically zero
    g.r = 0.0; g.ct = 1.0; g.st = 0.0; g.w = 0.0; g.k = -1; g.e = want_exp ? kZeroColumnExp : 0;
    geo[j] = g;
    if (exps) exps[j] = g.e;
    return;
  }
  const int64_t p = j / N, q = j - p * N;
  // Eqs. (2)-(3): centre offsets (q - (N-1)/2) S and (p - (N-1)/2) S.
  const double C = (double)(N - 1) * 0.5;
  const double x = ((double)q - C) * S;
  const double y = ((double)p - C) * S;
  const double r = sqrt(x * x + y * y);
  double ct = 1.0, st = 0.0;  // atan2(0, 0) = 0
  if (r > 0.0) {
    ct = x / r;
    st = y / r;
  }
  // Radial bracket: Q = (1-w) P_k + w P_{k+1}.
  int k = 0;
  double w = 0.0;
  bool zero = false;
  if (K > 1) {
    if (r <= radii[0]) {
      k = 0; w = 0.0;
    } else if (r >= radii[K - 1]) {
      k = K - 2; w = 1.0;
      if (oob == PSFLIB_OOB_ZERO && r > radii[K - 1]) zero = true;
    } else {
      int lo = 0, hi = K - 1;  // radii[lo] <= r < radii[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (radii[mid] <= r) lo = mid; else hi = mid;
      }
      k = lo;
      const double a = radii[lo], b = radii[lo + 1];
      if (interp == PSFLIB_INTERP_NEAREST)
        w = ((r - a) > (b - r)) ? 1.0 : 0.0;  // ties go to the lower sample
      else
        w = (r - a) / (b - a);
    }
  }
  g.r = r; g.ct = ct; g.st = st; g.w = zero ? 0.0 : w; g.k = zero ? -1 : k;
  g.e = want_exp ? kZeroColumnExp : 0;
  if (want_exp && !zero) {
    // Bound on the column's largest value: bilinear rotation is a convex
    // combination of Q's pixels (or zero), so max_i A_ij <= max Q.
    const double bound = (K == 1) ? (double)pmax[0]
                                  : (1.0 - w) * (double)pmax[k] + w * (double)pmax[k + 1];
    g.e = scale_exponent(bound);
  }
  geo[j] = g;
  if (exps) exps[j] = g.e;
}

__global__ __launch_bounds__(256) void export_geometry_kernel(const ColGeom* __restrict__ geo,
                                                              int64_t ncols,
                                                              double* __restrict__ geom,
                                                              int32_t* __restrict__ kout) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= ncols) return;
  const ColGeom g = geo[j];
  if (geom) {
    geom[4 * j + 0] = g.r;
    geom[4 * j + 1] = g.ct;
    geom[4 * j + 2] = g.st;
    geom[4 * j + 3] = g.w;
  }
  if (kout) kout[j] = g.k;
}

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_cube_max(const float* cube, int K, int64_t M, float* pmax, hipStream_t s) {
  cube_max_kernel<<<K, 1024, 0, s>>>(cube, M, pmax);
  return hipGetLastError();
}

hipError_t launch_pair_cube(const float* cube, int K, int64_t M, float* pairs, hipStream_t s) {
  const int64_t total = ((K > 1) ? (int64_t)(K - 1) : 1) * M;
  const int64_t want = (total + 255) / 256;
  const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
  pair_cube_kernel<<<grid, 256, 0, s>>>(cube, K, M, reinterpret_cast<float2*>(pairs));
  return hipGetLastError();
}

hipError_t launch_geometry(int N, double S, const double* radii, int K, int interp, int oob,
                           const float* pmax, bool want_exp, ColGeom* geo, int64_t ncols_pad,
                           int32_t* exps, hipStream_t s) {
  geometry_kernel<<<blocks_for(ncols_pad, 256), 256, 0, s>>>(N, S, radii, K, interp, oob, pmax,
                                                            want_exp ? 1 : 0, geo, ncols_pad, exps);
  return hipGetLastError();
}

hipError_t launch_export_geometry(const ColGeom* geo, int64_t ncols, double* geom, int32_t* k,
                                  hipStream_t s) {
  export_geometry_kernel<<<blocks_for(ncols, 256), 256, 0, s>>>(geo, ncols, geom, k);
  return hipGetLastError();
}

}  // namespace psflib
