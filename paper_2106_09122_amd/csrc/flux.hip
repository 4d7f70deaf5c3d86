// Optional flux-preserving column rescale.
//
// Rotating the radially interpolated PSF Q inside a fixed n x n frame (Sec. 2)
// loses the part of Q carried out of the frame, and a cubic spline's
// overshoot changes the total slightly.  With PSFLIB_FLUX_PRESERVE each
// column is scaled by t_j / tau_j, where t_j = (1-w) sum(P_k) + w sum(P_{k+1})
// is the flux of Q and tau_j the column's own sum, so the column carries the
// flux of the PSF it was interpolated from.  The scale is applied to the
// float32 column (one rounding), the column sum is recomputed from the
// stored values, and for the 16-bit forms the column exponent is recomputed
// from the rescaled bound before the column is rounded.  The orbit builds do
// this in two passes instead of rewriting the library: the column sums of the
// plain build (nothing stored), the scales (flux_scale_kernel), then the build
// with every value scaled as it is stored: the plain build's entries rescaled.
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

namespace {

__device__ inline int32_t exponent_of(double m) {  // m * 2^-e in [2^14, 2^15); kZeroColumnExp for m == 0
  if (m == 0.0) return kZeroColumnExp;
  int E;
  (void)frexp(m, &E);
  return E - 15;
}

// sums[k] = sum_p P_k[p] in float64, fixed-order tree; one workgroup per PSF.
__global__ __launch_bounds__(256) void psf_sums_kernel(const float* __restrict__ cube, int64_t M,
                                                       double* __restrict__ sums) {
  __shared__ double red[256];
  const float* P = cube + (int64_t)blockIdx.x * M;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < M; i += 256) acc += (double)P[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// One workgroup per column.
__global__ __launch_bounds__(256) void flux_rescale_kernel(
    float* __restrict__ A32, ColGeom* __restrict__ geo, int K, const double* __restrict__ sums,
    const float* __restrict__ pmax, int64_t M, double* __restrict__ tau,
    int32_t* __restrict__ exps, int want_exp) {
  __shared__ double red[256];
  const int64_t j = blockIdx.x;
  const ColGeom g = geo[j];
  if (g.k < 0) return;  // identically zero column: nothing to scale
  const double t = (K == 1) ? sums[0] : (1.0 - g.w) * sums[g.k] + g.w * sums[g.k + 1];
  const double old = tau[j];
  const double scale = (old != 0.0) ? t / old : 1.0;
  const float sf = (float)scale;
  float* col = A32 + j * M;
  double acc = 0.0;
  if ((M & 3) == 0 && (reinterpret_cast<uintptr_t>(col) & 15) == 0) {
    // 16-byte pieces, 8 loads of a thread in flight before their use
    f32x4* c4 = reinterpret_cast<f32x4*>(col);
    const int64_t nq = M >> 2;
    for (int64_t q0 = threadIdx.x; q0 < nq; q0 += 256 * 8) {
      f32x4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t q = q0 + 256 * u;
        if (q < nq) v[u] = __builtin_nontemporal_load(c4 + q);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t q = q0 + 256 * u;
        if (q < nq) {
          const f32x4 x = v[u] * sf;
          __builtin_nontemporal_store(x, c4 + q);
          acc += ((double)x[0] + (double)x[1]) + ((double)x[2] + (double)x[3]);
        }
      }
    }
  } else {
    for (int64_t i = threadIdx.x; i < M; i += 256) {
      const float v = col[i] * sf;
      col[i] = v;
      acc += (double)v;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tau[j] = red[0];
    if (want_exp) {
      const double bound = (K == 1) ? (double)pmax[0]
                                    : (1.0 - g.w) * (double)pmax[g.k] + g.w * (double)pmax[g.k + 1];
      const int32_t e = exponent_of(bound * fabs((double)sf));
      geo[j].e = e;
      exps[j] = e;
    }
  }
}

// The scales alone (the orbit builds apply them as they store): for column j
// the float32 scale t_j / tau_j of flux_rescale_kernel from the plain build's
// column sum, and for the 16-bit forms the exponent from the rescaled bound;
// identically zero columns keep scale 1 and their exponent.
__global__ __launch_bounds__(256) void flux_scale_kernel(ColGeom* __restrict__ geo, int K,
                                                         const double* __restrict__ sums,
                                                         const float* __restrict__ pmax,
                                                         int64_t ncols, const double* __restrict__ tau,
                                                         float* __restrict__ colscale,
                                                         int32_t* __restrict__ exps, int want_exp) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= ncols) return;
  const ColGeom g = geo[j];
  if (g.k < 0) {
    colscale[j] = 1.0f;
    return;
  }
  const double t = (K == 1) ? sums[0] : (1.0 - g.w) * sums[g.k] + g.w * sums[g.k + 1];
  const double old = tau[j];
  const double scale = (old != 0.0) ? t / old : 1.0;
  const float sf = (float)scale;
  colscale[j] = sf;
  if (want_exp) {
    const double bound = (K == 1) ? (double)pmax[0]
                                  : (1.0 - g.w) * (double)pmax[g.k] + g.w * (double)pmax[g.k + 1];
    const int32_t e = exponent_of(bound * fabs((double)sf));
    geo[j].e = e;
    exps[j] = e;
  }
}

}  // namespace

hipError_t launch_flux_scale(ColGeom* geo, int K, const double* sums, const float* pmax,
                             int64_t ncols, const double* tau, float* colscale, int32_t* exps,
                             bool want_exp, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  flux_scale_kernel<<<(unsigned)((ncols + 255) / 256), 256, 0, s>>>(geo, K, sums, pmax, ncols, tau,
                                                                    colscale, exps, want_exp ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_psf_sums(const float* cube, int K, int64_t M, double* sums, hipStream_t s) {
  psf_sums_kernel<<<K, 256, 0, s>>>(cube, M, sums);
  return hipGetLastError();
}

hipError_t launch_flux_rescale(float* A32, ColGeom* geo, int K, const double* sums,
                               const float* pmax, int64_t M, int64_t ncols, double* tau,
                               int32_t* exps, bool want_exp, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  flux_rescale_kernel<<<(unsigned)ncols, 256, 0, s>>>(A32, geo, K, sums, pmax, M, tau, exps,
                                                      want_exp ? 1 : 0);
  return hipGetLastError();
}

}  // namespace psflib
