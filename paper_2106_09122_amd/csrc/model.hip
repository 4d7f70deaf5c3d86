// Parametric exozodi disk rendered on the scene grid, and its parameter
// gradient: the model side of fitting a disk through the operator (the
// gradient analogue of the parameter retrieval the paper's conclusions plan).
//
// theta = (incl [rad], r0, width, gamma, flux), float64 in device memory:
//   rho = sqrt(x^2 + (y / cos incl)^2),  x = (q - (N-1)/2) S, y = (p - (N-1)/2) S
//   Z   = flux (rho/r0)^gamma exp(-(rho - r0)^2 / (2 width^2))
// and Z = 0 where rho = 0 or where the sky radius sqrt(x^2 + y^2) > rmax.
// Everything is evaluated in float64; the scene is stored as float32.
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

struct DiskTerms {
  bool live;
  double Z, dZdrho, rho, y;
};

__device__ __forceinline__ DiskTerms disk_terms(int64_t j, int N, double S, double rmax,
                                                const double* th) {
  DiskTerms d;
  const int64_t p = j / N, q = j - p * N;
  const double C = (double)(N - 1) * 0.5;
  const double x = ((double)q - C) * S, y = ((double)p - C) * S;
  const double ci = cos(th[0]);
  const double yc = y / ci;
  const double rho = sqrt(x * x + yc * yc);
  const double r = sqrt(x * x + y * y);
  d.live = rho > 0.0 && r <= rmax;
  d.rho = rho;
  d.y = y;
  d.Z = 0.0;
  d.dZdrho = 0.0;
  if (d.live) {
    const double r0 = th[1], w = th[2], g = th[3], F = th[4];
    const double dr = rho - r0;
    d.Z = F * exp(g * log(rho / r0) - dr * dr / (2.0 * w * w));
    d.dZdrho = d.Z * (g / rho - dr / (w * w));
  }
  return d;
}

__global__ __launch_bounds__(256) void render_disk_kernel(int N, double S, double rmax,
                                                          const double* __restrict__ theta,
                                                          float* __restrict__ Z) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= (int64_t)N * N) return;
  double th[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) th[k] = theta[k];
  Z[j] = (float)disk_terms(j, N, S, rmax, th).Z;
}

// dtheta_k = sum_j dZ_j dZ_j/dtheta_k in float64, in a fixed order: one
// pixel per thread, a tree per workgroup into partial[k][block], then one
// workgroup adds the block sums (each thread a strided run, then a tree).
constexpr int kGradThreads = 256;

__device__ __forceinline__ void tree256(double (*red)[kGradThreads], int tid) {
  for (int s = kGradThreads / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < 5; ++k) red[k][tid] += red[k][tid + s];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kGradThreads) void render_disk_grad_kernel(
    int N, double S, double rmax, const double* __restrict__ theta, const float* __restrict__ dZ,
    int64_t nblocks, double* __restrict__ partial) {
  __shared__ double red[5][kGradThreads];
  const int tid = threadIdx.x;
  double th[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) th[k] = theta[k];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t j = (int64_t)blockIdx.x * kGradThreads + tid;
  if (j < (int64_t)N * N) {
    const DiskTerms d = disk_terms(j, N, S, rmax, th);
    if (d.live) {
      const double ci = cos(th[0]), si = sin(th[0]);
      const double r0 = th[1], w = th[2], g = th[3], F = th[4];
      const double gz = (double)dZ[j] * d.Z;
      const double dr = d.rho - r0;
      acc[0] = (double)dZ[j] * d.dZdrho * (d.y * d.y * si / (ci * ci * ci * d.rho));
      acc[1] = gz * (-g / r0 + dr / (w * w));
      acc[2] = gz * dr * dr / (w * w * w);
      acc[3] = gz * log(d.rho / r0);
      acc[4] = gz / F;
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) red[k][tid] = acc[k];
  tree256(red, tid);
  if (tid < 5) partial[(int64_t)tid * nblocks + blockIdx.x] = red[tid][0];
}

__global__ __launch_bounds__(kGradThreads) void grad_sum_kernel(const double* __restrict__ partial,
                                                                int64_t nblocks,
                                                                double* __restrict__ dtheta) {
  __shared__ double red[5][kGradThreads];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double a = 0.0;
    for (int64_t b = tid; b < nblocks; b += kGradThreads) a += partial[k * nblocks + b];
    red[k][tid] = a;
  }
  tree256(red, tid);
  if (tid < 5) dtheta[tid] = red[tid][0];
}

// Chi-square misfit of a simulated image and its gradient in the image:
// t_i = (K S_i - D_i)^2 / var_i, grad_i = 2 K (K S_i - D_i) / var_i (float64,
// rounded once to float32).  Per-workgroup trees of t_i, then their sums in
// block order (chi2_sum_kernel), so the loss does not depend on scheduling.
__global__ __launch_bounds__(kGradThreads) void chi2_kernel(int64_t M, double K,
                                                            const float* __restrict__ S,
                                                            const double* __restrict__ D,
                                                            const double* __restrict__ var,
                                                            float* __restrict__ grad,
                                                            double* __restrict__ partial) {
  __shared__ double red[kGradThreads];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kGradThreads + tid;
  double t = 0.0;
  if (i < M) {
    const double r = K * (double)S[i] - D[i];
    const double v = var[i];
    t = r * r / v;
    if (grad) grad[i] = (float)((2.0 * K) * r / v);
  }
  red[tid] = t;
  for (int s2 = kGradThreads / 2; s2 > 0; s2 >>= 1) {
    __syncthreads();
    if (tid < s2) red[tid] += red[tid + s2];
  }
  if (tid == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kGradThreads) void chi2_sum_kernel(const double* __restrict__ partial,
                                                                int64_t nblocks,
                                                                double* __restrict__ loss) {
  __shared__ double red[kGradThreads];
  const int tid = threadIdx.x;
  double a = 0.0;
  for (int64_t b = tid; b < nblocks; b += kGradThreads) a += partial[b];
  red[tid] = a;
  for (int s2 = kGradThreads / 2; s2 > 0; s2 >>= 1) {
    __syncthreads();
    if (tid < s2) red[tid] += red[tid + s2];
  }
  if (tid == 0) *loss = red[0];
}

size_t chi2_scratch_bytes(int64_t M) {
  return (size_t)((M + kGradThreads - 1) / kGradThreads) * sizeof(double);
}

hipError_t launch_chi2(int64_t M, double K, const float* S, const double* D, const double* var,
                       double* loss, float* grad, void* scratch, hipStream_t s) {
  const int64_t nblocks = (M + kGradThreads - 1) / kGradThreads;
  double* partial = reinterpret_cast<double*>(scratch);
  chi2_kernel<<<(unsigned)nblocks, kGradThreads, 0, s>>>(M, K, S, D, var, grad, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  chi2_sum_kernel<<<1, kGradThreads, 0, s>>>(partial, nblocks, loss);
  return hipGetLastError();
}

size_t render_disk_grad_scratch_bytes(int N) {
  const int64_t nblocks = ((int64_t)N * N + kGradThreads - 1) / kGradThreads;
  return (size_t)nblocks * 5 * sizeof(double);
}

hipError_t launch_render_disk(int N, double S, double rmax, const double* theta, float* Z,
                              hipStream_t s) {
  const int64_t npix = (int64_t)N * N;
  render_disk_kernel<<<(unsigned)((npix + 255) / 256), 256, 0, s>>>(N, S, rmax, theta, Z);
  return hipGetLastError();
}

hipError_t launch_render_disk_grad(int N, double S, double rmax, const double* theta,
                                   const float* dZ, double* dtheta, void* scratch, hipStream_t s) {
  const int64_t nblocks = ((int64_t)N * N + kGradThreads - 1) / kGradThreads;
  double* partial = reinterpret_cast<double*>(scratch);
  render_disk_grad_kernel<<<(unsigned)nblocks, kGradThreads, 0, s>>>(N, S, rmax, theta, dZ,
                                                                     nblocks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  grad_sum_kernel<<<1, kGradThreads, 0, s>>>(partial, nblocks, dtheta);
  return hipGetLastError();
}

}  // namespace psflib
