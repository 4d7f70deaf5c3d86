// Cubic-spline rotation: spline coefficients of the sampled PSFs, which the
// cubic orbit build (build_lds.hip) and the cubic gather (build.hip) sample.
//
// The rotation step of Sec. 2 uses SciPy's rotate(), whose default
// interpolation is a cubic spline.  The spline that interpolates a PSF
// extended by zeros, f(x) = sum_m c_m beta3(x - m), has coefficients c that
// are the samples passed through the cubic B-spline interpolation filter.
// Here every sampled PSF P_k is padded by kSplinePad zero pixels per side and
// filtered (float64) along columns, then along rows, with the exact recursive
// filter for a mirror-symmetric extension of the padded array: gain 6, a
// causal and an anticausal first-order recursion with pole z = sqrt(3) - 2,
// the causal start summing the mirrored line over one period.  Because the
// filter is linear, the coefficients of a radially interpolated PSF
// Q = (1-w) P_k + w P_{k+1} are (1-w) C_k + w C_{k+1}, so the build blends
// coefficient pairs exactly as the bilinear build blends sample pairs.
//
// Output in scratch: the float64 coefficients [K][Np][Np] (Np = n + 2 pad),
// then radial pairs (C_k, C_{k+1}) rounded to float32, and per PSF the largest
// |coefficient| (which bounds the column for the 16-bit exponents: the spline
// value is a convex combination of coefficients).
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

namespace {

constexpr double kPole = -0.26794919243112270;  // sqrt(3) - 2

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// In-place interpolation filter of one line of N >= 2 float64 values with
// element stride st.
__device__ void spline_line(double* x, int64_t st, int N) {
#pragma clang fp contract(off)
  const double z = kPole;
  // causal start: sum over one period of the mirrored line (c = 6 s):
  // c_0 + z^{N-1} c_{N-1} + sum_{k=1}^{N-2} (z^k + z^{2N-2-k}) c_k, / (1 - z^{2N-2})
  double head = 0.0, zk = 1.0;
  for (int k = 0; k < N - 1; ++k) {  // z^k c_k, k = 0 .. N-2
    head += zk * (6.0 * x[k * st]);
    zk *= z;
  }
  // zk = z^{N-1}
  const double zN1 = zk;
  double tail = 0.0, q = z;
  for (int k = N - 2; k >= 1; --k) {  // z^{N-1-k} c_k
    tail += q * (6.0 * x[k * st]);
    q *= z;
  }
  const double start = (head + zN1 * (6.0 * x[(int64_t)(N - 1) * st]) + zN1 * tail) /
                       (1.0 - zN1 * zN1);
  // causal recursion c+_i = c_i + z c+_{i-1}, in place
  double prev = start;
  x[0] = start;
  for (int i = 1; i < N; ++i) {
    prev = 6.0 * x[i * st] + z * prev;
    x[i * st] = prev;
  }
  // anticausal: c-_{N-1} = z/(z^2-1) (c+_{N-1} + z c+_{N-2}); c-_i = z (c-_{i+1} - c+_i)
  double next = (z / (z * z - 1.0)) * (x[(int64_t)(N - 1) * st] + z * x[(int64_t)(N - 2) * st]);
  x[(int64_t)(N - 1) * st] = next;
  for (int i = N - 2; i >= 0; --i) {
    next = z * (next - x[i * st]);
    x[i * st] = next;
  }
}

// Column pass: thread = (k, column q) of the padded image; loads the padded
// column from the cube, filters it.
__global__ __launch_bounds__(256) void spline_cols_kernel(const float* __restrict__ cube, int K,
                                                          int n, int Np, double* __restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)K * Np) return;
  const int64_t k = t / Np;
  const int q = (int)(t - k * Np);
  double* col = T + k * (int64_t)Np * Np + q;
  const int b = q - kSplinePad;
  for (int i = 0; i < Np; ++i) {
    const int a = i - kSplinePad;
    const bool in = (unsigned)a < (unsigned)n && (unsigned)b < (unsigned)n;
    col[(int64_t)i * Np] = in ? (double)cube[(k * n + a) * (int64_t)n + b] : 0.0;
  }
  spline_line(col, Np, Np);
}

// Row pass: thread = (k, row i).
__global__ __launch_bounds__(256) void spline_rows_kernel(int K, int Np, double* __restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)K * Np) return;
  spline_line(T + t * Np, 1, Np);
}

// The same two passes with the lines staged in LDS: a workgroup loads a tile
// of W lines (coalesced, all 4 waves), one lane per line runs the recursion
// on LDS, and the tile is written back by all 4 waves.  The recursions are sequential
// along a line, so this trades global-memory latency per step for LDS latency.
// Column pass: tile = Np rows x W columns of one padded PSF, [row][column].
__global__ __launch_bounds__(256) void spline_cols_lds_kernel(const float* __restrict__ cube, int n,
                                                             int Np, int W,
                                                             double* __restrict__ T) {
  extern __shared__ double tile[];  // Np x W
  const int nblk = (Np + W - 1) / W;
  const int64_t k = blockIdx.x / nblk;
  const int q0 = (int)(blockIdx.x % nblk) * W;
  const int tid = threadIdx.x;
  for (int e = tid; e < Np * W; e += 256) {
    const int i = e / W, dq = e - i * W;
    const int a = i - kSplinePad, b = q0 + dq - kSplinePad;
    const bool in = (unsigned)a < (unsigned)n && (unsigned)b < (unsigned)n;
    tile[e] = in ? (double)cube[(k * n + a) * (int64_t)n + b] : 0.0;
  }
  __syncthreads();
  if (tid < W && q0 + tid < Np) spline_line(tile + tid, W, Np);
  __syncthreads();
  double* dst = T + k * (int64_t)Np * Np;
  for (int e = tid; e < Np * W; e += 256) {
    const int i = e / W, dq = e - i * W;
    if (q0 + dq < Np) dst[(int64_t)i * Np + q0 + dq] = tile[e];
  }
}

// Row pass: tile = W rows of Np, row stride Np + 1 (an odd number of doubles
// spreads the lanes' rows over the LDS banks).
__global__ __launch_bounds__(256) void spline_rows_lds_kernel(int Np, int W,
                                                             double* __restrict__ T) {
  extern __shared__ double tile[];  // W x (Np + 1)
  const int nblk = (Np + W - 1) / W;
  const int64_t k = blockIdx.x / nblk;
  const int i0 = (int)(blockIdx.x % nblk) * W;
  const int rows = (Np - i0 < W) ? Np - i0 : W;
  const int st = Np + 1;
  const int tid = threadIdx.x;
  double* src = T + (k * (int64_t)Np + i0) * Np;
  for (int e = tid; e < rows * Np; e += 256) {
    const int r = e / Np, c = e - r * Np;
    tile[r * st + c] = src[e];
  }
  __syncthreads();
  if (tid < rows) spline_line(tile + tid * st, 1, Np);
  __syncthreads();
  for (int e = tid; e < rows * Np; e += 256) {
    const int r = e / Np, c = e - r * Np;
    src[e] = tile[r * st + c];
  }
}

// Lines per LDS tile (64, 32 or 16 lines of Np doubles), 0 if none fits.
int spline_tile_lines(int Np) {
  for (int W = 64; W >= 16; W >>= 1)
    if ((size_t)W * (size_t)(Np + 1) * sizeof(double) <= (size_t)kLdsBuildMaxBytes) return W;
  return 0;
}

// pairs[k][p] = (C_k[p], C_{k+1}[p]) in float32 (C_1 reads as 0 when K == 1).
__global__ __launch_bounds__(256) void spline_pair_kernel(const double* __restrict__ T, int K,
                                                          int64_t P, float2* __restrict__ pairs) {
  const int64_t npairs = (K > 1) ? (int64_t)(K - 1) : 1;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < npairs * P;
       t += (int64_t)gridDim.x * 256) {
    const int64_t k = t / P, p = t - k * P;
    float2 v;
    v.x = (float)T[k * P + p];
    v.y = (K > 1) ? (float)T[(k + 1) * P + p] : 0.0f;
    pairs[t] = v;
  }
}

// cmax[k] = max_p |float(C_k[p])|, one workgroup per PSF.
__global__ __launch_bounds__(256) void spline_absmax_kernel(const double* __restrict__ T,
                                                            int64_t P, float* __restrict__ cmax) {
  __shared__ float red[256];
  const double* C = T + (int64_t)blockIdx.x * P;
  float m = 0.0f;
  for (int64_t i = threadIdx.x; i < P; i += 256) m = fmaxf(m, fabsf((float)C[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) cmax[blockIdx.x] = red[0];
}

}  // namespace

size_t spline_scratch_bytes(int K, int n) {
  const int64_t Np = (int64_t)n + 2 * kSplinePad, P = Np * Np;
  const int64_t npairs = (K > 1) ? (int64_t)(K - 1) : 1;
  return align256((size_t)K * (size_t)P * 8) + align256((size_t)npairs * (size_t)P * 8);
}

const float* spline_pairs_of(const void* scratch, int K, int n) {
  const int64_t Np = (int64_t)n + 2 * kSplinePad, P = Np * Np;
  return reinterpret_cast<const float*>(reinterpret_cast<const char*>(scratch) +
                                        align256((size_t)K * (size_t)P * 8));
}

hipError_t launch_spline_pairs(const float* cube, int K, int n, void* scratch, float* cmax,
                               hipStream_t s) {
  const int Np = n + 2 * kSplinePad;
  const int64_t P = (int64_t)Np * Np;
  double* T = reinterpret_cast<double*>(scratch);
  float2* pairs = reinterpret_cast<float2*>(const_cast<float*>(spline_pairs_of(scratch, K, n)));
  const int W = spline_tile_lines(Np);
  hipError_t e;
  if (W > 0) {
    const size_t lds = (size_t)W * (size_t)(Np + 1) * sizeof(double);
    const unsigned tiles = (unsigned)((int64_t)K * ((Np + W - 1) / W));
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(spline_cols_lds_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(spline_rows_lds_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    spline_cols_lds_kernel<<<tiles, 256, lds, s>>>(cube, n, Np, W, T);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    spline_rows_lds_kernel<<<tiles, 256, lds, s>>>(Np, W, T);
  } else {
    const unsigned lines = (unsigned)(((int64_t)K * Np + 255) / 256);
    spline_cols_kernel<<<lines, 256, 0, s>>>(cube, K, n, Np, T);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    spline_rows_kernel<<<lines, 256, 0, s>>>(K, Np, T);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = ((K > 1) ? (int64_t)(K - 1) : 1) * P;
  const int64_t want = (total + 255) / 256;
  spline_pair_kernel<<<(unsigned)(want < 65536 ? want : 65536), 256, 0, s>>>(T, K, P, pairs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (cmax) {
    spline_absmax_kernel<<<K, 256, 0, s>>>(T, P, cmax);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace psflib
