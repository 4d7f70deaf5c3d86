// Cubic-spline rotation, part 1: spline coefficients of the sampled PSFs.
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Rows per LDS band of the padded coefficient pair (Np pairs per row).
__host__ __device__ inline int cubic_band_rows(int Np) {
  const int h = (int)((size_t)kLdsBuildMaxBytes / ((size_t)Np * sizeof(float2)));
  return h < Np ? h : Np;
}

// Cubic-spline build with the bracket's coefficient pair (C_k, C_{k+1}) staged
// in LDS.  The padded pair has Np x Np entries; when that exceeds the LDS it
// is staged in bands of H rows that overlap by 3, band b holding rows
// [b (H-3), b (H-3) + H).  The 4 tap rows of an output pixel, r0-1 .. r0+2,
// all lie in band floor(max(r0-1, 0) / (H-3)) (the last band for rows near
// the bottom), so each pixel is produced in exactly one band.  A work item is
// up to kLdsCols columns of one bracket (columns grouped on the device), one
// wave per column, lane l owning image columns l, l+64, ...; coordinates and
// B-spline weights in float64 (weights rounded once to float32), the weight
// products, blended taps and the 16-term sum in float32 in the same order as
// the gather form, so both forms give identical values.
template <int E, bool FULL>
__global__ __launch_bounds__(1024) void build_cubic_lds_kernel(
    const float2* __restrict__ pairs, int Np, int H, int nbands, const ColGeom* __restrict__ geo,
    const int32_t* __restrict__ order, const int4* __restrict__ items,
    const int32_t* __restrict__ nitems, int nb, int n, int64_t M, float* __restrict__ A,
    double* __restrict__ tau) {
#pragma clang fp contract(off)
  extern __shared__ float2 band[];  // H rows of Np pairs
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, start = it.y, len = it.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (bkt == nb - 1) {  // identically zero columns (uniform per workgroup)
    if (wave >= len) return;
    const int64_t j = order[start + wave];
    float* col = A + j * M;
    for (int a = 0; a < n; ++a)
#pragma unroll
      for (int v = 0; v < E; ++v) {
        const int b = lane + 64 * v;
        if (FULL || b < n) __builtin_nontemporal_store(0.0f, col + a * n + b);
      }
    if (lane == 0) tau[j] = 0.0;
    return;
  }
  const float2* src = pairs + (int64_t)bkt * Np * Np;
  const bool live = wave < len;
  int64_t j = 0;
  ColGeom g;
  g.ct = 1.0; g.st = 0.0; g.w = 0.0;
  if (live) {
    j = order[start + wave];
    g = geo[j];
  }
  float* col = A + j * M;
  const double c = (double)(n - 1) * 0.5;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  double ctux[E], mstux[E];
#pragma unroll
  for (int v = 0; v < E; ++v) {
#pragma clang fp contract(off)
    const double ux = (double)(lane + 64 * v) - c;
    ctux[v] = g.ct * ux;
    mstux[v] = (-g.st) * ux;
  }
  const double pad = (double)kSplinePad;
  double tsum = 0.0;
  for (int bi = 0; bi < nbands; ++bi) {
    const int s0 = bi * (H - 3);
    const int rows = (Np - s0 < H) ? Np - s0 : H;
    __syncthreads();  // the previous band's reads are done
    const float2* bsrc = src + (int64_t)s0 * Np;
    for (int q = tid; q < rows * Np; q += 1024) band[q] = bsrc[q];
    __syncthreads();
    if (!live) continue;
    for (int a = 0; a < n; ++a) {
      double stuy, ctuy;
      {
#pragma clang fp contract(off)
        const double uy = (double)a - c;
        stuy = g.st * uy;
        ctuy = g.ct * uy;
      }
      float rowsum = 0.0f;
#pragma unroll
      for (int v = 0; v < E; ++v) {
        const int b = lane + 64 * v;
        if (!(FULL || b < n)) continue;
        const double sy = mstux[v] + ctuy;
        const double rowf = c + sy + pad;
        const double r0f = floor(rowf);
        const int r0 = (int)r0f;
        int rl = r0 - 1 > 0 ? r0 - 1 : 0;
        int mine = rl / (H - 3);
        if (mine > nbands - 1) mine = nbands - 1;
        if (mine != bi) continue;
        const double sx = ctux[v] + stuy;
        const double colf = c + sx + pad;
        const double c0f = floor(colf);
        const int c0 = (int)c0f;
        float wy[4], wx[4];
        cubic_weights(rowf - r0f, wy);
        cubic_weights(colf - c0f, wx);
        // taps outside the padded array are zero: their weight is zeroed and
        // their LDS address clamped into the band (no branches)
        int rofs[4], cidx[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int r = r0 + d - 1, cc = c0 + d - 1;
          if ((unsigned)r >= (unsigned)Np) wy[d] = 0.0f;
          if ((unsigned)cc >= (unsigned)Np) wx[d] = 0.0f;
          const int rb = r - s0;
          rofs[d] = (rb < 0 ? 0 : (rb > rows - 1 ? rows - 1 : rb)) * Np;
          cidx[d] = cc < 0 ? 0 : (cc > Np - 1 ? Np - 1 : cc);
        }
        float val = 0.0f;
#pragma unroll
        for (int dr = 0; dr < 4; ++dr) {
#pragma unroll
          for (int dc = 0; dc < 4; ++dc) {
            const float2 p = band[rofs[dr] + cidx[dc]];
            val = fmaf(wy[dr] * wx[dc], fmaf(wk1, p.y, wk0 * p.x), val);
          }
        }
        __builtin_nontemporal_store(val, col + a * n + b);
        rowsum += val;
      }
      tsum += (double)rowsum;
    }
  }
  if (!live) return;
  tsum = wave_sum(tsum);
  if (lane == 0) tau[j] = tsum;
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
  const unsigned lines = (unsigned)(((int64_t)K * Np + 255) / 256);
  spline_cols_kernel<<<lines, 256, 0, s>>>(cube, K, n, Np, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  spline_rows_kernel<<<lines, 256, 0, s>>>(K, Np, T);
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

bool build_cubic_lds_supported(int n) {
  const int Np = n + 2 * kSplinePad;
  return n <= 256 && cubic_band_rows(Np) >= 16;
}

size_t build_cubic_lds_scratch_bytes(int K, int64_t ncols) { return bucket_scratch_bytes(K, ncols); }

hipError_t launch_build_cubic_lds(const float* pairs, int K, const ColGeom* geo, int n, int64_t M,
                                  int64_t ncols, float* A32, double* tau, void* scratch,
                                  hipStream_t s) {
  BucketPlan bp;
  hipError_t e = launch_bucket_sort(geo, ncols, K, scratch, &bp, s);
  if (e != hipSuccess) return e;
  const int Np = n + 2 * kSplinePad;
  const int H = cubic_band_rows(Np);
  const int nbands = (H >= Np) ? 1 : (Np - 3 + (H - 3) - 1) / (H - 3);
  const size_t lds = (size_t)H * Np * sizeof(float2);
  const float2* P = reinterpret_cast<const float2*>(pairs);
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<(unsigned)bp.items_max, 1024, lds, s>>>(P, Np, H, nbands, geo, bp.order, bp.items,
                                                   bp.nitems, bp.nb, n, M, A32, tau);
    return hipGetLastError();
  };
  const bool full = (n % 64) == 0;
  switch ((n + 63) / 64) {
    case 1: return full ? launch(build_cubic_lds_kernel<1, true>) : launch(build_cubic_lds_kernel<1, false>);
    case 2: return full ? launch(build_cubic_lds_kernel<2, true>) : launch(build_cubic_lds_kernel<2, false>);
    case 3: return full ? launch(build_cubic_lds_kernel<3, true>) : launch(build_cubic_lds_kernel<3, false>);
    default: return full ? launch(build_cubic_lds_kernel<4, true>) : launch(build_cubic_lds_kernel<4, false>);
  }
}

}  // namespace psflib
