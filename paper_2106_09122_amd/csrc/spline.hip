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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The padded coefficient pair is staged in LDS with 4 more zero rows and
// columns on every side (the extended array, Ne = Np + 8 per side, row
// stride ls >= Ne).  A pixel's tap origin is clamped to padded indices
// [-3, Np+1]: where that moves it, all 4 x 4 taps lay outside the padded
// array and the clamped taps all read the zero margin, so the value is still
// exactly zero; every tap is then a plain LDS read at a fixed offset from one
// base address, with no bounds tests or weight masking.
constexpr int kCubicMargin = 4;

__host__ __device__ inline int cubic_ext(int Np) { return Np + 2 * kCubicMargin; }

// row stride of the extended array: Ne rounded up to 5 mod 8 (spreads the
// taps of a near-vertical line over the banks, as in the bilinear build)
__host__ __device__ inline int cubic_stride(int Np) {
  const int ne = cubic_ext(Np);
  return ne + ((5 - ne % 8) + 8) % 8;
}

// Rows per LDS band of the extended array.
__host__ __device__ inline int cubic_band_rows(int Np) {
  const int h = (int)((size_t)kLdsBuildMaxBytes / ((size_t)cubic_stride(Np) * sizeof(float2)));
  const int ne = cubic_ext(Np);
  return h < ne ? h : ne;
}

// Cubic-spline build with the bracket's coefficient pair (C_k, C_{k+1}) staged
// in LDS.  When the extended array exceeds the LDS it is staged in bands of H
// rows that overlap by 3, band b holding extended rows [b (H-3), b (H-3) + H);
// the 4 tap rows of a pixel, from its (clamped) origin row R - 1 on, all lie
// in band min((R - 1) / (H-3), last), so each pixel is produced in exactly
// one band.  A work item is up to kLdsCols columns of one bracket (columns of
// the first half of the scene grid, and the centre of an odd grid, grouped on
// the device), one wave per column, which writes every element also to the
// half-turned column N^2-1-j at the mirrored pixel (n-1-a, n-1-b): that
// column's tap coordinates there are the same float64 values, so its entry is
// the same.  A wave walks its column in
// tiles of 8 x 8 image pixels (lane l: row 8 a' + l / 8, column 8 b' + l % 8),
// so the 64 stencils of one LDS read cover a compact rotated patch of the
// array rather than a 64-pixel line: with the row stride at 5 mod 8 pairs
// their 16-byte reads spread over the banks at any angle.  A store
// instruction writes 8 runs of 32 bytes; plain stores let L2 merge the runs
// of neighbouring tiles into whole lines (non-temporal ones were ~11% slower
// end to end).  Coordinates and
// B-spline weights in float64 (weights rounded once to float32); the 16 taps
// are summed separably in float32 — each row's weighted sum of the k and k+1
// coefficients, those rows weighted, then the radial blend — in the same
// order as the gather form, so both give identical values.
__global__ __launch_bounds__(1024) void build_cubic_lds_kernel(
    const float2* __restrict__ pairs, int Np, int ls, int H, int nbands,
    const ColGeom* __restrict__ geo, const int32_t* __restrict__ order,
    const int4* __restrict__ items, const int32_t* __restrict__ nitems, int nb, int n, int64_t M,
    int64_t ncols, float* __restrict__ A, double* __restrict__ tau) {
#pragma clang fp contract(off)
  extern __shared__ float2 band[];  // H rows of the extended array, stride ls
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, start = it.y, len = it.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane >> 3, lj = lane & 7;  // row and column of the lane in its tile
  const int nt = (n + 7) / 8;               // tiles per side
  if (bkt == nb - 1) {  // identically zero columns (uniform per workgroup)
    if (wave >= len) return;
    const int64_t j = order[start + wave], j2 = ncols - 1 - j;
    float* col = A + j * M;
    float* col2 = A + j2 * M;
    for (int a = 0; a < n; ++a)
      for (int b = lane; b < n; b += 64) {
        __builtin_nontemporal_store(0.0f, col + a * n + b);
        __builtin_nontemporal_store(0.0f, col2 + a * n + b);
      }
    if (lane == 0) tau[j] = tau[j2] = 0.0;
    return;
  }
  const float2* src = pairs + (int64_t)bkt * Np * Np;
  const int Ne = cubic_ext(Np);
  const bool live = wave < len;
  int64_t j = 0;
  ColGeom g;
  g.ct = 1.0; g.st = 0.0; g.w = 0.0;
  if (live) {
    j = order[start + wave];
    g = geo[j];
  }
  // the half turn of column j: column ncols-1-j, entry (n-1-a, n-1-b) = entry (a, b)
  // (its tap coordinates are the same float64 values, the products negated twice)
  const int64_t j2 = ncols - 1 - j;
  const bool pair = j2 != j;
  float* col = A + j * M;
  float* col2 = A + j2 * M;
  const double c = (double)(n - 1) * 0.5;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  const double pad = (double)kSplinePad;
  double tsum = 0.0;
  for (int bi = 0; bi < nbands; ++bi) {
    const int s0 = bi * (H - 3);
    const int rows = (Ne - s0 < H) ? Ne - s0 : H;
    const int hi = (bi == nbands - 1) ? Ne : s0 + H - 4;  // last origin row of this band
    __syncthreads();  // the previous band's reads are done
    for (int q = tid; q < rows * Ne; q += 1024) {
      const int r = q / Ne, cc = q - r * Ne;
      const int pr = s0 + r - kCubicMargin, pc = cc - kCubicMargin;
      float2 v = make_float2(0.0f, 0.0f);
      if ((unsigned)pr < (unsigned)Np && (unsigned)pc < (unsigned)Np) v = src[(int64_t)pr * Np + pc];
      band[r * ls + cc] = v;
    }
    __syncthreads();
    if (!live) continue;
    for (int ta = 0; ta < nt; ++ta) {
      const int a = 8 * ta + li;
      double stuy, ctuy;
      {
        const double uy = (double)a - c;
        stuy = g.st * uy;
        ctuy = g.ct * uy;
      }
      for (int tb = 0; tb < nt; ++tb) {
        const int b = 8 * tb + lj;
        if (a >= n || b >= n) continue;
        const double ux = (double)b - c;
        const double rowf = c + ((-g.st) * ux + ctuy) + pad;
        const double r0f = floor(rowf);
        int r0 = (int)r0f;  // |rowf| < 3n + pad: exact
        r0 = r0 < -3 ? -3 : (r0 > Np + 1 ? Np + 1 : r0);
        const int R = r0 + kCubicMargin - 1;  // extended row of the first tap
        if (R < s0 || R > hi) continue;
        const double colf = c + (g.ct * ux + stuy) + pad;
        const double c0f = floor(colf);
        int c0 = (int)c0f;
        c0 = c0 < -3 ? -3 : (c0 > Np + 1 ? Np + 1 : c0);
        float wy[4], wx[4];
        cubic_weights(rowf - r0f, wy);
        cubic_weights(colf - c0f, wx);
        const float2* t0 = band + (R - s0) * ls + (c0 + kCubicMargin - 1);
        float X = 0.0f, Y = 0.0f;
#pragma unroll
        for (int dr = 0; dr < 4; ++dr) {
          const float2* tr = t0 + dr * ls;
          const float2 p0 = tr[0], p1 = tr[1], p2 = tr[2], p3 = tr[3];
          float x = wx[0] * p0.x, y = wx[0] * p0.y;
          x = fmaf(wx[1], p1.x, x);
          y = fmaf(wx[1], p1.y, y);
          x = fmaf(wx[2], p2.x, x);
          y = fmaf(wx[2], p2.y, y);
          x = fmaf(wx[3], p3.x, x);
          y = fmaf(wx[3], p3.y, y);
          X = fmaf(wy[dr], x, X);
          Y = fmaf(wy[dr], y, Y);
        }
        const float val = fmaf(wk1, Y, wk0 * X);
        col[a * n + b] = val;
        if (pair) col2[(n - 1 - a) * n + (n - 1 - b)] = val;
        tsum += (double)val;
      }
    }
  }
  if (!live) return;
  tsum = wave_sum(tsum);
  if (lane == 0) {
    tau[j] = tsum;
    if (pair) tau[j2] = tsum;
  }
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

bool build_cubic_lds_supported(int n) {
  const int Np = n + 2 * kSplinePad;
  return n <= 256 && cubic_band_rows(Np) >= 16;
}

size_t build_cubic_lds_scratch_bytes(int K, int64_t ncols) { return bucket_scratch_bytes(K, ncols); }

hipError_t launch_build_cubic_lds(const float* pairs, int K, const ColGeom* geo, int n, int64_t M,
                                  int64_t ncols, float* A32, double* tau, void* scratch,
                                  hipStream_t s) {
  // the first half of the columns (and the centre of an odd grid), each
  // written with its half turn
  BucketPlan bp;
  hipError_t e = launch_bucket_sort(geo, (ncols + 1) / 2, K, scratch, &bp, s);
  if (e != hipSuccess) return e;
  const int Np = n + 2 * kSplinePad, Ne = cubic_ext(Np), ls = cubic_stride(Np);
  const int H = cubic_band_rows(Np);
  const int nbands = (H >= Ne) ? 1 : (Ne - 3 + (H - 3) - 1) / (H - 3);
  const size_t lds = (size_t)H * ls * sizeof(float2);
  const float2* P = reinterpret_cast<const float2*>(pairs);
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<(unsigned)bp.items_max, 1024, lds, s>>>(P, Np, ls, H, nbands, geo, bp.order, bp.items,
                                                   bp.nitems, bp.nb, n, M, ncols, A32, tau);
    return hipGetLastError();
  };
  return launch(build_cubic_lds_kernel);
}

}  // namespace psflib
