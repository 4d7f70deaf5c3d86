// Single-scene products with the library: S = A Z (Sec. 3, Eq. (6)) and the
// adjoint G = A^T g.  Both stream the library once from HBM and are bound by
// memory bandwidth; the scene and image vectors are small and stay in cache.
//
// A is column-major (column j is contiguous), so the forward product is a sum
// of scaled columns.  It is split over (row block, column chunk) workgroups:
// each thread owns 4 consecutive rows, walks the chunk's columns with one
// 16-byte non-temporal load per column, and writes a partial image; a second
// kernel adds the partials in a fixed order.  Sums are blocked (16 columns per
// inner sum) so every rounding chain stays short.  Results are bitwise
// reproducible.
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

// ------------------------------------------------------------ forward -----
// Split-K with the reduction fused into the same launch: every workgroup
// writes its partial rows, then counts itself in per row block; the last
// workgroup of a row block to arrive adds the partials of that block in chunk
// order (so the result does not depend on which workgroup finishes last) and
// resets the counter for the next call.
__device__ __forceinline__ bool arrive_last(int32_t* counter, int expected) {
  __shared__ int last;
  __threadfence();  // publish this workgroup's partials device-wide
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1) == expected - 1);
  __syncthreads();
  if (last) __threadfence();  // see every other workgroup's partials
  return last;
}

template <bool VEC>
__global__ __launch_bounds__(kMvThreads) void matvec_f32_kernel(const float* __restrict__ A,
                                                                const float* __restrict__ Z,
                                                                float* __restrict__ part,
                                                                int32_t* __restrict__ counters,
                                                                float* __restrict__ out,
                                                                int64_t M, int64_t ncols) {
  const int64_t i0 = ((int64_t)blockIdx.x * kMvThreads + threadIdx.x) * 4;
  const int64_t c = blockIdx.y;
  const int64_t nchunks = gridDim.y;
  const int64_t j0 = c * kMvChunk;
  const int64_t j1 = (j0 + kMvChunk < ncols) ? j0 + kMvChunk : ncols;
  const bool active = i0 < M;
  const bool full = VEC && (i0 + 4 <= M);
  f32x4 outer = {0.f, 0.f, 0.f, 0.f};
  f32x4 inner = {0.f, 0.f, 0.f, 0.f};
  if (active) {
    int64_t j = j0;
    for (; j + 8 <= j1; j += 8) {
      f32x4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float* col = A + (j + u) * M + i0;
        if (full) {
          v[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[u][e] = (i0 + e < M) ? col[e] : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) inner += v[u] * Z[j + u];
      if (((j - j0) & 15) == 8) {
        outer += inner;
        inner = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
    }
    for (; j < j1; ++j) {
      const float* col = A + j * M + i0;
      f32x4 v;
      if (full) {
        v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (i0 + e < M) ? col[e] : 0.0f;
      }
      inner += v * Z[j];
    }
    outer += inner;
  }
  if (nchunks == 1) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < M) out[i0 + e] = outer[e];
    return;
  }
  float* dst = part + c * M + i0;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i0 + e < M) dst[e] = outer[e];
  if (!arrive_last(counters + blockIdx.x, (int)nchunks)) return;
  if (active) {
    f32x4 total = {0.f, 0.f, 0.f, 0.f};
    for (int64_t c0 = 0; c0 < nchunks; c0 += 16) {
      f32x4 blk = {0.f, 0.f, 0.f, 0.f};
      const int64_t c1 = (c0 + 16 < nchunks) ? c0 + 16 : nchunks;
      for (int64_t cc = c0; cc < c1; ++cc) {
        const float* src = part + cc * M + i0;
        if (full) {
          blk += *reinterpret_cast<const f32x4*>(src);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) blk[e] += (i0 + e < M) ? src[e] : 0.0f;
        }
      }
      total += blk;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < M) out[i0 + e] = total[e];
  }
  if (threadIdx.x == 0) counters[blockIdx.x] = 0;
}

// 16-bit storage: element (i, j) at ((j/8)*M + i)*8 + j%8.  One thread per
// row; one 16-byte load covers 8 columns.  Z_j is pre-scaled by 2^e_j.
__device__ __forceinline__ float h16_to_f32(uint32_t h, bool bf16) {
  if (bf16) return __uint_as_float(h << 16);
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

template <bool BF16>
__device__ __forceinline__ void unpack8(const u32x4 p, float* f) {
  f[0] = h16_to_f32(p.x & 0xFFFFu, BF16);
  f[1] = h16_to_f32(p.x >> 16, BF16);
  f[2] = h16_to_f32(p.y & 0xFFFFu, BF16);
  f[3] = h16_to_f32(p.y >> 16, BF16);
  f[4] = h16_to_f32(p.z & 0xFFFFu, BF16);
  f[5] = h16_to_f32(p.z >> 16, BF16);
  f[6] = h16_to_f32(p.w & 0xFFFFu, BF16);
  f[7] = h16_to_f32(p.w >> 16, BF16);
}

template <bool BF16>
__global__ __launch_bounds__(kMv16Threads) void matvec_h16_kernel(const u32x4* __restrict__ Mp,
                                                                  const int32_t* __restrict__ exps,
                                                                  const float* __restrict__ Z,
                                                                  float* __restrict__ part,
                                                                  int32_t* __restrict__ counters,
                                                                  float* __restrict__ out,
                                                                  int64_t M, int64_t ncols,
                                                                  int64_t ngroups) {
  const int64_t i = (int64_t)blockIdx.x * kMv16Threads + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t nchunks = gridDim.y;
  const int64_t g0 = c * kMv16Groups;
  const int64_t g1 = (g0 + kMv16Groups < ngroups) ? g0 + kMv16Groups : ngroups;
  const bool active = i < M;
  float outer = 0.0f;
  if (active) {
    for (int64_t g = g0; g < g1; g += 2) {
      u32x4 p[2];
      float zs[16];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bool ok = (g + t) < g1;
        p[t] = ok ? __builtin_nontemporal_load(Mp + (g + t) * M + i) : (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t j = (g + t) * 8 + u;
          zs[t * 8 + u] = (ok && j < ncols) ? ldexpf(Z[j], exps[j]) : 0.0f;
        }
      }
      float inner = 0.0f;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        float f[8];
        unpack8<BF16>(p[t], f);
#pragma unroll
        for (int u = 0; u < 8; ++u) inner = fmaf(f[u], zs[t * 8 + u], inner);
      }
      outer += inner;
    }
  }
  if (nchunks == 1) {
    if (active) out[i] = outer;
    return;
  }
  if (active) part[c * M + i] = outer;
  if (!arrive_last(counters + blockIdx.x, (int)nchunks)) return;
  if (active) {
    float total = 0.0f;
    for (int64_t c0 = 0; c0 < nchunks; c0 += 16) {
      float blk = 0.0f;
      const int64_t c1 = (c0 + 16 < nchunks) ? c0 + 16 : nchunks;
      for (int64_t cc = c0; cc < c1; ++cc) blk += part[cc * M + i];
      total += blk;
    }
    out[i] = total;
  }
  if (threadIdx.x == 0) counters[blockIdx.x] = 0;
}

int64_t matvec_partial_floats(int storage, int64_t M, int64_t ncols, int64_t ncols_pad) {
  if (storage == PSFLIB_FP32) return ((ncols + kMvChunk - 1) / kMvChunk) * M;
  const int64_t ngroups = ncols_pad / 8;
  return ((ngroups + kMv16Groups - 1) / kMv16Groups) * M;
}

int64_t matvec_counters(int storage, int64_t M) {
  if (storage == PSFLIB_FP32) return (M + 4 * kMvThreads - 1) / (4 * kMvThreads);
  return (M + kMv16Threads - 1) / kMv16Threads;
}

hipError_t launch_matvec(int storage, const void* lib, const int32_t* exps, const float* Z,
                         int64_t M, int64_t ncols, int64_t ncols_pad, float* partial,
                         int32_t* counters, float* out, hipStream_t s) {
  if (storage == PSFLIB_FP32) {
    const int64_t nchunks = (ncols + kMvChunk - 1) / kMvChunk;
    const dim3 grid((unsigned)matvec_counters(storage, M), (unsigned)nchunks);
    const float* A = reinterpret_cast<const float*>(lib);
    if (M % 4 == 0)
      matvec_f32_kernel<true><<<grid, kMvThreads, 0, s>>>(A, Z, partial, counters, out, M, ncols);
    else
      matvec_f32_kernel<false><<<grid, kMvThreads, 0, s>>>(A, Z, partial, counters, out, M, ncols);
  } else {
    const int64_t ngroups = ncols_pad / 8;
    const int64_t nchunks = (ngroups + kMv16Groups - 1) / kMv16Groups;
    const dim3 grid((unsigned)matvec_counters(storage, M), (unsigned)nchunks);
    const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
    if (storage == PSFLIB_BF16_POW2)
      matvec_h16_kernel<true><<<grid, kMv16Threads, 0, s>>>(Mp, exps, Z, partial, counters, out, M, ncols, ngroups);
    else
      matvec_h16_kernel<false><<<grid, kMv16Threads, 0, s>>>(Mp, exps, Z, partial, counters, out, M, ncols, ngroups);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ adjoint -----
// G_j = sum_i A_ij g_i.  A workgroup owns one row block (up to kAdjF32Rows
// rows, whose g values each thread keeps in registers) and a run of columns;
// a column is one wave-wide dot product per wave, then a 4-wave sum in LDS.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <bool VEC>
__global__ __launch_bounds__(kAdjThreads) void adjoint_f32_kernel(const float* __restrict__ A,
                                                                  const float* __restrict__ g,
                                                                  float* __restrict__ out,
                                                                  int64_t M, int64_t ncols,
                                                                  int64_t out_stride) {
  constexpr int U = kAdjF32Rows / (4 * kAdjThreads);  // float4 per thread per column
  __shared__ float red[2][kAdjThreads / 64];
  const int tid = threadIdx.x;
  const int64_t rb = blockIdx.y;
  const int64_t row0 = rb * kAdjF32Rows;
  f32x4 gr[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = row0 + 4 * ((int64_t)tid + (int64_t)kAdjThreads * u);
#pragma unroll
    for (int e = 0; e < 4; ++e) gr[u][e] = (i + e < M) ? g[i + e] : 0.0f;
  }
  const int64_t jb = (int64_t)blockIdx.x * kAdjColsPerBlock;
  for (int t = 0; t < kAdjColsPerBlock; ++t) {
    const int64_t j = jb + t;
    if (j >= ncols) break;  // uniform across the workgroup
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* col = A + j * M;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = row0 + 4 * ((int64_t)tid + (int64_t)kAdjThreads * u);
      f32x4 v;
      if (VEC && i + 4 <= M) {
        v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col + i));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (i + e < M) ? col[i + e] : 0.0f;
      }
      acc += v * gr[u];
    }
    float s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    s = wave_sum(s);
    if ((tid & 63) == 0) red[t & 1][tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
      float tot = 0.0f;
#pragma unroll
      for (int w = 0; w < kAdjThreads / 64; ++w) tot += red[t & 1][w];
      out[rb * out_stride + j] = tot;
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(kAdjThreads) void adjoint_h16_kernel(const u32x4* __restrict__ Mp,
                                                                  const int32_t* __restrict__ exps,
                                                                  const float* __restrict__ g,
                                                                  float* __restrict__ out,
                                                                  int64_t M, int64_t ncols,
                                                                  int64_t ngroups,
                                                                  int64_t out_stride,
                                                                  int apply_exp) {
  constexpr int U = kAdj16Rows / kAdjThreads;  // rows per thread
  __shared__ float red[2][kAdjThreads / 64][8];
  const int tid = threadIdx.x;
  const int64_t rb = blockIdx.y;
  const int64_t row0 = rb * kAdj16Rows;
  float gr[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = row0 + tid + (int64_t)kAdjThreads * u;
    gr[u] = (i < M) ? g[i] : 0.0f;
  }
  const int64_t gb = (int64_t)blockIdx.x * kAdjColsPerBlock;
  for (int t = 0; t < kAdjColsPerBlock; ++t) {
    const int64_t grp = gb + t;
    if (grp >= ngroups) break;
    float acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0f;
#pragma unroll 8
    for (int u = 0; u < U; ++u) {
      const int64_t i = row0 + tid + (int64_t)kAdjThreads * u;
      if (i < M) {
        const u32x4 p = __builtin_nontemporal_load(Mp + grp * M + i);
        float f[8];
        unpack8<BF16>(p, f);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fmaf(f[q], gr[u], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
    if ((tid & 63) == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) red[t & 1][tid >> 6][q] = acc[q];
    }
    __syncthreads();
    if (tid < 8) {
      const int64_t j = grp * 8 + tid;
      float tot = 0.0f;
#pragma unroll
      for (int w = 0; w < kAdjThreads / 64; ++w) tot += red[t & 1][w][tid];
      if (j < ncols) out[rb * out_stride + j] = apply_exp ? ldexpf(tot, exps[j]) : tot;
    }
  }
}

// out[j] = 2^e_j * sum over row blocks (fixed order), or the plain sum for FP32.
__global__ __launch_bounds__(256) void reduce_cols_kernel(const float* __restrict__ part,
                                                          int64_t nblocks, int64_t stride,
                                                          int64_t ncols,
                                                          const int32_t* __restrict__ exps,
                                                          float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= ncols) return;
  float tot = 0.0f;
  for (int64_t b = 0; b < nblocks; ++b) tot += part[b * stride + j];
  out[j] = exps ? ldexpf(tot, exps[j]) : tot;
}

int64_t adjoint_partial_floats(int storage, int64_t M, int64_t ncols, int64_t ncols_pad) {
  const int64_t rows = (storage == PSFLIB_FP32) ? kAdjF32Rows : kAdj16Rows;
  const int64_t nb = (M + rows - 1) / rows;
  return nb > 1 ? nb * ncols_pad : 0;
}

hipError_t launch_adjoint(int storage, const void* lib, const int32_t* exps, const float* g,
                          int64_t M, int64_t ncols, int64_t ncols_pad, float* partial, float* out,
                          hipStream_t s) {
  const int64_t rows = (storage == PSFLIB_FP32) ? kAdjF32Rows : kAdj16Rows;
  const int64_t nb = (M + rows - 1) / rows;
  float* dst = (nb > 1) ? partial : out;
  const int64_t stride = ncols_pad;
  if (storage == PSFLIB_FP32) {
    const dim3 grid((unsigned)((ncols + kAdjColsPerBlock - 1) / kAdjColsPerBlock), (unsigned)nb);
    const float* A = reinterpret_cast<const float*>(lib);
    if (M % 4 == 0)
      adjoint_f32_kernel<true><<<grid, kAdjThreads, 0, s>>>(A, g, dst, M, ncols, stride);
    else
      adjoint_f32_kernel<false><<<grid, kAdjThreads, 0, s>>>(A, g, dst, M, ncols, stride);
  } else {
    const int64_t ngroups = ncols_pad / 8;
    const dim3 grid((unsigned)((ngroups + kAdjColsPerBlock - 1) / kAdjColsPerBlock), (unsigned)nb);
    const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
    const int apply_exp = (nb > 1) ? 0 : 1;
    if (storage == PSFLIB_BF16_POW2)
      adjoint_h16_kernel<true><<<grid, kAdjThreads, 0, s>>>(Mp, exps, g, dst, M, ncols, ngroups, stride, apply_exp);
    else
      adjoint_h16_kernel<false><<<grid, kAdjThreads, 0, s>>>(Mp, exps, g, dst, M, ncols, ngroups, stride, apply_exp);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  reduce_cols_kernel<<<(unsigned)((ncols + 255) / 256), 256, 0, s>>>(
      partial, nb, stride, ncols, storage == PSFLIB_FP32 ? nullptr : exps, out);
  return hipGetLastError();
}

// ----------------------------------------------------------- columns ------
template <int STORE>
__global__ __launch_bounds__(256) void get_columns_kernel(const void* __restrict__ lib,
                                                          const int32_t* __restrict__ exps,
                                                          const int32_t* __restrict__ cols,
                                                          int64_t M, int64_t ncols,
                                                          float* __restrict__ out) {
  const int64_t t = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int64_t j = cols[t];
  float v = 0.0f;
  if (j >= 0 && j < ncols) {
    if constexpr (STORE == PSFLIB_FP32) {
      v = reinterpret_cast<const float*>(lib)[j * M + i];
    } else {
      const uint16_t* Mh = reinterpret_cast<const uint16_t*>(lib);
      const uint32_t h = Mh[((j >> 3) * M + i) * 8 + (j & 7)];
      v = ldexpf(h16_to_f32(h, STORE == PSFLIB_BF16_POW2), exps[j]);
    }
  }
  out[t * M + i] = v;
}

hipError_t launch_get_columns(int storage, const void* lib, const int32_t* exps,
                              const int32_t* cols, int count, int64_t M, int64_t ncols,
                              float* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const dim3 grid((unsigned)((M + 255) / 256), (unsigned)count);
  switch (storage) {
    case PSFLIB_FP32:
      get_columns_kernel<PSFLIB_FP32><<<grid, 256, 0, s>>>(lib, exps, cols, M, ncols, out);
      break;
    case PSFLIB_BF16_POW2:
      get_columns_kernel<PSFLIB_BF16_POW2><<<grid, 256, 0, s>>>(lib, exps, cols, M, ncols, out);
      break;
    default:
      get_columns_kernel<PSFLIB_FP16_POW2><<<grid, 256, 0, s>>>(lib, exps, cols, M, ncols, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace psflib
