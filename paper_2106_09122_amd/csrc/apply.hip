// Single-scene products with the library: S = A Z (Sec. 3, Eq. (6)) and the
// adjoint G = A^T g.  Both stream the library once from HBM and are bound by
// memory bandwidth; the scene and image vectors are small and stay in cache.
//
// A is column-major (column j is contiguous), so the forward product is a sum
// of scaled columns.  It is split over (row block, column chunk) workgroups:
// each thread owns 4 consecutive rows and walks the chunk's columns with 16
// independent 16-byte non-temporal loads in flight, and writes a partial
// image; a second kernel adds the partials of every row in chunk order.  (Doing
// that sum in the last workgroup to finish each row block needs a device-scope
// release per workgroup, which writes back the XCD's L2: measured slower than
// the extra launch.)  Sums are blocked (16 columns per inner sum) so every rounding chain
// stays short.  Results are bitwise reproducible.
#include <math.h>
#include <stdlib.h>

#include <map>
#include <mutex>

#include "psflib_internal.h"

namespace psflib {

// ------------------------------------------------------------ forward -----
// Split-K: workgroups own (row block, column chunk) tiles and write partial
// images; a second kernel adds the partials of every row in chunk order, so
// the result does not depend on scheduling.
// Rows of one 16-column block: v[u] = A[j+u][i0..i0+3] (zero past M).
template <bool FULL>
__device__ __forceinline__ void load_block16(const float* __restrict__ A, int64_t M, int64_t i0,
                                             int64_t j, f32x4* v) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const float* col = A + (j + u) * M + i0;
    if constexpr (FULL) {
      v[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[u][e] = (i0 + e < M) ? col[e] : 0.0f;
    }
  }
}

// sum_j A[j][i0..i0+3] Z[j] over [j0, j1), in three levels: 16 columns,
// 16 blocks of 16, then the rest, so no rounding chain exceeds ~16 + 16 +
// (j1-j0)/256 additions.
template <bool FULL>
__device__ __forceinline__ f32x4 matvec_rows(const float* __restrict__ A,
                                             const float* __restrict__ Z, int64_t M, int64_t i0,
                                             int64_t j0, int64_t j1) {
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 outer = zero, mid = zero;
  int nblk = 0;
  int64_t j = j0;
  for (; j + 16 <= j1; j += 16) {
    f32x4 v[16];
    load_block16<FULL>(A, M, i0, j, v);
    f32x4 inner = v[0] * Z[j];
#pragma unroll
    for (int u = 1; u < 16; ++u) inner += v[u] * Z[j + u];
    mid += inner;
    if (++nblk == 16) {
      outer += mid;
      mid = zero;
      nblk = 0;
    }
  }
  f32x4 inner = zero;
  for (; j < j1; ++j) {
    const float* col = A + j * M + i0;
    f32x4 v;
    if constexpr (FULL) {
      v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (i0 + e < M) ? col[e] : 0.0f;
    }
    inner += v * Z[j];
  }
  mid += inner;
  return outer + mid;
}

template <bool VEC>
__global__ __launch_bounds__(kMvThreads) void matvec_f32_kernel(const float* __restrict__ A,
                                                                const float* __restrict__ Z,
                                                                float* __restrict__ part,
                                                                float* __restrict__ out,
                                                                int64_t M, int64_t ncols,
                                                                int64_t chunk) {
  const int64_t i0 = ((int64_t)blockIdx.x * kMvThreads + threadIdx.x) * 4;
  const int64_t c = blockIdx.y;
  const int64_t nchunks = gridDim.y;
  const int64_t j0 = c * chunk;
  const int64_t j1 = (j0 + chunk < ncols) ? j0 + chunk : ncols;
  // uniform across the workgroup: every row of the block is inside the image
  const bool block_full = VEC && ((int64_t)(blockIdx.x + 1) * kMvThreads * 4 <= M);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (block_full)
    acc = matvec_rows<true>(A, Z, M, i0, j0, j1);
  else if (i0 < M)
    acc = matvec_rows<false>(A, Z, M, i0, j0, j1);
  float* dst = ((nchunks == 1) ? out : part + c * M) + i0;
  if (block_full) {
    *reinterpret_cast<f32x4*>(dst) = acc;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < M) dst[e] = acc[e];
  }
}

// 16-bit storage: element (i, slot s) at ((s/8)*M + i)*8 + s%8, slot s holding
// column perm[s].  One thread per row; one 16-byte load covers 8 slots.  The
// chunk's scene values Z[perm[s]] scaled by 2^eslot[s] are staged in LDS and
// read as broadcasts.
__device__ __forceinline__ float h16_to_f32(uint32_t h, bool bf16) {
  if (bf16) return __uint_as_float(h << 16);
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

template <bool BF16>
__device__ __forceinline__ void unpack8(const u32x4 p, float* f) {
  if constexpr (BF16) {
    f[0] = __uint_as_float(p.x << 16);
    f[1] = __uint_as_float(p.x & 0xFFFF0000u);
    f[2] = __uint_as_float(p.y << 16);
    f[3] = __uint_as_float(p.y & 0xFFFF0000u);
    f[4] = __uint_as_float(p.z << 16);
    f[5] = __uint_as_float(p.z & 0xFFFF0000u);
    f[6] = __uint_as_float(p.w << 16);
    f[7] = __uint_as_float(p.w & 0xFFFF0000u);
  } else {
    f[0] = h16_to_f32(p.x & 0xFFFFu, false);
    f[1] = h16_to_f32(p.x >> 16, false);
    f[2] = h16_to_f32(p.y & 0xFFFFu, false);
    f[3] = h16_to_f32(p.y >> 16, false);
    f[4] = h16_to_f32(p.z & 0xFFFFu, false);
    f[5] = h16_to_f32(p.z >> 16, false);
    f[6] = h16_to_f32(p.w & 0xFFFFu, false);
    f[7] = h16_to_f32(p.w >> 16, false);
  }
}

// Each thread owns kMv16RowsPerThread rows, kMv16Threads apart, so a
// workgroup reads kMv16RowsPerThread * 4 KiB of every group in one piece, and
// each broadcast of the group's 8 scene values serves that many loads.
template <bool BF16>
__global__ __launch_bounds__(kMv16Threads) void matvec_h16_kernel(const u32x4* __restrict__ Mp,
                                                                  const int32_t* __restrict__ perm,
                                                                  const int32_t* __restrict__ eslot,
                                                                  const float* __restrict__ Z,
                                                                  float* __restrict__ part,
                                                                  float* __restrict__ out,
                                                                  int64_t M, int64_t ngroups,
                                                                  int64_t chunk_g) {
  constexpr int R = kMv16RowsPerThread;
  constexpr int GB = 16 / R;  // groups per block of 16 loads
  __shared__ f32x4 zs[kMv16MaxChunkGroups * 2];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kMv16Threads * R + tid;
  const int64_t c = blockIdx.y;
  const int64_t nchunks = gridDim.y;
  const int64_t g0 = c * chunk_g;
  const int64_t g1 = (g0 + chunk_g < ngroups) ? g0 + chunk_g : ngroups;
  const int64_t ng = g1 - g0;
  float* zsf = reinterpret_cast<float*>(zs);
  for (int64_t t = tid; t < ng * 8; t += kMv16Threads) {
    const int64_t slot = g0 * 8 + t;
    const int32_t j = perm[slot];
    zsf[t] = (j >= 0) ? ldexpf(Z[j], eslot[slot]) : 0.0f;
  }
  __syncthreads();
  // rows past the image read row M-1 (in bounds) and are not written
  const u32x4* src[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + (int64_t)kMv16Threads * r;
    src[r] = Mp + (i < M ? i : M - 1);
  }
  float outer[R], mid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) outer[r] = mid[r] = 0.0f;
  // blocks of 16 groups per inner sum, 8 blocks per middle sum, per row
  float inner[R];
#pragma unroll
  for (int r = 0; r < R; ++r) inner[r] = 0.0f;
  int ing = 0, nblk = 0;
  int64_t g = g0;
  for (; g + GB <= g1; g += GB) {
    u32x4 p[GB][R];
#pragma unroll
    for (int u = 0; u < GB; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) p[u][r] = __builtin_nontemporal_load(src[r] + (g + u) * M);
#pragma unroll
    for (int u = 0; u < GB; ++u) {
      const f32x4 za = zs[2 * (g - g0 + u)], zb = zs[2 * (g - g0 + u) + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float f[8];
        unpack8<BF16>(p[u][r], f);
        float acc = inner[r];
        acc = fmaf(f[0], za.x, acc);
        acc = fmaf(f[1], za.y, acc);
        acc = fmaf(f[2], za.z, acc);
        acc = fmaf(f[3], za.w, acc);
        acc = fmaf(f[4], zb.x, acc);
        acc = fmaf(f[5], zb.y, acc);
        acc = fmaf(f[6], zb.z, acc);
        acc = fmaf(f[7], zb.w, acc);
        inner[r] = acc;
      }
    }
    ing += GB;
    if (ing == 16) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        mid[r] += inner[r];
        inner[r] = 0.0f;
      }
      ing = 0;
      if (++nblk == 8) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          outer[r] += mid[r];
          mid[r] = 0.0f;
        }
        nblk = 0;
      }
    }
  }
  for (; g < g1; ++g) {
    const f32x4 za = zs[2 * (g - g0)], zb = zs[2 * (g - g0) + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float f[8];
      unpack8<BF16>(__builtin_nontemporal_load(src[r] + g * M), f);
      float acc = inner[r];
      acc = fmaf(f[0], za.x, acc);
      acc = fmaf(f[1], za.y, acc);
      acc = fmaf(f[2], za.z, acc);
      acc = fmaf(f[3], za.w, acc);
      acc = fmaf(f[4], zb.x, acc);
      acc = fmaf(f[5], zb.y, acc);
      acc = fmaf(f[6], zb.z, acc);
      acc = fmaf(f[7], zb.w, acc);
      inner[r] = acc;
    }
  }
  float* dst = (nchunks == 1) ? out : part + c * M;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + (int64_t)kMv16Threads * r;
    if (i < M) dst[i] = outer[r] + (mid[r] + inner[r]);
  }
}

// out[i] = sum over chunks of part[chunk][i]: blocks of 16 partials loaded
// together and added in chunk order, then the block sums in order.  One row
// per thread, so the few megabytes of partials are spread over many waves.
__global__ __launch_bounds__(256) void reduce_rows_kernel(const float* __restrict__ part,
                                                          int64_t nchunks, int64_t M,
                                                          float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  float total = 0.0f;
  for (int64_t c0 = 0; c0 < nchunks; c0 += 16) {
    float p[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) p[u] = (c0 + u < nchunks) ? part[(c0 + u) * M + i] : 0.0f;
    float blk = p[0];
#pragma unroll
    for (int u = 1; u < 16; ++u) blk += p[u];
    total += blk;
  }
  out[i] = total;
}

// Split-K shape: about kMvTargetWorkgroups{32,16} workgroups in all (FP32:
// two per CU; 16-bit: one per CU of 8 rows x 16 B per thread and load step,
// measured at 128^2 against 192 or 384 workgroups: 80 us against 88-94 us,
// and against one row per thread at 768 workgroups: 85 us).  The value can be
// overridden with PSFLIB_MV_WORKGROUPS for tuning sweeps.
static int64_t mv_target_workgroups(int storage) {
  static const long env = [] {
    const char* e = getenv("PSFLIB_MV_WORKGROUPS");
    return e ? strtol(e, nullptr, 10) : 0L;
  }();
  if (env > 0) return env;
  return storage == PSFLIB_FP32 ? kMvTargetWorkgroups32 : kMvTargetWorkgroups16;
}

struct MvShape {
  int64_t rowblocks, chunk, nchunks;  // chunk: columns (FP32) or 8-column groups (16-bit)
};

static MvShape mv_shape(int storage, int64_t M, int64_t ncols, int64_t ncols_pad) {
  MvShape sh;
  const int64_t rows = (storage == PSFLIB_FP32) ? 4 * kMvThreads : kMv16Threads * kMv16RowsPerThread;
  const int64_t units = (storage == PSFLIB_FP32) ? ncols : ncols_pad / 8;
  sh.rowblocks = (M + rows - 1) / rows;
  int64_t want = (mv_target_workgroups(storage) + sh.rowblocks - 1) / sh.rowblocks;
  if (want < 1) want = 1;
  int64_t chunk = (units + want - 1) / want;
  chunk = (chunk + 15) / 16 * 16;
  if (storage != PSFLIB_FP32 && chunk > kMv16MaxChunkGroups) chunk = kMv16MaxChunkGroups;
  sh.chunk = chunk;
  sh.nchunks = (units + chunk - 1) / chunk;
  return sh;
}

int64_t matvec_partial_floats(int storage, int64_t M, int64_t ncols, int64_t ncols_pad) {
  const MvShape sh = mv_shape(storage, M, ncols, ncols_pad);
  return sh.nchunks > 1 ? sh.nchunks * M : 0;
}

hipError_t launch_matvec(int storage, const void* lib, const Cols16& cx, const float* Z,
                         int64_t M, int64_t ncols, int64_t ncols_pad, float* partial, float* out,
                         hipStream_t s) {
  const MvShape sh = mv_shape(storage, M, ncols, ncols_pad);
  const dim3 grid((unsigned)sh.rowblocks, (unsigned)sh.nchunks);
  if (storage == PSFLIB_FP32) {
    const float* A = reinterpret_cast<const float*>(lib);
    if (M % 4 == 0)
      matvec_f32_kernel<true><<<grid, kMvThreads, 0, s>>>(A, Z, partial, out, M, ncols, sh.chunk);
    else
      matvec_f32_kernel<false><<<grid, kMvThreads, 0, s>>>(A, Z, partial, out, M, ncols, sh.chunk);
  } else {
    const int64_t ngroups = ncols_pad / 8;
    const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
    if (storage == PSFLIB_BF16_POW2)
      matvec_h16_kernel<true><<<grid, kMv16Threads, 0, s>>>(Mp, cx.perm, cx.eslot, Z, partial, out, M, ngroups, sh.chunk);
    else
      matvec_h16_kernel<false><<<grid, kMv16Threads, 0, s>>>(Mp, cx.perm, cx.eslot, Z, partial, out, M, ngroups, sh.chunk);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sh.nchunks == 1) return e;
  reduce_rows_kernel<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(partial, sh.nchunks, M, out);
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

// 16-bit: the sums of group grp belong to slots 8 grp + q, i.e. columns
// perm[8 grp + q]; they are written at the column's index.
template <bool BF16>
__global__ __launch_bounds__(kAdjThreads) void adjoint_h16_kernel(const u32x4* __restrict__ Mp,
                                                                  const int32_t* __restrict__ perm,
                                                                  const int32_t* __restrict__ eslot,
                                                                  const float* __restrict__ g,
                                                                  float* __restrict__ out,
                                                                  int64_t M, int64_t ngroups,
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
  const int64_t gb = (int64_t)blockIdx.x * kAdj16GroupsPerBlock;
  for (int t = 0; t < kAdj16GroupsPerBlock; ++t) {
    const int64_t grp = gb + t;
    if (grp >= ngroups) break;
    float acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0f;
    const u32x4* src = Mp + grp * M + row0 + tid;
    if (row0 + kAdj16Rows <= M) {  // uniform: every row of the block is in the image
      // blocks of 16 loads issued together, then consumed in order
      for (int u0 = 0; u0 < U; u0 += 16) {
        u32x4 p[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) p[u] = __builtin_nontemporal_load(src + (int64_t)kAdjThreads * (u0 + u));
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          float f[8];
          unpack8<BF16>(p[u], f);
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[q] = fmaf(f[q], gr[u0 + u], acc[q]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = row0 + tid + (int64_t)kAdjThreads * u;
        if (i < M) {
          const u32x4 p = __builtin_nontemporal_load(src + (int64_t)kAdjThreads * u);
          float f[8];
          unpack8<BF16>(p, f);
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[q] = fmaf(f[q], gr[u], acc[q]);
        }
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
      const int64_t slot = grp * 8 + tid;
      const int32_t j = perm[slot];
      float tot = 0.0f;
#pragma unroll
      for (int w = 0; w < kAdjThreads / 64; ++w) tot += red[t & 1][w][tid];
      if (j >= 0) out[rb * out_stride + j] = apply_exp ? ldexpf(tot, eslot[slot]) : tot;
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

hipError_t launch_adjoint(int storage, const void* lib, const Cols16& cx, const float* g,
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
    const dim3 grid((unsigned)((ngroups + kAdj16GroupsPerBlock - 1) / kAdj16GroupsPerBlock), (unsigned)nb);
    const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
    const int apply_exp = (nb > 1) ? 0 : 1;
    if (storage == PSFLIB_BF16_POW2)
      adjoint_h16_kernel<true><<<grid, kAdjThreads, 0, s>>>(Mp, cx.perm, cx.eslot, g, dst, M, ngroups, stride, apply_exp);
    else
      adjoint_h16_kernel<false><<<grid, kAdjThreads, 0, s>>>(Mp, cx.perm, cx.eslot, g, dst, M, ngroups, stride, apply_exp);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  reduce_cols_kernel<<<(unsigned)((ncols + 255) / 256), 256, 0, s>>>(
      partial, nb, stride, ncols, storage == PSFLIB_FP32 ? nullptr : cx.exps, out);
  return hipGetLastError();
}

// ------------------------------------------- allocation-free scratch -----
// Partial sums of psflib_apply_noalloc: a fixed device array on every GPU the
// library runs on, held until the process ends and shared by every such call
// on that GPU.  In host code the array's name is not a device address: the
// address is looked up once per device with hipGetSymbolAddress (that device
// current) and kept, and only that address is passed to kernels.
static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

hipError_t noalloc_scratch(int dev, void** ptr) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) {
    *ptr = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  addr[dev] = p;
  *ptr = p;
  return hipSuccess;
}

// ----------------------------------------------------------- columns ------
template <int STORE>
__global__ __launch_bounds__(256) void get_columns_kernel(const void* __restrict__ lib,
                                                          const int32_t* __restrict__ exps,
                                                          const int32_t* __restrict__ slot_of,
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
      const int64_t slot = slot_of[j];
      const uint32_t h = Mh[((slot >> 3) * M + i) * 8 + (slot & 7)];
      v = ldexpf(h16_to_f32(h, STORE == PSFLIB_BF16_POW2), exps[j]);
    }
  }
  out[t * M + i] = v;
}

hipError_t launch_get_columns(int storage, const void* lib, const Cols16& cx,
                              const int32_t* cols, int count, int64_t M, int64_t ncols,
                              float* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const dim3 grid((unsigned)((M + 255) / 256), (unsigned)count);
  switch (storage) {
    case PSFLIB_FP32:
      get_columns_kernel<PSFLIB_FP32><<<grid, 256, 0, s>>>(lib, cx.exps, cx.slot_of, cols, M, ncols, out);
      break;
    case PSFLIB_BF16_POW2:
      get_columns_kernel<PSFLIB_BF16_POW2><<<grid, 256, 0, s>>>(lib, cx.exps, cx.slot_of, cols, M, ncols, out);
      break;
    default:
      get_columns_kernel<PSFLIB_FP16_POW2><<<grid, 256, 0, s>>>(lib, cx.exps, cx.slot_of, cols, M, ncols, out);
      break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------ column order -----
__global__ __launch_bounds__(256) void identity_order_kernel(int32_t* __restrict__ perm,
                                                             int32_t* __restrict__ eslot,
                                                             int32_t* __restrict__ slot_of,
                                                             const int32_t* __restrict__ exps,
                                                             int64_t ncols, int64_t ncols_pad) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= ncols_pad) return;
  perm[s] = s < ncols ? (int32_t)s : -1;
  eslot[s] = exps[s];
  if (s < ncols) slot_of[s] = (int32_t)s;
}

hipError_t launch_identity_order(int32_t* perm, int32_t* eslot, int32_t* slot_of,
                                 const int32_t* exps, int64_t ncols, int64_t ncols_pad,
                                 hipStream_t s) {
  identity_order_kernel<<<(unsigned)((ncols_pad + 255) / 256), 256, 0, s>>>(perm, eslot, slot_of,
                                                                           exps, ncols, ncols_pad);
  return hipGetLastError();
}

}  // namespace psflib
