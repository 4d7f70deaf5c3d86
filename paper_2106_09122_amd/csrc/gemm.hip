// Batched simulation: images of B scenes at once, out[b] = A Z_b, as one GEMM
// on the matrix cores.  In GEMM terms C (M x B) = A (M x K) * Z^T (K x B) with
// M = n^2 image pixels, K = N^2 scene pixels and B scenes.
//
// FP32 storage uses v_mfma_f32_32x32x2f32; the 16-bit forms use
// v_mfma_f32_32x32x16_{bf16,f16}.  The 16-bit library is stored in groups of
// 8 columns (16 bytes per row per group), which is exactly the per-lane K
// fragment of the 16-bit MFMA, so tiles are copied to LDS without reshaping.
// Scenes are rounded to the same 16-bit format with a per-scene power of two
// (applied back to the result), after folding in the per-column exponents.
//
// Tiling: a workgroup of 4 waves computes a 128 (image rows) x 64 (scenes)
// tile; each wave holds two 32x32 accumulators.  Tiles of K are
// double-buffered through LDS.  Accumulation is blocked in three levels (one
// K tile, 32 K tiles, the rest) so float32 rounding chains stay short; when
// the grid would be too small to fill the GPU, K is split across workgroups
// and a second kernel adds the slices in a fixed order.
#include <math.h>

#include "psflib_internal.h"

namespace psflib {

constexpr int kGemmThreads = 256;
constexpr int kGM = 128;  // image rows per workgroup tile
constexpr int kGN = 64;   // scenes per workgroup tile
constexpr int kGK32 = 16; // K per tile, FP32 path
constexpr int kGK16 = 32; // K per tile, 16-bit path (4 groups of 8)
constexpr int kMidTiles = 32;
constexpr int kMaxBatchChunk = 1024;  // scenes per internal pass (bounds the scratch)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Store a 32x32 accumulator: lane holds column n = lane%32 and rows
// 8*(r/4) + 4*(lane/32) + r%4 of the tile.
__device__ __forceinline__ void store_acc(const f32x16& acc, float* __restrict__ dst, int64_t M,
                                          int64_t B, int64_t mt, int64_t nt, int lane,
                                          const int32_t* fexp, bool scaled) {
  const int64_t n = nt + (lane & 31);
  if (n >= B) return;
  const int ex = scaled ? -fexp[n] : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t m = mt + 8 * q + 4 * (lane >> 5);
    f32x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = scaled ? ldexpf(acc[4 * q + e], ex) : acc[4 * q + e];
    float* p = dst + n * M + m;
    if (m + 4 <= M && (M % 4) == 0) {
      *reinterpret_cast<f32x4*>(p) = v;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (m + e < M) p[e] = v[e];
    }
  }
}

// ------------------------------------------------------------- FP32 -------
__global__ __launch_bounds__(kGemmThreads) void gemm_f32_kernel(const float* __restrict__ A,
                                                                const float* __restrict__ Z,
                                                                float* __restrict__ out,
                                                                int64_t M, int64_t K, int64_t B,
                                                                int64_t ktiles_per_split) {
  __shared__ float As[2][kGK32][kGM];
  __shared__ float Bs[2][kGK32][kGN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t m0 = (int64_t)blockIdx.x * kGM;
  const int64_t n0 = (int64_t)blockIdx.y * kGN;
  const int64_t ktiles = (K + kGK32 - 1) / kGK32;
  const int64_t kt0 = (int64_t)blockIdx.z * ktiles_per_split;
  int64_t kt1 = kt0 + ktiles_per_split;
  if (kt1 > ktiles) kt1 = ktiles;
  float* dst = out + (int64_t)blockIdx.z * B * M;
  const bool vecA = (M % 4) == 0, vecB = (K % 4) == 0;

  f32x4 ra[2], rbv;
  auto load_tile = [&](int64_t kt) {
    const int64_t k0 = kt * kGK32;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = tid + kGemmThreads * r;
      const int kk = idx >> 5, m4 = (idx & 31) * 4;
      const int64_t k = k0 + kk, m = m0 + m4;
      if (k < K && vecA && m + 4 <= M) {
        ra[r] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(A + k * M + m));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[r][e] = (k < K && m + e < M) ? A[k * M + m + e] : 0.0f;
      }
    }
    {
      const int nn = tid >> 2, k4 = (tid & 3) * 4;
      const int64_t n = n0 + nn, k = k0 + k4;
      if (n < B && vecB && k + 4 <= K) {
        rbv = *reinterpret_cast<const f32x4*>(Z + n * K + k);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rbv[e] = (n < B && k + e < K) ? Z[n * K + k + e] : 0.0f;
      }
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = tid + kGemmThreads * r;
      const int kk = idx >> 5, m4 = (idx & 31) * 4;
      *reinterpret_cast<f32x4*>(&As[buf][kk][m4]) = ra[r];
    }
    const int nn = tid >> 2, k4 = (tid & 3) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[buf][k4 + e][nn] = rbv[e];
  };

  const f32x16 zero16 = {};
  f32x16 acc_out[2] = {zero16, zero16}, acc_mid[2] = {zero16, zero16};
  if (kt0 < kt1) {
    load_tile(kt0);
    store_tile(0);
  }
  __syncthreads();
  int mid_count = 0;
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    const int cur = (int)((kt - kt0) & 1);
    if (kt + 1 < kt1) load_tile(kt + 1);
    f32x16 acc_t[2] = {zero16, zero16};
#pragma unroll
    for (int kk = 0; kk < kGK32 / 2; ++kk) {
      const int krow = 2 * kk + (lane >> 5);
      const float b = Bs[cur][krow][32 * wn + (lane & 31)];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float a = As[cur][krow][64 * wm + 32 * t + (lane & 31)];
        acc_t[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc_t[t], 0, 0, 0);
      }
    }
    acc_mid[0] += acc_t[0];
    acc_mid[1] += acc_t[1];
    if (++mid_count == kMidTiles) {
      acc_out[0] += acc_mid[0];
      acc_out[1] += acc_mid[1];
      acc_mid[0] = zero16;
      acc_mid[1] = zero16;
      mid_count = 0;
    }
    if (kt + 1 < kt1) store_tile(cur ^ 1);
    __syncthreads();
  }
  acc_out[0] += acc_mid[0];
  acc_out[1] += acc_mid[1];
#pragma unroll
  for (int t = 0; t < 2; ++t)
    store_acc(acc_out[t], dst, M, B, m0 + 64 * wm + 32 * t, n0 + 32 * wn, lane, nullptr, false);
}

// ------------------------------------------------------------- 16-bit -----
// Scene preparation: Zp[b][j] = RN16(Z[b][j] * 2^(e_j + f_b)), with f_b
// making max_j |Z[b][j]| 2^e_j land in [2^14, 2^15); padding columns are 0.
template <bool BF16>
__global__ __launch_bounds__(256) void prep_scenes_kernel(const float* __restrict__ Z,
                                                          const int32_t* __restrict__ exps,
                                                          int64_t ncols, int64_t ncols_pad,
                                                          uint16_t* __restrict__ Zp,
                                                          int32_t* __restrict__ fexp) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;
  const float* z = Z + b * ncols;
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < ncols; j += 256)
    m = fmax(m, ldexp((double)fabsf(z[j]), exps[j]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  int f = 0;
  if (red[0] > 0.0) {
    int E;
    (void)frexp(red[0], &E);
    f = 15 - E;
  }
  if (threadIdx.x == 0) fexp[b] = f;
  uint16_t* zp = Zp + b * ncols_pad;
  for (int64_t j = threadIdx.x; j < ncols_pad; j += 256) {
    uint32_t h = 0;
    if (j < ncols) {
      const float s = ldexpf(z[j], exps[j] + f);
      if (BF16) {
        uint32_t u = __float_as_uint(s);
        u += 0x7FFFu + ((u >> 16) & 1u);
        h = u >> 16;
      } else {
        h = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)s);
      }
    }
    zp[j] = (uint16_t)h;
  }
}

template <bool BF16>
__global__ __launch_bounds__(kGemmThreads) void gemm_h16_kernel(const u32x4* __restrict__ Mp,
                                                                const u32x4* __restrict__ Zp,
                                                                const int32_t* __restrict__ fexp,
                                                                float* __restrict__ out,
                                                                int64_t M, int64_t ngroups,
                                                                int64_t B,
                                                                int64_t ktiles_per_split) {
  __shared__ u32x4 As[2][kGK16 / 8][kGM];
  __shared__ u32x4 Bs[2][kGK16 / 8][kGN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t m0 = (int64_t)blockIdx.x * kGM;
  const int64_t n0 = (int64_t)blockIdx.y * kGN;
  const int64_t ktiles = ngroups / (kGK16 / 8);  // ngroups is a multiple of 8
  const int64_t kt0 = (int64_t)blockIdx.z * ktiles_per_split;
  int64_t kt1 = kt0 + ktiles_per_split;
  if (kt1 > ktiles) kt1 = ktiles;
  const bool split = gridDim.z > 1;
  float* dst = out + (int64_t)blockIdx.z * B * M;
  const u32x4 z4 = {0u, 0u, 0u, 0u};

  u32x4 ra[2], rbv;
  auto load_tile = [&](int64_t kt) {
    const int64_t g0 = kt * (kGK16 / 8);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = tid + kGemmThreads * r;
      const int gg = idx >> 7, m = idx & 127;
      ra[r] = (m0 + m < M) ? __builtin_nontemporal_load(Mp + (g0 + gg) * M + m0 + m) : z4;
    }
    const int nn = tid >> 2, gg = tid & 3;
    rbv = (n0 + nn < B) ? Zp[(n0 + nn) * ngroups + g0 + gg] : z4;
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = tid + kGemmThreads * r;
      As[buf][idx >> 7][idx & 127] = ra[r];
    }
    Bs[buf][tid & 3][tid >> 2] = rbv;
  };

  const f32x16 zero16 = {};
  f32x16 acc_out[2] = {zero16, zero16}, acc_mid[2] = {zero16, zero16};
  if (kt0 < kt1) {
    load_tile(kt0);
    store_tile(0);
  }
  __syncthreads();
  int mid_count = 0;
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    const int cur = (int)((kt - kt0) & 1);
    if (kt + 1 < kt1) load_tile(kt + 1);
    f32x16 acc_t[2] = {zero16, zero16};
#pragma unroll
    for (int kk = 0; kk < kGK16 / 16; ++kk) {
      const int gidx = 2 * kk + (lane >> 5);
      const u32x4 bw = Bs[cur][gidx][32 * wn + (lane & 31)];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const u32x4 aw = As[cur][gidx][64 * wm + 32 * t + (lane & 31)];
        if constexpr (BF16) {
          acc_t[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, aw),
                                                             __builtin_bit_cast(bf16x8, bw),
                                                             acc_t[t], 0, 0, 0);
        } else {
          acc_t[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, aw),
                                                            __builtin_bit_cast(f16x8, bw),
                                                            acc_t[t], 0, 0, 0);
        }
      }
    }
    acc_mid[0] += acc_t[0];
    acc_mid[1] += acc_t[1];
    if (++mid_count == kMidTiles) {
      acc_out[0] += acc_mid[0];
      acc_out[1] += acc_mid[1];
      acc_mid[0] = zero16;
      acc_mid[1] = zero16;
      mid_count = 0;
    }
    if (kt + 1 < kt1) store_tile(cur ^ 1);
    __syncthreads();
  }
  acc_out[0] += acc_mid[0];
  acc_out[1] += acc_mid[1];
  // Without a K split the per-scene power of two is undone here; with one, the
  // slice-reduction kernel does it.
#pragma unroll
  for (int t = 0; t < 2; ++t)
    store_acc(acc_out[t], dst, M, B, m0 + 64 * wm + 32 * t, n0 + 32 * wn, lane, fexp, !split);
}

// out[b][m] = 2^-f_b * sum over K slices (fixed order).
__global__ __launch_bounds__(256) void reduce_splits_kernel(const float* __restrict__ part,
                                                            int splits, int64_t BM, int64_t M,
                                                            const int32_t* __restrict__ fexp,
                                                            float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= BM) return;
  float s = 0.0f;
  for (int p = 0; p < splits; ++p) s += part[(int64_t)p * BM + t];
  out[t] = fexp ? ldexpf(s, -fexp[t / M]) : s;
}

// ------------------------------------------------------------ launch ------
static int choose_splits(int64_t mblocks, int64_t nblocks, int64_t ktiles) {
  const int64_t wgs = mblocks * nblocks;
  int64_t s = (1024 + wgs - 1) / wgs;
  if (s > 16) s = 16;
  if (s > ktiles) s = ktiles;
  if (s < 1) s = 1;
  return (int)s;
}

static int64_t chunk_of(int B) { return B < kMaxBatchChunk ? B : kMaxBatchChunk; }

static size_t split_partial_bytes(int storage, int64_t M, int64_t ncols_pad, int64_t bc) {
  const int64_t mblocks = (M + kGM - 1) / kGM, nblocks = (bc + kGN - 1) / kGN;
  const int64_t ktiles = (storage == PSFLIB_FP32) ? (ncols_pad + kGK32 - 1) / kGK32
                                                  : ncols_pad / kGK16;
  const int splits = choose_splits(mblocks, nblocks, ktiles);
  return splits > 1 ? (size_t)splits * (size_t)bc * (size_t)M * 4 : 0;
}

size_t batched_scratch_bytes(int storage, int64_t M, int64_t ncols_pad, int B) {
  // Passes run over up to kMaxBatchChunk scenes each: for the 16-bit forms the
  // prepared scenes and their exponents, then the K-split partial images of
  // the largest pass (a short final pass may split K more finely).
  if (B <= 0) return 0;
  const int64_t bc = chunk_of(B);
  size_t bytes = 0;
  if (storage != PSFLIB_FP32) {
    bytes += ((size_t)bc * (size_t)ncols_pad * 2 + 255) & ~(size_t)255;  // Zp
    bytes += ((size_t)bc * 4 + 255) & ~(size_t)255;                      // fexp
  }
  size_t part = split_partial_bytes(storage, M, ncols_pad, bc);
  const int64_t rem = B % bc;
  if (rem) {
    const size_t p2 = split_partial_bytes(storage, M, ncols_pad, rem);
    if (p2 > part) part = p2;
  }
  return bytes + part;
}

hipError_t launch_batched(int storage, const void* lib, const int32_t* exps, const float* Z,
                          float* out, int64_t M, int64_t ncols, int64_t ncols_pad, int B,
                          void* scratch, size_t scratch_bytes, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  char* sp = reinterpret_cast<char*>(scratch);
  uint16_t* Zp = nullptr;
  int32_t* fexp = nullptr;
  const int64_t bcmax = chunk_of(B);
  size_t off = 0;
  if (storage != PSFLIB_FP32) {
    Zp = reinterpret_cast<uint16_t*>(sp);
    off += ((size_t)bcmax * (size_t)ncols_pad * 2 + 255) & ~(size_t)255;
    fexp = reinterpret_cast<int32_t*>(sp + off);
    off += ((size_t)bcmax * 4 + 255) & ~(size_t)255;
  }
  float* part = reinterpret_cast<float*>(sp + off);
  for (int64_t b0 = 0; b0 < B; b0 += bcmax) {
    const int64_t bc = (B - b0 < bcmax) ? (B - b0) : bcmax;
    const int64_t mblocks = (M + kGM - 1) / kGM, nblocks = (bc + kGN - 1) / kGN;
    const float* Zc = Z + b0 * ncols;
    float* outc = out + b0 * M;
    int splits;
    hipError_t e;
    // every pass must fit the scratch sized by batched_scratch_bytes()
    if (off + split_partial_bytes(storage, M, ncols_pad, bc) > scratch_bytes) return hipErrorInvalidValue;
    if (storage == PSFLIB_FP32) {
      const int64_t ktiles = (ncols + kGK32 - 1) / kGK32;
      splits = choose_splits(mblocks, nblocks, ktiles);
      const int64_t per = (ktiles + splits - 1) / splits;
      const dim3 grid((unsigned)mblocks, (unsigned)nblocks, (unsigned)splits);
      gemm_f32_kernel<<<grid, kGemmThreads, 0, s>>>(reinterpret_cast<const float*>(lib), Zc,
                                                    splits > 1 ? part : outc, M, ncols, bc, per);
      e = hipGetLastError();
    } else {
      const bool bf = storage == PSFLIB_BF16_POW2;
      if (bf)
        prep_scenes_kernel<true><<<(unsigned)bc, 256, 0, s>>>(Zc, exps, ncols, ncols_pad, Zp, fexp);
      else
        prep_scenes_kernel<false><<<(unsigned)bc, 256, 0, s>>>(Zc, exps, ncols, ncols_pad, Zp, fexp);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      const int64_t ngroups = ncols_pad / 8;
      const int64_t ktiles = ncols_pad / kGK16;
      splits = choose_splits(mblocks, nblocks, ktiles);
      const int64_t per = (ktiles + splits - 1) / splits;
      const dim3 grid((unsigned)mblocks, (unsigned)nblocks, (unsigned)splits);
      const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
      const u32x4* Zq = reinterpret_cast<const u32x4*>(Zp);
      if (bf)
        gemm_h16_kernel<true><<<grid, kGemmThreads, 0, s>>>(Mp, Zq, fexp, splits > 1 ? part : outc,
                                                            M, ngroups, bc, per);
      else
        gemm_h16_kernel<false><<<grid, kGemmThreads, 0, s>>>(Mp, Zq, fexp, splits > 1 ? part : outc,
                                                             M, ngroups, bc, per);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (splits > 1) {
      const int64_t BM = bc * M;
      reduce_splits_kernel<<<(unsigned)((BM + 255) / 256), 256, 0, s>>>(
          part, splits, BM, M, storage == PSFLIB_FP32 ? nullptr : fexp, outc);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace psflib
