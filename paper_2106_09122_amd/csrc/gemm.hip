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
// Tiles are assigned to workgroups so that the workgroups one XCD runs
// together (hardware dispatch is round-robin over the 8 XCDs) share image-row
// blocks and scene blocks: each operand tile is then fetched from HBM once
// per XCD and re-read from that XCD's L2.  When the tile grid is too small to
// fill the GPU, K is split across workgroups and a second kernel adds the
// slices in a fixed order.
//
// FP32: a workgroup of 4 waves computes a 128 (image rows) x 64 (scenes) tile
// from K tiles of 16 double-buffered through LDS; accumulation is blocked in
// three levels (one K tile, 32 K tiles, the rest) so float32 rounding chains
// stay short.
//
// 16-bit: a workgroup of 4 waves computes a 256 x 128 tile; each wave owns 64
// image rows and all 128 scenes (2 x 4 accumulators of 32 x 32).  Library
// fragments go straight from HBM into registers (each is used by one wave
// only, for 4 MFMAs), one K stage ahead; scene fragments are shared by the 4
// waves through a double-buffered LDS tile of 64 K.  The 16-bit rounding of
// the inputs dominates the error, so accumulation is a single float32 level.
#include <math.h>
#include <stdlib.h>

#include "psflib_internal.h"

namespace psflib {

constexpr int kGemmThreads = 256;
constexpr int kGM = 128;  // FP32: image rows per workgroup tile
constexpr int kGN = 64;   // FP32: scenes per workgroup tile
constexpr int kGK32 = 16; // FP32: K per tile
constexpr int kMidTiles = 32;
constexpr int kHM = 256;  // 16-bit: image rows per workgroup tile (64 per wave)
constexpr int kHN = 128;  // 16-bit: scenes per workgroup tile
constexpr int kHG = 8;    // 16-bit: 8-column groups per K stage (64 columns)
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

// XCD-aware tile order.  Workgroup w runs on XCD w % 8; give XCD x a
// contiguous run of tile indices (scenes fastest, then image rows, then K
// slices), so the tiles resident on one XCD share operand blocks in its L2.
// A bijection of [0, T) for any T.
__device__ __forceinline__ int64_t xcd_tile(int64_t w, int64_t T) {
  const int64_t x = w & 7, q = w >> 3;
  const int64_t base = T >> 3, rem = T & 7;
  return x * base + (x < rem ? x : rem) + q;
}

// ------------------------------------------------------------- FP32 -------
__global__ __launch_bounds__(kGemmThreads) void gemm_f32_kernel(const float* __restrict__ A,
                                                                const float* __restrict__ Z,
                                                                float* __restrict__ out,
                                                                int64_t M, int64_t K, int64_t B,
                                                                int64_t mblocks, int64_t nblocks,
                                                                int64_t splits,
                                                                int64_t ktiles_per_split) {
  __shared__ float As[2][kGK32][kGM];
  __shared__ float Bs[2][kGK32][kGN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t tile = xcd_tile(blockIdx.x, mblocks * nblocks * splits);
  const int64_t nb = tile % nblocks, mb = (tile / nblocks) % mblocks, sp = tile / (nblocks * mblocks);
  const int64_t m0 = mb * kGM;
  const int64_t n0 = nb * kGN;
  const int64_t ktiles = (K + kGK32 - 1) / kGK32;
  const int64_t kt0 = sp * ktiles_per_split;
  int64_t kt1 = kt0 + ktiles_per_split;
  if (kt1 > ktiles) kt1 = ktiles;
  float* dst = out + sp * B * M;
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
        ra[r] = *reinterpret_cast<const f32x4*>(A + k * M + m);  // cached: re-read per scene block
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
// One workgroup per scene; each thread handles whole 8-column groups (two
// 16-byte loads of Z and of the exponents, one 16-byte store).
__device__ __forceinline__ uint32_t to16(float s, bool bf16) {
  if (bf16) {
    uint32_t u = __float_as_uint(s);
    u += 0x7FFFu + ((u >> 16) & 1u);  // finite: round to nearest, ties to even
    return u >> 16;
  }
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)s);
}

template <bool BF16, bool VEC>
__global__ __launch_bounds__(256) void prep_scenes_kernel(const float* __restrict__ Z,
                                                          const int32_t* __restrict__ exps,
                                                          int64_t ncols, int64_t ncols_pad,
                                                          uint16_t* __restrict__ Zp,
                                                          int32_t* __restrict__ fexp) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;
  const float* z = Z + b * ncols;
  const int64_t ngroups = ncols_pad / 8;
  // group g of this scene, values and exponents (zeros past ncols)
  auto load8 = [&](int64_t g, float* v, int32_t* e) {
    const int64_t j0 = g * 8;
    if (VEC && j0 + 8 <= ncols) {
      const f32x4 v0 = *reinterpret_cast<const f32x4*>(z + j0);
      const f32x4 v1 = *reinterpret_cast<const f32x4*>(z + j0 + 4);
      typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
      const i32x4 e0 = *reinterpret_cast<const i32x4*>(exps + j0);
      const i32x4 e1 = *reinterpret_cast<const i32x4*>(exps + j0 + 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = v0[q]; v[4 + q] = v1[q];
        e[q] = e0[q]; e[4 + q] = e1[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const bool in = j0 + q < ncols;
        v[q] = in ? z[j0 + q] : 0.0f;
        e[q] = in ? exps[j0 + q] : 0;
      }
    }
  };
  double m = 0.0;
  for (int64_t g = threadIdx.x; g < ngroups; g += 256) {
    float v[8];
    int32_t e[8];
    load8(g, v, e);
#pragma unroll
    for (int q = 0; q < 8; ++q) m = fmax(m, ldexp((double)fabsf(v[q]), e[q]));
  }
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
  u32x4* zp = reinterpret_cast<u32x4*>(Zp + b * ncols_pad);
  for (int64_t g = threadIdx.x; g < ngroups; g += 256) {
    float v[8];
    int32_t e[8];
    load8(g, v, e);
    uint32_t h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q] = to16(ldexpf(v[q], e[q] + f), BF16);
    u32x4 pk;
    pk.x = h[0] | (h[1] << 16);
    pk.y = h[2] | (h[3] << 16);
    pk.z = h[4] | (h[5] << 16);
    pk.w = h[6] | (h[7] << 16);
    zp[g] = pk;
  }
}

template <bool BF16>
__device__ __forceinline__ f32x16 mfma16(const u32x4 a, const u32x4 b, const f32x16 c) {
  if constexpr (BF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

template <bool BF16>
__global__ __launch_bounds__(kGemmThreads, 2) void gemm_h16_kernel(
    const u32x4* __restrict__ Mp, const u32x4* __restrict__ Zp, const int32_t* __restrict__ fexp,
    float* __restrict__ out, int64_t M, int64_t ngroups, int64_t B, int64_t mblocks,
    int64_t nblocks, int64_t splits, int64_t stages_per_split) {
  __shared__ u32x4 Bs[2][kHG][kHN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile = xcd_tile(blockIdx.x, mblocks * nblocks * splits);
  const int64_t nb = tile % nblocks, mb = (tile / nblocks) % mblocks, sp = tile / (nblocks * mblocks);
  const int64_t m0 = mb * kHM, n0 = nb * kHN;
  const int64_t nstages = ngroups / kHG;  // ngroups is a multiple of 8
  const int64_t st0 = sp * stages_per_split;
  int64_t st1 = st0 + stages_per_split;
  if (st1 > nstages) st1 = nstages;
  float* dst = out + sp * B * M;
  const u32x4 z4 = {0u, 0u, 0u, 0u};

  // this lane's library rows (one per 32-row MFMA tile) and their validity
  const int64_t row0 = m0 + 64 * wave + (lane & 31);
  const bool ok0 = row0 < M, ok1 = row0 + 32 < M;
  const int half = lane >> 5;  // which 8-group of a 16-wide K step this lane feeds

  // A fragments of one stage: [k16 step][m tile]
  u32x4 a_cur[4][2], a_nxt[4][2];
  auto load_a = [&](int64_t st, u32x4 (&a)[4][2]) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int64_t g = st * kHG + 2 * ks + half;
      const u32x4* src = Mp + g * M + row0;
      a[ks][0] = ok0 ? src[0] : z4;  // cached: the XCD's other scene blocks re-read it
      a[ks][1] = ok1 ? src[32] : z4;
    }
  };
  // scene tile of one stage: thread -> scene n = tid / 2, groups 4*(tid%2) .. +3
  u32x4 b_reg[4];
  const int bn = tid >> 1, bg = (tid & 1) * 4;
  const bool bok = n0 + bn < B;
  auto load_b = [&](int64_t st) {
    const u32x4* src = Zp + (n0 + bn) * ngroups + st * kHG + bg;
#pragma unroll
    for (int q = 0; q < 4; ++q) b_reg[q] = bok ? src[q] : z4;
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[buf][bg + q][bn] = b_reg[q];
  };

  const f32x16 zero16 = {};
  f32x16 acc[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = zero16;

  if (st0 < st1) {
    load_a(st0, a_cur);
    load_b(st0);
    store_b(0);
  }
  __syncthreads();
  for (int64_t st = st0; st < st1; ++st) {
    const int cur = (int)((st - st0) & 1);
    const bool more = st + 1 < st1;
    if (more) {
      load_a(st + 1, a_nxt);
      load_b(st + 1);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      u32x4 bf[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) bf[u] = Bs[cur][2 * ks + half][32 * u + (lane & 31)];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = mfma16<BF16>(a_cur[ks][t], bf[u], acc[t][u]);
    }
    if (more) {
      store_b(cur ^ 1);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        a_cur[ks][0] = a_nxt[ks][0];
        a_cur[ks][1] = a_nxt[ks][1];
      }
    }
    __syncthreads();
  }
  // Without a K split the per-scene power of two is undone here; with one,
  // the slice-reduction kernel does it.
  const bool split = splits > 1;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u)
      store_acc(acc[t][u], dst, M, B, m0 + 64 * wave + 32 * t, n0 + 32 * u, lane, fexp, !split);
}

// Large batches: a 256 x 256 tile per workgroup, one workgroup per CU.  Each
// wave owns 64 image rows and all 256 scenes (2 x 8 accumulators of 32 x 32,
// held in the accumulation registers); library fragments are prefetched one
// K stage ahead into registers; the scene tile of the next stage is staged
// through registers, half a stage at a time, into the other half of a
// double-buffered LDS tile (2 x 32 KiB).  Scene fragments are double-buffered
// across the four 16-wide K steps of a stage so LDS reads overlap the MFMAs.
// Per flop it moves half the L2 traffic of the 256 x 128 tile.
template <bool BF16>
__global__ __launch_bounds__(kGemmThreads, 1) void gemm_h16_wide_kernel(
    const u32x4* __restrict__ Mp, const u32x4* __restrict__ Zp, const int32_t* __restrict__ fexp,
    float* __restrict__ out, int64_t M, int64_t ngroups, int64_t B, int64_t mblocks,
    int64_t nblocks, int64_t splits, int64_t stages_per_split) {
  constexpr int TN = 2 * kHN;  // 256 scenes
  __shared__ u32x4 Bs[2][kHG][TN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile = xcd_tile(blockIdx.x, mblocks * nblocks * splits);
  const int64_t nb = tile % nblocks, mb = (tile / nblocks) % mblocks, sp = tile / (nblocks * mblocks);
  const int64_t m0 = mb * kHM, n0 = nb * TN;
  const int64_t nstages = ngroups / kHG;
  const int64_t st0 = sp * stages_per_split;
  int64_t st1 = st0 + stages_per_split;
  if (st1 > nstages) st1 = nstages;
  float* dst = out + sp * B * M;
  const u32x4 z4 = {0u, 0u, 0u, 0u};

  const int64_t row0 = m0 + 64 * wave + (lane & 31);
  const bool ok0 = row0 < M, ok1 = row0 + 32 < M;
  const int half = lane >> 5;

  u32x4 a_cur[4][2], a_nxt[4][2];
  auto load_a = [&](int64_t st, u32x4 (&a)[4][2]) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int64_t g = st * kHG + 2 * ks + half;
      const u32x4* src = Mp + g * M + row0;
      a[ks][0] = ok0 ? src[0] : z4;
      a[ks][1] = ok1 ? src[32] : z4;
    }
  };
  u32x4 b_reg[kHG / 2];  // scene n = tid, 4 of the 8 groups of a stage
  const bool bok = n0 + tid < B;
  auto load_b = [&](int64_t st, int h) {
    const u32x4* src = Zp + (n0 + tid) * ngroups + st * kHG + 4 * h;
#pragma unroll
    for (int q = 0; q < 4; ++q) b_reg[q] = bok ? src[q] : z4;
  };
  auto store_b = [&](int buf, int h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[buf][4 * h + q][tid] = b_reg[q];
  };

  const f32x16 zero16 = {};
  f32x16 acc[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[t][u] = zero16;

  if (st0 < st1) {
    load_a(st0, a_cur);
    load_b(st0, 0);
    store_b(0, 0);
    load_b(st0, 1);
    store_b(0, 1);
  }
  __syncthreads();
  for (int64_t st = st0; st < st1; ++st) {
    const int cur = (int)((st - st0) & 1);
    const bool more = st + 1 < st1;
    if (more) {
      load_a(st + 1, a_nxt);
      load_b(st + 1, 0);
    }
    u32x4 bfr[2][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) bfr[0][u] = Bs[cur][half][32 * u + (lane & 31)];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks < 3) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          bfr[(ks + 1) & 1][u] = Bs[cur][2 * (ks + 1) + half][32 * u + (lane & 31)];
      }
      if (ks == 1 && more) {
        store_b(cur ^ 1, 0);
        load_b(st + 1, 1);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc[0][u] = mfma16<BF16>(a_cur[ks][0], bfr[ks & 1][u], acc[0][u]);
        acc[1][u] = mfma16<BF16>(a_cur[ks][1], bfr[ks & 1][u], acc[1][u]);
      }
    }
    if (more) {
      store_b(cur ^ 1, 1);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        a_cur[ks][0] = a_nxt[ks][0];
        a_cur[ks][1] = a_nxt[ks][1];
      }
    }
    __syncthreads();
  }
  const bool split = splits > 1;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u)
      store_acc(acc[t][u], dst, M, B, m0 + 64 * wave + 32 * t, n0 + 32 * u, lane, fexp, !split);
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
struct GemmPlan {
  int64_t mblocks, nblocks, kunits, splits, per;  // kunits: K tiles (FP32) or K stages (16-bit)
  bool wide;  // 16-bit: 256 x 256 tiles, one workgroup per CU
};

static GemmPlan plan_gemm(int storage, int64_t M, int64_t ncols, int64_t ncols_pad, int64_t bc) {
  GemmPlan p;
  const bool f32 = storage == PSFLIB_FP32;
  static const long wide_env = [] {
    const char* e = getenv("PSFLIB_GEMM_WIDE");  // tuning override: 0 off, 1 on
    return e ? strtol(e, nullptr, 10) : -1L;
  }();
  p.wide = !f32 && bc > kHN && wide_env == 1;
  const int64_t tm = f32 ? kGM : kHM, tn = f32 ? kGN : (p.wide ? 2 * kHN : kHN);
  p.mblocks = (M + tm - 1) / tm;
  p.nblocks = (bc + tn - 1) / tn;
  p.kunits = f32 ? (ncols + kGK32 - 1) / kGK32 : (ncols_pad / 8) / kHG;
  // about two workgroups per CU (512), split K if the tile grid is smaller
  const int64_t want = f32 ? 1024 : (p.wide ? 256 : 512);
  const int64_t tiles = p.mblocks * p.nblocks;
  int64_t s = (want + tiles - 1) / tiles;
  if (s > 16) s = 16;
  if (s > p.kunits) s = p.kunits;
  if (s < 1) s = 1;
  p.per = (p.kunits + s - 1) / s;
  p.splits = (p.kunits + p.per - 1) / p.per;  // no empty slice
  if (p.splits < 1) p.splits = 1;
  return p;
}

static int64_t chunk_of(int B) { return B < kMaxBatchChunk ? B : kMaxBatchChunk; }

static size_t split_partial_bytes(int storage, int64_t M, int64_t ncols, int64_t ncols_pad,
                                  int64_t bc) {
  const GemmPlan p = plan_gemm(storage, M, ncols, ncols_pad, bc);
  return p.splits > 1 ? (size_t)p.splits * (size_t)bc * (size_t)M * 4 : 0;
}

size_t batched_scratch_bytes(int storage, int64_t M, int64_t ncols, int64_t ncols_pad, int B) {
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
  size_t part = split_partial_bytes(storage, M, ncols, ncols_pad, bc);
  const int64_t rem = B % bc;
  if (rem) {
    const size_t p2 = split_partial_bytes(storage, M, ncols, ncols_pad, rem);
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
    const GemmPlan p = plan_gemm(storage, M, ncols, ncols_pad, bc);
    const float* Zc = Z + b0 * ncols;
    float* outc = out + b0 * M;
    hipError_t e;
    // every pass must fit the scratch sized by batched_scratch_bytes()
    if (off + split_partial_bytes(storage, M, ncols, ncols_pad, bc) > scratch_bytes)
      return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(p.mblocks * p.nblocks * p.splits);
    float* dst = p.splits > 1 ? part : outc;
    if (storage == PSFLIB_FP32) {
      gemm_f32_kernel<<<grid, kGemmThreads, 0, s>>>(reinterpret_cast<const float*>(lib), Zc, dst,
                                                    M, ncols, bc, p.mblocks, p.nblocks, p.splits,
                                                    p.per);
      e = hipGetLastError();
    } else {
      const bool bf = storage == PSFLIB_BF16_POW2;
      const bool vec = (ncols % 8) == 0 && (reinterpret_cast<uintptr_t>(Zc) % 16) == 0;
      if (bf && vec)
        prep_scenes_kernel<true, true><<<(unsigned)bc, 256, 0, s>>>(Zc, exps, ncols, ncols_pad, Zp, fexp);
      else if (bf)
        prep_scenes_kernel<true, false><<<(unsigned)bc, 256, 0, s>>>(Zc, exps, ncols, ncols_pad, Zp, fexp);
      else if (vec)
        prep_scenes_kernel<false, true><<<(unsigned)bc, 256, 0, s>>>(Zc, exps, ncols, ncols_pad, Zp, fexp);
      else
        prep_scenes_kernel<false, false><<<(unsigned)bc, 256, 0, s>>>(Zc, exps, ncols, ncols_pad, Zp, fexp);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      const int64_t ngroups = ncols_pad / 8;
      const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
      const u32x4* Zq = reinterpret_cast<const u32x4*>(Zp);
      if (p.wide && bf)
        gemm_h16_wide_kernel<true><<<grid, kGemmThreads, 0, s>>>(Mp, Zq, fexp, dst, M, ngroups, bc,
                                                                 p.mblocks, p.nblocks, p.splits, p.per);
      else if (p.wide)
        gemm_h16_wide_kernel<false><<<grid, kGemmThreads, 0, s>>>(Mp, Zq, fexp, dst, M, ngroups, bc,
                                                                  p.mblocks, p.nblocks, p.splits, p.per);
      else if (bf)
        gemm_h16_kernel<true><<<grid, kGemmThreads, 0, s>>>(Mp, Zq, fexp, dst, M, ngroups, bc,
                                                            p.mblocks, p.nblocks, p.splits, p.per);
      else
        gemm_h16_kernel<false><<<grid, kGemmThreads, 0, s>>>(Mp, Zq, fexp, dst, M, ngroups, bc,
                                                             p.mblocks, p.nblocks, p.splits, p.per);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (p.splits > 1) {
      const int64_t BM = bc * M;
      reduce_splits_kernel<<<(unsigned)((BM + 255) / 256), 256, 0, s>>>(
          part, (int)p.splits, BM, M, storage == PSFLIB_FP32 ? nullptr : fexp, outc);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace psflib
