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
// FP32: each wave computes 64 image rows x 64 scenes (32 for batches of at
// most 32) on its own, streaming library rows from HBM straight into
// registers and pre-arranged scene fragments from L2, four groups of 8
// columns ahead; accumulation is blocked in two levels so float32 rounding
// chains stay short.
//
// 16-bit, up to 256 scenes: a workgroup of 4 waves computes a 256 x TN tile
// (TN = 128 or 256 scenes); each wave owns 64 image rows and all TN scenes
// (2 x TN/32 accumulators of 32 x 32).  K advances in stages of 32 columns
// through a 4-slot ring, three stages ahead of use: library fragments (each
// used by one wave only) go from HBM straight into registers, and the scene
// tile (shared by the 4 waves) is copied from a group-major packed copy of
// the scenes into LDS by the buffer unit, with no register staging.  Above
// 256 scenes a workgroup of 8 waves (two per SIMD) computes a 256 x 256 tile
// with both operand tiles copied into LDS.  The 16-bit rounding of the inputs
// dominates the error, so accumulation is a single float32 level.
#include <math.h>
#include <stdlib.h>

#include <algorithm>

#include "psflib_internal.h"

namespace psflib {

constexpr int kGemmThreads = 256;
constexpr int kGM = 256;  // FP32: image rows per workgroup (64 per wave)
constexpr int kHM = 256;  // 16-bit: image rows per workgroup tile (64 per wave)
constexpr int kHG = 4;    // 16-bit: 8-column groups per K stage (32 columns)
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
// Scenes are first copied into a fragment-major form Zp: for each 8-column
// group g and block of 32 scenes sb, 64 lanes x 4 floats (1 KiB), lane
// l = 32h + n holding Z[32 sb + n][8g + 4h .. 8g + 4h + 3] (zeros past the
// batch and past K).  One 16-byte load per lane is then the scene operand
// of four MFMA steps.
constexpr int kF32Ring = 4;    // 8-column groups in flight per wave
constexpr int kF32Block = 16;  // groups per inner accumulation block (a multiple of kF32Ring)

template <bool VEC>
__global__ __launch_bounds__(256) void pack_f32_scenes_kernel(const float* __restrict__ Z,
                                                              int64_t K, int64_t B, int64_t ngroups,
                                                              int64_t SB, f32x4* __restrict__ Zp) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ngroups * SB * 64) return;
  const int l = (int)(t & 63);
  const int64_t sb = (t >> 6) % SB, g = (t >> 6) / SB;
  const int64_t n = 32 * sb + (l & 31), k = 8 * g + 4 * (l >> 5);
  f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
  if (n < B) {
    const float* src = Z + n * K + k;
    if (VEC && k + 4 <= K) {
      v = *reinterpret_cast<const f32x4*>(src);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (k + c < K) v[c] = src[c];
    }
  }
  Zp[t] = v;
}

// A workgroup is 4 independent waves, each computing 64 image rows x 32*NB
// scenes with v_mfma_f32_32x32x2f32.  Nothing is shared between waves, so
// there is no LDS and no barrier: each wave streams its library rows straight
// from HBM into registers and its scene fragments from L2, kF32Ring groups
// of 8 columns ahead of use.
//
// Operand mapping for group g and MFMA step s (0..3): lane (i = l % 32,
// h = l / 32) supplies column k = 8g + 4h + s for the two k-slots of the
// MFMA, with A rows m0 + 2i (MFMA t = 0) and m0 + 2i + 1 (t = 1) read as one
// 8-byte load, and the scene value of the same column from its Zp fragment.
// Output row i of MFMA t is image row m0 + 2i + t.
//
// All loads are buffer loads whose descriptor covers only live data: columns
// past K and groups past the slice read as zero, so the loop runs whole
// accumulation blocks with no bounds tests.  Rows past the image read the
// next column (finite values, never stored) or zero.
//
// Accumulation is blocked in two levels (kF32Block groups, then the slice)
// so float32 rounding chains stay short; split-K slices are added by
// reduce_splits_kernel in a fixed order.
//
// NT: library loads carry the non-temporal hint, for grids with one scene
// tile, where no other workgroup reads the same library rows.
template <int NB, bool VEC, bool NT>
__global__ __launch_bounds__(kGemmThreads, 2) void gemm_f32_kernel(
    const float* __restrict__ A, const f32x4* __restrict__ Zp, float* __restrict__ out, int64_t M,
    int64_t K, int64_t B, int64_t SB, int64_t mblocks, int64_t nblocks, int64_t splits,
    int64_t gper) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tile = xcd_tile(blockIdx.x, mblocks * nblocks * splits);
  const int64_t nb = tile % nblocks, mb = (tile / nblocks) % mblocks, sp = tile / (nblocks * mblocks);
  const int64_t m0 = mb * kGM + 64 * wave;
  if (m0 >= M) return;  // no barriers: a wave past the image leaves at once
  // group indices fit 32 bits (K < 2^31); 32-bit scalar compares are native
  const int ngroups = (int)((K + 7) / 8);
  const int g0 = (int)(sp * gper);
  const int g1 = (g0 + (int)gper < ngroups) ? g0 + (int)gper : ngroups;
  const uint32_t colbytes = (uint32_t)(M * 4);
  const int i = lane & 31, h = lane >> 5;
  uint32_t voff[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) voff[s] = (uint32_t)(((4 * h + s) * M + m0 + 2 * i) * 4);
  const uint32_t zoff = (uint32_t)((nb * NB * 64 + lane) * 16);

  constexpr int kAux = NT ? 2 : 0;  // cache-policy bits of the library loads
  f32x2 ra[kF32Ring][4];
  f32x4 rb[kF32Ring][NB];
  auto issue = [&](int g, int slot) {
    const bool live = g < g1;
    const int gc = live ? g : g1 - 1;
    // the descriptor ends with the group's last live column (8 M floats <= 2^31
    // bytes; the record count is an unsigned 32-bit field): rows a wave reads
    // past the image read zero there, never past the library
    const int left = (int)(K - 8 * (int64_t)gc);
    const int abytes = !live ? 0 : (int)((uint32_t)(left < 8 ? left : 8) * colbytes);
    const __amdgpu_buffer_rsrc_t ra_d = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(A + 8 * (int64_t)gc * M), (short)0, abytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rb_d = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Zp + (int64_t)gc * SB * 64), (short)0, live ? (int)(SB * 1024) : 0, 0x00020000);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (VEC) {
        ra[slot][s] = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(ra_d, voff[s], 0, kAux));
      } else {
        ra[slot][s][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra_d, voff[s], 0, kAux));
        ra[slot][s][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra_d, voff[s] + 4, 0, kAux));
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
      rb[slot][q] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb_d, zoff + 1024 * q, 0, 0));
  };

  const f32x16 zero16 = {};
  f32x16 acc[2][NB], tot[2][NB];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < NB; ++q) tot[t][q] = zero16;

  const int nblk = g1 > g0 ? (g1 - g0 + kF32Block - 1) / kF32Block : 0;
  if (nblk > 0) {
#pragma unroll
    for (int r = 0; r < kF32Ring; ++r) issue(g0 + r, r);
  }
  for (int blk = 0; blk < nblk; ++blk) {
    const int gb = g0 + blk * kF32Block;
#pragma unroll
    for (int j = 0; j < kF32Block; ++j) {
      const int slot = j % kF32Ring;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int t = 0; t < 2; ++t)
            acc[t][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(ra[slot][s][t], rb[slot][q][s],
                                                            (j == 0 && s == 0) ? zero16 : acc[t][q],
                                                            0, 0, 0);
      issue(gb + j + kF32Ring, slot);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < NB; ++q) tot[t][q] += acc[t][q];
  }

  // lane holds scene column l % 32 and MFMA rows 8(r/4) + 4h + r%4, i.e. image
  // rows m0 + 16(r/4) + 8h + 2(r%4) + t: 8 consecutive rows per r/4
  float* dst = out + sp * B * M;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int64_t n = (nb * NB + q) * 32 + i;
    if (n >= B) continue;
    float* row = dst + n * M;
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      const int64_t m = m0 + 16 * r4 + 8 * h;
      f32x4 lo, hi;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        lo[2 * e] = tot[0][q][4 * r4 + e];
        lo[2 * e + 1] = tot[1][q][4 * r4 + e];
        hi[2 * e] = tot[0][q][4 * r4 + 2 + e];
        hi[2 * e + 1] = tot[1][q][4 * r4 + 2 + e];
      }
      if ((M % 4) == 0 && m + 8 <= M) {
        *reinterpret_cast<f32x4*>(row + m) = lo;
        *reinterpret_cast<f32x4*>(row + m + 4) = hi;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (m + e < M) row[m + e] = lo[e];
          if (m + 4 + e < M) row[m + 4 + e] = hi[e];
        }
      }
    }
  }
}

// ------------------------------------------------------------- 16-bit -----
// Scene preparation, in two passes over the fp32 scenes:
//   f_b:  max_j |Z[b][j]| 2^(e_j + f_b) lands in [2^14, 2^15)  (0 for an empty
//         scene), so no scene underflows or overflows the 16-bit format
//         whatever its units (one workgroup of 1024 threads per scene);
//   Zg[g][b] = RN16(Z[b][8g .. 8g+7] * 2^(e_j + f_b)), 16 bytes per (group, scene),
// stored group-major with the batch padded to whole scene tiles (zeros), so
// one K stage of a scene tile is a contiguous run the GEMM copies straight to LDS.
__device__ __forceinline__ uint32_t to16(float s, bool bf16) {
  if (bf16) {
    uint32_t u = __float_as_uint(s);
    u += 0x7FFFu + ((u >> 16) & 1u);  // finite: round to nearest, ties to even
    return u >> 16;
  }
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)s);
}

// 8 values and column exponents of group g of one scene (zeros past ncols)
template <bool VEC>
__device__ __forceinline__ void load_group(const float* __restrict__ z,
                                           const int32_t* __restrict__ exps, int64_t ncols,
                                           int64_t g, float* v, int32_t* e) {
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
}

// f_b of one scene per workgroup of 1024 threads: the maximum of
// |Z_bj| 2^e_j in float64 (exact: a power-of-two scaling of a float32), each
// thread over a few 8-column groups (two loads of each in flight), then a
// wave and a workgroup reduction.  The maximum does not depend on the order.
template <bool VEC>
__global__ __launch_bounds__(1024) void scene_exponent_kernel(const float* __restrict__ Z,
                                                              const int32_t* __restrict__ exps,
                                                              int64_t ncols, int64_t ngroups,
                                                              int32_t* __restrict__ fexp) {
  __shared__ double red[16];
  const int64_t b = blockIdx.x;
  const float* z = Z + b * ncols;
  double m = 0.0;
  int64_t g = threadIdx.x;
  for (; g + 1024 < ngroups; g += 2048) {
    float v[2][8];
    int32_t e[2][8];
    load_group<VEC>(z, exps, ncols, g, v[0], e[0]);
    load_group<VEC>(z, exps, ncols, g + 1024, v[1], e[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 8; ++q) m = fmax(m, ldexp((double)fabsf(v[h][q]), e[h][q]));
  }
  if (g < ngroups) {
    float v[8];
    int32_t e[8];
    load_group<VEC>(z, exps, ncols, g, v, e);
#pragma unroll
    for (int q = 0; q < 8; ++q) m = fmax(m, ldexp((double)fabsf(v[q]), e[q]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = red[0];
#pragma unroll
    for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
    int f = 0;
    if (m > 0.0) {
      int E;
      (void)frexp(m, &E);
      f = 15 - E;  // max |Z_bj| 2^(e_j + f) in [2^14, 2^15)
    }
    fexp[b] = f;
  }
}

// Thread = (slot group g, scene n): 8 lanes cover one group of 8 consecutive
// scenes and write 8 whole 128-byte lines of Zg per wave.  Slot s of the
// group holds column perm[s] of the library (the scene value gathered from
// it) with exponent eslot[s]; padding slots (perm -1) get zeros.
template <bool BF16>
__global__ __launch_bounds__(256) void pack_scenes_kernel(const float* __restrict__ Z,
                                                          const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ eslot,
                                                          const int32_t* __restrict__ fexp,
                                                          int64_t ncols, int64_t ngroups,
                                                          int64_t bc, int64_t Bp,
                                                          u32x4* __restrict__ Zg) {
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  const int64_t g = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
  if (g >= ngroups) return;
  const int64_t n = (int64_t)blockIdx.y * 8 + (threadIdx.x & 7);
  u32x4 pk = {0u, 0u, 0u, 0u};
  if (n < bc) {
    const i32x4 p0 = *reinterpret_cast<const i32x4*>(perm + 8 * g);
    const i32x4 p1 = *reinterpret_cast<const i32x4*>(perm + 8 * g + 4);
    const i32x4 e0 = *reinterpret_cast<const i32x4*>(eslot + 8 * g);
    const i32x4 e1 = *reinterpret_cast<const i32x4*>(eslot + 8 * g + 4);
    const float* z = Z + n * ncols;
    float v[8];
    int32_t e[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = p0[q] >= 0 ? z[p0[q]] : 0.0f;
      v[4 + q] = p1[q] >= 0 ? z[p1[q]] : 0.0f;
      e[q] = e0[q];
      e[4 + q] = e1[q];
    }
    const int f = fexp[n];
    uint32_t h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q] = to16(ldexpf(v[q], e[q] + f), BF16);
    pk.x = h[0] | (h[1] << 16);
    pk.y = h[2] | (h[3] << 16);
    pk.z = h[4] | (h[5] << 16);
    pk.w = h[6] | (h[7] << 16);
  }
  Zg[g * Bp + n] = pk;
}

// Scenes of at most kStageMaxCols columns are packed by one workgroup of 1024
// threads per scene that reads the scene once, coalesced (the slot order
// gathers columns from all over the scene: read straight from HBM, each
// 4-byte value would cost a sector): the scene into LDS (16-byte loads, all
// of a thread's issued before their use), f_b
// from it (as scene_exponent_kernel), then the slots in order, gathered from
// LDS, scaled by 2^(eslot + f_b) and rounded, each group's 16 bytes written to
// its place Zg[g][b] of the operand.  A workgroup writes one 16-byte piece of
// every 128-byte line of the operand; the 8 scenes of a line are numbered to
// land on one XCD back to back (dispatch is round-robin over the 8 XCDs), so
// each line fills in that XCD's L2.  Workgroups of the padding scenes (b >= bc)
// write zeros.  (A [scene][group] copy followed by a transpose kernel took
// 27 + 12 us at B = 1024 against 34 us.)
template <bool BF16, bool VEC>
__global__ __launch_bounds__(1024) void stage_slots16_kernel(const float* __restrict__ Z,
                                                             const int32_t* __restrict__ exps,
                                                             const int32_t* __restrict__ perm,
                                                             const int32_t* __restrict__ eslot,
                                                             int64_t ncols, int64_t ngroups,
                                                             int64_t bc, int64_t Bp,
                                                             int32_t* __restrict__ fexp,
                                                             u32x4* __restrict__ Zg) {
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  extern __shared__ float zl[];  // the scene, ncols floats
  __shared__ double red[16];
  __shared__ int s_f;
  // Bp is a multiple of 64: workgroups x, x + 8, ..., x + 56 (one XCD) take
  // scenes 8x .. 8x + 7, and so on per 64 scenes
  const int64_t wg = blockIdx.x, xcd = wg % 8, rnd = wg / 8;
  const int64_t b = 8 * (xcd + 8 * (rnd / 8)) + rnd % 8;
  const int tid = threadIdx.x;
  if (b >= bc) {
    for (int64_t g = tid; g < ngroups; g += 1024) Zg[g * Bp + b] = (u32x4){0u, 0u, 0u, 0u};
    return;
  }
  const float* z = Z + b * ncols;
  double m = 0.0;
  if constexpr (VEC) {
    // batches of 4 independent 16-byte loads per thread (all of a 16384-column
    // scene in one batch), then their use
    for (int64_t j0 = 4 * (int64_t)tid; j0 < ncols; j0 += 4 * 4 * 1024) {
      f32x4 v[4];
      i32x4 e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + 4 * 1024 * u;
        if (j < ncols) {
          v[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(z + j));
          e[u] = *reinterpret_cast<const i32x4*>(exps + j);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + 4 * 1024 * u;
        if (j < ncols) {
          *reinterpret_cast<f32x4*>(zl + j) = v[u];
#pragma unroll
          for (int q = 0; q < 4; ++q) m = fmax(m, ldexp((double)fabsf(v[u][q]), e[u][q]));
        }
      }
    }
  } else {
    for (int64_t j = tid; j < ncols; j += 1024) {
      const float v = z[j];
      zl[j] = v;
      m = fmax(m, ldexp((double)fabsf(v), exps[j]));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    m = red[0];
#pragma unroll
    for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
    int f = 0;
    if (m > 0.0) {
      int E;
      (void)frexp(m, &E);
      f = 15 - E;  // max |Z_bj| 2^(e_j + f) in [2^14, 2^15)
    }
    s_f = f;
    fexp[b] = f;
  }
  __syncthreads();
  const int f = s_f;
  // two groups per thread per batch: the slot maps of both loaded first
  for (int64_t g0 = tid; g0 < ngroups; g0 += 2 * 1024) {
    i32x4 p0[2], p1[2], e0[2], e1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t g = g0 + 1024 * u;
      if (g < ngroups) {
        p0[u] = *reinterpret_cast<const i32x4*>(perm + 8 * g);
        p1[u] = *reinterpret_cast<const i32x4*>(perm + 8 * g + 4);
        e0[u] = *reinterpret_cast<const i32x4*>(eslot + 8 * g);
        e1[u] = *reinterpret_cast<const i32x4*>(eslot + 8 * g + 4);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t g = g0 + 1024 * u;
      if (g < ngroups) {
        uint32_t h[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          h[q] = to16(ldexpf(p0[u][q] >= 0 ? zl[p0[u][q]] : 0.0f, e0[u][q] + f), BF16);
          h[4 + q] = to16(ldexpf(p1[u][q] >= 0 ? zl[p1[u][q]] : 0.0f, e1[u][q] + f), BF16);
        }
        Zg[g * Bp + b] = (u32x4){h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                 h[6] | (h[7] << 16)};
      }
    }
  }
}

// Two scenes per workgroup, for scenes of at most kStagePairCols columns (both
// in LDS): the same steps as stage_slots16_kernel, with lanes 2i and 2i+1
// packing one group of the two scenes, so each pair of lanes writes 32
// contiguous bytes of the operand line (half as many L2 write requests).
// Scenes 2q, 2q+1 of the 4 pairs of an 8-scene line are numbered to run on
// one XCD back to back.
template <bool BF16, bool VEC>
__global__ __launch_bounds__(1024) void stage_pairs16_kernel(const float* __restrict__ Z,
                                                             const int32_t* __restrict__ exps,
                                                             const int32_t* __restrict__ perm,
                                                             const int32_t* __restrict__ eslot,
                                                             int64_t ncols, int64_t ngroups,
                                                             int64_t bc, int64_t Bp,
                                                             int32_t* __restrict__ fexp,
                                                             u32x4* __restrict__ Zg) {
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  extern __shared__ float zl[];  // the two scenes, ncols floats each
  __shared__ double red[2][16];
  __shared__ int s_f[2];
  const int64_t wg = blockIdx.x, xcd = wg % 8, rnd = wg / 8;
  const int64_t b0 = 2 * (4 * (xcd + 8 * (rnd / 4)) + rnd % 4);
  const int tid = threadIdx.x;
  if (b0 >= bc) {
    for (int64_t t = tid; t < 2 * ngroups; t += 1024) Zg[(t >> 1) * Bp + b0 + (t & 1)] = (u32x4){0u, 0u, 0u, 0u};
    return;
  }
  const bool live1 = b0 + 1 < bc;
  const float* z0 = Z + b0 * ncols;
  const float* z1 = live1 ? z0 + ncols : z0;
  float* zl1 = zl + ncols;
  double m0 = 0.0, m1 = 0.0;
  if constexpr (VEC) {
    for (int64_t j0 = 4 * (int64_t)tid; j0 < ncols; j0 += 4 * 4 * 1024) {
      f32x4 v0[4], v1[4];
      i32x4 e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + 4 * 1024 * u;
        if (j < ncols) {
          v0[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(z0 + j));
          v1[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(z1 + j));
          e[u] = *reinterpret_cast<const i32x4*>(exps + j);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + 4 * 1024 * u;
        if (j < ncols) {
          if (!live1) v1[u] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
          *reinterpret_cast<f32x4*>(zl + j) = v0[u];
          *reinterpret_cast<f32x4*>(zl1 + j) = v1[u];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            m0 = fmax(m0, ldexp((double)fabsf(v0[u][q]), e[u][q]));
            m1 = fmax(m1, ldexp((double)fabsf(v1[u][q]), e[u][q]));
          }
        }
      }
    }
  } else {
    for (int64_t j = tid; j < ncols; j += 1024) {
      const float v0 = z0[j], v1 = live1 ? z1[j] : 0.0f;
      zl[j] = v0;
      zl1[j] = v1;
      m0 = fmax(m0, ldexp((double)fabsf(v0), exps[j]));
      m1 = fmax(m1, ldexp((double)fabsf(v1), exps[j]));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m0 = fmax(m0, __shfl_xor(m0, off, 64));
    m1 = fmax(m1, __shfl_xor(m1, off, 64));
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = m0;
    red[1][tid >> 6] = m1;
  }
  __syncthreads();
  if (tid < 2) {
    double m = red[tid][0];
#pragma unroll
    for (int w = 1; w < 16; ++w) m = fmax(m, red[tid][w]);
    int f = 0;
    if (m > 0.0) {
      int E;
      (void)frexp(m, &E);
      f = 15 - E;  // max |Z_bj| 2^(e_j + f) in [2^14, 2^15)
    }
    s_f[tid] = f;
    if (b0 + tid < bc) fexp[b0 + tid] = f;
  }
  __syncthreads();
  const int sc = tid & 1;
  const int f = s_f[sc];
  const float* zs = sc ? zl1 : zl;
  // item t = 2 g + sc; two items per thread per batch, slot maps loaded first
  for (int64_t g0 = tid >> 1; g0 < ngroups; g0 += 2 * 512) {
    i32x4 p0[2], p1[2], e0[2], e1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t g = g0 + 512 * u;
      if (g < ngroups) {
        p0[u] = *reinterpret_cast<const i32x4*>(perm + 8 * g);
        p1[u] = *reinterpret_cast<const i32x4*>(perm + 8 * g + 4);
        e0[u] = *reinterpret_cast<const i32x4*>(eslot + 8 * g);
        e1[u] = *reinterpret_cast<const i32x4*>(eslot + 8 * g + 4);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t g = g0 + 512 * u;
      if (g < ngroups) {
        uint32_t h[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          h[q] = to16(ldexpf(p0[u][q] >= 0 ? zs[p0[u][q]] : 0.0f, e0[u][q] + f), BF16);
          h[4 + q] = to16(ldexpf(p1[u][q] >= 0 ? zs[p1[u][q]] : 0.0f, e1[u][q] + f), BF16);
        }
        Zg[g * Bp + b0 + sc] = (u32x4){h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                      h[6] | (h[7] << 16)};
      }
    }
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

// The 16-bit GEMM.  Workgroup = 4 waves, tile 256 image rows x TN scenes,
// K stages of 32 columns (4 groups); each wave owns 64 rows and all TN scenes
// (2 x TN/32 accumulators of 32 x 32: 128 registers at TN = 128, two
// workgroups per CU; 256 at TN = 256, one).  Operands of a stage travel on
// two paths into a 4-slot ring, three stages ahead of use:
//   library fragments (each used by one wave only) go from memory straight to
//   registers, 4 x 16 bytes per lane per stage;
//   the scene tile (shared by the 4 waves) is copied from memory into LDS by
//   the buffer unit (buffer_load ... lds), TN x 16 bytes per wave per stage
//   (C = TN/64 copies per lane), with no register staging.
// Each lane issues exactly 4 + C vector-memory operations per stage, and
// those complete in issue order, so "at most 2 (4 + C) outstanding" means
// this wave's copies for the stage about to be used have landed; the barrier
// after that wait makes every wave's copies visible, and the lgkmcnt(0)
// before it ends this wave's LDS reads of the slot the next copy overwrites.
// Each ring slot is its own LDS array, so the compiler can tell that the
// scene-fragment reads of one slot do not alias the copies in flight into
// the others: it waits only for the copy into the slot being read (the same
// bound), and schedules the reads between the products with partial lgkmcnt
// waits (at B = 512, one workgroup per CU, ~306 -> 272-290 us against
// whole-block reads that waited for all four fragments before any product).
constexpr int kHRing = 4;    // ring slots
constexpr int kHUnroll = 16; // stages per main-loop iteration (a multiple of kHRing)

// NT: library loads with the non-temporal hint, for grids with one scene
// tile (no other workgroup re-reads a library block; B <= 128: 130 -> 120 us
// at 128^2; the 256-scene tile, 128 < B <= 256: ~2.4% at B = 160 and 256,
// re-measured with the current staging).  With several scene tiles the hint
// costs the L2 reuse (B = 1024: +12%).
template <bool BF16, int TN, bool NT>
__global__ __launch_bounds__(kGemmThreads, TN == 128 ? 2 : 1) void gemm_h16_kernel(
    const u32x4* Mp, const u32x4* Zg, const int32_t* __restrict__ fexp,
    float* __restrict__ out, int64_t M, int64_t ngroups, int64_t B, int64_t Bp, int64_t mblocks,
    int64_t nblocks, int64_t splits, int64_t stages_per_split) {
  constexpr int NU = TN / 32;     // 32-scene accumulator columns per wave
  constexpr int NC = TN / 64;     // LDS copies per lane per stage
  __shared__ u32x4 Bs0[kHG][TN], Bs1[kHG][TN], Bs2[kHG][TN], Bs3[kHG][TN];  // ring slots
  auto slot_of = [&](int slot) -> u32x4 (*)[TN] {
    return slot == 0 ? Bs0 : slot == 1 ? Bs1 : slot == 2 ? Bs2 : Bs3;
  };
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t tile = xcd_tile(blockIdx.x, mblocks * nblocks * splits);
  const int64_t nb = tile % nblocks, mb = (tile / nblocks) % mblocks, sp = tile / (nblocks * mblocks);
  const int64_t m0 = mb * kHM, n0 = nb * TN;
  const int64_t nstages = ngroups / kHG;  // ngroups is a multiple of 8
  const int64_t st0 = sp * stages_per_split;
  const int64_t ns = (nstages - st0 < stages_per_split ? nstages - st0 : stages_per_split);
  float* dst = out + sp * B * M;

  // library rows of this lane (one per 32-row MFMA tile); rows past M read
  // row M-1 (valid addresses; those results are never stored)
  int64_t row0 = m0 + 64 * wave + (lane & 31), row1 = row0 + 32;
  if (row0 > M - 1) row0 = M - 1;
  if (row1 > M - 1) row1 = M - 1;
  const int half = lane >> 5;  // which group of a 16-wide K step this lane feeds
  const uint32_t offa0 = (uint32_t)((half * M + row0) * 16);
  const uint32_t offa1 = (uint32_t)((half * M + row1) * 16);
  const char* Ab = reinterpret_cast<const char*>(Mp);
  // this wave copies group `wave` of each stage: scenes n0 .. n0+TN-1
  const char* Zb = reinterpret_cast<const char*>(Zg + (int64_t)wave * Bp + n0);
  const int offb = lane * 16;

  u32x4 a[kHRing][2][2];  // [slot][k16 step][m tile]
  auto issue = [&](int64_t ls, int slot) {  // local stage ls of this K slice
    const int64_t st = st0 + ls;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const char* base = Ab + (st * kHG + 2 * ks) * M * 16;
      if constexpr (NT) {
        a[slot][ks][0] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base + offa0));
        a[slot][ks][1] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base + offa1));
      } else {
        a[slot][ks][0] = *reinterpret_cast<const u32x4*>(base + offa0);
        a[slot][ks][1] = *reinterpret_cast<const u32x4*>(base + offa1);
      }
    }
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Zb + st * kHG * Bp * 16), (short)0, 0x7FFFFFFF, 0x00020000);
#pragma unroll
    for (int h = 0; h < NC; ++h)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rb, (void __attribute__((address_space(3)))*)(&slot_of(slot)[wave][64 * h]), 16,
          offb + 1024 * h, 0, 0, 0);
  };

  const f32x16 zero16 = {};
  f32x16 acc[2][NU];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < NU; ++u) acc[t][u] = zero16;

  u32x4 bf[2][NU];
  auto readb = [&](int slot) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int u = 0; u < NU; ++u) bf[ks][u] = slot_of(slot)[2 * ks + half][32 * u + (lane & 31)];
  };
  auto compute = [&](int slot) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[t][u] = mfma16<BF16>(a[slot][ks][t], bf[ks][u], acc[t][u]);
  };
  // stage ls: issue stage ls + 3 (clamped to the last one: the extra copies
  // land in a slot nobody reads again) and multiply stage ls
  auto step = [&](int64_t ls, int j) {
    // 4 + NC operations per stage, two stages issued after this one
    if constexpr (NC == 2)
      asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(16) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    readb(j % kHRing);
    const int64_t nx = ls + kHRing - 1;
    issue(nx < ns ? nx : ns - 1, (j + kHRing - 1) % kHRing);
    compute(j % kHRing);
  };
#pragma unroll
  for (int s = 0; s < kHRing - 1; ++s) issue(s < ns ? s : ns - 1, s);
  int64_t l0 = 0;
  for (; l0 + kHUnroll <= ns; l0 += kHUnroll) {
#pragma unroll
    for (int j = 0; j < kHUnroll; ++j) step(l0 + j, j);
  }
  for (; l0 < ns; l0 += kHRing) {
#pragma unroll
    for (int j = 0; j < kHRing; ++j)
      if (l0 + j < ns) step(l0 + j, j);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // no copy into LDS outlives the workgroup

  // Without a K split the per-scene power of two is undone here; with one,
  // the slice-reduction kernel does it.
  const bool split = splits > 1;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < NU; ++u)
      store_acc(acc[t][u], dst, M, B, m0 + 64 * wave + 32 * t, n0 + 32 * u, lane, fexp, !split);
}

// The 16-bit GEMM for batches above 256 scenes: 8 waves (two per SIMD, so one
// wave's waits are filled with the other's products), tile 256 image rows x
// 256 scenes, wave (wm = w & 3, wn = w >> 2) owning rows 64 wm .. +63 and
// scenes 128 wn .. +127 (2 x 4 accumulators of 32 x 32).  Both operand
// tiles of a K stage are copied into LDS by the buffer unit (each wave 2
// library and 2 scene copies of 16 bytes per lane), into a 4-slot ring three
// stages ahead of use, and every wave reads its fragments from LDS: the two
// waves that share a row block read one copy of it.  The wait before each
// stage barrier allows 2 x 4 operations outstanding.  Against the 4-wave
// 256-scene tile (one wave per SIMD, library fragments straight to
// registers) the matrix cores are busy 73% instead of 65% of the cycles at
// B = 1024 (SQ_VALU_MFMA_BUSY_CYCLES), 352-370 against 353-417 us for the
// kernel; products and accumulation order per output are unchanged.
template <bool BF16>
__global__ __launch_bounds__(512, 1) void gemm_h16_w8_kernel(
    const u32x4* Mp, const u32x4* Zg, const int32_t* __restrict__ fexp,
    float* __restrict__ out, int64_t M, int64_t ngroups, int64_t B, int64_t Bp, int64_t mblocks,
    int64_t nblocks, int64_t splits, int64_t stages_per_split) {
  constexpr int TN = 256, NU = 4;
  __shared__ u32x4 Bs0[kHG][TN], Bs1[kHG][TN], Bs2[kHG][TN], Bs3[kHG][TN];  // scene ring
  __shared__ u32x4 As0[kHG][kHM], As1[kHG][kHM], As2[kHG][kHM], As3[kHG][kHM];  // library ring
  auto bslot = [&](int slot) -> u32x4 (*)[TN] {
    return slot == 0 ? Bs0 : slot == 1 ? Bs1 : slot == 2 ? Bs2 : Bs3;
  };
  auto aslot = [&](int slot) -> u32x4 (*)[kHM] {
    return slot == 0 ? As0 : slot == 1 ? As1 : slot == 2 ? As2 : As3;
  };
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 3, wn = wave >> 2;
  const int64_t tile = xcd_tile(blockIdx.x, mblocks * nblocks * splits);
  const int64_t nb = tile % nblocks, mb = (tile / nblocks) % mblocks, sp = tile / (nblocks * mblocks);
  const int64_t m0 = mb * kHM, n0 = nb * TN;
  const int64_t nstages = ngroups / kHG;  // ngroups is a multiple of 8
  const int64_t st0 = sp * stages_per_split;
  const int64_t ns = (nstages - st0 < stages_per_split ? nstages - st0 : stages_per_split);
  float* dst = out + sp * B * M;
  const int half = lane >> 5;
  // copies of this wave: group wm of each stage; library rows m0 + 128 wn + lane
  // and + 64 (rows past M read row M-1: valid addresses, results never
  // stored), scenes n0 + 128 wn .. +127
  int64_t arow0 = m0 + 128 * wn + lane, arow1 = arow0 + 64;
  if (arow0 > M - 1) arow0 = M - 1;
  if (arow1 > M - 1) arow1 = M - 1;
  const char* Ab = reinterpret_cast<const char*>(Mp);
  const char* Zb = reinterpret_cast<const char*>(Zg + (int64_t)wm * Bp + n0 + 128 * wn);
  const int offb = lane * 16;
  auto issue = [&](int64_t ls, int slot) {
    const int64_t st = st0 + ls;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Ab + (st * kHG + wm) * M * 16), (short)0, 0x7FFFFFFF, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        ra, (void __attribute__((address_space(3)))*)(&aslot(slot)[wm][128 * wn]), 16,
        (uint32_t)(arow0 * 16), 0, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        ra, (void __attribute__((address_space(3)))*)(&aslot(slot)[wm][128 * wn + 64]), 16,
        (uint32_t)(arow1 * 16), 0, 0, 0);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Zb + st * kHG * Bp * 16), (short)0, 0x7FFFFFFF, 0x00020000);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rb, (void __attribute__((address_space(3)))*)(&bslot(slot)[wm][128 * wn + 64 * h]), 16,
          offb + 1024 * h, 0, 0, 0);
  };
  const f32x16 zero16 = {};
  f32x16 acc[2][NU];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < NU; ++u) acc[t][u] = zero16;
  u32x4 af[2][2], bf[2][NU];
  auto readf = [&](int slot) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
      for (int u = 0; u < NU; ++u) bf[ks][u] = bslot(slot)[2 * ks + half][128 * wn + 32 * u + (lane & 31)];
#pragma unroll
      for (int t = 0; t < 2; ++t) af[ks][t] = aslot(slot)[2 * ks + half][64 * wm + 32 * t + (lane & 31)];
    }
  };
  auto compute = [&]() {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) acc[t][u] = mfma16<BF16>(af[ks][t], bf[ks][u], acc[t][u]);
  };
  auto step = [&](int64_t ls, int j) {
    // 4 copies per lane and stage; the two stages issued after this one may
    // still be in flight
    asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    readf(j % kHRing);
    const int64_t nx = ls + kHRing - 1;
    issue(nx < ns ? nx : ns - 1, (j + kHRing - 1) % kHRing);
    compute();
  };
#pragma unroll
  for (int s = 0; s < kHRing - 1; ++s) issue(s < ns ? s : ns - 1, s);
  int64_t l0 = 0;
  for (; l0 + kHUnroll <= ns; l0 += kHUnroll) {
#pragma unroll
    for (int j = 0; j < kHUnroll; ++j) step(l0 + j, j);
  }
  for (; l0 < ns; l0 += kHRing) {
#pragma unroll
    for (int j = 0; j < kHRing; ++j)
      if (l0 + j < ns) step(l0 + j, j);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // no copy into LDS outlives the workgroup
  const bool split = splits > 1;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < NU; ++u)
      store_acc(acc[t][u], dst, M, B, m0 + 64 * wm + 32 * t, n0 + 128 * wn + 32 * u, lane, fexp, !split);
}

// out[b][m] = 2^-f_b * sum over K slices (fixed order).  VEC: 4 outputs per
// thread (M % 4 == 0, so the 4 share one scene).
template <bool VEC>
__global__ __launch_bounds__(256) void reduce_splits_kernel(const float* __restrict__ part,
                                                            int splits, int64_t BM, int64_t M,
                                                            const int32_t* __restrict__ fexp,
                                                            float* __restrict__ out) {
  if constexpr (VEC) {
    const int64_t t = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (t >= BM) return;
    f32x4 s = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int p = 0; p < splits; ++p)
      s += __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(part + (int64_t)p * BM + t));
    if (fexp) {
      const int ex = -fexp[t / M];
#pragma unroll
      for (int e = 0; e < 4; ++e) s[e] = ldexpf(s[e], ex);
    }
    *reinterpret_cast<f32x4*>(out + t) = s;
  } else {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= BM) return;
    float s = 0.0f;
    for (int p = 0; p < splits; ++p) s += part[(int64_t)p * BM + t];
    out[t] = fexp ? ldexpf(s, -fexp[t / M]) : s;
  }
}

// ------------------------------------------------------------ launch ------
struct GemmPlan {
  int64_t mblocks, nblocks, kunits, splits, per;  // kunits: 8-column groups (FP32) or K stages (16-bit)
};

// 16-bit kernel by batch: the 4-wave 128-scene tile up to 128 scenes (a wider
// tile would be mostly padding; two workgroups per CU), the 4-wave 256-scene
// tile for 128 < B <= 256 (~5% faster than two 128-wide tiles), and the
// 8-wave 256 x 256 tile above (B = 512: 237-244 against 241-248 us per
// product with the 128-wide tile, K split in two; B = 1024: 400-403 against
// 406-416 us).
enum H16Kind { kH128 = 0, kH256 = 1, kHW8 = 2 };
static H16Kind h16_kind(int64_t bc) { return bc <= 128 ? kH128 : bc <= 256 ? kH256 : kHW8; }
static int64_t h16_tile(int64_t bc) { return h16_kind(bc) == kH128 ? 128 : 256; }

// FP32 scene blocks of 32 per workgroup tile: 1 for batches of at most 32
static int f32_nb(int64_t bc) { return bc <= 32 ? 1 : 2; }

// scene blocks of 32 in the FP32 fragment-major scene copy (whole tiles)
static int64_t f32_scene_blocks(int64_t bc) {
  const int nb = f32_nb(bc);
  return (bc + 32 * nb - 1) / (32 * nb) * nb;
}

static GemmPlan plan_gemm(int storage, int64_t M, int64_t ncols, int64_t ncols_pad, int64_t bc) {
  GemmPlan p;
  const bool f32 = storage == PSFLIB_FP32;
  const int64_t tm = f32 ? kGM : kHM, tn = f32 ? 32 * f32_nb(bc) : h16_tile(bc);
  p.mblocks = (M + tm - 1) / tm;
  p.nblocks = (bc + tn - 1) / tn;
  p.kunits = f32 ? (ncols + 7) / 8 : (ncols_pad / 8) / kHG;
  // split K if the tile grid is smaller than the GPU: FP32 aims at two
  // workgroups per CU; the 16-bit kernels at one (an extra K slice costs a
  // partial-image round trip that a second workgroup per CU does not repay).
  // The 8-wave kernel splits only while whole extra rounds of tiles fit
  // (192 tiles stay unsplit: 384 workgroups would leave half the GPU idle in
  // their second round too).
  const int64_t want = f32 ? 512 : 256;
  const int64_t tiles = p.mblocks * p.nblocks;
  int64_t s = (!f32 && h16_kind(bc) == kHW8) ? want / tiles : (want + tiles - 1) / tiles;
  if (s > 16) s = 16;
  if (s > p.kunits) s = p.kunits;
  if (s < 1) s = 1;
  p.per = (p.kunits + s - 1) / s;
  if (f32) p.per = (p.per + kF32Block - 1) / kF32Block * kF32Block;  // whole accumulation blocks
  p.splits = (p.kunits + p.per - 1) / p.per;  // no empty slice
  if (p.splits < 1) p.splits = 1;
  return p;
}

template <int NB, bool VEC, bool NT>
static hipError_t launch_gemm_f32_t(unsigned grid, const float* A, const f32x4* Zp, float* dst,
                                    int64_t M, int64_t K, int64_t B, int64_t SB, const GemmPlan& p,
                                    hipStream_t s) {
  gemm_f32_kernel<NB, VEC, NT><<<grid, kGemmThreads, 0, s>>>(A, Zp, dst, M, K, B, SB, p.mblocks,
                                                             p.nblocks, p.splits, p.per);
  return hipGetLastError();
}

// variant bits: 4 = two scene blocks per wave, 2 = even M (8-byte row pairs), 1 = non-temporal
static hipError_t launch_gemm_f32(int variant, unsigned grid, const float* A, const f32x4* Zp,
                                  float* dst, int64_t M, int64_t K, int64_t B, int64_t SB,
                                  const GemmPlan& p, hipStream_t s) {
  switch (variant) {
    case 0: return launch_gemm_f32_t<1, false, false>(grid, A, Zp, dst, M, K, B, SB, p, s);
    case 1: return launch_gemm_f32_t<1, false, true>(grid, A, Zp, dst, M, K, B, SB, p, s);
    case 2: return launch_gemm_f32_t<1, true, false>(grid, A, Zp, dst, M, K, B, SB, p, s);
    case 3: return launch_gemm_f32_t<1, true, true>(grid, A, Zp, dst, M, K, B, SB, p, s);
    case 4: return launch_gemm_f32_t<2, false, false>(grid, A, Zp, dst, M, K, B, SB, p, s);
    case 5: return launch_gemm_f32_t<2, false, true>(grid, A, Zp, dst, M, K, B, SB, p, s);
    case 6: return launch_gemm_f32_t<2, true, false>(grid, A, Zp, dst, M, K, B, SB, p, s);
    default: return launch_gemm_f32_t<2, true, true>(grid, A, Zp, dst, M, K, B, SB, p, s);
  }
}

template <bool BF16, int TN, bool NT>
static hipError_t launch_gemm_h16_t(unsigned grid, const u32x4* Mp, const u32x4* Zg,
                                    const int32_t* fexp, float* dst, int64_t M, int64_t ngroups,
                                    int64_t B, int64_t Bp, const GemmPlan& p, hipStream_t s) {
  gemm_h16_kernel<BF16, TN, NT><<<grid, kGemmThreads, 0, s>>>(Mp, Zg, fexp, dst, M, ngroups, B, Bp,
                                                             p.mblocks, p.nblocks, p.splits, p.per);
  return hipGetLastError();
}

static hipError_t launch_gemm_h16(bool bf, H16Kind kind, bool nt, unsigned grid, const u32x4* Mp,
                                  const u32x4* Zg, const int32_t* fexp, float* dst, int64_t M,
                                  int64_t ngroups, int64_t B, int64_t Bp, const GemmPlan& p,
                                  hipStream_t s) {
  if (kind == kHW8) {
    if (bf)
      gemm_h16_w8_kernel<true><<<grid, 512, 0, s>>>(Mp, Zg, fexp, dst, M, ngroups, B, Bp, p.mblocks,
                                                    p.nblocks, p.splits, p.per);
    else
      gemm_h16_w8_kernel<false><<<grid, 512, 0, s>>>(Mp, Zg, fexp, dst, M, ngroups, B, Bp, p.mblocks,
                                                     p.nblocks, p.splits, p.per);
    return hipGetLastError();
  }
  const bool wide = kind == kH256;
  const int v = (bf ? 4 : 0) + (wide ? 2 : 0) + (nt ? 1 : 0);
  switch (v) {
    case 0: return launch_gemm_h16_t<false, 128, false>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    case 1: return launch_gemm_h16_t<false, 128, true>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    case 2: return launch_gemm_h16_t<false, 256, false>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    case 3: return launch_gemm_h16_t<false, 256, true>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    case 4: return launch_gemm_h16_t<true, 128, false>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    case 5: return launch_gemm_h16_t<true, 128, true>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    case 6: return launch_gemm_h16_t<true, 256, false>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
    default: return launch_gemm_h16_t<true, 256, true>(grid, Mp, Zg, fexp, dst, M, ngroups, B, Bp, p, s);
  }
}

static int64_t chunk_of(int B) { return B < kMaxBatchChunk ? B : kMaxBatchChunk; }

// scenes per group row of the packed 16-bit scene copy (whole scene tiles)
static int64_t padded_batch(int64_t bc) { return (bc + h16_tile(bc) - 1) / h16_tile(bc) * h16_tile(bc); }

static size_t split_partial_bytes(int storage, int64_t M, int64_t ncols, int64_t ncols_pad,
                                  int64_t bc) {
  const GemmPlan p = plan_gemm(storage, M, ncols, ncols_pad, bc);
  return p.splits > 1 ? (size_t)p.splits * (size_t)bc * (size_t)M * 4 : 0;
}

size_t batched_scratch_bytes(int storage, int64_t M, int64_t ncols, int64_t ncols_pad, int B) {
  // Passes run over up to kMaxBatchChunk scenes each: for the 16-bit forms the
  // packed scenes and their exponents, then the K-split partial images of
  // the largest pass (a short final pass may split K more finely).
  if (B <= 0) return 0;
  const int64_t bc = chunk_of(B);
  size_t bytes = 0;
  if (storage != PSFLIB_FP32) {
    bytes += ((size_t)padded_batch(bc) * (size_t)ncols_pad * 2 + 255) & ~(size_t)255;  // Zg
    bytes += ((size_t)bc * 4 + 255) & ~(size_t)255;                                    // fexp
  } else {
    bytes += (size_t)((ncols + 7) / 8) * (size_t)f32_scene_blocks(bc) * 1024;          // Zp
  }
  size_t part = split_partial_bytes(storage, M, ncols, ncols_pad, bc);
  const int64_t rem = B % bc;
  if (rem) {
    const size_t p2 = split_partial_bytes(storage, M, ncols, ncols_pad, rem);
    if (p2 > part) part = p2;
  }
  return bytes + part;
}

hipError_t launch_batched(int storage, const void* lib, const Cols16& cx, const float* Z,
                          float* out, int64_t M, int64_t ncols, int64_t ncols_pad, int B,
                          void* scratch, size_t scratch_bytes, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  char* sp = reinterpret_cast<char*>(scratch);
  u32x4* Zg = nullptr;
  int32_t* fexp = nullptr;
  const int64_t bcmax = chunk_of(B);
  size_t off = 0;
  f32x4* Zp = nullptr;
  if (storage != PSFLIB_FP32) {
    Zg = reinterpret_cast<u32x4*>(sp);
    off += ((size_t)padded_batch(bcmax) * (size_t)ncols_pad * 2 + 255) & ~(size_t)255;
    fexp = reinterpret_cast<int32_t*>(sp + off);
    off += ((size_t)bcmax * 4 + 255) & ~(size_t)255;
  } else {
    Zp = reinterpret_cast<f32x4*>(sp);
    off += (size_t)((ncols + 7) / 8) * (size_t)f32_scene_blocks(bcmax) * 1024;
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
      const int64_t ngroups = (ncols + 7) / 8, SB = f32_scene_blocks(bc);
      const bool zvec = (ncols % 4) == 0 && (reinterpret_cast<uintptr_t>(Zc) % 16) == 0;
      const unsigned pgrid = (unsigned)((ngroups * SB * 64 + 255) / 256);
      if (zvec)
        pack_f32_scenes_kernel<true><<<pgrid, 256, 0, s>>>(Zc, ncols, bc, ngroups, SB, Zp);
      else
        pack_f32_scenes_kernel<false><<<pgrid, 256, 0, s>>>(Zc, ncols, bc, ngroups, SB, Zp);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      const int variant = (f32_nb(bc) == 2 ? 4 : 0) + ((M % 2) == 0 ? 2 : 0) + (p.nblocks == 1 ? 1 : 0);
      e = launch_gemm_f32(variant, grid, reinterpret_cast<const float*>(lib), Zp, dst, M, ncols, bc,
                          SB, p, s);
    } else {
      const bool bf = storage == PSFLIB_BF16_POW2;
      const bool vec = (ncols % 8) == 0 && (reinterpret_cast<uintptr_t>(Zc) % 16) == 0;
      const int64_t ngroups = ncols_pad / 8, Bp = padded_batch(bc);
      const dim3 pgrid((unsigned)((ngroups + 31) / 32), (unsigned)(Bp / 8));
      if (ncols <= kStageMaxCols) {
        const bool pairs = ncols <= kStagePairCols;
        const size_t lds = (size_t)ncols * 4 * (pairs ? 2 : 1);
        const unsigned sgrid = (unsigned)(pairs ? Bp / 2 : Bp);
        auto stage = [&](auto kern) -> hipError_t {
          hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          if (err != hipSuccess) return err;
          kern<<<sgrid, 1024, lds, s>>>(Zc, cx.exps, cx.perm, cx.eslot, ncols, ngroups, bc, Bp,
                                        fexp, Zg);
          return hipGetLastError();
        };
        if (pairs)
          e = bf ? (vec ? stage(stage_pairs16_kernel<true, true>) : stage(stage_pairs16_kernel<true, false>))
                 : (vec ? stage(stage_pairs16_kernel<false, true>) : stage(stage_pairs16_kernel<false, false>));
        else
          e = bf ? (vec ? stage(stage_slots16_kernel<true, true>) : stage(stage_slots16_kernel<true, false>))
                 : (vec ? stage(stage_slots16_kernel<false, true>) : stage(stage_slots16_kernel<false, false>));
        if (e != hipSuccess) return e;
      } else {
        if (vec)
          scene_exponent_kernel<true><<<(unsigned)bc, 1024, 0, s>>>(Zc, cx.exps, ncols, ngroups, fexp);
        else
          scene_exponent_kernel<false><<<(unsigned)bc, 1024, 0, s>>>(Zc, cx.exps, ncols, ngroups, fexp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (bf)
          pack_scenes_kernel<true><<<pgrid, 256, 0, s>>>(Zc, cx.perm, cx.eslot, fexp, ncols, ngroups, bc, Bp, Zg);
        else
          pack_scenes_kernel<false><<<pgrid, 256, 0, s>>>(Zc, cx.perm, cx.eslot, fexp, ncols, ngroups, bc, Bp, Zg);
      }
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      const u32x4* Mp = reinterpret_cast<const u32x4*>(lib);
      const H16Kind kind = h16_kind(bc);
      e = launch_gemm_h16(bf, kind, (kind == kH128 || kind == kH256) && p.nblocks == 1, grid, Mp, Zg, fexp, dst, M,
                          ngroups, bc, Bp, p, s);
    }
    if (e != hipSuccess) return e;
    if (p.splits > 1) {
      const int64_t BM = bc * M;
      const int32_t* fx = storage == PSFLIB_FP32 ? nullptr : fexp;
      const bool v4 = (M % 4) == 0 && (reinterpret_cast<uintptr_t>(outc) % 16) == 0;
      if (v4)
        reduce_splits_kernel<true><<<(unsigned)((BM / 4 + 255) / 256), 256, 0, s>>>(
            part, (int)p.splits, BM, M, fx, outc);
      else
        reduce_splits_kernel<false><<<(unsigned)((BM + 255) / 256), 256, 0, s>>>(
            part, (int)p.splits, BM, M, fx, outc);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace psflib
