// Grouped simulation: many scenes, each with its own library (different image
// and scene sizes, different wavelengths), in one persistent launch captured
// in a HIP graph.  Sec. 5 of the paper points at simulating many complex
// scenes at once; with a few scenes per library the product streams every
// library once from HBM and is bandwidth bound: a multi-right-hand-side
// matvec.  It still runs on the matrix cores, because they multiply a library
// tile by 16 scenes at the rate HBM delivers it where the vector ALUs manage
// about 8, and a library whose scenes fit one pass is read once.
//
// Work items are (library, scene group of <= 16, row block, column chunk)
// tiles, listed on the host when the plan is made.  A persistent grid
// walks the list; each workgroup streams its tile of the library once and
// multiplies it with every scene of the group.  An item that covers every
// column of its library writes the images directly; otherwise items write
// partial images and a second kernel adds the partials of each (scene, row
// block) in chunk order (bitwise reproducible).  The tile shape -- rows per
// item (16-bit: 256, 128 or 64, the workgroup's four waves splitting the
// columns of the smaller tiles and adding their sums through LDS) and chunk
// length (or whole columns) -- is chosen by timing the candidate shapes on the
// plan itself (psflib_grouped_create with autotune), and the choice is cached
// per plan signature for the process.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "psflib_internal.h"

namespace psflib {

constexpr int kGrpScenes = 16;  // scenes multiplied per pass (the library is read once per pass)
constexpr int kGrpThreads = 256;  // 4 waves of 64 image rows

struct GItem {
  const void* A;          // library matrix (FP32 column-major or 16-bit 8-column groups)
  const int32_t* exps;    // 16-bit per-column exponents (nullptr for FP32)
  int64_t M, ncols;       // rows, scene pixels of this library
  int64_t row0;           // first row of the block
  int64_t j0, j1;         // columns (FP32) or 8-column groups (16-bit) of the chunk
  int32_t scene0, nscenes;  // scenes (index into the plan's scene table)
  int64_t part;           // float offset of this item's partials: [scenes per pass][rows]
  int64_t bpk;            // packed scene operand of the scene group (16-byte units)
  int32_t direct;         // the item covers every column: images written directly, no partials
  int32_t pad;
};

// A scene slot of the plan: its values and its library's column exponents.
struct GScene {
  const float* z;
  const int32_t* exps;
  int64_t ncols;
};

// A scene group: slots slot0 .. slot0+nscenes-1 of one library, packed into
// the matrix-core operand at bpk: 16-bit, ngroups 8-slot groups x 32 columns
// x 16 bytes (library slot s holds column perm[s], exponent eslot[s]); FP32,
// ngroups 16-column blocks x 64 lanes x 16 bytes.
struct GPack {
  int64_t bpk, ncols, ngroups;
  const int32_t* perm;
  const int32_t* eslot;
  int32_t slot0, nscenes;
};

struct GReduce {
  int64_t M, row0, rows;
  int64_t part0;          // partials of the first chunk; chunk c at part0 + c * stride
  int64_t stride;         // floats between consecutive chunks' partials
  int32_t nchunks, scene0, nscenes, pad;
};

// ------------------------------------------------------------- kernels ----
// FP32, on the matrix cores (v_mfma_f32_16x16x4f32: 16 rows x 16 scenes x 4
// columns per instruction).  The scene group is packed once per run into
// blocks of 16 columns: block b holds 64 lanes x 4 floats, lane l = 16q + n
// holding Z_n[16b + 4s + q] for s = 0..3 (scene slot n, zeros past the
// group's scenes and past ncols), the B operand of the four MFMA steps s of
// the block.  A wave owns 64 image rows: lane (n = l % 16, q = l / 16) loads
// rows m0 + 4n .. m0 + 4n + 3 of column 16b + 4s + q as one 16-byte load,
// whose component t is the A operand of MFMA t; output row i of MFMA t is
// image row m0 + 4i + t.  Loads go through buffer descriptors that end at the
// live data (columns past ncols and blocks past the item read as zero), kGrpRing
// blocks ahead of use, with no LDS and no barriers.  Accumulation is blocked
// (64 columns, then the chunk).
constexpr int kGrpRing = 2;

template <bool VEC>
__device__ __forceinline__ void grouped_f32_item(const GItem& w, const f32x4* __restrict__ zpk,
                                                 int lane, int wave, float* __restrict__ part,
                                                 float* const* __restrict__ images) {
  const int64_t m0 = w.row0 + 64 * wave;
  if (m0 >= w.M) return;  // no barriers: a wave past the image leaves at once
  const int n = lane & 15, q = lane >> 4;
  // 16 columns of M floats span < 2^31 bytes (M <= 2^25, checked when the plan is made)
  const int M4 = (int)(w.M * 4);
  uint32_t voff[4];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4)
    voff[s4] = (uint32_t)((int64_t)(4 * s4 + q) * w.M * 4 + (m0 + 4 * n) * 4);
  const float* A = reinterpret_cast<const float*>(w.A);
  const int b0 = (int)(w.j0 / 16), b1 = (int)((w.j1 + 15) / 16);
  const int ncols = (int)w.ncols;
  f32x4 ra[kGrpRing][4], rb[kGrpRing];
  auto issue = [&](int b, int slot) {
    const bool live = b < b1;
    const int bc = live ? b : b1 - 1;
    // the descriptor ends with the block's last library column: rows a wave
    // reads past the image read zero there, never past the library
    const int left = ncols - 16 * bc;  // columns of the library from this block on
    // (the record count is an unsigned 32-bit field: 16 M4 <= 2^31 fits)
    const int abytes = !live ? 0 : (int)((uint32_t)(left < 16 ? left : 16) * (uint32_t)M4);
    const __amdgpu_buffer_rsrc_t ad = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(A + (int64_t)16 * bc * w.M), (short)0, abytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t bd = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(zpk + w.bpk + (int64_t)bc * 64), (short)0, live ? 1024 : 0, 0x00020000);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      if (VEC) {
        ra[slot][s4] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ad, voff[s4], 0, 2));
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          ra[slot][s4][t] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ad, voff[s4] + 4 * t, 0, 2));
      }
    }
    rb[slot] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(bd, (uint32_t)lane * 16, 0, 0));
  };
  const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc[4], tot[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) tot[t] = zero4;
  const int nblk = (b1 - b0 + 3) / 4;  // groups of 4 blocks = 64 columns
#pragma unroll
  for (int r = 0; r < kGrpRing; ++r) issue(b0 + r, r);
  for (int kb = 0; kb < nblk; ++kb) {
    const int bb = b0 + 4 * kb;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int slot = u % kGrpRing;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[slot][s4][t], rb[slot][s4],
                                                        (u == 0 && s4 == 0) ? zero4 : acc[t], 0, 0, 0);
      issue(bb + u + kGrpRing, slot);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) tot[t] += acc[t];
  }
  // lane holds scene n and MFMA rows 4q + r, i.e. image rows m0 + 16q + 4r + t
  if (n < w.nscenes) {
    if (w.direct) {
      float* img = images[w.scene0 + n];
      const int64_t rr = m0 + 16 * q;
      const bool whole = VEC && rr + 16 <= w.M;  // images are 16-byte aligned; M % 4 == 0
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const f32x4 v = {tot[0][r], tot[1][r], tot[2][r], tot[3][r]};
        if (whole) {
          *reinterpret_cast<f32x4*>(img + rr + 4 * r) = v;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (rr + 4 * r + t < w.M) img[rr + 4 * r + t] = v[t];
        }
      }
    } else {
      float* dst = part + w.part + (int64_t)n * kGrpThreads + 64 * wave + 16 * q;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const f32x4 v = {tot[0][r], tot[1][r], tot[2][r], tot[3][r]};
        *reinterpret_cast<f32x4*>(dst + 4 * r) = v;
      }
    }
  }
}

__global__ __launch_bounds__(kGrpThreads) void grouped_f32_kernel(
    const GItem* __restrict__ items, int64_t nitems, const f32x4* __restrict__ zpk,
    float* __restrict__ part, float* const* __restrict__ images) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GItem w = items[it];
    if ((w.M & 3) == 0)
      grouped_f32_item<true>(w, zpk, lane, wave, part, images);
    else
      grouped_f32_item<false>(w, zpk, lane, wave, part, images);
  }
}

// FP32 packed scene operand: thread = (scene group, 16-column block b, lane l).
__global__ __launch_bounds__(256) void grouped_pack_f32_kernel(const GPack* __restrict__ packs,
                                                               const float* const* __restrict__ scenes,
                                                               f32x4* __restrict__ zpk) {
  const GPack pk = packs[blockIdx.x];
  for (int64_t t = (int64_t)blockIdx.y * 256 + threadIdx.x; t < pk.ngroups * 64;
       t += (int64_t)gridDim.y * 256) {
    const int l = (int)(t & 63);
    const int64_t b = t >> 6;
    const int n = l & 15, q = l >> 4;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (n < pk.nscenes) {
      const float* z = scenes[pk.slot0 + n];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int64_t j = 16 * b + 4 * s4 + q;
        if (j < pk.ncols) v[s4] = z[j];
      }
    }
    zpk[pk.bpk + t] = v;
  }
}

// 16-bit, on the matrix cores (v_mfma_f32_32x32x16_{bf16,f16}).  A pass
// multiplies a library tile by up to 16 scenes, so a library with up to 16
// scenes is streamed from HBM once.  The 16-bit product needs 16-bit scene
// values; to keep the error that of the stored library alone, each scaled
// scene value v = Z_j 2^(e_j + f_s) is split into hi = RN16(v) and
// lo = RN16(v - hi) (v = hi + lo to about u^2), and the 32 columns of the
// B operand are the 16 scenes' hi parts followed by their lo parts; the two
// halves are added after the products.  f_s is the per-scene power of two
// that puts the scene's largest scaled value in [2^14, 2^15) (so FP16 neither
// overflows nor loses the faint end to underflow).
//
// The split scene values are packed once per run into the B operand of every
// (scene group, 8-column group): 32 columns x 16 bytes, 512 bytes per group,
// all of it small enough to stay in L2/MALL.  Workgroup = 4 waves = 256 image
// rows, wave = 64 rows (two 32-row tiles); library fragments (8 columns of one
// row = 16 bytes = the MFMA A fragment) stream from HBM straight into
// registers and scene fragments from the packed operand, a block of 4 K steps
// ahead, with no LDS and no barriers.

// f_s of every scene slot (one 1024-thread workgroup per slot; 16-byte loads
// of the scene and the exponents when both are aligned).
__global__ __launch_bounds__(1024) void grouped_scene_exp_kernel(const GScene* __restrict__ slots,
                                                                 int32_t* __restrict__ fexp) {
  __shared__ double red[1024];
  const GScene sc = slots[blockIdx.x];
  double m = 0.0;
  const bool vec = (sc.ncols % 4) == 0 && (reinterpret_cast<uintptr_t>(sc.z) % 16) == 0 &&
                   (reinterpret_cast<uintptr_t>(sc.exps) % 16) == 0;
  if (vec) {
    for (int64_t j = 4 * (int64_t)threadIdx.x; j < sc.ncols; j += 4 * 1024) {
      const f32x4 z = *reinterpret_cast<const f32x4*>(sc.z + j);
      const int4 e = *reinterpret_cast<const int4*>(sc.exps + j);
      m = fmax(m, ldexp((double)fabsf(z[0]), e.x));
      m = fmax(m, ldexp((double)fabsf(z[1]), e.y));
      m = fmax(m, ldexp((double)fabsf(z[2]), e.z));
      m = fmax(m, ldexp((double)fabsf(z[3]), e.w));
    }
  } else {
    for (int64_t j = threadIdx.x; j < sc.ncols; j += 1024)
      m = fmax(m, ldexp((double)fabsf(sc.z[j]), sc.exps[j]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int f = 0;
    if (red[0] > 0.0) {
      int E;
      (void)frexp(red[0], &E);
      f = 15 - E;
    }
    fexp[blockIdx.x] = f;
  }
}

template <bool BF16>
__device__ __forceinline__ uint16_t g16_round(float x) {
  if constexpr (BF16) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // finite: round to nearest, ties to even
    return (uint16_t)(u >> 16);
  } else {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
  }
}

template <bool BF16>
__device__ __forceinline__ float g16_value(uint16_t h) {
  if constexpr (BF16)
    return __uint_as_float((uint32_t)h << 16);
  else
    return (float)__builtin_bit_cast(_Float16, h);
}

// Packed operand: thread = (scene group, 8-column group g, quarter r4 of the
// scene slots); loads the group's 8 column indices and exponents once and
// writes columns r (hi parts) and 16 + r (lo parts) of group g for its four
// slots r = 4 r4 .. 4 r4 + 3, 16 bytes each (zeros for slots past the group's
// scenes).  Grid: one row of workgroups per scene group, (group, quarter)
// pairs strided across the row.
template <bool BF16>
__global__ __launch_bounds__(256) void grouped_pack_kernel(const GPack* __restrict__ packs,
                                                           const float* const* __restrict__ scenes,
                                                           const int32_t* __restrict__ fexp,
                                                           u32x4* __restrict__ bpk) {
  const GPack pk = packs[blockIdx.x];
  for (int64_t t = (int64_t)blockIdx.y * 256 + threadIdx.x; t < pk.ngroups * 4;
       t += (int64_t)gridDim.y * 256) {
    const int64_t g = t >> 2;
    const int r4 = (int)(t & 3);
    u32x4* dst = bpk + pk.bpk + g * 32;
    int32_t jj[8], es[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      jj[u] = pk.perm[g * 8 + u];
      es[u] = pk.eslot[g * 8 + u];
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int r = 4 * r4 + rr;
      uint32_t hi[4] = {0u, 0u, 0u, 0u}, lo[4] = {0u, 0u, 0u, 0u};
      if (r < pk.nscenes) {
        const float* z = scenes[pk.slot0 + r];
        const int f = fexp[pk.slot0 + r];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float v = (jj[u] >= 0) ? ldexpf(z[jj[u]], es[u] + f) : 0.0f;
          const uint16_t h = g16_round<BF16>(v);
          const uint16_t l = g16_round<BF16>(v - g16_value<BF16>(h));
          hi[u >> 1] |= (uint32_t)h << (16 * (u & 1));
          lo[u >> 1] |= (uint32_t)l << (16 * (u & 1));
        }
      }
      dst[r] = (u32x4){hi[0], hi[1], hi[2], hi[3]};
      dst[16 + r] = (u32x4){lo[0], lo[1], lo[2], lo[3]};
    }
  }
}

// Scene exponents and packing in one kernel when every library of the plan
// has at most kStageMaxCols columns: one 1024-thread workgroup per (scene
// group, slot r < 16) stages its scene in LDS (coalesced loads), takes f_s
// from the LDS copy (as grouped_scene_exp_kernel) and writes columns r and
// 16 + r of every 8-slot group of the group's operand, gathering the slots
// from LDS (gathered straight from HBM, every 4-byte value costs a sector).
// The 16 slots of a scene group write the 512-byte blocks of its operand
// together; they are numbered to land on one XCD back to back (dispatch is
// round-robin over the 8 XCDs), so the blocks fill in that XCD's L2.  Slots
// past the group's scenes write zeros.
template <bool BF16>
__global__ __launch_bounds__(1024) void grouped_stage_pack_kernel(const GPack* __restrict__ packs,
                                                                  int64_t npacks,
                                                                  const GScene* __restrict__ slots,
                                                                  int32_t* __restrict__ fexp,
                                                                  u32x4* __restrict__ bpk) {
  typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
  extern __shared__ float zl[];  // the scene
  __shared__ double red[16];
  __shared__ int s_f;
  const int64_t wg = blockIdx.x, xcd = wg % 8, rnd = wg / 8;
  const int64_t gi = xcd + 8 * (rnd / kGrpScenes);
  const int r = (int)(rnd % kGrpScenes);
  if (gi >= npacks) return;  // uniform: padding workgroups of the grid
  const GPack pk = packs[gi];
  const int tid = threadIdx.x;
  u32x4* dst = bpk + pk.bpk;
  if (r >= pk.nscenes) {
    for (int64_t g = tid; g < pk.ngroups; g += 1024) {
      dst[g * 32 + r] = (u32x4){0u, 0u, 0u, 0u};
      dst[g * 32 + 16 + r] = (u32x4){0u, 0u, 0u, 0u};
    }
    return;
  }
  const GScene sc = slots[pk.slot0 + r];
  double m = 0.0;
  const bool vec = (sc.ncols % 4) == 0 && (reinterpret_cast<uintptr_t>(sc.z) % 16) == 0 &&
                   (reinterpret_cast<uintptr_t>(sc.exps) % 16) == 0;
  if (vec) {
    for (int64_t j = 4 * (int64_t)tid; j < sc.ncols; j += 4 * 1024) {
      const f32x4 z = *reinterpret_cast<const f32x4*>(sc.z + j);
      const i32x4 e = *reinterpret_cast<const i32x4*>(sc.exps + j);
      *reinterpret_cast<f32x4*>(zl + j) = z;
#pragma unroll
      for (int q = 0; q < 4; ++q) m = fmax(m, ldexp((double)fabsf(z[q]), e[q]));
    }
  } else {
    for (int64_t j = tid; j < sc.ncols; j += 1024) {
      const float z = sc.z[j];
      zl[j] = z;
      m = fmax(m, ldexp((double)fabsf(z), sc.exps[j]));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double mm = red[0];
#pragma unroll
    for (int w = 1; w < 16; ++w) mm = fmax(mm, red[w]);
    int f = 0;
    if (mm > 0.0) {
      int E;
      (void)frexp(mm, &E);
      f = 15 - E;
    }
    s_f = f;
    fexp[pk.slot0 + r] = f;
  }
  __syncthreads();
  const int f = s_f;
  for (int64_t g = tid; g < pk.ngroups; g += 1024) {
    const i32x4 p0 = *reinterpret_cast<const i32x4*>(pk.perm + 8 * g);
    const i32x4 p1 = *reinterpret_cast<const i32x4*>(pk.perm + 8 * g + 4);
    const i32x4 e0 = *reinterpret_cast<const i32x4*>(pk.eslot + 8 * g);
    const i32x4 e1 = *reinterpret_cast<const i32x4*>(pk.eslot + 8 * g + 4);
    uint32_t hi[4] = {0u, 0u, 0u, 0u}, lo[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t j = u < 4 ? p0[u] : p1[u - 4];
      const int32_t e = u < 4 ? e0[u] : e1[u - 4];
      const float v = (j >= 0) ? ldexpf(zl[j], e + f) : 0.0f;
      const uint16_t h = g16_round<BF16>(v);
      const uint16_t l = g16_round<BF16>(v - g16_value<BF16>(h));
      hi[u >> 1] |= (uint32_t)h << (16 * (u & 1));
      lo[u >> 1] |= (uint32_t)l << (16 * (u & 1));
    }
    dst[g * 32 + r] = (u32x4){hi[0], hi[1], hi[2], hi[3]};
    dst[g * 32 + 16 + r] = (u32x4){lo[0], lo[1], lo[2], lo[3]};
  }
}

template <bool BF16>
__device__ __forceinline__ f32x16 g16_mfma(const u32x4 a, const u32x4 b, const f32x16 c) {
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
  if constexpr (BF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// KS = waves splitting an item's columns: an item is 256 / KS rows, row wave
// rw = wave % (4 / KS) takes 64 of them and split ks = wave / (4 / KS) a
// contiguous run of the item's K steps (whole blocks of 4); the splits' sums
// go through LDS and are added in split order by split 0, which writes the
// item's rows.
template <bool BF16, int KS>
__global__ __launch_bounds__(kGrpThreads) void grouped_h16_kernel(
    const GItem* __restrict__ items, int64_t nitems, const u32x4* __restrict__ bpk,
    const int32_t* __restrict__ fexp, float* __restrict__ part, float* const* __restrict__ images) {
  constexpr int RW = 4 / KS;   // row waves
  constexpr int R = 64 * RW;   // rows per item
  __shared__ f32x16 red[(KS > 1) ? (KS - 1) * RW * 2 : 1][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rw = wave % RW, ks = wave / RW;
  const int half = lane >> 5;  // which group of a 16-wide K step this lane feeds
  const u32x4 z4 = {0u, 0u, 0u, 0u};
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GItem w = items[it];
    const u32x4* Mp = reinterpret_cast<const u32x4*>(w.A);
    const int ng = (int)(w.j1 - w.j0);  // even (chunks and libraries are whole 8-group blocks)
    const int nsteps = ng / 2;
    const int nq = (nsteps + 3) / 4;  // blocks of 4 K steps, shared out among the splits
    const int sa = 4 * ((nq * ks) / KS);
    const int sb = (4 * ((nq * (ks + 1)) / KS) < nsteps) ? 4 * ((nq * (ks + 1)) / KS) : nsteps;
    const int gend = 2 * sb;
    // this lane's library rows; rows past M read row M-1 (never stored)
    int64_t r0 = w.row0 + 64 * rw + (lane & 31), r1 = r0 + 32;
    if (r0 > w.M - 1) r0 = w.M - 1;
    if (r1 > w.M - 1) r1 = w.M - 1;
    const u32x4* A0 = Mp + w.j0 * w.M + r0;
    const u32x4* A1 = Mp + w.j0 * w.M + r1;
    // scene operand of this item's chunk: group g at Bg[g * 32 + column]
    const u32x4* Bg = bpk + w.bpk + w.j0 * 32 + (lane & 31);
    auto load4 = [&](int s0, u32x4 (&a)[4][3]) {  // K steps s0 .. s0+3 (groups 2s + half)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int g = 2 * (s0 + q) + half;
        const bool ok = g < gend;
        a[q][0] = ok ? __builtin_nontemporal_load(A0 + (int64_t)g * w.M) : z4;
        a[q][1] = ok ? __builtin_nontemporal_load(A1 + (int64_t)g * w.M) : z4;
        a[q][2] = ok ? Bg[g * 32] : z4;
      }
    };
    u32x4 pa[4][3], pb[4][3];
    const f32x16 zero16 = {};
    f32x16 acc[2] = {zero16, zero16};
    auto mult4 = [&](int s0, const u32x4 (&a)[4][3]) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (s0 + q >= sb) break;  // uniform
        acc[0] = g16_mfma<BF16>(a[q][0], a[q][2], acc[0]);
        acc[1] = g16_mfma<BF16>(a[q][1], a[q][2], acc[1]);
      }
    };
    if (sa < sb) {
      load4(sa, pa);
      for (int s0 = sa; s0 < sb; s0 += 8) {
        load4(s0 + 4, pb);
        mult4(s0, pa);
        if (s0 + 4 >= sb) break;
        load4(s0 + 8, pa);
        mult4(s0 + 4, pb);
      }
    }
    if constexpr (KS > 1) {
      if (ks > 0) {
        red[((ks - 1) * RW + rw) * 2 + 0][lane] = acc[0];
        red[((ks - 1) * RW + rw) * 2 + 1][lane] = acc[1];
      }
      __syncthreads();
      if (ks == 0) {
#pragma unroll
        for (int k2 = 1; k2 < KS; ++k2) {
          acc[0] += red[((k2 - 1) * RW + rw) * 2 + 0][lane];
          acc[1] += red[((k2 - 1) * RW + rw) * 2 + 1][lane];
        }
      }
    }
    if (ks == 0) {
      // column n = lane % 32 holds scene n's hi part (n < 16) or scene n-16's lo part
      const int n = lane & 31;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const float v = acc[t][q] + __shfl_xor(acc[t][q], 16, 64);
          if (n < w.nscenes) {
            const int rl = 64 * rw + 32 * t + 8 * (q >> 2) + 4 * half + (q & 3);
            const float x = ldexpf(v, -fexp[w.scene0 + n]);
            if (w.direct) {
              if (w.row0 + rl < w.M) images[w.scene0 + n][w.row0 + rl] = x;
            } else {
              part[w.part + (int64_t)n * R + rl] = x;
            }
          }
        }
      }
    }
    if constexpr (KS > 1) __syncthreads();  // the LDS sums are read before the next item
  }
}

// image[b][row0 + t] = sum over the chunks (in order) of the partials.
__global__ __launch_bounds__(256) void grouped_reduce_kernel(const GReduce* __restrict__ red,
                                                             const float* __restrict__ part,
                                                             float* const* __restrict__ images) {
  const GReduce w = red[blockIdx.x];
  for (int64_t t = threadIdx.x; t < w.rows * w.nscenes; t += 256) {
    const int r = (int)(t / w.rows);
    const int64_t row = t - (int64_t)r * w.rows;
    if (w.row0 + row >= w.M) continue;
    const float* src = part + w.part0 + (int64_t)r * w.rows + row;
    float total = 0.0f;
    for (int32_t c0 = 0; c0 < w.nchunks; c0 += 16) {
      float p[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) p[u] = (c0 + u < w.nchunks) ? src[(int64_t)(c0 + u) * w.stride] : 0.0f;
      float blk = p[0];
#pragma unroll
      for (int u = 1; u < 16; ++u) blk += p[u];
      total += blk;
    }
    images[w.scene0 + r][w.row0 + row] = total;
  }
}

}  // namespace psflib

// ------------------------------------------------------------ host side ----
struct psflib_grouped {
  int storage;
  int device;
  hipGraph_t graph;
  hipGraphExec_t exec;
  void* dev;        // items | reductions | scene/image tables | slots | packed operands | partials
  int64_t chunk;    // chosen chunk length (columns, or 8-column groups for 16-bit; 0: whole)
  int32_t rows;     // chosen rows per item
  float ms_tuned;   // time of the chosen shape during autotuning (0 if not tuned)
  mutable psflib::StreamUses uses;  // streams the graph was launched on
};

namespace {

struct LibInfo {
  const void* A;
  psflib::Cols16 cx;
  int64_t M, ncols, ncols_pad;
};

// What a plan is made of, kept for a later change of tile shape.
struct PlanInputs {
  std::vector<LibInfo> libs;
  std::vector<int32_t> lib_of_scene;
  std::vector<const float*> scenes;
  std::vector<float*> images;
};
std::mutex g_inputs_mu;
std::map<const psflib_grouped*, PlanInputs> g_inputs;

struct Plan {
  std::vector<psflib::GItem> items;
  std::vector<psflib::GReduce> reds;
  std::vector<const float*> scenes;
  std::vector<float*> images;
  std::vector<psflib::GScene> slots;  // per scene slot: values, exponents (16-bit scaling)
  std::vector<psflib::GPack> packs;   // 16-bit: per scene group, its packed operand
  int64_t part_floats = 0;
  int64_t bpk_vecs = 0;               // 16-byte entries of the packed operands
};

// Tile shape: rows per item and chunk length (0: every column of the library
// in one item, whose rows are then written directly).
struct Shape {
  int64_t chunk;
  int32_t rows;
};

// Items for a given shape.  Scenes are grouped by library (kept in the
// caller's order inside a library) and cut into groups of kGrpScenes.
Plan make_plan(int storage, const std::vector<LibInfo>& libs, const int32_t* lib_of_scene,
               const float* const* scenes, float* const* images, int B, Shape shape) {
  Plan p;
  const bool f32 = storage == PSFLIB_FP32;
  const int64_t rows_per = shape.rows;
  for (size_t L = 0; L < libs.size(); ++L) {
    std::vector<int> sc;
    for (int b = 0; b < B; ++b)
      if (lib_of_scene[b] == (int)L) sc.push_back(b);
    const LibInfo& li = libs[L];
    const int64_t units = f32 ? li.ncols : li.ncols_pad / 8;  // chunks count columns or 8-column groups
    const int64_t pk_units = f32 ? (li.ncols + 15) / 16 : units;  // packed operand blocks
    const int64_t chunk = shape.chunk > 0 ? shape.chunk : std::max<int64_t>(units, 1);
    const int64_t nchunks = (units + chunk - 1) / chunk;
    const int64_t nrb = (li.M + rows_per - 1) / rows_per;
    const size_t spg = psflib::kGrpScenes;
    for (size_t g0 = 0; g0 < sc.size(); g0 += spg) {
      const int ns = (int)std::min<size_t>(spg, sc.size() - g0);
      const int32_t scene0 = (int32_t)p.scenes.size();
      for (int r = 0; r < ns; ++r) {
        p.scenes.push_back(scenes[sc[g0 + r]]);
        p.images.push_back(images[sc[g0 + r]]);
        p.slots.push_back(psflib::GScene{scenes[sc[g0 + r]], li.cx.exps, li.ncols});
      }
      const int64_t bpk = p.bpk_vecs;
      p.packs.push_back(psflib::GPack{bpk, li.ncols, pk_units, li.cx.perm, li.cx.eslot, scene0, ns});
      p.bpk_vecs += pk_units * (f32 ? 64 : 32);
      for (int64_t rb = 0; rb < nrb; ++rb) {
        psflib::GReduce rd;
        rd.M = li.M;
        rd.row0 = rb * rows_per;
        rd.rows = rows_per;
        rd.part0 = p.part_floats;
        rd.stride = (int64_t)spg * rows_per;
        rd.nchunks = (int32_t)nchunks;
        rd.scene0 = scene0;
        rd.nscenes = ns;
        rd.pad = 0;
        if (nchunks > 1) p.reds.push_back(rd);
        for (int64_t c = 0; c < nchunks; ++c) {
          psflib::GItem it;
          it.A = li.A;
          it.exps = li.cx.exps;
          it.M = li.M;
          it.ncols = li.ncols;
          it.row0 = rb * rows_per;
          it.j0 = c * chunk;
          it.j1 = std::min(units, (c + 1) * chunk);
          it.scene0 = scene0;
          it.nscenes = ns;
          it.bpk = bpk;
          it.direct = nchunks == 1;
          it.pad = 0;
          it.part = it.direct ? 0 : p.part_floats;
          if (!it.direct) p.part_floats += rd.stride;
          p.items.push_back(it);
        }
      }
    }
  }
  return p;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune_cache;  // plan signature -> chosen shape

}  // namespace

namespace psflib {

// Build (or rebuild) the plan's device tables and graph for one tile shape.
static hipError_t instantiate(psflib_grouped* g, const std::vector<LibInfo>& libs,
                              const int32_t* lib_of_scene, const float* const* scenes,
                              float* const* images, int B, Shape shape, hipStream_t s) {
  const Plan p = make_plan(g->storage, libs, lib_of_scene, scenes, images, B, shape);
  const size_t o_items = 0;
  const size_t o_reds = align256(o_items + p.items.size() * sizeof(GItem));
  const size_t o_sc = align256(o_reds + p.reds.size() * sizeof(GReduce));
  const size_t o_im = align256(o_sc + p.scenes.size() * sizeof(void*));
  const size_t o_slots = align256(o_im + p.images.size() * sizeof(void*));
  const size_t o_fexp = align256(o_slots + p.slots.size() * sizeof(GScene));
  const size_t o_packs = align256(o_fexp + p.slots.size() * sizeof(int32_t));
  const size_t o_bpk = align256(o_packs + p.packs.size() * sizeof(GPack));
  const size_t o_part = align256(o_bpk + (size_t)p.bpk_vecs * 16);
  const size_t total = align256(o_part + (size_t)p.part_floats * 4);
  if (g->exec) { (void)hipGraphExecDestroy(g->exec); g->exec = nullptr; }
  if (g->graph) { (void)hipGraphDestroy(g->graph); g->graph = nullptr; }
  // the previous tables are idle: every launch of the previous graph was
  // waited for on `s` (autotuning) before a new shape is instantiated
  if (g->dev) { (void)pool_release(g->dev, g->device); g->dev = nullptr; }
  hipError_t e = hipSuccess;
  if (total > 0) {
    e = pool_alloc(&g->dev, total, g->device, s);
    if (e != hipSuccess) { g->dev = nullptr; return e; }
  }
  char* d = reinterpret_cast<char*>(g->dev);
  if (!p.items.empty()) {
    const struct { size_t off; const void* src; size_t bytes; } up[] = {
        {o_items, p.items.data(), p.items.size() * sizeof(GItem)},
        {o_reds, p.reds.data(), p.reds.size() * sizeof(GReduce)},
        {o_sc, p.scenes.data(), p.scenes.size() * sizeof(void*)},
        {o_im, p.images.data(), p.images.size() * sizeof(void*)},
        {o_slots, p.slots.data(), p.slots.size() * sizeof(GScene)},
        {o_packs, p.packs.data(), p.packs.size() * sizeof(GPack)}};
    for (const auto& u : up) {
      if (u.bytes == 0) continue;
      e = hipMemcpyAsync(d + u.off, u.src, u.bytes, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return e;
    }
  }
  // the tables are on the device before any launch of the graph
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const GItem* items = reinterpret_cast<const GItem*>(d + o_items);
  const GReduce* reds = reinterpret_cast<const GReduce*>(d + o_reds);
  const float* const* sc = reinterpret_cast<const float* const*>(d + o_sc);
  float* const* im = reinterpret_cast<float* const*>(d + o_im);
  const GScene* slots = reinterpret_cast<const GScene*>(d + o_slots);
  int32_t* fexp = reinterpret_cast<int32_t*>(d + o_fexp);
  const GPack* packs = reinterpret_cast<const GPack*>(d + o_packs);
  u32x4* bpk = reinterpret_cast<u32x4*>(d + o_bpk);
  float* part = reinterpret_cast<float*>(d + o_part);
  const int64_t nitems = (int64_t)p.items.size();
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device);
  const int64_t per_cu = 4;  // resident workgroups per CU the persistent grid aims at
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)cus * per_cu));

  // 16-bit scenes staged whole in LDS for packing when every library allows
  int64_t maxcols = 0;
  for (const GPack& pk : p.packs) maxcols = std::max<int64_t>(maxcols, pk.ncols);
  const bool staged = g->storage != PSFLIB_FP32 && maxcols <= kStageMaxCols;
  const size_t stage_lds = (size_t)maxcols * 4;
  if (staged) {
    e = hipFuncSetAttribute(g->storage == PSFLIB_BF16_POW2
                                ? reinterpret_cast<const void*>(grouped_stage_pack_kernel<true>)
                                : reinterpret_cast<const void*>(grouped_stage_pack_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)stage_lds);
    if (e != hipSuccess) return e;
  }
  hipStream_t cap;
  e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    if (nitems > 0) {
      if (g->storage == PSFLIB_FP32) {
        const dim3 np((unsigned)p.packs.size(), 64);
        grouped_pack_f32_kernel<<<np, 256, 0, cap>>>(packs, sc, reinterpret_cast<f32x4*>(bpk));
        grouped_f32_kernel<<<grid, kGrpThreads, 0, cap>>>(items, nitems,
                                                          reinterpret_cast<const f32x4*>(bpk), part, im);
      } else {
        const bool bf = g->storage == PSFLIB_BF16_POW2;
        if (staged) {
          // whole rounds of 8 XCDs x 16 slots
          const int64_t npk = (int64_t)p.packs.size();
          const unsigned sgrid = (unsigned)((npk + 7) / 8 * 8 * kGrpScenes);
          if (bf)
            grouped_stage_pack_kernel<true><<<sgrid, 1024, stage_lds, cap>>>(packs, npk, slots, fexp, bpk);
          else
            grouped_stage_pack_kernel<false><<<sgrid, 1024, stage_lds, cap>>>(packs, npk, slots, fexp, bpk);
        } else {
          grouped_scene_exp_kernel<<<(unsigned)p.slots.size(), 1024, 0, cap>>>(slots, fexp);
          const dim3 np((unsigned)p.packs.size(), 64);  // 64 workgroups per scene group
          if (bf)
            grouped_pack_kernel<true><<<np, 256, 0, cap>>>(packs, sc, fexp, bpk);
          else
            grouped_pack_kernel<false><<<np, 256, 0, cap>>>(packs, sc, fexp, bpk);
        }
        auto run = [&](auto kern) { kern<<<grid, kGrpThreads, 0, cap>>>(items, nitems, bpk, fexp, part, im); };
        switch (shape.rows) {
          case 64: bf ? run(grouped_h16_kernel<true, 4>) : run(grouped_h16_kernel<false, 4>); break;
          case 128: bf ? run(grouped_h16_kernel<true, 2>) : run(grouped_h16_kernel<false, 2>); break;
          default: bf ? run(grouped_h16_kernel<true, 1>) : run(grouped_h16_kernel<false, 1>); break;
        }
      }
      if (!p.reds.empty())
        grouped_reduce_kernel<<<(unsigned)p.reds.size(), 256, 0, cap>>>(reds, part, im);
    }
    hipError_t e2 = hipStreamEndCapture(cap, &g->graph);
    e = (e2 != hipSuccess) ? e2 : hipGetLastError();
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  g->chunk = shape.chunk;
  g->rows = shape.rows;
  return e;
}

}  // namespace psflib

extern "C" {

psflib_status psflib_grouped_create(const psflib_handle* const* h_libs, int32_t nlibs,
                                    const int32_t* h_lib_of_scene, const float* const* h_scenes,
                                    float* const* h_images, int32_t B, int32_t autotune,
                                    void* stream, psflib_grouped** out) {
  if (!h_libs || nlibs < 1 || !out || B < 0 || (B > 0 && (!h_lib_of_scene || !h_scenes || !h_images)))
    return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: bad arguments");
  std::vector<LibInfo> libs;
  int storage = -1, dev = -1;
  for (int L = 0; L < nlibs; ++L) {
    if (!h_libs[L]) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: NULL library handle");
    LibInfo li;
    int st, d;
    psflib::handle_info(h_libs[L], &li.A, &li.cx, &li.M, &li.ncols, &li.ncols_pad, &st, &d);
    if (storage < 0) { storage = st; dev = d; }
    if (st != storage)
      return psflib::fail_status(PSFLIB_ERR_UNSUPPORTED, "grouped: all libraries must share one storage form");
    if (d != dev) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: libraries on different devices");
    if (st == PSFLIB_FP32 && li.M > ((int64_t)1 << 25))
      return psflib::fail_status(PSFLIB_ERR_UNSUPPORTED,
                                 "grouped: FP32 libraries need n*n <= 2^25 (n <= 5792)");
    libs.push_back(li);
  }
  for (int b = 0; b < B; ++b) {
    if (h_lib_of_scene[b] < 0 || h_lib_of_scene[b] >= nlibs)
      return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: scene library index out of range");
    if (!h_scenes[b] || !h_images[b])
      return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: NULL scene or image pointer");
    if (((uintptr_t)h_scenes[b] & 15u) != 0 || ((uintptr_t)h_images[b] & 15u) != 0)
      return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: scene and image arrays must be 16-byte aligned");
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != dev)
    return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: current device differs from the libraries'");
  psflib_status pst = psflib::check_pending_error();
  if (pst != PSFLIB_OK) return pst;
  psflib_grouped* g = new (std::nothrow) psflib_grouped();
  if (!g) return psflib::fail_status(PSFLIB_ERR_DEVICE, "host allocation failed");
  g->storage = storage;
  g->device = dev;
  g->graph = nullptr;
  g->exec = nullptr;
  g->dev = nullptr;
  g->ms_tuned = 0.0f;
  g->chunk = 0;
  g->rows = 256;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the libraries may still be building on `stream`
  hipError_t e = hipStreamSynchronize(s);
  auto bail = [&](hipError_t err, const char* what) {
    psflib_grouped_destroy(g);
    return psflib::device_fail_status(err, what);
  };
  if (e != hipSuccess) return bail(e, "hipStreamSynchronize");

  // Candidate shapes.  Chunk lengths: columns (FP32) or 8-column groups
  // (16-bit), 0 = every column in one item (images written directly, no
  // partials); rows per item: 256 for FP32, 256, 128 or 64 for 16-bit.
  const bool f32 = storage == PSFLIB_FP32;
  std::vector<Shape> cands;
  if (f32) {
    for (int64_t c : {0, 256, 512, 1024, 2048}) cands.push_back(Shape{c, 256});
  } else {
    for (int32_t r : {256, 128, 64})
      for (int64_t c : {0, 128, 256, 512, 1024}) cands.push_back(Shape{c, r});
  }
  std::string sig = std::to_string(storage) + ":";
  for (int b = 0; b < B; ++b) {
    const LibInfo& li = libs[h_lib_of_scene[b]];
    sig += std::to_string(li.M) + "x" + std::to_string(li.ncols) + ",";
  }
  Shape chosen = f32 ? Shape{512, 256} : Shape{256, 256};
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto itc = g_tune_cache.find(sig);
    if (itc != g_tune_cache.end()) { chosen = itc->second; cached = true; }
  }
  if (autotune && !cached && B > 0) {
    float best = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return bail(hipErrorUnknown, "hipEventCreate");
    for (const Shape& c : cands) {
      e = psflib::instantiate(g, libs, h_lib_of_scene, h_scenes, h_images, B, c, s);
      if (e != hipSuccess) break;
      float t = 1e30f;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = hipGraphLaunch(g->exec, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < t) t = ms;  // the first launch warms the caches
      }
      if (e == hipSuccess && t < best) { best = t; chosen = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return bail(e, "grouped autotune");
    g->ms_tuned = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[sig] = chosen;
  }
  e = psflib::instantiate(g, libs, h_lib_of_scene, h_scenes, h_images, B, chosen, s);
  if (e != hipSuccess) return bail(e, "grouped plan");
  {
    PlanInputs in;
    in.libs = libs;
    in.lib_of_scene.assign(h_lib_of_scene, h_lib_of_scene + B);
    in.scenes.assign(h_scenes, h_scenes + B);
    in.images.assign(h_images, h_images + B);
    std::lock_guard<std::mutex> lk(g_inputs_mu);
    g_inputs[g] = std::move(in);
  }
  *out = g;
  return PSFLIB_OK;
}

psflib_status psflib_grouped_set_shape(psflib_grouped* g, int64_t chunk, int32_t rows, void* stream) {
  if (!g) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped plan is NULL");
  const bool f32 = g->storage == PSFLIB_FP32;
  if (chunk < 0 || chunk % (f32 ? 16 : 8) != 0 ||
      (f32 ? rows != 256 : (rows != 64 && rows != 128 && rows != 256)))
    return psflib::fail_status(PSFLIB_ERR_INVALID_ARG,
                               "grouped: chunk must be a non-negative multiple of 16 columns (FP32) or "
                               "8 groups (16-bit); rows 256 (FP32) or 64, 128, 256 (16-bit)");
  PlanInputs in;
  {
    std::lock_guard<std::mutex> lk(g_inputs_mu);
    auto it = g_inputs.find(g);
    if (it == g_inputs.end()) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: unknown plan");
    in = it->second;
  }
  if (in.scenes.empty()) return PSFLIB_OK;
  psflib_status pst = psflib::check_pending_error();
  if (pst != PSFLIB_OK) return pst;
  // the plan's earlier launches finish before its tables are replaced
  g->uses.wait_all();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = psflib::instantiate(g, in.libs, in.lib_of_scene.data(), in.scenes.data(),
                                     in.images.data(), (int)in.scenes.size(), Shape{chunk, rows}, s);
  if (e != hipSuccess) return psflib::device_fail_status(e, "grouped plan");
  g->ms_tuned = 0.0f;
  return PSFLIB_OK;
}

psflib_status psflib_grouped_run(const psflib_grouped* g, void* stream) {
  if (!g) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped plan is NULL");
  if (!g->exec) return PSFLIB_OK;  // no scenes
  psflib_status pst = psflib::check_pending_error();
  if (pst != PSFLIB_OK) return pst;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipGraphLaunch(g->exec, s);
  if (e != hipSuccess) return psflib::device_fail_status(e, "hipGraphLaunch");
  e = g->uses.note(s);
  if (e != hipSuccess) return psflib::device_fail_status(e, "hipEventRecord(grouped run)");
  return PSFLIB_OK;
}

psflib_status psflib_grouped_chunk(const psflib_grouped* g, int64_t* chunk, float* tuned_ms) {
  return psflib_grouped_shape(g, chunk, nullptr, tuned_ms);
}

psflib_status psflib_grouped_shape(const psflib_grouped* g, int64_t* chunk, int32_t* rows,
                                   float* tuned_ms) {
  if (!g || !chunk) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "NULL argument");
  *chunk = g->chunk;
  if (rows) *rows = g->rows;
  if (tuned_ms) *tuned_ms = g->ms_tuned;
  return PSFLIB_OK;
}

void psflib_grouped_destroy(psflib_grouped* g) {
  if (!g) return;
  {
    std::lock_guard<std::mutex> lk(g_inputs_mu);
    g_inputs.erase(g);
  }
  // wait for the plan's own launches (not for the device)
  g->uses.wait_all();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->dev) (void)psflib::pool_release(g->dev, g->device);
  delete g;
}

}  // extern "C"
