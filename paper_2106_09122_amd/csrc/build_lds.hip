// Library build with the radial sample pair staged in LDS (Sec. 2; Eqs. (4)-(5)).
//
// Columns are grouped by their radial bracket k on the device (a counting sort:
// histogram, scan, scatter), so a workgroup can stage the two sampled PSFs it
// needs, P_k and P_{k+1}, once in LDS and build many columns from them.  The
// pair is stored interleaved (one 8-byte LDS read returns both radial
// neighbours of a tap) inside a one-pixel zero border, so the bilinear taps of
// the rotated sample need no per-tap bounds tests.
//
// Coordinates follow the oracle's float64 operations exactly (same products,
// no contraction): per column the products cos*(b-c) and -sin*(b-c) of an
// image column and sin*(a-c), cos*(a-c) of an image row are formed once and
// each element adds them.  The fractional offsets and their complements are
// exact float64 values rounded once to float32; the bilinear weights are their
// float32 products, the radial blend and the weighted sum are float32
// (relative error a few float32 units, as the entries are non-negative
// combinations).
//
// Paths, by what fits:
//  * rotation orbits: the four quarter turns of a scene pixel about the star
//    have bitwise-rotated columns, so one wave forms a base column and writes
//    all four (float32: 16-byte runs straight from registers; 16-bit: rounded
//    into an LDS tile of 8-slot units, slots ordered so that a group holds one
//    quarter turn of 8 base columns).  The pair is staged whole when it fits
//    the LDS; larger pairs (up to 8192 x 8192) are read through a small box per
//    32 x 32 pixel tile, staged by each wave in its own LDS region;
//  * columns in bracket order (16-bit forms whose scene size is not a multiple
//    of 8, pairs that fit the LDS): one wave per column, 16 columns per
//    workgroup, units assembled from an LDS tile.
// The 16-bit forms of the other builds (and of columns that need float32
// post-processing, the flux-preserving rescale) are built as float32 columns
// into scratch and packed by a second kernel (scale by 2^-e_j, round to
// nearest even, 8 columns per 16 B).
#include <math.h>

#include <type_traits>

#include "psflib_internal.h"

namespace psflib {

// ------------------------------------------------------------ buckets -----
__global__ __launch_bounds__(256) void zero_ints_kernel(int32_t* __restrict__ p, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0;
}

// bucket of column j: its bracket k, or nb-1 for an identically zero column.
// Counts are gathered in an LDS histogram per workgroup and added to the
// global counts with one atomic per non-empty bucket (few buckets, many
// columns: direct global atomics would serialise on a handful of addresses).
__device__ __forceinline__ int bucket_of(const ColGeom* __restrict__ geo, int64_t j, int nb) {
  const int k = geo[j].k;
  return k >= 0 ? k : nb - 1;
}

__global__ __launch_bounds__(256) void bucket_count_kernel(const ColGeom* __restrict__ geo,
                                                           int64_t ncols, int nb,
                                                           int32_t* __restrict__ cnt) {
  extern __shared__ int32_t hist[];  // nb
  for (int b = threadIdx.x; b < nb; b += 256) hist[b] = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < ncols) atomicAdd(hist + bucket_of(geo, j, nb), 1);
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += 256)
    if (hist[b]) atomicAdd(cnt + b, hist[b]);
}

// One workgroup: bucket starts (exclusive scan of the counts) and the work
// items (bucket, first sorted position, length <= kLdsCols).
__global__ __launch_bounds__(1024) void bucket_scan_kernel(const int32_t* __restrict__ cnt, int nb,
                                                           int32_t* __restrict__ bstart,
                                                           int4* __restrict__ items,
                                                           int32_t* __restrict__ nitems) {
  __shared__ int32_t s_cols[1024], s_items[1024];
  const int tid = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = tid * per, b1 = (b0 + per < nb) ? b0 + per : nb;
  int my_cols = 0, my_items = 0;
  for (int b = b0; b < b1; ++b) {
    my_cols += cnt[b];
    my_items += (cnt[b] + kLdsCols - 1) / kLdsCols;
  }
  s_cols[tid] = my_cols;
  s_items[tid] = my_items;
  __syncthreads();
  // inclusive Hillis-Steele scan of both arrays
  for (int off = 1; off < 1024; off <<= 1) {
    int c = 0, it = 0;
    if (tid >= off) {
      c = s_cols[tid - off];
      it = s_items[tid - off];
    }
    __syncthreads();
    s_cols[tid] += c;
    s_items[tid] += it;
    __syncthreads();
  }
  int col = s_cols[tid] - my_cols, item = s_items[tid] - my_items;
  for (int b = b0; b < b1; ++b) {
    bstart[b] = col;
    for (int s = 0; s < cnt[b]; s += kLdsCols) {
      const int len = (cnt[b] - s < kLdsCols) ? cnt[b] - s : kLdsCols;
      items[item++] = make_int4(b, col + s, len, 0);
    }
    col += cnt[b];
  }
  if (tid == 1023) *nitems = s_items[1023];
}

// Positions: a local rank from LDS atomics, one global atomic per non-empty
// bucket to reserve this workgroup's run of positions.  (The order inside a
// bucket only decides which workgroup builds a column, not its values.)
__global__ __launch_bounds__(256) void bucket_scatter_kernel(const ColGeom* __restrict__ geo,
                                                             int64_t ncols, int nb,
                                                             const int32_t* __restrict__ bstart,
                                                             int32_t* __restrict__ cursor,
                                                             int32_t* __restrict__ order) {
  extern __shared__ int32_t sh[];  // nb local counts, then nb bases
  int32_t* lcnt = sh;
  int32_t* base = sh + nb;
  for (int b = threadIdx.x; b < nb; b += 256) lcnt[b] = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int b = 0, r = 0;
  if (j < ncols) {
    b = bucket_of(geo, j, nb);
    r = atomicAdd(lcnt + b, 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nb; q += 256)
    if (lcnt[q]) base[q] = bstart[q] + atomicAdd(cursor + q, lcnt[q]);
  __syncthreads();
  if (j < ncols) order[base[b] + r] = (int32_t)j;
}

// --------------------------------------------------------------- build -----
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Float64 coordinate work of one element, in the oracle's order:
// sx = ct*ux + st*uy, sy = (-st)*ux + ct*uy, col = c + sx, row = c + sy.
struct Tap {
  int idx;           // LDS index of (r0, c0) in the bordered array
  bool ok;           // all four taps inside the bordered array
  float fx, gx, fy, gy;  // fx, 1-fx, fy, 1-fy (float32 of the float64 values)
};

__device__ __forceinline__ Tap tap_coords(double ctux, double mstux, double stuy, double ctuy,
                                          double c, int n, int ls) {
#pragma clang fp contract(off)
  const double sx = ctux + stuy;
  const double sy = mstux + ctuy;
  const double colf = c + sx;
  const double rowf = c + sy;
  const double c0f = floor(colf);
  const double r0f = floor(rowf);
  const double fx = colf - c0f;
  const double fy = rowf - r0f;
  Tap t;
  t.fx = (float)fx;
  t.gx = (float)(1.0 - fx);
  t.fy = (float)fy;
  t.gy = (float)(1.0 - fy);
  // |colf|, |rowf| < 3n, so the integer conversions are exact.  Taps r0, r0+1
  // (c0, c0+1) lie in the bordered array iff -1 <= r0, c0 <= n-1.
  const int c0 = (int)c0f, r0 = (int)r0f;
  t.ok = ((unsigned)(r0 + 1) <= (unsigned)n) && ((unsigned)(c0 + 1) <= (unsigned)n);
  t.idx = t.ok ? (r0 + 1) * ls + (c0 + 1) : 0;
  return t;
}

template <int E, bool FULL>
__global__ __launch_bounds__(1024) void build_lds_kernel(const float* __restrict__ cube, int K,
                                                         const ColGeom* __restrict__ geo,
                                                         const int32_t* __restrict__ order,
                                                         const int4* __restrict__ items,
                                                         const int32_t* __restrict__ nitems,
                                                         int nb, int n, int ls, int64_t M,
                                                         float* __restrict__ A,
                                                         double* __restrict__ tau) {
  // (n+2) rows of pairs (P_k, P_{k+1}) with a zero border, row stride ls >= n+2
  extern __shared__ float2 P2[];
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, start = it.y, len = it.z;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int np = n + 2;
  if (!zero_bucket) {
    const float* Pk = cube + (int64_t)bkt * M;
    const float* Pk1 = (K > 1) ? Pk + M : nullptr;
    // zero border
    for (int idx = tid; idx < 4 * np; idx += 1024) {
      const int side = idx / np, t = idx % np;
      const int pos = side == 0 ? t : side == 1 ? (np - 1) * ls + t
                    : side == 2 ? t * ls : t * ls + np - 1;
      P2[pos] = make_float2(0.0f, 0.0f);
    }
    // interior, 4 pixels (16 B of each PSF) per thread and step when rows allow
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(cube) & 15) == 0) {
      const int nq = n >> 2;
      for (int q = tid; q < n * nq; q += 1024) {
        const int rr = q / nq, cc = 4 * (q - rr * nq);
        const f32x4 a = *reinterpret_cast<const f32x4*>(Pk + rr * n + cc);
        const f32x4 b = Pk1 ? *reinterpret_cast<const f32x4*>(Pk1 + rr * n + cc)
                            : (f32x4){0.f, 0.f, 0.f, 0.f};
        float2* dst = P2 + (rr + 1) * ls + cc + 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = make_float2(a[e], b[e]);
      }
    } else {
      for (int q = tid; q < n * n; q += 1024) {
        const int rr = q / n, cc = q - rr * n;
        P2[(rr + 1) * ls + cc + 1] = make_float2(Pk[q], Pk1 ? Pk1[q] : 0.0f);
      }
    }
  }
  __syncthreads();
  if (wave >= len) return;  // no barrier below
  const int64_t j = order[start + wave];
  float* col = A + j * M;
  if (zero_bucket) {
    for (int a = 0; a < n; ++a)
#pragma unroll
      for (int v = 0; v < E; ++v) {
        const int b = lane + 64 * v;
        if (FULL || b < n) __builtin_nontemporal_store(0.0f, col + a * n + b);
      }
    if (lane == 0) tau[j] = 0.0;
    return;
  }
  const ColGeom g = geo[j];
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
  double tsum = 0.0;
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
      if (FULL || b < n) {
        const Tap t = tap_coords(ctux[v], mstux[v], stuy, ctuy, c, n, ls);
        const float2 p00 = P2[t.idx], p01 = P2[t.idx + 1];
        const float2 p10 = P2[t.idx + ls], p11 = P2[t.idx + ls + 1];
        const float q00 = fmaf(wk1, p00.y, wk0 * p00.x);
        const float q01 = fmaf(wk1, p01.y, wk0 * p01.x);
        const float q10 = fmaf(wk1, p10.y, wk0 * p10.x);
        const float q11 = fmaf(wk1, p11.y, wk0 * p11.x);
        float val = (t.gy * t.gx) * q00;
        val = fmaf(t.gy * t.fx, q01, val);
        val = fmaf(t.fy * t.gx, q10, val);
        val = fmaf(t.fy * t.fx, q11, val);
        val = t.ok ? val : 0.0f;
        __builtin_nontemporal_store(val, col + a * n + b);
        rowsum += val;
      }
    }
    tsum += (double)rowsum;
  }
  tsum = wave_sum_f64(tsum);
  if (lane == 0) tau[j] = tsum;
}

// ------------------------------------------- 16-bit build, slot order -----
// The 16-bit forms store columns in groups of 8 slots.  So that one workgroup
// can write whole 16-byte groups straight from LDS-staged PSFs, the slots
// are ordered by radial bracket: a stable counting sort (bracket, then column
// index) gives slot s -> column perm[s], and the buckets are cut into work
// items along 16-slot windows.  A workgroup builds the (up to 16) columns of
// one item from its bracket's pair, one wave per column, a few image rows at
// a time: each wave rounds its values to the 16-bit format into an LDS tile,
// and after a barrier every thread gathers the 8 slots of one (group, pixel)
// and writes them as one 16-byte store (2-byte stores for the slots of a
// group that belong to the neighbouring bucket's item).  The float32 values,
// their rounding and the column sums are those of the float32 build.

constexpr int kSortBlock = 1024;  // columns per block of the stable sort

// counts of every bucket in every block of kSortBlock columns: cnt[blk][b]
__global__ __launch_bounds__(kSortBlock) void sort_count_kernel(const ColGeom* __restrict__ geo,
                                                                int64_t ncols, int nb,
                                                                int32_t* __restrict__ cnt) {
  extern __shared__ int32_t hist[];  // nb
  for (int b = threadIdx.x; b < nb; b += kSortBlock) hist[b] = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kSortBlock + threadIdx.x;
  if (j < ncols) atomicAdd(hist + bucket_of(geo, j, nb), 1);  // counts: order-free
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += kSortBlock) cnt[(int64_t)blockIdx.x * nb + b] = hist[b];
}

// One workgroup.  cnt[blk][b] becomes the first slot of bucket b's columns of
// block blk (bucket start + the bucket's columns in earlier blocks); items
// (bucket, first slot, length, 16-slot window start) cover every bucket along
// 16-slot windows.
__global__ __launch_bounds__(1024) void sort_scan_kernel(int32_t* __restrict__ cnt, int64_t nblk,
                                                         int nb, int4* __restrict__ items,
                                                         int32_t* __restrict__ nitems) {
  __shared__ int32_t s_cols[1024], s_items[1024];
  __shared__ int32_t tot[kLdsMaxBuckets];
  const int tid = threadIdx.x;
  for (int b = tid; b < nb; b += 1024) {  // independent loads: no store in between
    int32_t run = 0;
    for (int64_t k = 0; k < nblk; ++k) run += cnt[k * nb + b];
    tot[b] = run;
  }
  __syncthreads();
  const int per = (nb + 1023) / 1024;
  const int b0 = tid * per, b1 = (b0 + per < nb) ? b0 + per : nb;
  int my_cols = 0;
  for (int b = b0; b < b1; ++b) my_cols += tot[b];
  s_cols[tid] = my_cols;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int c = tid >= off ? s_cols[tid - off] : 0;
    __syncthreads();
    s_cols[tid] += c;
    __syncthreads();
  }
  // bucket starts, then the items of each bucket
  int start = s_cols[tid] - my_cols, my_items = 0;
  for (int b = b0; b < b1; ++b) {
    const int c = tot[b];
    if (c > 0) my_items += (start + c - 1) / 16 - start / 16 + 1;
    start += c;
  }
  s_items[tid] = my_items;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int c = tid >= off ? s_items[tid - off] : 0;
    __syncthreads();
    s_items[tid] += c;
    __syncthreads();
  }
  start = s_cols[tid] - my_cols;
  int item = s_items[tid] - my_items;
  for (int b = b0; b < b1; ++b) {
    const int c = tot[b];
    int32_t run = start;  // first slot of bucket b in each block
    for (int64_t k0 = 0; k0 < nblk; k0 += 16) {
      int32_t v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = (k0 + u < nblk) ? cnt[(k0 + u) * nb + b] : 0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (k0 + u < nblk) {
          cnt[(k0 + u) * nb + b] = run;
          run += v[u];
        }
    }
    for (int w = start / 16 * 16; c > 0 && w < start + c; w += 16) {
      const int lo = w > start ? w : start;
      const int hi = (w + 16 < start + c) ? w + 16 : start + c;
      items[item++] = make_int4(b, lo, hi - lo, w);
    }
    start += c;
  }
  if (tid == 1023) *nitems = s_items[1023];
}

// Slots: a column's slot is its block's first slot of the bucket plus its
// rank among the block's earlier columns of the same bucket.  Each wave ranks
// its 64 columns with one ballot per bucket present; then the waves take
// their slots in order, each adding its counts to a per-bucket cursor in LDS
// that starts at the block's first slots.  Also the slot's exponent.
__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(const ColGeom* __restrict__ geo,
                                                                  int64_t ncols, int nb,
                                                                  const int32_t* __restrict__ first,
                                                                  int32_t* __restrict__ perm,
                                                                  int32_t* __restrict__ slot_of,
                                                                  int32_t* __restrict__ eslot) {
  extern __shared__ int32_t cursor[];  // nb
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = tid; q < nb; q += kSortBlock) cursor[q] = first[(int64_t)blockIdx.x * nb + q];
  const int64_t j = (int64_t)blockIdx.x * kSortBlock + tid;
  const bool valid = j < ncols;
  const int b = valid ? bucket_of(geo, j, nb) : -1;
  uint64_t todo = __ballot(valid);
  int rank = 0, count = 0;
  while (todo) {  // uniform: one pass per bucket present in the wave
    const int bl = __shfl(b, __builtin_ctzll(todo), 64);
    const uint64_t m = __ballot(valid && b == bl);
    if (valid && b == bl) {
      rank = __popcll(m & ((1ull << lane) - 1ull));
      count = __popcll(m);
    }
    todo &= ~m;
  }
  __syncthreads();
  int slot = 0;
  for (int w = 0; w < kSortBlock / 64; ++w) {
    if (wave == w && valid) {
      slot = cursor[b] + rank;  // every lane reads before the wave's leaders add
      __builtin_amdgcn_wave_barrier();
      if (rank == 0) cursor[b] += count;
    }
    __syncthreads();
  }
  if (!valid) return;
  perm[slot] = (int32_t)j;
  slot_of[j] = slot;
  eslot[slot] = geo[j].e;
}

template <int E, bool FULL, bool BF16>
__global__ __launch_bounds__(1024) void build_lds16_kernel(const float* __restrict__ cube, int K,
                                                           const ColGeom* __restrict__ geo,
                                                           const int32_t* __restrict__ perm,
                                                           const int4* __restrict__ items,
                                                           const int32_t* __restrict__ nitems,
                                                           int nb, int n, int ls, int R, int64_t M,
                                                           uint16_t* __restrict__ Mh,
                                                           double* __restrict__ tau) {
  extern __shared__ float2 P2[];  // bordered pair, (n+2) rows of stride ls; then the 16-bit tile
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, first = it.y, len = it.z, w0 = it.w;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int np = n + 2;
  uint16_t* T = reinterpret_cast<uint16_t*>(P2 + (size_t)np * ls);  // [16][R * n]
  const int tstride = R * n;
  if (!zero_bucket) {
    const float* Pk = cube + (int64_t)bkt * M;
    const float* Pk1 = (K > 1) ? Pk + M : nullptr;
    for (int idx = tid; idx < 4 * np; idx += 1024) {
      const int side = idx / np, t = idx % np;
      const int pos = side == 0 ? t : side == 1 ? (np - 1) * ls + t
                    : side == 2 ? t * ls : t * ls + np - 1;
      P2[pos] = make_float2(0.0f, 0.0f);
    }
    if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(cube) & 15) == 0) {
      const int nq = n >> 2;
      for (int q = tid; q < n * nq; q += 1024) {
        const int rr = q / nq, cc = 4 * (q - rr * nq);
        const f32x4 a = *reinterpret_cast<const f32x4*>(Pk + rr * n + cc);
        const f32x4 b = Pk1 ? *reinterpret_cast<const f32x4*>(Pk1 + rr * n + cc)
                            : (f32x4){0.f, 0.f, 0.f, 0.f};
        float2* dst = P2 + (rr + 1) * ls + cc + 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = make_float2(a[e], b[e]);
      }
    } else {
      for (int q = tid; q < n * n; q += 1024) {
        const int rr = q / n, cc = q - rr * n;
        P2[(rr + 1) * ls + cc + 1] = make_float2(Pk[q], Pk1 ? Pk1[q] : 0.0f);
      }
    }
  }
  const int slot = w0 + wave;
  const bool live = slot >= first && slot < first + len;  // uniform per wave
  int64_t j = 0;
  ColGeom g;
  g.ct = 1.0; g.st = 0.0; g.w = 0.0; g.e = 0;
  if (live) {
    j = perm[slot];
    g = geo[j];
  }
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
  double tsum = 0.0;
  // the slots of this item among the item's two groups
  const int64_t grp0 = w0 / 8;
  for (int a0 = 0; a0 < n; a0 += R) {
    const int rows = (n - a0 < R) ? n - a0 : R;
    __syncthreads();  // the pair is staged; the previous tile has been stored
    if (live) {
      for (int r = 0; r < rows; ++r) {
        const int a = a0 + r;
        double stuy, ctuy;
        {
#pragma clang fp contract(off)
          const double uy = (double)a - c;
          stuy = g.st * uy;
          ctuy = g.ct * uy;
        }
#pragma unroll
        for (int v = 0; v < E; ++v) {
          const int b = lane + 64 * v;
          if (FULL || b < n) {
            float val = 0.0f;
            if (!zero_bucket) {
              const Tap t = tap_coords(ctux[v], mstux[v], stuy, ctuy, c, n, ls);
              const float2 p00 = P2[t.idx], p01 = P2[t.idx + 1];
              const float2 p10 = P2[t.idx + ls], p11 = P2[t.idx + ls + 1];
              const float q00 = fmaf(wk1, p00.y, wk0 * p00.x);
              const float q01 = fmaf(wk1, p01.y, wk0 * p01.x);
              const float q10 = fmaf(wk1, p10.y, wk0 * p10.x);
              const float q11 = fmaf(wk1, p11.y, wk0 * p11.x);
              val = (t.gy * t.gx) * q00;
              val = fmaf(t.gy * t.fx, q01, val);
              val = fmaf(t.fy * t.gx, q10, val);
              val = fmaf(t.fy * t.fx, q11, val);
              val = t.ok ? val : 0.0f;
            }
            tsum += (double)val;
            const float x = ldexpf(val, -g.e);  // exact power-of-two scaling
            uint32_t h;
            if constexpr (BF16) {
              uint32_t u = __float_as_uint(x);
              u += 0x7FFFu + ((u >> 16) & 1u);  // finite: round to nearest, ties to even
              h = u >> 16;
            } else {
              h = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
            }
            T[wave * tstride + r * n + b] = (uint16_t)h;
          }
        }
      }
    }
    __syncthreads();
    // (group gi, pixel p of the tile): the 8 slots of the group at that pixel
    const int units = 2 * rows * n;
    for (int u = tid; u < units; u += 1024) {
      const int gi = u / (rows * n), p = u - gi * (rows * n);
      const int s0 = 8 * gi;  // first slot of the group, relative to w0
      const int lo = (first - w0 > s0) ? first - w0 : s0;
      const int hi = (first + len - w0 < s0 + 8) ? first + len - w0 : s0 + 8;
      if (lo >= hi) continue;  // no slot of this group in the item
      const int64_t i = (int64_t)a0 * n + p;
      uint16_t* dst = Mh + ((grp0 + gi) * M + i) * 8;
      if (lo == s0 && hi == s0 + 8) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          w[q] = (uint32_t)T[(s0 + 2 * q) * tstride + p] | ((uint32_t)T[(s0 + 2 * q + 1) * tstride + p] << 16);
        __builtin_nontemporal_store((u32x4){w[0], w[1], w[2], w[3]}, reinterpret_cast<u32x4*>(dst));
      } else {
        for (int q = lo; q < hi; ++q) dst[q - s0] = T[q * tstride + p];
      }
    }
  }
  if (!live) return;
  tsum = wave_sum_f64(tsum);
  if (lane == 0) tau[j] = tsum;
}

// 16-bit packing: M16[g][i][u] = RN16(A32[8g+u][i] * 2^-e), zeros past ncols.
// Two rows per thread: 8 x 8-byte loads (one per column; 512 B per wave and
// column) and 32 contiguous bytes stored.
template <bool BF16>
__global__ __launch_bounds__(256) void pack16_kernel(const float* __restrict__ A32,
                                                     const ColGeom* __restrict__ geo,
                                                     int64_t M, int64_t ncols,
                                                     u32x4* __restrict__ Mp, int64_t g0,
                                                     int64_t col0) {
  // groups g0 + blockIdx.y; column j of the float32 source at A32 + (j - col0) M
  const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  const int64_t grp = g0 + blockIdx.y;
  if (i0 >= M) return;
  const bool pair = (M % 2) == 0;  // then i0 + 1 < M and the 8-byte loads are aligned
  float v[8][2];
  int32_t ex[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t j = grp * 8 + u;
    v[u][0] = v[u][1] = 0.0f;
    ex[u] = 0;
    if (j < ncols) {
      ex[u] = geo[j].e;
      const float* src = A32 + (j - col0) * M + i0;
      if (pair) {
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        const f32x2 t = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(src));
        v[u][0] = t.x;
        v[u][1] = t.y;
      } else {
        v[u][0] = src[0];
        v[u][1] = (i0 + 1 < M) ? src[1] : 0.0f;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (i0 + r >= M) break;
    uint32_t h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float x = ldexpf(v[u][r], -ex[u]);
      if (BF16) {
        uint32_t w = __float_as_uint(x);
        w += 0x7FFFu + ((w >> 16) & 1u);
        h[u] = w >> 16;
      } else {
        h[u] = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
      }
    }
    u32x4 pk;
    pk.x = h[0] | (h[1] << 16);
    pk.y = h[2] | (h[3] << 16);
    pk.z = h[4] | (h[5] << 16);
    pk.w = h[6] | (h[7] << 16);
    __builtin_nontemporal_store(pk, Mp + grp * M + i0 + r);
  }
}

// Zero mantissas of the padding slots [ncols, ncols_pad): thread = (group, row).
__global__ __launch_bounds__(256) void zero_pad16_kernel(uint16_t* __restrict__ Mh, int64_t M,
                                                         int64_t ncols, int64_t g0) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int64_t grp = g0 + blockIdx.y;
  uint16_t* dst = Mh + (grp * M + i) * 8;
  for (int q = 0; q < 8; ++q)
    if (grp * 8 + q >= ncols) dst[q] = 0;
}

// --------------------------------------------- rotation-orbit builds -----
// The scene grid (centre ((N-1)/2, (N-1)/2)) and the PSF grid (centre
// ((n-1)/2, (n-1)/2)) are both invariant under quarter turns.  Turning a
// scene pixel by 90 degrees about the star maps (x, y) to (-y, x) exactly
// (index arithmetic: (p, q) -> (q, N-1-p)), so the turned column has
// cos' = -sin and sin' = cos exactly and the same radius, bracket and
// weight; its source coordinates at image pixel (b', a') = (N-1-a, b) are
// the base column's at (b, a) -- the same float64 products added in the
// other order, which is exact.  Every entry of the turned column is
// therefore bitwise the base column's at the turned image pixel:
//   C1[b][n-1-a] = C2[n-1-a][n-1-b] = C3[n-1-b][a] = C0[a][b]
// for the orbit (j0, j1, j2, j3) of a base column j0 in the quadrant
// x > 0, y >= 0 (the centre pixel of an odd grid is its own orbit).  The
// orbit builds compute C0 once and write all four columns: a quarter of the
// coordinate and interpolation work per stored entry.  Base columns are
// sorted by bracket (stable), cut into windows of 16; a work item is the run
// of one bracket inside a window times a range of image rows (so a launch has
// many more items than compute units), and each wave builds one base column
// over the item's rows.  Column sums: per (row range, base column) partial
// sums in float64, added in row-range order by a last kernel.

// quadrant bases p in [N/2, N), q in [(N+1)/2, N); the centre last (odd N)
struct OrbitGrid {
  int N, plo, qlo, hq;
  int64_t n4;      // base columns with a 4-column orbit
  int64_t nreps;   // n4, plus the centre for odd N
};

__host__ __device__ inline OrbitGrid orbit_grid(int N) {
  OrbitGrid o;
  o.N = N;
  o.plo = N / 2;
  o.qlo = (N + 1) / 2;
  o.hq = N - o.qlo;
  o.n4 = (int64_t)(N - o.plo) * o.hq;
  o.nreps = o.n4 + (N & 1);
  return o;
}

__device__ __forceinline__ int64_t orbit_base(const OrbitGrid& o, int64_t t) {
  if (t < o.n4) {
    const int64_t p = o.plo + t / o.hq, q = o.qlo + t % o.hq;
    return p * o.N + q;
  }
  return (int64_t)(o.N / 2) * o.N + o.N / 2;  // centre
}

// rotation partners of base column j0 = p N + q (k quarter turns)
__device__ __forceinline__ int64_t orbit_member(int64_t j0, int N, int k) {
  const int64_t p = j0 / N, q = j0 - p * N;
  switch (k) {
    case 0: return j0;
    case 1: return q * N + (N - 1 - p);
    case 2: return (N - 1 - p) * N + (N - 1 - q);
    default: return (N - 1 - q) * N + p;
  }
}

__device__ __forceinline__ bool orbit_is_centre(int64_t j0, int N) {
  return (N & 1) && j0 == (int64_t)(N / 2) * N + N / 2;
}

// rows of an image-row range: a multiple of 32, about a quarter of the image
static inline int orbit_rows_per_range(int n) {
  const int q = (n + 3) / 4;
  return ((q + 31) / 32) * 32;
}

__global__ __launch_bounds__(kSortBlock) void orbit_count_kernel(const ColGeom* __restrict__ geo,
                                                                 OrbitGrid o, int nb,
                                                                 int32_t* __restrict__ cnt) {
  extern __shared__ int32_t hist[];  // nb
  for (int b = threadIdx.x; b < nb; b += kSortBlock) hist[b] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kSortBlock + threadIdx.x;
  if (t < o.nreps) atomicAdd(hist + bucket_of(geo, orbit_base(o, t), nb), 1);  // order-free
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += kSortBlock) cnt[(int64_t)blockIdx.x * nb + b] = hist[b];
}

// Stable placement of the base columns (as sort_scatter_kernel); with
// `perm` set (16-bit forms, N a multiple of 8, no centre) also the slots of
// every orbit member: base position s in block s/8 of 8 bases, member k in
// group 4 (s/8) + k, slot 32 (s/8) + 8 k + s%8.
__global__ __launch_bounds__(kSortBlock) void orbit_scatter_kernel(const ColGeom* __restrict__ geo,
                                                                   OrbitGrid o, int nb,
                                                                   const int32_t* __restrict__ first,
                                                                   int32_t* __restrict__ reps,
                                                                   int32_t* __restrict__ perm,
                                                                   int32_t* __restrict__ slot_of,
                                                                   int32_t* __restrict__ eslot) {
  extern __shared__ int32_t cursor[];  // nb
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = tid; q < nb; q += kSortBlock) cursor[q] = first[(int64_t)blockIdx.x * nb + q];
  const int64_t t = (int64_t)blockIdx.x * kSortBlock + tid;
  const bool valid = t < o.nreps;
  const int64_t j0 = valid ? orbit_base(o, t) : 0;
  const int b = valid ? bucket_of(geo, j0, nb) : -1;
  uint64_t todo = __ballot(valid);
  int rank = 0, count = 0;
  while (todo) {  // uniform: one pass per bucket present in the wave
    const int bl = __shfl(b, __builtin_ctzll(todo), 64);
    const uint64_t m = __ballot(valid && b == bl);
    if (valid && b == bl) {
      rank = __popcll(m & ((1ull << lane) - 1ull));
      count = __popcll(m);
    }
    todo &= ~m;
  }
  __syncthreads();
  int pos = 0;
  for (int w = 0; w < kSortBlock / 64; ++w) {
    if (wave == w && valid) {
      pos = cursor[b] + rank;  // every lane reads before the wave's leaders add
      __builtin_amdgcn_wave_barrier();
      if (rank == 0) cursor[b] += count;
    }
    __syncthreads();
  }
  if (!valid) return;
  reps[pos] = (int32_t)j0;
  if (perm) {
    const int32_t e = geo[j0].e;  // the members share the radius, hence the exponent
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t j = orbit_member(j0, o.N, k);
      const int32_t slot = (pos / 8) * 32 + 8 * k + pos % 8;
      perm[slot] = (int32_t)j;
      slot_of[j] = slot;
      eslot[slot] = e;
    }
  }
}

// column sums: the partial sums of the row ranges in order, for every member
__global__ __launch_bounds__(256) void orbit_tau_kernel(const int32_t* __restrict__ reps,
                                                        const double* __restrict__ part,
                                                        int nranges, int64_t nreps, int N,
                                                        double* __restrict__ tau) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nreps) return;
  double t = 0.0;
  for (int r = 0; r < nranges; ++r) t += part[(int64_t)r * nreps + s];
  const int64_t j0 = reps[s];
  if (orbit_is_centre(j0, N)) {
    tau[j0] = t;
    return;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) tau[orbit_member(j0, N, k)] = t;
}

// the bordered pair (P_k, P_{k+1}) with its zero border, as the LDS build
__device__ __forceinline__ void stage_pair(float2* __restrict__ P2, const float* __restrict__ cube,
                                           int bkt, int K, int n, int ls, int64_t M, int tid) {
  const int np = n + 2;
  const float* Pk = cube + (int64_t)bkt * M;
  const float* Pk1 = (K > 1) ? Pk + M : nullptr;
  for (int idx = tid; idx < 4 * np; idx += 1024) {
    const int side = idx / np, t = idx % np;
    const int pos = side == 0 ? t : side == 1 ? (np - 1) * ls + t : side == 2 ? t * ls : t * ls + np - 1;
    P2[pos] = make_float2(0.0f, 0.0f);
  }
  if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(cube) & 15) == 0) {
    const int nq = n >> 2;
    for (int q = tid; q < n * nq; q += 1024) {
      const int rr = q / nq, cc = 4 * (q - rr * nq);
      const f32x4 a = *reinterpret_cast<const f32x4*>(Pk + rr * n + cc);
      const f32x4 b = Pk1 ? *reinterpret_cast<const f32x4*>(Pk1 + rr * n + cc) : (f32x4){0.f, 0.f, 0.f, 0.f};
      float2* dst = P2 + (rr + 1) * ls + cc + 1;
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = make_float2(a[e], b[e]);
    }
  } else {
    for (int q = tid; q < n * n; q += 1024) {
      const int rr = q / n, cc = q - rr * n;
      P2[(rr + 1) * ls + cc + 1] = make_float2(Pk[q], Pk1 ? Pk1[q] : 0.0f);
    }
  }
}

// One element of the base column (the LDS build's arithmetic).
__device__ __forceinline__ float orbit_value(const float2* __restrict__ P2, double ctux, double mstux,
                                             double stuy, double ctuy, double c, int n, int ls,
                                             float wk0, float wk1) {
  const Tap t = tap_coords(ctux, mstux, stuy, ctuy, c, n, ls);
  const float2 p00 = P2[t.idx], p01 = P2[t.idx + 1];
  const float2 p10 = P2[t.idx + ls], p11 = P2[t.idx + ls + 1];
  const float q00 = fmaf(wk1, p00.y, wk0 * p00.x);
  const float q01 = fmaf(wk1, p01.y, wk0 * p01.x);
  const float q10 = fmaf(wk1, p10.y, wk0 * p10.x);
  const float q11 = fmaf(wk1, p11.y, wk0 * p11.x);
  float val = (t.gy * t.gx) * q00;
  val = fmaf(t.gy * t.fx, q01, val);
  val = fmaf(t.fy * t.gx, q10, val);
  val = fmaf(t.fy * t.fx, q11, val);
  return t.ok ? val : 0.0f;
}

// Modes of the float32 orbit kernels: the plain build; only the column sums
// (no stores: the first pass of a flux-preserving build); or every value
// multiplied by its column's float32 scale before it is stored and summed
// (the second pass).
constexpr int kPlain = kOrbitPlain, kSumsOnly = kOrbitSumsOnly, kScaled = kOrbitScaled;

// Float32 orbit build.  Wave = base column over the item's rows in tiles of
// 32 x 32 pixels; lane (i, k) = (lane / 8, lane % 8) forms the 4 x 4 block
// at rows 4i.., columns 4k.. of a tile.  Each lane then holds four runs of
// four entries for every member (C0, C2 along rows; C1, C3 along the base
// column's image columns), so every store is 16 bytes and each store
// instruction fills eight whole 128-byte lines of one member (VEC: n % 4 ==
// 0, every 4 x 4 block is wholly inside or outside the image, runs 16-byte
// aligned; otherwise scalar stores).
template <bool VEC, int MODE>
__global__ __launch_bounds__(1024) void build_orbit_kernel(const float* __restrict__ cube, int K,
                                                           const ColGeom* __restrict__ geo,
                                                           const int32_t* __restrict__ reps,
                                                           const int4* __restrict__ items,
                                                           const int32_t* __restrict__ nitems,
                                                           int nb, int n, int ls, int N, int64_t M,
                                                           int rpr, int64_t nreps,
                                                           float* __restrict__ A,
                                                           double* __restrict__ part,
    const float* __restrict__ colscale) {
  extern __shared__ float2 P2[];
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, first = it.y, len = it.z, w0 = it.w;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ra = (int)blockIdx.y * rpr, rb = (ra + rpr < n) ? ra + rpr : n;
  if (!zero_bucket) stage_pair(P2, cube, bkt, K, n, ls, M, tid);
  __syncthreads();
  const int sp = w0 + wave;
  if (sp < first || sp >= first + len) return;  // uniform per wave; no barrier below
  const int64_t j0 = reps[sp];
  const bool centre = orbit_is_centre(j0, N);
  float* C0 = A + j0 * M;
  float* C1 = A + orbit_member(j0, N, 1) * M;
  float* C2 = A + orbit_member(j0, N, 2) * M;
  float* C3 = A + orbit_member(j0, N, 3) * M;
  if (zero_bucket) {  // identically zero orbit: rows [ra, rb) of every member
    for (int x = lane; MODE != kSumsOnly && x < (rb - ra) * n; x += 64) {
      const int64_t p = (int64_t)ra * n + x;
      __builtin_nontemporal_store(0.0f, C0 + p);
      if (!centre) {
        __builtin_nontemporal_store(0.0f, C1 + p);
        __builtin_nontemporal_store(0.0f, C2 + p);
        __builtin_nontemporal_store(0.0f, C3 + p);
      }
    }
    if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = 0.0;
    return;
  }
  const ColGeom g = geo[j0];
  const float sf = (MODE == kScaled) ? colscale[j0] : 1.0f;  // flux-preserving scale
  const double c = (double)(n - 1) * 0.5;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  const int li = lane >> 3, lk = lane & 7;
  double tsum = 0.0;
  for (int a0 = ra; a0 < rb; a0 += 32) {
    const int ab = a0 + 4 * li;
    if (ab >= rb) continue;  // VEC: the whole block is below the range
    for (int b0 = 0; b0 < n; b0 += 32) {
      const int bb = b0 + 4 * lk;
      if (bb >= n) continue;
      double ctux[4], mstux[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma clang fp contract(off)
        const double ux = (double)(bb + q) - c;
        ctux[q] = g.ct * ux;
        mstux[q] = (-g.st) * ux;
      }
      float x[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = ab + r;
        double stuy, ctuy;
        {
#pragma clang fp contract(off)
          const double uy = (double)a - c;
          stuy = g.st * uy;
          ctuy = g.ct * uy;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[r][q] = 0.0f;
          if (VEC || (a < rb && bb + q < n)) {
            x[r][q] = orbit_value(P2, ctux[q], mstux[q], stuy, ctuy, c, n, ls, wk0, wk1);
            if constexpr (MODE == kScaled) x[r][q] *= sf;
            tsum += (double)x[r][q];
          }
          if (q == 1) __builtin_amdgcn_sched_barrier(0);  // two elements in flight
        }
        if constexpr (VEC && MODE != kSumsOnly) {  // the row's runs of C0 and C2
          __builtin_nontemporal_store((f32x4){x[r][0], x[r][1], x[r][2], x[r][3]},
                                      reinterpret_cast<f32x4*>(C0 + (int64_t)a * n + bb));
          if (!centre)
            __builtin_nontemporal_store((f32x4){x[r][3], x[r][2], x[r][1], x[r][0]},
                                        reinterpret_cast<f32x4*>(C2 + (int64_t)(n - 1 - a) * n + (n - 4 - bb)));
        }
        // one row of the block at a time: bounds the live coordinate temporaries
        __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (MODE == kSumsOnly) {
      } else if constexpr (VEC) {
        if (!centre) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b = bb + q;
            __builtin_nontemporal_store((f32x4){x[3][q], x[2][q], x[1][q], x[0][q]},
                                        reinterpret_cast<f32x4*>(C1 + (int64_t)b * n + (n - 4 - ab)));
            __builtin_nontemporal_store((f32x4){x[0][q], x[1][q], x[2][q], x[3][q]},
                                        reinterpret_cast<f32x4*>(C3 + (int64_t)(n - 1 - b) * n + ab));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int a = ab + r, b = bb + q;
            if (a >= rb || b >= n) continue;
            __builtin_nontemporal_store(x[r][q], C0 + (int64_t)a * n + b);
            if (centre) continue;
            __builtin_nontemporal_store(x[r][q], C1 + (int64_t)b * n + (n - 1 - a));
            __builtin_nontemporal_store(x[r][q], C2 + (int64_t)(n - 1 - a) * n + (n - 1 - b));
            __builtin_nontemporal_store(x[r][q], C3 + (int64_t)(n - 1 - b) * n + a);
          }
      }
    }
  }
  tsum = wave_sum_f64(tsum);
  if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = tsum;
}

// Float32 orbit build for pairs larger than the LDS (n > 141).  The
// rotation map is affine, so a 32 x 32 tile of the base column draws its taps
// from a small box of the bordered pair: every float64 step of the source
// coordinates (the products with the cosine and sine, the two sums) is
// correctly rounded, hence monotone in the pixel's column for a fixed row and
// in its row for a fixed column, so the extreme source rows and columns over a
// tile are those of its four corners, exactly.  The box spans at most
// 31 (|cos| + |sin|) <= 43.85 source units, i.e. at most 45 tap origins and 46
// rows (columns) of the bordered array.  Each wave stages its tile's box in a
// private LDS region, already blended along the radius (the value
// (1-w) P_k + w P_{k+1} at each pixel, formed with the same float32 operations
// as the pair kernels' taps, so the entries are bitwise theirs), then forms the
// tile's 4 x 4 blocks and writes the four quarter turns as build_orbit_kernel
// does.  Sixteen waves per workgroup, 8.6 KiB of LDS each; no workgroup
// barrier (a wave orders its own LDS writes and reads).
constexpr int kFpSpan = 46;                     // box rows or columns, at most
constexpr int kFpRegion = kFpSpan * (kFpSpan + 1);  // floats per wave (odd row stride)
constexpr int kBoxMaxN = 8192;  // PSF side: pixel offsets n^2 and row-range sizes stay in int

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// floor of the source row and column of image pixel (a, b) (tap_coords' steps)
__device__ __forceinline__ void tap_origin(const ColGeom& g, double c, int a, int b, int& r0, int& c0) {
#pragma clang fp contract(off)
  const double ux = (double)b - c, uy = (double)a - c;
  const double ctux = g.ct * ux, mstux = (-g.st) * ux;
  const double stuy = g.st * uy, ctuy = g.ct * uy;
  const double colf = c + (ctux + stuy);
  const double rowf = c + (mstux + ctuy);
  c0 = (int)floor(colf);
  r0 = (int)floor(rowf);
}

// one element from the staged box (origin: bordered row Rlo, column Clo)
__device__ __forceinline__ float box_value(const float* __restrict__ Q, double ctux, double mstux,
                                           double stuy, double ctuy, double c, int n, int bs,
                                           int base) {
  const Tap t = tap_coords(ctux, mstux, stuy, ctuy, c, n, bs);
  const int i = t.ok ? t.idx - base : 0;
  const float q00 = Q[i], q01 = Q[i + 1];
  const float q10 = Q[i + bs], q11 = Q[i + bs + 1];
  float val = (t.gy * t.gx) * q00;
  val = fmaf(t.gy * t.fx, q01, val);
  val = fmaf(t.fy * t.gx, q10, val);
  val = fmaf(t.fy * t.fx, q11, val);
  return t.ok ? val : 0.0f;
}

// Stage rows [Rlo, Rlo + bh) x columns [Clo, Clo + bw) of a box into Q (row
// stride bs), each entry the radial blend (1-w) x + w y of its pair, formed as
// the pair kernels form their taps.  Bilinear: bordered indices of the
// sample pair Pk, Pk1 (zero border); cubic: padded indices of the coefficient
// pairs Pc (zero outside the Np x Np array).  The box is taken in row-major
// order 64 entries at a time, lane l taking entry l of each step, 8 steps'
// loads in flight before their LDS writes.
template <bool CUBIC>
__device__ __forceinline__ void stage_box(float* __restrict__ Q, const float* __restrict__ Pk,
                                          const float* __restrict__ Pk1,
                                          const float2* __restrict__ Pc, int n, int Np, int Rlo,
                                          int Clo, int bh, int bw, int bs, float wk0, float wk1,
                                          int lane) {
  if (bh <= 0 || bw <= 0) return;  // uniform
  const int q64 = 64 / bw, r64 = 64 - q64 * bw;
  int rr = lane / bw, cc = lane - rr * bw;
  while (__builtin_amdgcn_readfirstlane(rr) < bh) {  // lane 0 has the lowest entry
    float xv[8], yv[8];
    int dst[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int R = Rlo + rr, C = Clo + cc;
      const bool in = rr < bh;
      if constexpr (CUBIC) {
        const bool inner = in && (unsigned)R < (unsigned)Np && (unsigned)C < (unsigned)Np;
        const float2 p = inner ? Pc[R * Np + C] : make_float2(0.0f, 0.0f);
        xv[k] = p.x;
        yv[k] = p.y;
      } else {
        const bool inner = in && (unsigned)(R - 1) < (unsigned)n && (unsigned)(C - 1) < (unsigned)n;
        const int off = (R - 1) * n + (C - 1);
        xv[k] = inner ? Pk[off] : 0.0f;
        yv[k] = (inner && Pk1) ? Pk1[off] : 0.0f;
      }
      dst[k] = in ? rr * bs + cc : -1;
      cc += r64;
      rr += q64;
      if (cc >= bw) {
        cc -= bw;
        ++rr;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (dst[k] >= 0) Q[dst[k]] = fmaf(wk1, yv[k], wk0 * xv[k]);
  }
}

template <bool VEC, int MODE>
__global__ __launch_bounds__(1024) void build_orbit_box_kernel(const float* __restrict__ cube, int K,
                                                               const ColGeom* __restrict__ geo,
                                                               const int32_t* __restrict__ reps,
                                                               const int4* __restrict__ items,
                                                               const int32_t* __restrict__ nitems,
                                                               int nb, int n, int N, int64_t M,
                                                               int rpr, int64_t nreps,
                                                               float* __restrict__ A,
                                                               double* __restrict__ part,
    const float* __restrict__ colscale) {
  extern __shared__ float QS[];  // 16 regions of kFpRegion floats
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, first = it.y, len = it.z, w0 = it.w;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ra = (int)blockIdx.y * rpr, rb = (ra + rpr < n) ? ra + rpr : n;
  const int sp = w0 + wave;
  if (sp < first || sp >= first + len) return;  // uniform per wave; no workgroup barrier
  const int64_t j0 = reps[sp];
  const bool centre = orbit_is_centre(j0, N);
  float* C0 = A + j0 * M;
  float* C1 = A + orbit_member(j0, N, 1) * M;
  float* C2 = A + orbit_member(j0, N, 2) * M;
  float* C3 = A + orbit_member(j0, N, 3) * M;
  if (zero_bucket) {  // identically zero orbit: rows [ra, rb) of every member
    for (int x = lane; MODE != kSumsOnly && x < (rb - ra) * n; x += 64) {
      const int64_t p = (int64_t)ra * n + x;
      __builtin_nontemporal_store(0.0f, C0 + p);
      if (!centre) {
        __builtin_nontemporal_store(0.0f, C1 + p);
        __builtin_nontemporal_store(0.0f, C2 + p);
        __builtin_nontemporal_store(0.0f, C3 + p);
      }
    }
    if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = 0.0;
    return;
  }
  float* Q = QS + wave * kFpRegion;
  const float* Pk = cube + (int64_t)bkt * M;
  const float* Pk1 = (K > 1) ? Pk + M : nullptr;
  const ColGeom g = geo[j0];
  const float sf = (MODE == kScaled) ? colscale[j0] : 1.0f;  // flux-preserving scale
  const double c = (double)(n - 1) * 0.5;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  const int li = lane >> 3, lk = lane & 7;
  double tsum = 0.0;
  for (int a0 = ra; a0 < rb; a0 += 32) {
    const int ae = (a0 + 32 < rb) ? a0 + 32 : rb;
    const int ab = a0 + 4 * li;
    for (int b0 = 0; b0 < n; b0 += 32) {
      const int be = (b0 + 32 < n) ? b0 + 32 : n;
      // the tile's box of bordered rows [Rlo, Rlo + bh) and columns [Clo, Clo + bw)
      int rmin, rmax, cmin, cmax;
      {
        int r0, c0;
        tap_origin(g, c, a0, b0, r0, c0);
        rmin = rmax = r0;
        cmin = cmax = c0;
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          tap_origin(g, c, (k & 1) ? ae - 1 : a0, (k & 2) ? be - 1 : b0, r0, c0);
          rmin = min(rmin, r0);
          rmax = max(rmax, r0);
          cmin = min(cmin, c0);
          cmax = max(cmax, c0);
        }
      }
      const int Rlo = max(rmin + 1, 0), Clo = max(cmin + 1, 0);
      const int bh = min(max(min(rmax + 2, n + 1) - Rlo + 1, 0), kFpSpan);
      const int bw = min(max(min(cmax + 2, n + 1) - Clo + 1, 0), kFpSpan);
      const int bs = bw | 1;
      wave_lds_sync();  // the previous tile's reads are done
      stage_box<false>(Q, Pk, Pk1, nullptr, n, 0, Rlo, Clo, bh, bw, bs, wk0, wk1, lane);
      wave_lds_sync();  // the box is staged
      const int base = Rlo * bs + Clo;
      const int bb = b0 + 4 * lk;
      if (ab >= ae || bb >= be) continue;  // VEC: the whole block is outside the tile
      double ctux[4], mstux[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma clang fp contract(off)
        const double ux = (double)(bb + q) - c;
        ctux[q] = g.ct * ux;
        mstux[q] = (-g.st) * ux;
      }
      float x[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = ab + r;
        double stuy, ctuy;
        {
#pragma clang fp contract(off)
          const double uy = (double)a - c;
          stuy = g.st * uy;
          ctuy = g.ct * uy;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[r][q] = 0.0f;
          if (VEC || (a < ae && bb + q < be)) {
            x[r][q] = box_value(Q, ctux[q], mstux[q], stuy, ctuy, c, n, bs, base);
            if constexpr (MODE == kScaled) x[r][q] *= sf;
            tsum += (double)x[r][q];
          }
          if (q == 1) __builtin_amdgcn_sched_barrier(0);  // two elements in flight
        }
        if constexpr (VEC && MODE != kSumsOnly) {  // the row's runs of C0 and C2
          __builtin_nontemporal_store((f32x4){x[r][0], x[r][1], x[r][2], x[r][3]},
                                      reinterpret_cast<f32x4*>(C0 + (int64_t)a * n + bb));
          if (!centre)
            __builtin_nontemporal_store((f32x4){x[r][3], x[r][2], x[r][1], x[r][0]},
                                        reinterpret_cast<f32x4*>(C2 + (int64_t)(n - 1 - a) * n + (n - 4 - bb)));
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (MODE == kSumsOnly) {
      } else if constexpr (VEC) {
        if (!centre) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b = bb + q;
            __builtin_nontemporal_store((f32x4){x[3][q], x[2][q], x[1][q], x[0][q]},
                                        reinterpret_cast<f32x4*>(C1 + (int64_t)b * n + (n - 4 - ab)));
            __builtin_nontemporal_store((f32x4){x[0][q], x[1][q], x[2][q], x[3][q]},
                                        reinterpret_cast<f32x4*>(C3 + (int64_t)(n - 1 - b) * n + ab));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int a = ab + r, b = bb + q;
            if (a >= ae || b >= be) continue;
            __builtin_nontemporal_store(x[r][q], C0 + (int64_t)a * n + b);
            if (centre) continue;
            __builtin_nontemporal_store(x[r][q], C1 + (int64_t)b * n + (n - 1 - a));
            __builtin_nontemporal_store(x[r][q], C2 + (int64_t)(n - 1 - a) * n + (n - 1 - b));
            __builtin_nontemporal_store(x[r][q], C3 + (int64_t)(n - 1 - b) * n + a);
          }
      }
    }
  }
  tsum = wave_sum_f64(tsum);
  if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = tsum;
}

// 16-bit orbit build (N a multiple of 8: no centre, whole blocks of 8 bases).
// A window of 16 bases is two blocks; block h's member k is group
// 4 (w0/8 + h) + k, whose unit at an image pixel holds the 8 bases' member
// values there.  The item's rows are walked in tiles of 8 x 32 pixels: every
// wave forms its base column's tile (lane (i, k): row i, columns 4k..4k+3),
// rounds the values into an LDS tile [2][8][33][8] (unit-major: the 8 bases of
// a block and pixel are one 16-byte LDS word; one unit of padding per row
// keeps the column-wise reads conflict-free), and after one barrier half the
// threads copy the tile's units along rows to members 0 and 2 (runs of 32
// units in rows a and n-1-a) and half along columns to members 1 and 3 (runs
// of 8 units, one 128-byte line, in rows b and n-1-b).  The LDS tile is
// double-buffered, so that one barrier per tile suffices: a tile's buffer is
// written again two tiles later, after every thread has passed the barrier
// behind the copy that read it.  Slots of a block outside the item (the block
// straddles two brackets) are left to the other item: 2-byte stores.
template <bool BF16, bool SCALED>
__global__ __launch_bounds__(1024) void build_orbit16_kernel(const float* __restrict__ cube, int K,
                                                             const ColGeom* __restrict__ geo,
                                                             const int32_t* __restrict__ reps,
                                                             const int4* __restrict__ items,
                                                             const int32_t* __restrict__ nitems,
                                                             int nb, int n, int ls, int64_t M,
                                                             int rpr, int64_t nreps,
                                                             uint16_t* __restrict__ Mh,
                                                             double* __restrict__ part,
    const float* __restrict__ colscale) {
  constexpr int TA = 8, TB = 32, TP = TB + 1;
  constexpr int TILE = 2 * TA * TP * 8;  // uint16 per buffer
  extern __shared__ float2 P2[];  // bordered pair, then the two tile buffers
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, first = it.y, len = it.z, w0 = it.w;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ra = (int)blockIdx.y * rpr, rb = (ra + rpr < n) ? ra + rpr : n;
  uint16_t* tiles = reinterpret_cast<uint16_t*>(P2 + ((((size_t)(n + 2) * ls) + 1) & ~(size_t)1));
  if (!zero_bucket) stage_pair(P2, cube, bkt, K, n, ls, M, tid);
  const int sp = w0 + wave;
  const bool live = sp >= first && sp < first + len;  // uniform per wave
  const int h = wave >> 3, u = wave & 7;
  ColGeom g;
  g.ct = 1.0; g.st = 0.0; g.w = 0.0; g.e = 0;
  if (live) g = geo[reps[sp]];
  const float sf = (SCALED && live) ? colscale[reps[sp]] : 1.0f;  // flux-preserving scale
  const double c = (double)(n - 1) * 0.5;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  const int64_t G0 = (int64_t)(w0 / 8) * 4;
  int lo[2], hi[2];  // the item's slots of each block, relative to the block
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int s0 = w0 + 8 * q;
    lo[q] = (first > s0) ? first - s0 : 0;
    hi[q] = (first + len < s0 + 8) ? first + len - s0 : 8;
  }
  const int li = lane >> 3, lk = lane & 7;
  // copy roles: threads 0..511 along rows, 512..1023 along columns
  const bool along_cols = tid >= 512;
  const int cq = (tid & 511) >> 8, crem = tid & 255;
  double tsum = 0.0;
  __syncthreads();  // the pair is staged
  int buf = 0;
  for (int a0 = ra; a0 < rb; a0 += TA) {
    for (int b0 = 0; b0 < n; b0 += TB, buf ^= 1) {
      uint16_t* tile = tiles + buf * TILE;
      if (live) {
        const int a = a0 + li, bb = b0 + 4 * lk;
        if (a < rb) {
          double stuy, ctuy;
          {
#pragma clang fp contract(off)
            const double uy = (double)a - c;
            stuy = g.st * uy;
            ctuy = g.ct * uy;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (bb + q >= n) continue;
            double ctux, mstux;
            {
#pragma clang fp contract(off)
              const double ux = (double)(bb + q) - c;
              ctux = g.ct * ux;
              mstux = (-g.st) * ux;
            }
            float val = zero_bucket ? 0.0f
                                    : orbit_value(P2, ctux, mstux, stuy, ctuy, c, n, ls, wk0, wk1);
            if constexpr (SCALED) val *= sf;
            tsum += (double)val;
            const float xs = ldexpf(val, -g.e);  // exact power-of-two scaling
            uint32_t hv;
            if constexpr (BF16) {
              uint32_t w = __float_as_uint(xs);
              w += 0x7FFFu + ((w >> 16) & 1u);  // finite: round to nearest, ties to even
              hv = w >> 16;
            } else {
              hv = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)xs);
            }
            tile[((h * TA + li) * TP + 4 * lk + q) * 8 + u] = (uint16_t)hv;
          }
        }
      }
      __syncthreads();
      // one unit per thread: block cq, 8 rows x 32 columns
      if (lo[cq] < hi[cq]) {
        int r, cb;
        if (along_cols) {
          cb = crem >> 3;
          r = crem & 7;
        } else {
          r = crem >> 5;
          cb = crem & 31;
        }
        const int a = a0 + r, b = b0 + cb;
        if (a < rb && b < n) {
          const uint16_t* src = tile + ((cq * TA + r) * TP + cb) * 8;
          uint16_t* dA;
          uint16_t* dB;
          if (along_cols) {
            dA = Mh + ((G0 + 4 * cq + 1) * M + (int64_t)b * n + (n - 1 - a)) * 8;
            dB = Mh + ((G0 + 4 * cq + 3) * M + (int64_t)(n - 1 - b) * n + a) * 8;
          } else {
            dA = Mh + ((G0 + 4 * cq + 0) * M + (int64_t)a * n + b) * 8;
            dB = Mh + ((G0 + 4 * cq + 2) * M + (int64_t)(n - 1 - a) * n + (n - 1 - b)) * 8;
          }
          if (lo[cq] == 0 && hi[cq] == 8) {
            const u32x4 w = *reinterpret_cast<const u32x4*>(src);
            __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(dA));
            __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(dB));
          } else {
            for (int s = lo[cq]; s < hi[cq]; ++s) {
              dA[s] = src[s];
              dB[s] = src[s];
            }
          }
        }
      }
    }
  }
  if (!live) return;
  tsum = wave_sum_f64(tsum);
  if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = tsum;
}

// Cubic-spline orbit build: the quarter-turn orbits of the bilinear builds
// (the four members of an orbit sample the spline at the same source points,
// so one base column is computed and four are written), each 32 x 32 pixel
// tile reading its 4 x 4 B-spline taps from a box of the padded coefficient
// pair that the wave stages in its own LDS region.  A pixel's tap origin is
// clamped to padded indices [-3, Np+1] (where that moves it, all its taps lay
// outside the padded array and read zeros, as before the clamp); the clamp and
// the floors are monotone, so the tile's extreme origins are those of its
// corners and the box spans at most 44 + 4 = 48 rows and columns.  The box
// holds the radial blend (1-w) C_k + w C_{k+1} (zero outside the array), and a
// pixel is the 4 x 4 weighted sum of the blend, row by row, in the order of
// the gather form, so both give identical values.
constexpr int kCbSpan = 48;                        // box rows or columns, at most
constexpr int kCbRegion = kCbSpan * (kCbSpan + 1);  // floats per wave (odd row stride)

__device__ __forceinline__ int clamp_origin(int v, int Np) { return v < -3 ? -3 : (v > Np + 1 ? Np + 1 : v); }

// clamped tap origin (padded row and column) of image pixel (a, b)
__device__ __forceinline__ void cubic_origin(const ColGeom& g, double c, int a, int b, int Np,
                                             int& r0, int& c0) {
#pragma clang fp contract(off)
  const double ux = (double)b - c, uy = (double)a - c;
  const double pad = (double)kSplinePad;
  const double rowf = c + ((-g.st) * ux + g.ct * uy) + pad;
  const double colf = c + (g.ct * ux + g.st * uy) + pad;
  r0 = clamp_origin((int)floor(rowf), Np);
  c0 = clamp_origin((int)floor(colf), Np);
}

template <bool VEC, int MODE>
__global__ __launch_bounds__(1024) void build_cubic_orbit_kernel(const float2* __restrict__ pairs,
                                                                 int Np,
                                                                 const ColGeom* __restrict__ geo,
                                                                 const int32_t* __restrict__ reps,
                                                                 const int4* __restrict__ items,
                                                                 const int32_t* __restrict__ nitems,
                                                                 int nb, int n, int N, int64_t M,
                                                                 int rpr, int64_t nreps,
                                                                 float* __restrict__ A,
                                                                 double* __restrict__ part,
    const float* __restrict__ colscale) {
  extern __shared__ float QS[];  // 16 regions of kCbRegion floats
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, first = it.y, len = it.z, w0 = it.w;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ra = (int)blockIdx.y * rpr, rb = (ra + rpr < n) ? ra + rpr : n;
  const int sp = w0 + wave;
  if (sp < first || sp >= first + len) return;  // uniform per wave; no workgroup barrier
  const int64_t j0 = reps[sp];
  const bool centre = orbit_is_centre(j0, N);
  float* C0 = A + j0 * M;
  float* C1 = A + orbit_member(j0, N, 1) * M;
  float* C2 = A + orbit_member(j0, N, 2) * M;
  float* C3 = A + orbit_member(j0, N, 3) * M;
  if (zero_bucket) {  // identically zero orbit: rows [ra, rb) of every member
    for (int x = lane; MODE != kSumsOnly && x < (rb - ra) * n; x += 64) {
      const int64_t p = (int64_t)ra * n + x;
      __builtin_nontemporal_store(0.0f, C0 + p);
      if (!centre) {
        __builtin_nontemporal_store(0.0f, C1 + p);
        __builtin_nontemporal_store(0.0f, C2 + p);
        __builtin_nontemporal_store(0.0f, C3 + p);
      }
    }
    if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = 0.0;
    return;
  }
  float* Q = QS + wave * kCbRegion;
  const float2* src = pairs + (int64_t)bkt * Np * Np;
  const ColGeom g = geo[j0];
  const float sf = (MODE == kScaled) ? colscale[j0] : 1.0f;  // flux-preserving scale
  const double c = (double)(n - 1) * 0.5;
  const double pad = (double)kSplinePad;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  const int li = lane >> 3, lk = lane & 7;
  double tsum = 0.0;
  for (int a0 = ra; a0 < rb; a0 += 32) {
    const int ae = (a0 + 32 < rb) ? a0 + 32 : rb;
    const int ab = a0 + 4 * li;
    for (int b0 = 0; b0 < n; b0 += 32) {
      const int be = (b0 + 32 < n) ? b0 + 32 : n;
      // the tile's box of padded rows [Rlo, Rlo + bh) and columns [Clo, Clo + bw)
      int rmin, rmax, cmin, cmax;
      {
        int r0, c0;
        cubic_origin(g, c, a0, b0, Np, r0, c0);
        rmin = rmax = r0;
        cmin = cmax = c0;
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          cubic_origin(g, c, (k & 1) ? ae - 1 : a0, (k & 2) ? be - 1 : b0, Np, r0, c0);
          rmin = min(rmin, r0);
          rmax = max(rmax, r0);
          cmin = min(cmin, c0);
          cmax = max(cmax, c0);
        }
      }
      const int Rlo = rmin - 1, Clo = cmin - 1;
      const int bh = min(rmax - rmin + 4, kCbSpan), bw = min(cmax - cmin + 4, kCbSpan);
      const int bs = bw | 1;
      wave_lds_sync();  // the previous tile's reads are done
      stage_box<true>(Q, nullptr, nullptr, src, n, Np, Rlo, Clo, bh, bw, bs, wk0, wk1, lane);
      wave_lds_sync();  // the box is staged
      const int bb = b0 + 4 * lk;
      if (ab >= ae || bb >= be) continue;  // VEC: the whole block is outside the tile
      double ctux[4], mstux[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma clang fp contract(off)
        const double ux = (double)(bb + q) - c;
        ctux[q] = g.ct * ux;
        mstux[q] = (-g.st) * ux;
      }
      float x[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = ab + r;
        double stuy, ctuy;
        {
#pragma clang fp contract(off)
          const double uy = (double)a - c;
          stuy = g.st * uy;
          ctuy = g.ct * uy;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[r][q] = 0.0f;
          if (VEC || (a < ae && bb + q < be)) {
#pragma clang fp contract(off)
            const double rowf = c + (mstux[q] + ctuy) + pad;
            const double colf = c + (ctux[q] + stuy) + pad;
            const double r0f = floor(rowf), c0f = floor(colf);
            const int r0 = clamp_origin((int)r0f, Np), c0 = clamp_origin((int)c0f, Np);
            float wy[4], wx[4];
            cubic_weights(rowf - r0f, wy);
            cubic_weights(colf - c0f, wx);
            const float* t = Q + (r0 - 1 - Rlo) * bs + (c0 - 1 - Clo);
            float V = 0.0f;
#pragma unroll
            for (int dr = 0; dr < 4; ++dr) {
              const float* tr = t + dr * bs;
              float v = wx[0] * tr[0];
              v = fmaf(wx[1], tr[1], v);
              v = fmaf(wx[2], tr[2], v);
              v = fmaf(wx[3], tr[3], v);
              V = fmaf(wy[dr], v, V);
            }
            if constexpr (MODE == kScaled) V *= sf;
            x[r][q] = V;
            tsum += (double)V;
          }
        }
        if constexpr (VEC && MODE != kSumsOnly) {  // the row's runs of C0 and C2
          __builtin_nontemporal_store((f32x4){x[r][0], x[r][1], x[r][2], x[r][3]},
                                      reinterpret_cast<f32x4*>(C0 + (int64_t)a * n + bb));
          if (!centre)
            __builtin_nontemporal_store((f32x4){x[r][3], x[r][2], x[r][1], x[r][0]},
                                        reinterpret_cast<f32x4*>(C2 + (int64_t)(n - 1 - a) * n + (n - 4 - bb)));
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (MODE == kSumsOnly) {
      } else if constexpr (VEC) {
        if (!centre) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b = bb + q;
            __builtin_nontemporal_store((f32x4){x[3][q], x[2][q], x[1][q], x[0][q]},
                                        reinterpret_cast<f32x4*>(C1 + (int64_t)b * n + (n - 4 - ab)));
            __builtin_nontemporal_store((f32x4){x[0][q], x[1][q], x[2][q], x[3][q]},
                                        reinterpret_cast<f32x4*>(C3 + (int64_t)(n - 1 - b) * n + ab));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int a = ab + r, b = bb + q;
            if (a >= ae || b >= be) continue;
            __builtin_nontemporal_store(x[r][q], C0 + (int64_t)a * n + b);
            if (centre) continue;
            __builtin_nontemporal_store(x[r][q], C1 + (int64_t)b * n + (n - 1 - a));
            __builtin_nontemporal_store(x[r][q], C2 + (int64_t)(n - 1 - a) * n + (n - 1 - b));
            __builtin_nontemporal_store(x[r][q], C3 + (int64_t)(n - 1 - b) * n + a);
          }
      }
    }
  }
  tsum = wave_sum_f64(tsum);
  if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = tsum;
}

// 16-bit orbit build for pairs larger than the LDS (n > 141, N a multiple of
// 8), bilinear or cubic-spline: build_orbit16_kernel's unit tiles and copies,
// with each wave's taps read from a staged box (as build_orbit_box_kernel and
// build_cubic_orbit_kernel) of the 32 x 32 pixels it forms as 32 / TA tiles of
// TA x 32.  LDS: 16 box regions, then the two unit tiles; the cubic boxes are
// larger (48 x 49 floats), so the cubic form takes 4-row tiles (each lane two
// pixels of a tile row) where the bilinear form takes 8-row ones (four).
template <bool BF16, bool CUBIC, bool SCALED>
__global__ __launch_bounds__(1024) void build_orbit16_box_kernel(const float* __restrict__ src0, int K,
                                                                 const ColGeom* __restrict__ geo,
                                                                 const int32_t* __restrict__ reps,
                                                                 const int4* __restrict__ items,
                                                                 const int32_t* __restrict__ nitems,
                                                                 int nb, int n, int64_t M, int Np,
                                                                 int rpr, int64_t nreps,
                                                                 uint16_t* __restrict__ Mh,
                                                                 double* __restrict__ part,
    const float* __restrict__ colscale) {
  constexpr int TA = CUBIC ? 4 : 8, TB = 32, TP = TB + 1;
  constexpr int CPL = (TA * TB) / 64;      // pixels of a tile row per lane
  constexpr int LPR = TB / CPL;            // lanes per tile row
  constexpr int TILE = 2 * TA * TP * 8;    // uint16 per buffer
  constexpr int REGION = CUBIC ? kCbRegion : kFpRegion;
  extern __shared__ float QS[];
  if ((int)blockIdx.x >= *nitems) return;  // uniform: surplus workgroups of the upper bound
  const int4 it = items[blockIdx.x];
  const int bkt = it.x, first = it.y, len = it.z, w0 = it.w;
  const bool zero_bucket = bkt == nb - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ra = (int)blockIdx.y * rpr, rb = (ra + rpr < n) ? ra + rpr : n;
  uint16_t* tiles = reinterpret_cast<uint16_t*>(QS + 16 * REGION);
  float* Q = QS + wave * REGION;
  const int sp = w0 + wave;
  const bool live = sp >= first && sp < first + len;  // uniform per wave
  const int h = wave >> 3, u = wave & 7;
  ColGeom g;
  g.ct = 1.0; g.st = 0.0; g.w = 0.0; g.e = 0;
  if (live) g = geo[reps[sp]];
  const float sf = (SCALED && live) ? colscale[reps[sp]] : 1.0f;  // flux-preserving scale
  const double c = (double)(n - 1) * 0.5;
  const double pad = (double)kSplinePad;
  const float wk0 = (float)(1.0 - g.w), wk1 = (float)g.w;
  const int pb = zero_bucket ? 0 : bkt;
  const float* Pk = CUBIC ? src0 : src0 + (int64_t)pb * M;  // bilinear: the sample pair
  const float* Pk1 = (!CUBIC && K > 1) ? Pk + M : nullptr;
  const float2* Pc = reinterpret_cast<const float2*>(src0) + (CUBIC ? (int64_t)pb * Np * Np : 0);  // cubic
  const int64_t G0 = (int64_t)(w0 / 8) * 4;
  int lo[2], hi[2];  // the item's slots of each block, relative to the block
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int s0 = w0 + 8 * q;
    lo[q] = (first > s0) ? first - s0 : 0;
    hi[q] = (first + len < s0 + 8) ? first + len - s0 : 8;
  }
  const int li = lane / LPR, lk = lane % LPR;
  // copy roles: threads 0..511 along rows, 512..1023 along columns; unit cu of
  // a direction is block cu / (TA TB), row and column from cu % (TA TB)
  const bool along_cols = tid >= 512;
  const int cu = tid & 511, cq = cu / (TA * TB), crem = cu % (TA * TB);
  double tsum = 0.0;
  int buf = 0;
  for (int a0 = ra; a0 < rb; a0 += 32) {
    const int ae = (a0 + 32 < rb) ? a0 + 32 : rb;
    for (int b0 = 0; b0 < n; b0 += TB) {
      const int be = (b0 + TB < n) ? b0 + TB : n;
      int bs = 1, base = 0, Rlo = 0, Clo = 0;
      if (live && !zero_bucket) {  // uniform per wave: stage the box of rows [a0, ae), columns [b0, be)
        int rmin, rmax, cmin, cmax;
        {
          int r0, c0;
          if constexpr (CUBIC) cubic_origin(g, c, a0, b0, Np, r0, c0);
          else tap_origin(g, c, a0, b0, r0, c0);
          rmin = rmax = r0;
          cmin = cmax = c0;
#pragma unroll
          for (int k = 1; k < 4; ++k) {
            if constexpr (CUBIC)
              cubic_origin(g, c, (k & 1) ? ae - 1 : a0, (k & 2) ? be - 1 : b0, Np, r0, c0);
            else
              tap_origin(g, c, (k & 1) ? ae - 1 : a0, (k & 2) ? be - 1 : b0, r0, c0);
            rmin = min(rmin, r0);
            rmax = max(rmax, r0);
            cmin = min(cmin, c0);
            cmax = max(cmax, c0);
          }
        }
        int bh, bw;
        if constexpr (CUBIC) {
          Rlo = rmin - 1;
          Clo = cmin - 1;
          bh = min(rmax - rmin + 4, kCbSpan);
          bw = min(cmax - cmin + 4, kCbSpan);
        } else {
          Rlo = max(rmin + 1, 0);
          Clo = max(cmin + 1, 0);
          bh = min(max(min(rmax + 2, n + 1) - Rlo + 1, 0), kFpSpan);
          bw = min(max(min(cmax + 2, n + 1) - Clo + 1, 0), kFpSpan);
        }
        bs = bw | 1;
        base = Rlo * bs + Clo;
        stage_box<CUBIC>(Q, Pk, Pk1, Pc, n, Np, Rlo, Clo, bh, bw, bs, wk0, wk1, lane);
        wave_lds_sync();  // the box is staged
      }
      for (int a1 = a0; a1 < ae; a1 += TA, buf ^= 1) {  // uniform over the workgroup
        uint16_t* tile = tiles + buf * TILE;
        if (live) {
          const int a = a1 + li, bb = b0 + CPL * lk;
          if (a < ae) {
            double stuy, ctuy;
            {
#pragma clang fp contract(off)
              const double uy = (double)a - c;
              stuy = g.st * uy;
              ctuy = g.ct * uy;
            }
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
              if (bb + q >= n) continue;
              double ctux, mstux;
              {
#pragma clang fp contract(off)
                const double ux = (double)(bb + q) - c;
                ctux = g.ct * ux;
                mstux = (-g.st) * ux;
              }
              float val = 0.0f;
              if (!zero_bucket) {
                if constexpr (CUBIC) {
#pragma clang fp contract(off)
                  const double rowf = c + (mstux + ctuy) + pad;
                  const double colf = c + (ctux + stuy) + pad;
                  const double r0f = floor(rowf), c0f = floor(colf);
                  const int r0 = clamp_origin((int)r0f, Np), c0 = clamp_origin((int)c0f, Np);
                  float wy[4], wx[4];
                  cubic_weights(rowf - r0f, wy);
                  cubic_weights(colf - c0f, wx);
                  const float* t = Q + (r0 - 1 - Rlo) * bs + (c0 - 1 - Clo);
#pragma unroll
                  for (int dr = 0; dr < 4; ++dr) {
                    const float* tr = t + dr * bs;
                    float v = wx[0] * tr[0];
                    v = fmaf(wx[1], tr[1], v);
                    v = fmaf(wx[2], tr[2], v);
                    v = fmaf(wx[3], tr[3], v);
                    val = fmaf(wy[dr], v, val);
                  }
                } else {
                  val = box_value(Q, ctux, mstux, stuy, ctuy, c, n, bs, base);
                }
              }
              if constexpr (SCALED) val *= sf;
              tsum += (double)val;
              const float xs = ldexpf(val, -g.e);  // exact power-of-two scaling
              uint32_t hv;
              if constexpr (BF16) {
                uint32_t w = __float_as_uint(xs);
                w += 0x7FFFu + ((w >> 16) & 1u);  // finite: round to nearest, ties to even
                hv = w >> 16;
              } else {
                hv = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)xs);
              }
              tile[((h * TA + li) * TP + CPL * lk + q) * 8 + u] = (uint16_t)hv;
            }
          }
        }
        __syncthreads();
        // one unit per thread: block cq, TA rows x 32 columns
        if (cq < 2 && lo[cq] < hi[cq]) {
          int r, cb;
          if (along_cols) {
            cb = crem / TA;
            r = crem % TA;
          } else {
            r = crem >> 5;
            cb = crem & 31;
          }
          const int a = a1 + r, b = b0 + cb;
          if (a < ae && b < n) {
            const uint16_t* src = tile + ((cq * TA + r) * TP + cb) * 8;
            uint16_t* dA;
            uint16_t* dB;
            if (along_cols) {
              dA = Mh + ((G0 + 4 * cq + 1) * M + (int64_t)b * n + (n - 1 - a)) * 8;
              dB = Mh + ((G0 + 4 * cq + 3) * M + (int64_t)(n - 1 - b) * n + a) * 8;
            } else {
              dA = Mh + ((G0 + 4 * cq + 0) * M + (int64_t)a * n + b) * 8;
              dB = Mh + ((G0 + 4 * cq + 2) * M + (int64_t)(n - 1 - a) * n + (n - 1 - b)) * 8;
            }
            if (lo[cq] == 0 && hi[cq] == 8) {
              const u32x4 w = *reinterpret_cast<const u32x4*>(src);
              __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(dA));
              __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(dB));
            } else {
              for (int s = lo[cq]; s < hi[cq]; ++s) {
                dA[s] = src[s];
                dB[s] = src[s];
              }
            }
          }
        }
      }
    }
  }
  if (!live) return;
  tsum = wave_sum_f64(tsum);
  if (lane == 0) part[(int64_t)blockIdx.y * nreps + sp] = tsum;
}

// ------------------------------------------------------------- launch -----
static int lds_e(int n) { return (n + 63) / 64; }

// LDS row stride (in pairs) of the bordered array: n+2 rounded up to 5 mod 8
// when that still fits.  The taps of a wave follow a rotated line through the
// array; with an even stride, near-vertical lines put lanes two rows apart on
// the same banks, an odd stride spreads them (about 13% fewer LDS cycles over
// random angles at n = 128 in a bank model).
static int lds_stride(int n) {
  const int np = n + 2, ls = np + ((5 - np % 8) + 8) % 8;
  return (size_t)np * ls * sizeof(float2) <= (size_t)kLdsBuildMaxBytes ? ls : np;
}

static bool pair_fits_lds(int n) {
  return (size_t)(n + 2) * (n + 2) * sizeof(float2) <= (size_t)kLdsBuildMaxBytes;
}

static bool orbit_sort_fits(int K, int N);

bool build_lds_supported(int n, int K, int N) {
  // the bordered pair fits the LDS whole, or (up to kBoxMaxN) the orbit
  // builds stage a box of it per tile; the bucket histograms (8 B per bucket)
  // must fit the sort kernels' LDS
  if (K > 8192) return false;
  return pair_fits_lds(n) || (n <= kBoxMaxN && orbit_sort_fits(K, N));
}

static int nbuckets(int K) { return ((K > 1) ? K - 1 : 1) + 1; }

size_t bucket_scratch_bytes(int K, int64_t ncols) {
  const int64_t nb = nbuckets(K);
  const int64_t items_max = (ncols + kLdsCols - 1) / kLdsCols + nb;
  size_t b = 0;
  b += ((size_t)nb * 4 * 3 + 255) & ~(size_t)255;           // cnt, cursor, bstart
  b += ((size_t)items_max * 16 + 16 + 255) & ~(size_t)255;  // items + nitems
  b += ((size_t)ncols * 4 + 255) & ~(size_t)255;            // order
  return b;
}



hipError_t launch_bucket_sort(const ColGeom* geo, int64_t ncols, int K, void* scratch,
                              BucketPlan* plan, hipStream_t s) {
  const int nb = nbuckets(K);
  const int64_t items_max = (ncols + kLdsCols - 1) / kLdsCols + nb;
  char* p = reinterpret_cast<char*>(scratch);
  int32_t* cnt = reinterpret_cast<int32_t*>(p);
  int32_t* cursor = cnt + nb;
  int32_t* bstart = cursor + nb;
  p += ((size_t)nb * 4 * 3 + 255) & ~(size_t)255;
  int4* items = reinterpret_cast<int4*>(p);
  int32_t* nitems = reinterpret_cast<int32_t*>(items + items_max);
  p += ((size_t)items_max * 16 + 16 + 255) & ~(size_t)255;
  int32_t* order = reinterpret_cast<int32_t*>(p);
  // cnt and cursor start at zero (a fill kernel, not hipMemsetAsync, so a
  // captured build replays correctly)
  zero_ints_kernel<<<(unsigned)((2 * nb + 255) / 256), 256, 0, s>>>(cnt, 2 * nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned cgrid = (unsigned)((ncols + 255) / 256);
  bucket_count_kernel<<<cgrid, 256, (size_t)nb * 4, s>>>(geo, ncols, nb, cnt);
  bucket_scan_kernel<<<1, 1024, 0, s>>>(cnt, nb, bstart, items, nitems);
  bucket_scatter_kernel<<<cgrid, 256, (size_t)nb * 8, s>>>(geo, ncols, nb, bstart, cursor, order);
  plan->order = order;
  plan->items = items;
  plan->nitems = nitems;
  plan->items_max = items_max;
  plan->nb = nb;
  return hipGetLastError();
}

hipError_t launch_pack16(int storage, const float* A32, const ColGeom* geo, int64_t M,
                         int64_t ncols, int64_t ncols_pad, void* lib, hipStream_t s) {
  return launch_pack16_range(storage, A32, 0, 0, ncols_pad / 8, geo, M, ncols, lib, s);
}

hipError_t launch_pack16_range(int storage, const float* A32, int64_t col0, int64_t g0, int64_t g1,
                               const ColGeom* geo, int64_t M, int64_t ncols, void* lib,
                               hipStream_t s) {
  if (g1 <= g0) return hipSuccess;
  const dim3 pgrid((unsigned)((M + 511) / 512), (unsigned)(g1 - g0));
  u32x4* Mp = reinterpret_cast<u32x4*>(lib);
  if (storage == PSFLIB_BF16_POW2)
    pack16_kernel<true><<<pgrid, 256, 0, s>>>(A32, geo, M, ncols, Mp, g0, col0);
  else
    pack16_kernel<false><<<pgrid, 256, 0, s>>>(A32, geo, M, ncols, Mp, g0, col0);
  return hipGetLastError();
}

// rows of the 16-bit tile that fit next to the bordered pair (0: none)
static int lds16_rows(int n) {
  const size_t pair = (size_t)(n + 2) * lds_stride(n) * sizeof(float2);
  for (int R = 4; R >= 1; R >>= 1)
    if (pair + (size_t)16 * R * n * 2 <= (size_t)kLdsBuildMaxBytes) return R;
  return 0;
}

bool build_lds16_supported(int n, int K, int64_t ncols) {
  if (K > kLdsMaxBuckets - 1 || n > 141 || lds16_rows(n) == 0) return false;
  const int64_t nblk = (ncols + kSortBlock - 1) / kSortBlock;
  return nblk * nbuckets(K) <= ((int64_t)1 << 24) && ncols < ((int64_t)1 << 31);
}

size_t build_lds16_scratch_bytes(int K, int64_t ncols) {
  const int64_t nb = nbuckets(K);
  const int64_t nblk = (ncols + kSortBlock - 1) / kSortBlock;
  const int64_t items_max = (ncols + 15) / 16 + 2 * nb + 1;
  return (((size_t)nblk * nb * 4 + 255) & ~(size_t)255) + (((size_t)items_max * 16 + 16 + 255) & ~(size_t)255);
}

hipError_t launch_build_lds16(int storage, const float* cube, int K, const ColGeom* geo, int n,
                              int64_t M, int64_t ncols, int64_t ncols_pad, const int32_t* exps,
                              int32_t* perm, int32_t* eslot, int32_t* slot_of, void* lib,
                              double* tau, void* scratch, hipStream_t s) {
  const int nb = nbuckets(K);
  const int64_t nblk = (ncols + kSortBlock - 1) / kSortBlock;
  const int64_t items_max = (ncols + 15) / 16 + 2 * nb + 1;
  char* p = reinterpret_cast<char*>(scratch);
  int32_t* cnt = reinterpret_cast<int32_t*>(p);
  p += ((size_t)nblk * nb * 4 + 255) & ~(size_t)255;
  int4* items = reinterpret_cast<int4*>(p);
  int32_t* nitems = reinterpret_cast<int32_t*>(items + items_max);
  // padding slots (and defaults) first; the sort then places every column
  hipError_t e = launch_identity_order(perm, eslot, slot_of, exps, ncols, ncols_pad, s);
  if (e != hipSuccess) return e;
  sort_count_kernel<<<(unsigned)nblk, kSortBlock, (size_t)nb * 4, s>>>(geo, ncols, nb, cnt);
  sort_scan_kernel<<<1, 1024, 0, s>>>(cnt, nblk, nb, items, nitems);
  sort_scatter_kernel<<<(unsigned)nblk, kSortBlock, (size_t)nb * 4, s>>>(geo, ncols, nb, cnt, perm,
                                                                         slot_of, eslot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ls = lds_stride(n), R = lds16_rows(n);
  const size_t lds = (size_t)(n + 2) * ls * sizeof(float2) + (size_t)16 * R * n * 2;
  const bool full = (n % 64) == 0;
  const bool bf = storage == PSFLIB_BF16_POW2;
  uint16_t* Mh = reinterpret_cast<uint16_t*>(lib);
  auto launch = [&](auto kern) -> hipError_t {
    const void* fn = reinterpret_cast<const void*>(kern);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<(unsigned)items_max, 1024, lds, s>>>(cube, K, geo, perm, items, nitems, nb, n, ls, R, M,
                                                Mh, tau);
    return hipGetLastError();
  };
  switch (lds_e(n)) {
    case 1:
      e = full ? (bf ? launch(build_lds16_kernel<1, true, true>) : launch(build_lds16_kernel<1, true, false>))
               : (bf ? launch(build_lds16_kernel<1, false, true>) : launch(build_lds16_kernel<1, false, false>));
      break;
    case 2:
      e = full ? (bf ? launch(build_lds16_kernel<2, true, true>) : launch(build_lds16_kernel<2, true, false>))
               : (bf ? launch(build_lds16_kernel<2, false, true>) : launch(build_lds16_kernel<2, false, false>));
      break;
    default:
      e = bf ? launch(build_lds16_kernel<3, false, true>) : launch(build_lds16_kernel<3, false, false>);
      break;
  }
  if (e != hipSuccess) return e;
  if (ncols_pad > ncols) {
    const int64_t g0 = ncols / 8;
    zero_pad16_kernel<<<dim3((unsigned)((M + 255) / 256), (unsigned)(ncols_pad / 8 - g0)), 256, 0, s>>>(
        Mh, M, ncols, g0);
    e = hipGetLastError();
  }
  return e;
}

static bool build_orbit_supported(int n, int K, int N);
static hipError_t launch_build_orbit(const float* cube, int K, const ColGeom* geo, int n, int N,
                                     int64_t M, float* A32, double* tau, void* scratch, int mode,
                                     const float* colscale, hipStream_t s);

hipError_t launch_build_lds(const float* cube, int K, const ColGeom* geo, int n, int N, int64_t M,
                            float* A32, double* tau, void* scratch, hipStream_t s) {
  if (build_orbit_supported(n, K, N))
    return launch_build_orbit(cube, K, geo, n, N, M, A32, tau, scratch, kPlain, nullptr, s);
  if (!pair_fits_lds(n)) return hipErrorInvalidValue;  // larger pairs: the orbit builds only
  const int64_t ncols = (int64_t)N * N;
  BucketPlan bp;
  hipError_t e = launch_bucket_sort(geo, ncols, K, scratch, &bp, s);
  if (e != hipSuccess) return e;
  const int32_t* order = bp.order;
  const int4* items = bp.items;
  const int32_t* nitems = bp.nitems;
  const int nb = bp.nb;
  const int64_t items_max = bp.items_max;

  const unsigned grid = (unsigned)items_max;
  const bool full = (n % 64) == 0;
  const int ls = lds_stride(n);
  const size_t lds = (size_t)(n + 2) * ls * sizeof(float2);
  const void* fn;
  auto launch = [&](auto kern) -> hipError_t {
    fn = reinterpret_cast<const void*>(kern);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<grid, 1024, lds, s>>>(cube, K, geo, order, items, nitems, nb, n, ls, M, A32, tau);
    return hipSuccess;
  };
  switch (lds_e(n)) {
    case 1: e = full ? launch(build_lds_kernel<1, true>) : launch(build_lds_kernel<1, false>); break;
    case 2: e = full ? launch(build_lds_kernel<2, true>) : launch(build_lds_kernel<2, false>); break;
    default: e = launch(build_lds_kernel<3, false>); break;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ------------------------------------------------- orbit launches -----
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct OrbitPlan {
  OrbitGrid o;
  int nb, rpr, nranges;
  int64_t nblk, items_max;
  int32_t* cnt;
  int4* items;
  int32_t* nitems;
  int32_t* reps;
  double* part;
};

static OrbitPlan orbit_plan(int K, int N, int n, void* scratch) {
  OrbitPlan pl;
  pl.o = orbit_grid(N);
  pl.nb = nbuckets(K);
  pl.rpr = orbit_rows_per_range(n);
  pl.nranges = (n + pl.rpr - 1) / pl.rpr;
  pl.nblk = (pl.o.nreps + kSortBlock - 1) / kSortBlock;
  pl.items_max = (pl.o.nreps + 15) / 16 + 2 * (int64_t)pl.nb + 1;
  char* p = reinterpret_cast<char*>(scratch);
  pl.cnt = reinterpret_cast<int32_t*>(p);
  p += al256((size_t)pl.nblk * pl.nb * 4);
  pl.items = reinterpret_cast<int4*>(p);
  pl.nitems = reinterpret_cast<int32_t*>(pl.items + pl.items_max);
  p += al256((size_t)pl.items_max * 16 + 16);
  pl.reps = reinterpret_cast<int32_t*>(p);
  p += al256((size_t)pl.o.nreps * 4);
  pl.part = reinterpret_cast<double*>(p);
  return pl;
}

size_t build_orbit_scratch_bytes(int K, int N, int n) {
  const OrbitPlan pl = orbit_plan(K, N, n, nullptr);
  return al256((size_t)pl.nblk * pl.nb * 4) + al256((size_t)pl.items_max * 16 + 16) +
         al256((size_t)pl.o.nreps * 4) + al256((size_t)pl.nranges * pl.o.nreps * 8);
}

static bool orbit_sort_fits(int K, int N) {
  const OrbitGrid o = orbit_grid(N);
  const int64_t nblk = (o.nreps + kSortBlock - 1) / kSortBlock;
  return K <= kLdsMaxBuckets - 1 && nblk * nbuckets(K) <= ((int64_t)1 << 24) &&
         (int64_t)N * N < ((int64_t)1 << 31);
}

// counting sort of the base columns by bracket, and the work items
static hipError_t orbit_sort(const ColGeom* geo, const OrbitPlan& pl, int32_t* perm,
                             int32_t* slot_of, int32_t* eslot, hipStream_t s) {
  orbit_count_kernel<<<(unsigned)pl.nblk, kSortBlock, (size_t)pl.nb * 4, s>>>(geo, pl.o, pl.nb, pl.cnt);
  sort_scan_kernel<<<1, 1024, 0, s>>>(pl.cnt, pl.nblk, pl.nb, pl.items, pl.nitems);
  orbit_scatter_kernel<<<(unsigned)pl.nblk, kSortBlock, (size_t)pl.nb * 4, s>>>(
      geo, pl.o, pl.nb, pl.cnt, pl.reps, perm, slot_of, eslot);
  return hipGetLastError();
}

static hipError_t orbit_finish(const OrbitPlan& pl, double* tau, hipStream_t s) {
  orbit_tau_kernel<<<(unsigned)((pl.o.nreps + 255) / 256), 256, 0, s>>>(pl.reps, pl.part, pl.nranges,
                                                                       pl.o.nreps, pl.o.N, tau);
  return hipGetLastError();
}

static hipError_t launch_build_orbit(const float* cube, int K, const ColGeom* geo, int n, int N,
                                     int64_t M, float* A32, double* tau, void* scratch, int mode,
                                     const float* colscale, hipStream_t s) {
  const OrbitPlan pl = orbit_plan(K, N, n, scratch);
  hipError_t e = orbit_sort(geo, pl, nullptr, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  const bool vec = (n % 4) == 0;
  const dim3 grid((unsigned)pl.items_max, (unsigned)pl.nranges);
  if (!pair_fits_lds(n)) {  // a staged box per 32 x 32 tile
    const size_t lds = (size_t)16 * kFpRegion * sizeof(float);
    auto launch = [&](auto kern) -> hipError_t {
      const void* fn = reinterpret_cast<const void*>(kern);
      hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (err != hipSuccess) return err;
      kern<<<grid, 1024, lds, s>>>(cube, K, geo, pl.reps, pl.items, pl.nitems, pl.nb, n, N, M, pl.rpr,
                                   pl.o.nreps, A32, pl.part, colscale);
      return hipGetLastError();
    };
    switch (mode) {
      case kSumsOnly:
        e = vec ? launch(build_orbit_box_kernel<true, kSumsOnly>) : launch(build_orbit_box_kernel<false, kSumsOnly>);
        break;
      case kScaled:
        e = vec ? launch(build_orbit_box_kernel<true, kScaled>) : launch(build_orbit_box_kernel<false, kScaled>);
        break;
      default:
        e = vec ? launch(build_orbit_box_kernel<true, kPlain>) : launch(build_orbit_box_kernel<false, kPlain>);
    }
    if (e != hipSuccess) return e;
    return orbit_finish(pl, tau, s);
  }
  const int ls = lds_stride(n);
  const size_t lds = (size_t)(n + 2) * ls * sizeof(float2);
  auto launch = [&](auto kern) -> hipError_t {
    const void* fn = reinterpret_cast<const void*>(kern);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<grid, 1024, lds, s>>>(cube, K, geo, pl.reps, pl.items, pl.nitems, pl.nb, n, ls, N, M,
                                 pl.rpr, pl.o.nreps, A32, pl.part, colscale);
    return hipGetLastError();
  };
  switch (mode) {
    case kSumsOnly:
      e = vec ? launch(build_orbit_kernel<true, kSumsOnly>) : launch(build_orbit_kernel<false, kSumsOnly>);
      break;
    case kScaled:
      e = vec ? launch(build_orbit_kernel<true, kScaled>) : launch(build_orbit_kernel<false, kScaled>);
      break;
    default:
      e = vec ? launch(build_orbit_kernel<true, kPlain>) : launch(build_orbit_kernel<false, kPlain>);
  }
  if (e != hipSuccess) return e;
  return orbit_finish(pl, tau, s);
}

// The two float32 passes of a flux-preserving orbit build (see the modes above).
bool build_orbit_flux_supported(int n, int K, int N) { return K <= 8192 && build_orbit_supported(n, K, N); }

hipError_t launch_build_orbit_sums(const float* cube, int K, const ColGeom* geo, int n, int N,
                                   int64_t M, float* A32, double* tau, void* scratch, hipStream_t s) {
  return launch_build_orbit(cube, K, geo, n, N, M, A32, tau, scratch, kSumsOnly, nullptr, s);
}

hipError_t launch_build_orbit_scaled(const float* cube, int K, const ColGeom* geo, int n, int N,
                                     int64_t M, const float* colscale, float* A32, double* tau,
                                     void* scratch, hipStream_t s) {
  return launch_build_orbit(cube, K, geo, n, N, M, A32, tau, scratch, kScaled, colscale, s);
}

// cubic-spline orbit build from staged boxes of the padded coefficient pairs
bool build_cubic_orbit_supported(int n, int K, int N) {
  return K <= 8192 && n <= kBoxMaxN && orbit_sort_fits(K, N) &&
         (size_t)16 * kCbRegion * sizeof(float) <= (size_t)kLdsBuildMaxBytes;
}

hipError_t launch_build_cubic_orbit(const float* pairs, int K, const ColGeom* geo, int n, int N,
                                    int64_t M, float* A32, double* tau, void* scratch, int mode,
                                    const float* colscale, hipStream_t s) {
  const OrbitPlan pl = orbit_plan(K, N, n, scratch);
  hipError_t e = orbit_sort(geo, pl, nullptr, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  const int Np = n + 2 * kSplinePad;
  const dim3 grid((unsigned)pl.items_max, (unsigned)pl.nranges);
  const size_t lds = (size_t)16 * kCbRegion * sizeof(float);
  const float2* P = reinterpret_cast<const float2*>(pairs);
  auto launch = [&](auto kern) -> hipError_t {
    const void* fn = reinterpret_cast<const void*>(kern);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<grid, 1024, lds, s>>>(P, Np, geo, pl.reps, pl.items, pl.nitems, pl.nb, n, N, M, pl.rpr,
                                 pl.o.nreps, A32, pl.part, colscale);
    return hipGetLastError();
  };
  const bool vec = (n % 4) == 0;
  switch (mode) {
    case kSumsOnly:
      e = vec ? launch(build_cubic_orbit_kernel<true, kSumsOnly>) : launch(build_cubic_orbit_kernel<false, kSumsOnly>);
      break;
    case kScaled:
      e = vec ? launch(build_cubic_orbit_kernel<true, kScaled>) : launch(build_cubic_orbit_kernel<false, kScaled>);
      break;
    default:
      e = vec ? launch(build_cubic_orbit_kernel<true, kPlain>) : launch(build_cubic_orbit_kernel<false, kPlain>);
  }
  if (e != hipSuccess) return e;
  return orbit_finish(pl, tau, s);
}

// 16-bit orbit build: the pair (ending 16-byte aligned), then two 2 x 8 x 33 unit tiles
static size_t orbit16_pair_bytes(int n) {
  return (((size_t)(n + 2) * lds_stride(n) * sizeof(float2)) + 15) & ~(size_t)15;
}
static size_t orbit16_lds_bytes(int n) { return orbit16_pair_bytes(n) + (size_t)2 * (2 * 8 * 33 * 16); }

// LDS of the 16-bit box kernel: 16 box regions, then the two unit tiles
static size_t orbit16_box_lds_bytes(bool cubic) {
  return cubic ? (size_t)16 * kCbRegion * sizeof(float) + (size_t)2 * (2 * 4 * 33 * 16)
               : (size_t)16 * kFpRegion * sizeof(float) + (size_t)2 * (2 * 8 * 33 * 16);
}

// the pair in LDS with the unit tiles, or (up to kBoxMaxN) staged boxes
bool build_orbit16_supported(int n, int K, int N) {
  if (N % 8 != 0 || !orbit_sort_fits(K, N)) return false;
  if (pair_fits_lds(n)) return orbit16_lds_bytes(n) <= (size_t)kLdsBuildMaxBytes;
  return n <= kBoxMaxN && orbit16_box_lds_bytes(false) <= (size_t)kLdsBuildMaxBytes;
}

// float32: the pair in LDS, or (up to kBoxMaxN) a staged box per tile
static bool build_orbit_supported(int n, int K, int N) {
  return (pair_fits_lds(n) || n <= kBoxMaxN) && orbit_sort_fits(K, N);
}

size_t build_lds_scratch_bytes(int K, int N, int n) {
  return build_orbit_supported(n, K, N) ? build_orbit_scratch_bytes(K, N, n)
                                        : bucket_scratch_bytes(K, (int64_t)N * N);
}

hipError_t launch_build_orbit16(int storage, const float* cube, int K, const ColGeom* geo, int n,
                                int N, int64_t M, int32_t* perm, int32_t* eslot, int32_t* slot_of,
                                void* lib, double* tau, void* scratch, const float* colscale,
                                hipStream_t s) {
  const OrbitPlan pl = orbit_plan(K, N, n, scratch);
  hipError_t e = orbit_sort(geo, pl, perm, slot_of, eslot, s);
  if (e != hipSuccess) return e;
  uint16_t* Mh = reinterpret_cast<uint16_t*>(lib);
  const dim3 grid((unsigned)pl.items_max, (unsigned)pl.nranges);
  if (!pair_fits_lds(n)) {  // a staged box per 32 x 32 pixels
    const size_t lds = orbit16_box_lds_bytes(false);
    auto launch = [&](auto kern) -> hipError_t {
      const void* fn = reinterpret_cast<const void*>(kern);
      hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (err != hipSuccess) return err;
      kern<<<grid, 1024, lds, s>>>(cube, K, geo, pl.reps, pl.items, pl.nitems, pl.nb, n, M, 0, pl.rpr,
                                   pl.o.nreps, Mh, pl.part, colscale);
      return hipGetLastError();
    };
    const bool bf = storage == PSFLIB_BF16_POW2;
    if (colscale)
      e = bf ? launch(build_orbit16_box_kernel<true, false, true>) : launch(build_orbit16_box_kernel<false, false, true>);
    else
      e = bf ? launch(build_orbit16_box_kernel<true, false, false>) : launch(build_orbit16_box_kernel<false, false, false>);
    if (e != hipSuccess) return e;
    return orbit_finish(pl, tau, s);
  }
  const int ls = lds_stride(n);
  const size_t lds = orbit16_lds_bytes(n);
  auto launch = [&](auto kern) -> hipError_t {
    const void* fn = reinterpret_cast<const void*>(kern);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<grid, 1024, lds, s>>>(cube, K, geo, pl.reps, pl.items, pl.nitems, pl.nb, n, ls, M,
                                 pl.rpr, pl.o.nreps, Mh, pl.part, colscale);
    return hipGetLastError();
  };
  const bool bf = storage == PSFLIB_BF16_POW2;
  if (colscale)
    e = bf ? launch(build_orbit16_kernel<true, true>) : launch(build_orbit16_kernel<false, true>);
  else
    e = bf ? launch(build_orbit16_kernel<true, false>) : launch(build_orbit16_kernel<false, false>);
  if (e != hipSuccess) return e;
  return orbit_finish(pl, tau, s);
}

bool build_cubic_orbit16_supported(int n, int K, int N) {
  return N % 8 == 0 && build_cubic_orbit_supported(n, K, N) &&
         orbit16_box_lds_bytes(true) <= (size_t)kLdsBuildMaxBytes;
}

hipError_t launch_build_cubic_orbit16(int storage, const float* pairs, int K, const ColGeom* geo,
                                      int n, int N, int64_t M, int32_t* perm, int32_t* eslot,
                                      int32_t* slot_of, void* lib, double* tau, void* scratch,
                                      const float* colscale, hipStream_t s) {
  const OrbitPlan pl = orbit_plan(K, N, n, scratch);
  hipError_t e = orbit_sort(geo, pl, perm, slot_of, eslot, s);
  if (e != hipSuccess) return e;
  uint16_t* Mh = reinterpret_cast<uint16_t*>(lib);
  const dim3 grid((unsigned)pl.items_max, (unsigned)pl.nranges);
  const size_t lds = orbit16_box_lds_bytes(true);
  const int Np = n + 2 * kSplinePad;
  auto launch = [&](auto kern) -> hipError_t {
    const void* fn = reinterpret_cast<const void*>(kern);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    kern<<<grid, 1024, lds, s>>>(pairs, K, geo, pl.reps, pl.items, pl.nitems, pl.nb, n, M, Np, pl.rpr,
                                 pl.o.nreps, Mh, pl.part, colscale);
    return hipGetLastError();
  };
  const bool bf = storage == PSFLIB_BF16_POW2;
  if (colscale)
    e = bf ? launch(build_orbit16_box_kernel<true, true, true>) : launch(build_orbit16_box_kernel<false, true, true>);
  else
    e = bf ? launch(build_orbit16_box_kernel<true, true, false>) : launch(build_orbit16_box_kernel<false, true, false>);
  if (e != hipSuccess) return e;
  return orbit_finish(pl, tau, s);
}


}  // namespace psflib
