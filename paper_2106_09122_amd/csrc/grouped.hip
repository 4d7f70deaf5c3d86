// Grouped simulation: many scenes, each with its own library (different image
// and scene sizes, different wavelengths), in one persistent launch captured
// in a HIP graph.  Sec. 5 of the paper points at simulating many complex
// scenes at once; with a few scenes per library the product streams every
// library once from HBM and is bandwidth bound, so it is a multi-right-hand-
// side matvec rather than a matrix-core GEMM.
//
// Work items are (library, scene group of <= kGrpScenes, row block, column
// chunk) tiles, listed on the host when the plan is made.  A persistent grid
// walks the list; each workgroup streams its tile of the library once and
// multiplies it with every scene of the group, writing partial images; a
// second kernel adds the partials of each (scene, row block) in chunk order
// (bitwise reproducible).  The chunk length is chosen by timing the candidate
// shapes on the plan itself (psflib_grouped_create with autotune), and the
// choice is cached per plan signature for the process.
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

constexpr int kGrpScenes = 8;   // scenes multiplied per pass over a tile
constexpr int kGrpThreads = 256;

struct GItem {
  const void* A;          // library matrix (FP32 column-major or 16-bit 8-column groups)
  const int32_t* exps;    // 16-bit per-column exponents (nullptr for FP32)
  int64_t M, ncols;       // rows, scene pixels of this library
  int64_t row0;           // first row of the block
  int64_t j0, j1;         // columns (FP32) or 8-column groups (16-bit) of the chunk
  int32_t scene0, nscenes;  // scenes (index into the plan's scene table)
  int64_t part;           // float offset of this item's partials: [kGrpScenes][rows]
};

struct GReduce {
  int64_t M, row0, rows;
  int64_t part0;          // partials of the first chunk; chunk c at part0 + c * stride
  int64_t stride;         // floats between consecutive chunks' partials
  int32_t nchunks, scene0, nscenes, pad;
};

// ------------------------------------------------------------- kernels ----
// FP32: each thread owns 4 consecutive rows (1024 rows per workgroup) and one
// accumulator per scene; the chunk's scene values are staged in LDS (zeros for
// the unused scene slots, so every slot is computed without branches) and read
// as broadcasts; 8 columns of 16-byte non-temporal loads are in flight.
template <bool FULL>
__device__ __forceinline__ void grouped_f32_block8(const float* __restrict__ A, int64_t M,
                                                   int64_t i0, int64_t j, const float* zrow,
                                                   int zstride, f32x4* inner) {
  f32x4 v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const float* col = A + (j + u) * M + i0;
    if constexpr (FULL) {
      v[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[u][e] = (i0 + e < M) ? col[e] : 0.0f;
    }
  }
#pragma unroll
  for (int r = 0; r < kGrpScenes; ++r) {
    const f32x4 za = *reinterpret_cast<const f32x4*>(zrow + r * zstride);
    const f32x4 zb = *reinterpret_cast<const f32x4*>(zrow + r * zstride + 4);
    inner[r] += v[0] * za.x;
    inner[r] += v[1] * za.y;
    inner[r] += v[2] * za.z;
    inner[r] += v[3] * za.w;
    inner[r] += v[4] * zb.x;
    inner[r] += v[5] * zb.y;
    inner[r] += v[6] * zb.z;
    inner[r] += v[7] * zb.w;
  }
}

template <bool FULL>
__device__ __forceinline__ void grouped_f32_rows(const float* __restrict__ A, int64_t M,
                                                 int64_t i0, int64_t j0, int nc,
                                                 const float* zs, f32x4* acc) {
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  int q = 0;
  for (; q + 16 <= nc; q += 16) {  // blocked sums: 16 columns per inner sum
    f32x4 inner[kGrpScenes];
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) inner[r] = zero;
    grouped_f32_block8<FULL>(A, M, i0, j0 + q, zs + q, kGrpMaxChunkCols, inner);
    grouped_f32_block8<FULL>(A, M, i0, j0 + q + 8, zs + q + 8, kGrpMaxChunkCols, inner);
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) acc[r] += inner[r];
  }
  f32x4 inner[kGrpScenes];
#pragma unroll
  for (int r = 0; r < kGrpScenes; ++r) inner[r] = zero;
  for (; q < nc; ++q) {
    const float* col = A + (j0 + q) * M + i0;
    f32x4 v;
    if constexpr (FULL) {
      v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(col));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (i0 + e < M) ? col[e] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) inner[r] += v * zs[r * kGrpMaxChunkCols + q];
  }
#pragma unroll
  for (int r = 0; r < kGrpScenes; ++r) acc[r] += inner[r];
}

__global__ __launch_bounds__(kGrpThreads, 2) void grouped_f32_kernel(
    const GItem* __restrict__ items, int64_t nitems, const float* const* __restrict__ scenes,
    float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) float zs[kGrpScenes * kGrpMaxChunkCols];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GItem w = items[it];
    const float* A = reinterpret_cast<const float*>(w.A);
    const int nc = (int)(w.j1 - w.j0);
    __syncthreads();  // the previous item is done with zs
    for (int t = threadIdx.x; t < kGrpScenes * nc; t += kGrpThreads) {
      const int r = t / nc, q = t - r * nc;
      zs[r * kGrpMaxChunkCols + q] = (r < w.nscenes) ? scenes[w.scene0 + r][w.j0 + q] : 0.0f;
    }
    __syncthreads();
    const int64_t i0 = w.row0 + 4 * (int64_t)threadIdx.x;
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    f32x4 acc[kGrpScenes];
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) acc[r] = zero;
    // uniform across the workgroup: every row of the block is inside the image
    const bool block_full = (w.M % 4 == 0) && w.row0 + 4 * kGrpThreads <= w.M;
    if (block_full)
      grouped_f32_rows<true>(A, w.M, i0, w.j0, nc, zs, acc);
    else if (i0 < w.M)
      grouped_f32_rows<false>(A, w.M, i0, w.j0, nc, zs, acc);
    const int64_t rows = 4 * kGrpThreads;
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r)
      *reinterpret_cast<f32x4*>(part + w.part + r * rows + 4 * threadIdx.x) = acc[r];
  }
}

// 16-bit: one thread per row (256 rows per workgroup), one 16-byte load per
// 8-column group; the chunk's scene values times 2^e_j are staged in LDS.
// Library loads run one batch of 8 groups ahead of the multiply (two
// register sets), and the first batch of an item is issued before its scene
// values are staged, so the loads stay in flight across both.
template <bool BF16>
__device__ __forceinline__ void grouped_h16_batch(const u32x4 (&pk)[8], int64_t g, int64_t ng,
                                                  int nscenes, const float (*zs)[kGrpMaxChunkGroups * 8],
                                                  float (&acc)[kGrpScenes]) {
  float inner[kGrpScenes];
#pragma unroll
  for (int r = 0; r < kGrpScenes; ++r) inner[r] = 0.0f;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (g + t >= ng) break;
    const uint32_t wd[4] = {pk[t].x, pk[t].y, pk[t].z, pk[t].w};
    float f[8];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      if (BF16) {
        f[2 * h] = __uint_as_float(wd[h] << 16);
        f[2 * h + 1] = __uint_as_float(wd[h] & 0xFFFF0000u);
      } else {
        f[2 * h] = (float)__builtin_bit_cast(_Float16, (uint16_t)(wd[h] & 0xFFFFu));
        f[2 * h + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(wd[h] >> 16));
      }
    }
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) {
      if (r >= nscenes) break;
      const float* z = &zs[r][(g + t) * 8];
#pragma unroll
      for (int u = 0; u < 8; ++u) inner[r] = fmaf(f[u], z[u], inner[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < kGrpScenes; ++r) acc[r] += inner[r];
}

template <bool BF16>
__global__ __launch_bounds__(kGrpThreads) void grouped_h16_kernel(
    const GItem* __restrict__ items, int64_t nitems, const float* const* __restrict__ scenes,
    float* __restrict__ part) {
  __shared__ float zs[kGrpScenes][kGrpMaxChunkGroups * 8];
  const u32x4 z4 = {0u, 0u, 0u, 0u};
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GItem w = items[it];
    const u32x4* Mp = reinterpret_cast<const u32x4*>(w.A);
    const int64_t ng = w.j1 - w.j0;
    const int64_t i = w.row0 + threadIdx.x;
    const bool row_ok = i < w.M;
    auto load = [&](int64_t g, u32x4 (&pk)[8]) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        pk[t] = (row_ok && g + t < ng) ? __builtin_nontemporal_load(Mp + (w.j0 + g + t) * w.M + i) : z4;
    };
    u32x4 pa[8], pb[8];
    load(0, pa);
    __syncthreads();  // the previous item is done with zs
    for (int64_t t = threadIdx.x; t < ng * 8 * kGrpScenes; t += kGrpThreads) {
      const int r = (int)(t / (ng * 8));
      const int64_t q = t - (int64_t)r * ng * 8;
      const int64_t j = w.j0 * 8 + q;
      float v = 0.0f;
      if (r < w.nscenes && j < w.ncols) v = ldexpf(scenes[w.scene0 + r][j], w.exps[j]);
      zs[r][q] = v;
    }
    __syncthreads();
    float acc[kGrpScenes];
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) acc[r] = 0.0f;
    if (row_ok) {
      for (int64_t g = 0; g < ng; g += 16) {
        load(g + 8, pb);
        grouped_h16_batch<BF16>(pa, g, ng, w.nscenes, zs, acc);
        if (g + 8 >= ng) break;
        load(g + 16, pa);
        grouped_h16_batch<BF16>(pb, g + 8, ng, w.nscenes, zs, acc);
      }
    }
#pragma unroll
    for (int r = 0; r < kGrpScenes; ++r) part[w.part + r * kGrpThreads + threadIdx.x] = acc[r];
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
  void* dev;        // items | reductions | scene table | image table | partials
  int64_t chunk;    // chosen chunk length (columns, or 8-column groups for 16-bit)
  float ms_tuned;   // time of the chosen shape during autotuning (0 if not tuned)
};

namespace {

struct LibInfo {
  const void* A;
  const int32_t* exps;
  int64_t M, ncols, ncols_pad;
};

struct Plan {
  std::vector<psflib::GItem> items;
  std::vector<psflib::GReduce> reds;
  std::vector<const float*> scenes;
  std::vector<float*> images;
  int64_t part_floats = 0;
};

// Items for a given chunk length.  Scenes are grouped by library (kept in the
// caller's order inside a library) and cut into groups of kGrpScenes.
Plan make_plan(int storage, const std::vector<LibInfo>& libs, const int32_t* lib_of_scene,
               const float* const* scenes, float* const* images, int B, int64_t chunk) {
  Plan p;
  const bool f32 = storage == PSFLIB_FP32;
  const int64_t rows_per = f32 ? 4 * psflib::kGrpThreads : psflib::kGrpThreads;
  for (size_t L = 0; L < libs.size(); ++L) {
    std::vector<int> sc;
    for (int b = 0; b < B; ++b)
      if (lib_of_scene[b] == (int)L) sc.push_back(b);
    const LibInfo& li = libs[L];
    const int64_t units = f32 ? li.ncols : li.ncols_pad / 8;
    const int64_t nchunks = (units + chunk - 1) / chunk;
    const int64_t nrb = (li.M + rows_per - 1) / rows_per;
    for (size_t g0 = 0; g0 < sc.size(); g0 += psflib::kGrpScenes) {
      const int ns = (int)std::min<size_t>(psflib::kGrpScenes, sc.size() - g0);
      const int32_t scene0 = (int32_t)p.scenes.size();
      for (int r = 0; r < ns; ++r) {
        p.scenes.push_back(scenes[sc[g0 + r]]);
        p.images.push_back(images[sc[g0 + r]]);
      }
      for (int64_t rb = 0; rb < nrb; ++rb) {
        psflib::GReduce rd;
        rd.M = li.M;
        rd.row0 = rb * rows_per;
        rd.rows = rows_per;
        rd.part0 = p.part_floats;
        rd.stride = (int64_t)psflib::kGrpScenes * rows_per;
        rd.nchunks = (int32_t)nchunks;
        rd.scene0 = scene0;
        rd.nscenes = ns;
        rd.pad = 0;
        p.reds.push_back(rd);
        for (int64_t c = 0; c < nchunks; ++c) {
          psflib::GItem it;
          it.A = li.A;
          it.exps = li.exps;
          it.M = li.M;
          it.ncols = li.ncols;
          it.row0 = rb * rows_per;
          it.j0 = c * chunk;
          it.j1 = std::min(units, (c + 1) * chunk);
          it.scene0 = scene0;
          it.nscenes = ns;
          it.part = p.part_floats;
          p.part_floats += rd.stride;
          p.items.push_back(it);
        }
      }
    }
  }
  return p;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

std::mutex g_tune_mu;
std::map<std::string, int64_t> g_tune_cache;  // plan signature -> chosen chunk

}  // namespace

namespace psflib {

// Build (or rebuild) the plan's device tables and graph for one chunk length.
static hipError_t instantiate(psflib_grouped* g, const std::vector<LibInfo>& libs,
                              const int32_t* lib_of_scene, const float* const* scenes,
                              float* const* images, int B, int64_t chunk, hipStream_t s) {
  const Plan p = make_plan(g->storage, libs, lib_of_scene, scenes, images, B, chunk);
  const size_t o_items = 0;
  const size_t o_reds = align256(o_items + p.items.size() * sizeof(GItem));
  const size_t o_sc = align256(o_reds + p.reds.size() * sizeof(GReduce));
  const size_t o_im = align256(o_sc + p.scenes.size() * sizeof(void*));
  const size_t o_part = align256(o_im + p.images.size() * sizeof(void*));
  const size_t total = align256(o_part + (size_t)p.part_floats * 4);
  if (g->exec) { (void)hipGraphExecDestroy(g->exec); g->exec = nullptr; }
  if (g->graph) { (void)hipGraphDestroy(g->graph); g->graph = nullptr; }
  if (g->dev) { (void)hipFree(g->dev); g->dev = nullptr; }
  hipError_t e = hipSuccess;
  if (total > 0) {
    e = hipMalloc(&g->dev, total);
    if (e != hipSuccess) { g->dev = nullptr; return e; }
  }
  char* d = reinterpret_cast<char*>(g->dev);
  if (!p.items.empty()) {
    e = hipMemcpy(d + o_items, p.items.data(), p.items.size() * sizeof(GItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipMemcpy(d + o_reds, p.reds.data(), p.reds.size() * sizeof(GReduce), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipMemcpy(d + o_sc, p.scenes.data(), p.scenes.size() * sizeof(void*), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipMemcpy(d + o_im, p.images.data(), p.images.size() * sizeof(void*), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  const GItem* items = reinterpret_cast<const GItem*>(d + o_items);
  const GReduce* reds = reinterpret_cast<const GReduce*>(d + o_reds);
  const float* const* sc = reinterpret_cast<const float* const*>(d + o_sc);
  float* const* im = reinterpret_cast<float* const*>(d + o_im);
  float* part = reinterpret_cast<float*>(d + o_part);
  const int64_t nitems = (int64_t)p.items.size();
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device);
  const int64_t per_cu = 4;  // resident workgroups per CU the persistent grid aims at
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)cus * per_cu));

  hipStream_t cap;
  e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    if (nitems > 0) {
      if (g->storage == PSFLIB_FP32)
        grouped_f32_kernel<<<grid, kGrpThreads, 0, cap>>>(items, nitems, sc, part);
      else if (g->storage == PSFLIB_BF16_POW2)
        grouped_h16_kernel<true><<<grid, kGrpThreads, 0, cap>>>(items, nitems, sc, part);
      else
        grouped_h16_kernel<false><<<grid, kGrpThreads, 0, cap>>>(items, nitems, sc, part);
      grouped_reduce_kernel<<<(unsigned)p.reds.size(), 256, 0, cap>>>(reds, part, im);
    }
    hipError_t e2 = hipStreamEndCapture(cap, &g->graph);
    e = (e2 != hipSuccess) ? e2 : hipGetLastError();
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  g->chunk = chunk;
  (void)s;
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
    psflib::handle_info(h_libs[L], &li.A, &li.exps, &li.M, &li.ncols, &li.ncols_pad, &st, &d);
    if (storage < 0) { storage = st; dev = d; }
    if (st != storage)
      return psflib::fail_status(PSFLIB_ERR_UNSUPPORTED, "grouped: all libraries must share one storage form");
    if (d != dev) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: libraries on different devices");
    libs.push_back(li);
  }
  for (int b = 0; b < B; ++b) {
    if (h_lib_of_scene[b] < 0 || h_lib_of_scene[b] >= nlibs)
      return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: scene library index out of range");
    if (!h_scenes[b] || !h_images[b])
      return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: NULL scene or image pointer");
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != dev)
    return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped: current device differs from the libraries'");
  psflib_grouped* g = new (std::nothrow) psflib_grouped();
  if (!g) return psflib::fail_status(PSFLIB_ERR_DEVICE, "host allocation failed");
  g->storage = storage;
  g->device = dev;
  g->graph = nullptr;
  g->exec = nullptr;
  g->dev = nullptr;
  g->ms_tuned = 0.0f;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the libraries may still be building on `stream`
  hipError_t e = hipStreamSynchronize(s);
  auto bail = [&](hipError_t err, const char* what) {
    psflib_grouped_destroy(g);
    return psflib::device_fail_status(err, what);
  };
  if (e != hipSuccess) return bail(e, "hipStreamSynchronize");

  // Candidate chunk lengths: columns (FP32) or 8-column groups (16-bit).
  const bool f32 = storage == PSFLIB_FP32;
  std::vector<int64_t> cands = f32 ? std::vector<int64_t>{256, 512, 1024}
                                   : std::vector<int64_t>{32, 64, 128};
  std::string sig = std::to_string(storage) + ":";
  for (int b = 0; b < B; ++b) {
    const LibInfo& li = libs[h_lib_of_scene[b]];
    sig += std::to_string(li.M) + "x" + std::to_string(li.ncols) + ",";
  }
  int64_t chosen = f32 ? 512 : 64;
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
    for (int64_t c : cands) {
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
  *out = g;
  return PSFLIB_OK;
}

psflib_status psflib_grouped_run(const psflib_grouped* g, void* stream) {
  if (!g) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "grouped plan is NULL");
  if (!g->exec) return PSFLIB_OK;  // no scenes
  hipError_t e = hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return psflib::device_fail_status(e, "hipGraphLaunch");
  return PSFLIB_OK;
}

psflib_status psflib_grouped_chunk(const psflib_grouped* g, int64_t* chunk, float* tuned_ms) {
  if (!g || !chunk) return psflib::fail_status(PSFLIB_ERR_INVALID_ARG, "NULL argument");
  *chunk = g->chunk;
  if (tuned_ms) *tuned_ms = g->ms_tuned;
  return PSFLIB_OK;
}

void psflib_grouped_destroy(psflib_grouped* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->dev) (void)hipFree(g->dev);
  delete g;
}

}  // extern "C"
