// Measurement probes: the ceilings the products are compared against, taken
// on the part itself rather than from the datasheet.
//
//  * HBM read: a stream of 16-byte non-temporal loads over a caller buffer
//    (much larger than the 256 MB last-level cache), U loads in flight per
//    thread, grid-stride or one contiguous slice per workgroup -- the
//    access pattern of the matvec without its arithmetic.  The best rate
//    over a sweep of launch shapes is the bandwidth the matvec can hope for.
//  * Matrix cores: every wave issues chains of independent MFMA
//    instructions on register operands (no memory traffic), 4 accumulators
//    per wave so consecutive instructions never wait for each other -- the
//    throughput the batched products can hope for at the clock the part
//    actually holds under load.
#include "psflib_internal.h"

namespace psflib {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// SLICE false: grid-stride (workgroup w reads 4 KiB runs w, w + grid, ...);
// SLICE true: workgroup w streams its own contiguous 1/grid of the buffer,
// 4 KiB runs one after another, U of them in flight.
template <int U, bool SLICE>
__global__ __launch_bounds__(256) void hbm_read_kernel(const f32x4* __restrict__ p, int64_t n16,
                                                       float* __restrict__ sink) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  int64_t i, end, stride;
  if constexpr (SLICE) {
    const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
    i = (int64_t)blockIdx.x * per + threadIdx.x;
    end = min((int64_t)(blockIdx.x + 1) * per, n16);
    stride = 256;
  } else {
    i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    end = n16;
    stride = (int64_t)gridDim.x * 256;
  }
  for (; i + (U - 1) * stride < end; i += U * stride) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  for (; i < end; i += stride) acc += __builtin_nontemporal_load(p + i);
  const float s = (acc.x + acc.y) + (acc.z + acc.w);
  // a store the compiler cannot drop, taken only for a value the probe's
  // input (zeros or finite data) makes practically impossible
  if (s == -1.2345e-37f) sink[blockIdx.x] = s;
}

// KIND 0: v_mfma_f32_32x32x2f32; 1: v_mfma_f32_32x32x16_bf16; 2: ..._f16.
template <int KIND>
__global__ __launch_bounds__(256) void mfma_issue_kernel(int iters, float* __restrict__ sink) {
  const int lane = threadIdx.x & 63;
  f32x16 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
  const float x = 1e-3f * (float)(lane + 1);
  if constexpr (KIND == 0) {
    const float a = x, b = 1.0f - x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
    }
  } else if constexpr (KIND == 1) {
    bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] = (__bf16)(x + 0.01f * k);
      b[k] = (__bf16)(1.0f - x);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    }
  } else {
    f16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] = (_Float16)(x + 0.01f * k);
      b[k] = (_Float16)(1.0f - x);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[c][r];
  if (s == -1.2345e-37f) sink[blockIdx.x] = s;
}

}  // namespace

hipError_t launch_probe_hbm_read(const void* buf, size_t bytes, int workgroups, int unroll,
                                 bool slice, float* sink, hipStream_t s) {
  const f32x4* p = reinterpret_cast<const f32x4*>(buf);
  const int64_t n16 = (int64_t)(bytes / 16);
  if (slice) {
    switch (unroll) {
      case 4: hbm_read_kernel<4, true><<<workgroups, 256, 0, s>>>(p, n16, sink); break;
      case 8: hbm_read_kernel<8, true><<<workgroups, 256, 0, s>>>(p, n16, sink); break;
      default: hbm_read_kernel<16, true><<<workgroups, 256, 0, s>>>(p, n16, sink); break;
    }
  } else {
    switch (unroll) {
      case 4: hbm_read_kernel<4, false><<<workgroups, 256, 0, s>>>(p, n16, sink); break;
      case 8: hbm_read_kernel<8, false><<<workgroups, 256, 0, s>>>(p, n16, sink); break;
      default: hbm_read_kernel<16, false><<<workgroups, 256, 0, s>>>(p, n16, sink); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_probe_mfma(int kind, int iters, int workgroups, float* sink, hipStream_t s) {
  switch (kind) {
    case 0: mfma_issue_kernel<0><<<workgroups, 256, 0, s>>>(iters, sink); break;
    case 1: mfma_issue_kernel<1><<<workgroups, 256, 0, s>>>(iters, sink); break;
    default: mfma_issue_kernel<2><<<workgroups, 256, 0, s>>>(iters, sink); break;
  }
  return hipGetLastError();
}

}  // namespace psflib
