// Internal declarations shared by the psflib translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <utility>
#include <vector>

#include "psflib.h"

namespace psflib {

// Per-column geometry and radial bracket, written by the geometry kernel.
struct ColGeom {
  double r, ct, st, w;  // offset, cos/sin of the position angle, radial weight
  int32_t k;            // lower radial sample; -1 for an identically zero column
  int32_t e;            // power-of-two exponent of the 16-bit storage (0 for FP32)
  int32_t pad[2];
};
static_assert(sizeof(ColGeom) == 48, "ColGeom layout");

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Launch-shape constants shared between the host code and the kernels.
constexpr int kBuildThreads = 256;   // build kernel: one workgroup per group of 8 columns
constexpr int kMvThreads = 256;      // FP32 matvec threads per workgroup (4 rows each)
constexpr int kMvTargetWorkgroups32 = 512;  // split-K FP32 matvec: workgroups per launch (about)
constexpr int kMvTargetWorkgroups16 = 256;  // split-K 16-bit matvec: workgroups per launch (about)
constexpr int kMv16Threads = 256;    // 16-bit matvec threads per workgroup
constexpr int kMv16RowsPerThread = 8;  // 16-bit matvec rows per thread (kMv16Threads apart)
constexpr int kMv16MaxChunkGroups = 512;  // 16-bit matvec: 8-column groups per chunk, at most
constexpr int64_t kStageMaxCols = 32768;  // batched 16-bit: scenes staged whole in LDS up to this many columns
constexpr int64_t kStagePairCols = 16384;  // batched 16-bit: two scenes per staging workgroup up to this many columns
constexpr int kAdjThreads = 256;     // adjoint threads per workgroup
constexpr int kAdjF32Rows = 16384;   // rows per FP32 adjoint row block (16 float4 per thread)
constexpr int kAdj16Rows = 16384;    // rows per 16-bit adjoint row block (64 rows per thread)
constexpr int kAdjColsPerBlock = 16; // FP32 adjoint: columns per workgroup
constexpr int kAdj16GroupsPerBlock = 2;  // 16-bit adjoint: 8-column groups per workgroup
constexpr int kColPad = 64;          // 16-bit column count padded to a multiple of this
constexpr int32_t kZeroColumnExp = PSFLIB_ZERO_COLUMN_EXPONENT;  // exponent of an identically zero column
constexpr int kLdsCols = 16;         // LDS build: columns per work item (one wave each)
constexpr int kLdsBuildMaxBytes = 163840;  // LDS build: bordered PSF pair must fit the CU's LDS
constexpr int kSplinePad = 12;       // cubic rotation: zero pixels padded on each side before the spline filter
constexpr int kLdsMaxBuckets = 8193; // LDS builds: radial brackets + the zero-column bucket, at most

struct Layout {
  int64_t M;          // n*n image pixels (rows of A)
  int64_t ncols;      // N*N scene pixels (columns of A)
  int64_t ncols_pad;  // columns stored (multiple of kColPad for 16-bit forms)
  // byte offsets in the library buffer: column sums; 16-bit forms: exponents
  // per column, slot -> column map, exponents per slot, column -> slot map
  size_t off_tau, off_exp, off_perm, off_eslot, off_slot, total;
};

// Column order of the 16-bit storage forms: mantissa slot s (in groups of 8
// slots) holds column perm[s] (-1 for padding) with exponent eslot[s];
// column j sits in slot slot_of[j] and has exponent exps[j].  All nullptr for
// FP32 storage (natural column order).
struct Cols16 {
  const int32_t* exps;     // [ncols_pad] per column
  const int32_t* perm;     // [ncols_pad] slot -> column
  const int32_t* eslot;    // [ncols_pad] per slot
  const int32_t* slot_of;  // [ncols] column -> slot
};

bool compute_layout(const psflib_desc& d, Layout* L);

// Error helpers of the ABI layer (record the message for psflib_last_error).
psflib_status fail_status(psflib_status s, const char* msg);
psflib_status device_fail_status(hipError_t e, const char* what);
// PSFLIB_ERR_DEVICE if a HIP error is pending on this thread from earlier
// work (an asynchronous fault, or a failed runtime call): checked after
// validation and before anything is enqueued.
psflib_status check_pending_error();

// Stream-ordered device memory from the library's pool for `dev` (one pool
// per device, kept until the process ends; freed blocks are reused).
hipError_t pool_alloc(void** p, size_t bytes, int dev, hipStream_t s);
// Return pool memory that no queued work uses any more (the caller has waited
// for its users): freed on a library-internal stream of `dev`, so nothing
// the caller enqueued waits for it.
hipError_t pool_release(void* p, int dev);

// The streams that used an object's device memory: one event per stream,
// re-recorded at every use, so that releasing the object waits for its own
// work only, not for the whole device.  Uses on a stream that is being
// captured are not recorded (a graph that uses the object must finish before
// the object is released).
class StreamUses {
 public:
  hipError_t note(hipStream_t s);
  void wait_all();  // host-wait for every recorded use, then forget them
  ~StreamUses();

 private:
  std::mutex mu_;
  std::vector<std::pair<hipStream_t, hipEvent_t>> ev_;
};

// Fixed device scratch of the allocation-free apply (psflib_apply_noalloc):
// a file-scope device array of kNoAllocScratchBytes on every GPU the library
// runs on.  noalloc_scratch gives its address on device `dev` (the current
// device), looked up once per device.
constexpr size_t kNoAllocScratchBytes = PSFLIB_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch(int dev, void** ptr);

// Read-only view of a built library for the grouped apply.
void handle_info(const psflib_handle* h, const void** A, Cols16* cx, int64_t* M,
                 int64_t* ncols, int64_t* ncols_pad, int* storage, int* device);
// Natural column order for a 16-bit library (slot s = column s) and the
// per-slot exponents, once the per-column exponents are final.
hipError_t launch_identity_order(int32_t* perm, int32_t* eslot, int32_t* slot_of,
                                 const int32_t* exps, int64_t ncols, int64_t ncols_pad,
                                 hipStream_t s);

// The four cubic B-spline weights of the taps at offsets -1, 0, +1, +2 from
// floor(x), for t = x - floor(x) in [0, 1): beta3 at distances 1+t, t, 1-t,
// 2-t (all exact in float64), evaluated in float64 and rounded to float32.
__device__ __forceinline__ void cubic_weights(double t, float w[4]) {
#pragma clang fp contract(off)
  constexpr double sixth = 1.0 / 6.0;  // a product, not a float64 division (within an ulp)
  const double s = 1.0 - t;
  w[0] = (float)(s * s * s * sixth);
  w[1] = (float)(2.0 / 3.0 - t * t + t * t * t * 0.5);
  w[2] = (float)(2.0 / 3.0 - s * s + s * s * s * 0.5);
  w[3] = (float)(t * t * t * sixth);
}

// ---- kernel launchers (each returns hipGetLastError() after its launch) ----
hipError_t launch_cube_max(const float* cube, int K, int64_t M, float* pmax, hipStream_t s);
hipError_t launch_pair_cube(const float* cube, int K, int64_t M, float* pairs, hipStream_t s);
hipError_t launch_geometry(int N, double S, const double* radii, int K, int interp, int oob,
                           const float* pmax, bool want_exp, ColGeom* geo, int64_t ncols_pad,
                           int32_t* exps, hipStream_t s);
// Cubic-spline rotation: coefficients of every sampled PSF padded by
// kSplinePad zeros per side ([K][Np][Np], Np = n + 2 kSplinePad) as
// radial pairs (float2 [max(K-1,1)][Np*Np]) and their largest magnitude per
// PSF; scratch must hold spline_scratch_bytes(K, n) bytes.
size_t spline_scratch_bytes(int K, int n);
hipError_t launch_spline_pairs(const float* cube, int K, int n, void* scratch, float* cmax,
                               hipStream_t s);
const float* spline_pairs_of(const void* scratch, int K, int n);
hipError_t launch_build_cubic(int storage, const float* pairs, const ColGeom* geo, int n, int64_t M,
                              int64_t ncols, int64_t ncols_pad, void* lib, double* tau,
                              hipStream_t s);
// Modes of the float32 orbit builds: plain; column sums only (nothing
// stored); every value times its column's scale colscale[j] before it is
// stored and summed.  The 16-bit orbit builds scale when colscale is given.
constexpr int kOrbitPlain = 0, kOrbitSumsOnly = 1, kOrbitScaled = 2;
// The two passes of a flux-preserving bilinear orbit build: the column sums
// of the plain build (tau), then the build scaled per column.
bool build_orbit_flux_supported(int n, int K, int N);
hipError_t launch_build_orbit_sums(const float* cube, int K, const ColGeom* geo, int n, int N,
                                   int64_t M, float* A32, double* tau, void* scratch, hipStream_t s);
hipError_t launch_build_orbit_scaled(const float* cube, int K, const ColGeom* geo, int n, int N,
                                     int64_t M, const float* colscale, float* A32, double* tau,
                                     void* scratch, hipStream_t s);
// Cubic build by quarter-turn orbits, the taps read from a box of the padded
// coefficient pair staged per tile in LDS (float32 columns); scratch of
// build_orbit_scratch_bytes(K, N, n) bytes.
bool build_cubic_orbit_supported(int n, int K, int N);
hipError_t launch_build_cubic_orbit(const float* pairs, int K, const ColGeom* geo, int n, int N,
                                    int64_t M, float* A32, double* tau, void* scratch, int mode,
                                    const float* colscale, hipStream_t s);
// 16-bit cubic storage built by the same orbits (N % 8 == 0), slots as
// launch_build_orbit16's; scratch of build_orbit_scratch_bytes(K, N, n) bytes.
bool build_cubic_orbit16_supported(int n, int K, int N);
hipError_t launch_build_cubic_orbit16(int storage, const float* pairs, int K, const ColGeom* geo,
                                      int n, int N, int64_t M, int32_t* perm, int32_t* eslot,
                                      int32_t* slot_of, void* lib, double* tau, void* scratch,
                                      const float* colscale, hipStream_t s);
hipError_t launch_build(int storage, const float* pairs, const ColGeom* geo, int n, int64_t M,
                        int64_t ncols, int64_t ncols_pad, void* lib, double* tau, hipStream_t s);
bool build_lds_supported(int n, int K, int N);
// scratch of launch_build_lds for an N x N scene
size_t build_lds_scratch_bytes(int K, int N, int n);
// Columns grouped by radial bracket on the device: order[] lists the columns
// bucket by bucket (bucket k = bracket k, the last bucket = zero columns);
// items[t] = (bucket, first position in order, length <= kLdsCols, 0) for
// t < *nitems <= items_max.
struct BucketPlan {
  const int32_t* order;
  const int4* items;
  const int32_t* nitems;
  int64_t items_max;
  int nb;
};
size_t bucket_scratch_bytes(int K, int64_t ncols);
hipError_t launch_bucket_sort(const ColGeom* geo, int64_t ncols, int K, void* scratch,
                              BucketPlan* plan, hipStream_t s);
// float32 columns (A32[j*M + i]) and their float64 sums: the rotation-orbit
// build (the pair in LDS, or a staged box of it per tile), else columns in
// bracket order with the pair in LDS
hipError_t launch_build_lds(const float* cube, int K, const ColGeom* geo, int n, int N, int64_t M,
                            float* A32, double* tau, void* scratch, hipStream_t s);
// 16-bit storage built by rotation orbits (N % 8 == 0; the pair, or a box of
// it per tile, and the unit tiles in LDS):
// slot 32 (s/8) + 8 k + s%8 holds member k of the s-th base column in
// bracket order (perm, slot_of, eslot written here); column sums in tau.
bool build_orbit16_supported(int n, int K, int N);
size_t build_orbit_scratch_bytes(int K, int N, int n);
hipError_t launch_build_orbit16(int storage, const float* cube, int K, const ColGeom* geo, int n,
                                int N, int64_t M, int32_t* perm, int32_t* eslot, int32_t* slot_of,
                                void* lib, double* tau, void* scratch, const float* colscale,
                                hipStream_t s);
// 16-bit storage built directly (bilinear rotation, no column rescale, the
// pair and a 16-bit tile in LDS): columns ordered by radial bracket (perm,
// slot_of, eslot written here, exps per column given), mantissas written as
// whole 8-slot groups; column sums in tau.
bool build_lds16_supported(int n, int K, int64_t ncols);
size_t build_lds16_scratch_bytes(int K, int64_t ncols);
hipError_t launch_build_lds16(int storage, const float* cube, int K, const ColGeom* geo, int n,
                              int64_t M, int64_t ncols, int64_t ncols_pad, const int32_t* exps,
                              int32_t* perm, int32_t* eslot, int32_t* slot_of, void* lib,
                              double* tau, void* scratch, hipStream_t s);
// 16-bit storage from float32 columns with the exponents in geo
hipError_t launch_pack16(int storage, const float* A32, const ColGeom* geo, int64_t M,
                         int64_t ncols, int64_t ncols_pad, void* lib, hipStream_t s);
// the same for groups [g0, g1), column j of the source at A32 + (j - col0) M
hipError_t launch_pack16_range(int storage, const float* A32, int64_t col0, int64_t g0, int64_t g1,
                               const ColGeom* geo, int64_t M, int64_t ncols, void* lib,
                               hipStream_t s);
// Flux-preserving rescale of float32 columns: sums[k] = sum(P_k) (float64),
// column j scaled by t_j / tau_j, tau_j recomputed; with want_exp the 16-bit
// exponents (geo[j].e and exps[j]) follow the rescaled bound.
hipError_t launch_psf_sums(const float* cube, int K, int64_t M, double* sums, hipStream_t s);
// Per-column flux scales (and, with want_exp, exponents) from the plain
// build's column sums, for the orbit builds' scaled pass.
hipError_t launch_flux_scale(ColGeom* geo, int K, const double* sums, const float* pmax,
                             int64_t ncols, const double* tau, float* colscale, int32_t* exps,
                             bool want_exp, hipStream_t s);
hipError_t launch_flux_rescale(float* A32, ColGeom* geo, int K, const double* sums,
                               const float* pmax, int64_t M, int64_t ncols, double* tau,
                               int32_t* exps, bool want_exp, hipStream_t s);
hipError_t launch_matvec(int storage, const void* lib, const Cols16& cx, const float* Z,
                         int64_t M, int64_t ncols, int64_t ncols_pad, float* partial, float* out,
                         hipStream_t s);
int64_t matvec_partial_floats(int storage, int64_t M, int64_t ncols, int64_t ncols_pad);
hipError_t launch_adjoint(int storage, const void* lib, const Cols16& cx, const float* g,
                          int64_t M, int64_t ncols, int64_t ncols_pad, float* partial, float* out,
                          hipStream_t s);
int64_t adjoint_partial_floats(int storage, int64_t M, int64_t ncols, int64_t ncols_pad);
hipError_t launch_batched(int storage, const void* lib, const Cols16& cx, const float* Z,
                          float* out, int64_t M, int64_t ncols, int64_t ncols_pad, int B,
                          void* scratch, size_t scratch_bytes, hipStream_t s);
size_t batched_scratch_bytes(int storage, int64_t M, int64_t ncols, int64_t ncols_pad, int B);
hipError_t launch_get_columns(int storage, const void* lib, const Cols16& cx,
                              const int32_t* cols, int count, int64_t M, int64_t ncols,
                              float* out, hipStream_t s);
hipError_t launch_render_disk(int N, double S, double rmax, const double* theta, float* Z,
                              hipStream_t s);
size_t render_disk_grad_scratch_bytes(int N);
size_t chi2_scratch_bytes(int64_t M);
hipError_t launch_chi2(int64_t M, double K, const float* S, const double* D, const double* var,
                       double* loss, float* grad, void* scratch, hipStream_t s);
hipError_t launch_render_disk_grad(int N, double S, double rmax, const double* theta,
                                   const float* dZ, double* dtheta, void* scratch, hipStream_t s);
// Measurement probes (probe.hip): a 16-byte-load read stream over `bytes`
// of `buf` (unroll 4, 8 or 16 loads in flight per thread; grid-stride, or one
// contiguous slice per workgroup), and chains of
// independent MFMAs (kind 0 FP32 32x32x2, 1 BF16 32x32x16, 2 FP16 32x32x16;
// 4 waves per workgroup, 4 chains per wave); `sink` holds >= workgroups
// floats and is written only for an impossible value.
hipError_t launch_probe_hbm_read(const void* buf, size_t bytes, int workgroups, int unroll,
                                 bool slice, float* sink, hipStream_t s);
hipError_t launch_probe_mfma(int kind, int iters, int workgroups, float* sink, hipStream_t s);
hipError_t launch_export_geometry(const ColGeom* geo, int64_t ncols, double* geom, int32_t* k,
                                  hipStream_t s);

}  // namespace psflib
