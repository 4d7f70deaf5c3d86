// C ABI of psflib: argument validation, the library layout, the handle and
// its workspace, and dispatch to the kernels.  Every argument is checked
// before anything is enqueued, so a failed call leaves the stream untouched.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "psflib_internal.h"

struct psflib_handle {
  psflib_desc desc;
  psflib::Layout L;
  int device;
  void* lib;            // caller-owned library buffer
  void* ws;             // device workspace (owned, from the library's pool)
  psflib::ColGeom* geo;
  double* radii_dev;
  float* pmax;
  std::vector<double> radii;  // host copy (source of the radii upload)
  // streams that used the workspace (the build, geometry exports)
  mutable psflib::StreamUses ws_uses;
};

namespace {

thread_local std::string g_last_error;

psflib_status fail(psflib_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

psflib_status device_fail(hipError_t e, const char* what) {
  return fail(PSFLIB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
// Kernels read and write caller arrays with 16-byte vector accesses where the
// sizes allow; every device array passed in must therefore be 16-byte aligned.
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Stream-ordered device memory (the handle's workspace, build temporaries,
// packed scenes, K-split partial images) comes from a memory pool the library
// owns, one per device, which keeps freed blocks for reuse: after the first
// call of a given size no call pays for a fresh device allocation.  The pools
// live until the process ends.
struct DevicePool {
  hipMemPool_t pool = nullptr;
  hipStream_t release = nullptr;  // internal stream for pool_release
};

std::mutex g_pool_mu;
std::map<int, DevicePool> g_pools;

hipError_t device_pool(int dev, DevicePool** out) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  auto it = g_pools.find(dev);
  if (it != g_pools.end()) {
    *out = &it->second;
    return hipSuccess;
  }
  hipMemPoolProps props;
  memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  DevicePool dp;
  hipError_t e = hipMemPoolCreate(&dp.pool, &props);
  if (e != hipSuccess) return e;
  uint64_t keep = ~(uint64_t)0;
  e = hipMemPoolSetAttribute(dp.pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) {
    (void)hipMemPoolDestroy(dp.pool);
    return e;
  }
  *out = &(g_pools[dev] = dp);
  return hipSuccess;
}

constexpr int32_t kMaxN = 8192;   // image side: n^2 rows fit comfortably in 32-bit pixel indices
constexpr int32_t kMaxScene = 46340;  // scene side: N^2 < 2^31 columns

psflib_status check_desc(const psflib_desc* d) {
  if (!d) return fail(PSFLIB_ERR_INVALID_ARG, "desc is NULL");
  if (d->n < 1 || d->n > kMaxN) return fail(PSFLIB_ERR_INVALID_ARG, "n must be in [1, 8192]");
  if (d->N < 1 || d->N > kMaxScene) return fail(PSFLIB_ERR_INVALID_ARG, "N must be in [1, 46340]");
  if (d->n_psf < 1) return fail(PSFLIB_ERR_INVALID_ARG, "n_psf must be >= 1");
  if (!(d->scene_pixscale > 0.0) || !isfinite(d->scene_pixscale))
    return fail(PSFLIB_ERR_INVALID_ARG, "scene_pixscale must be finite and > 0");
  if (d->interp != PSFLIB_INTERP_LINEAR && d->interp != PSFLIB_INTERP_NEAREST)
    return fail(PSFLIB_ERR_INVALID_ARG, "unknown interp");
  if (d->oob != PSFLIB_OOB_CLAMP && d->oob != PSFLIB_OOB_ZERO)
    return fail(PSFLIB_ERR_INVALID_ARG, "unknown oob mode");
  if (d->storage != PSFLIB_FP32 && d->storage != PSFLIB_BF16_POW2 && d->storage != PSFLIB_FP16_POW2)
    return fail(PSFLIB_ERR_INVALID_ARG, "unknown storage");
  if (d->rotate != PSFLIB_ROTATE_BILINEAR && d->rotate != PSFLIB_ROTATE_CUBIC)
    return fail(PSFLIB_ERR_INVALID_ARG, "unknown rotate mode");
  if (d->flux != PSFLIB_FLUX_NONE && d->flux != PSFLIB_FLUX_PRESERVE)
    return fail(PSFLIB_ERR_INVALID_ARG, "unknown flux mode");
  return PSFLIB_OK;
}

psflib_status check_handle(const psflib_handle* h) {
  if (!h) return fail(PSFLIB_ERR_INVALID_ARG, "handle is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev != h->device)
    return fail(PSFLIB_ERR_INVALID_ARG, "current device differs from the device the library was built on");
  return PSFLIB_OK;
}

}  // namespace

namespace psflib {

psflib_status fail_status(psflib_status s, const char* msg) { return fail(s, msg); }
psflib_status device_fail_status(hipError_t e, const char* what) { return device_fail(e, what); }

psflib_status check_pending_error() {
  // hipErrorNotReady only says that queried work is still running
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess || e == hipErrorNotReady) return PSFLIB_OK;
  return device_fail(e, "HIP error pending from earlier work");
}

hipError_t pool_alloc(void** p, size_t bytes, int dev, hipStream_t s) {
  DevicePool* dp = nullptr;
  hipError_t e = device_pool(dev, &dp);
  if (e != hipSuccess) return e;
  return hipMallocFromPoolAsync(p, bytes, dp->pool, s);
}

hipError_t pool_release(void* p, int dev) {
  if (!p) return hipSuccess;
  DevicePool* dp = nullptr;
  hipError_t e = device_pool(dev, &dp);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (!dp->release) {
      e = hipStreamCreateWithFlags(&dp->release, hipStreamNonBlocking);
      if (e != hipSuccess) {
        dp->release = nullptr;
        return e;
      }
    }
  }
  return hipFreeAsync(p, dp->release);
}

hipError_t StreamUses::note(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusNone) return hipSuccess;
  std::lock_guard<std::mutex> lock(mu_);
  for (auto& se : ev_)
    if (se.first == s) return hipEventRecord(se.second, s);
  hipEvent_t ev;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  ev_.emplace_back(s, ev);
  return hipEventRecord(ev, s);
}

void StreamUses::wait_all() {
  std::lock_guard<std::mutex> lock(mu_);
  for (auto& se : ev_) {
    (void)hipEventSynchronize(se.second);
    (void)hipEventDestroy(se.second);
  }
  ev_.clear();
}

StreamUses::~StreamUses() { wait_all(); }

Cols16 cols16_of(const psflib_handle* h) {
  Cols16 cx = {nullptr, nullptr, nullptr, nullptr};
  if (h->desc.storage == PSFLIB_FP32) return cx;
  const char* lib = reinterpret_cast<const char*>(h->lib);
  cx.exps = reinterpret_cast<const int32_t*>(lib + h->L.off_exp);
  cx.perm = reinterpret_cast<const int32_t*>(lib + h->L.off_perm);
  cx.eslot = reinterpret_cast<const int32_t*>(lib + h->L.off_eslot);
  cx.slot_of = reinterpret_cast<const int32_t*>(lib + h->L.off_slot);
  return cx;
}

void handle_info(const psflib_handle* h, const void** A, Cols16* cx, int64_t* M,
                 int64_t* ncols, int64_t* ncols_pad, int* storage, int* device) {
  *A = h->lib;
  *cx = cols16_of(h);
  *M = h->L.M;
  *ncols = h->L.ncols;
  *ncols_pad = h->L.ncols_pad;
  *storage = h->desc.storage;
  *device = h->device;
}

bool compute_layout(const psflib_desc& d, Layout* L) {
  const int64_t M = (int64_t)d.n * d.n;
  const int64_t ncols = (int64_t)d.N * d.N;
  const int64_t ncols_pad =
      (d.storage == PSFLIB_FP32) ? ncols : ((ncols + kColPad - 1) / kColPad) * kColPad;
  const int64_t esize = (d.storage == PSFLIB_FP32) ? 4 : 2;
  // M <= 2^26 and ncols_pad < 2^31 + 64: the product stays below 2^60.
  const unsigned __int128 mat = (unsigned __int128)M * (unsigned __int128)ncols_pad * esize;
  if (mat > ((unsigned __int128)1 << 62)) return false;
  size_t off = align256((size_t)mat);
  L->M = M;
  L->ncols = ncols;
  L->ncols_pad = ncols_pad;
  L->off_tau = off;
  off = align256(off + (size_t)ncols * 8);
  L->off_exp = L->off_perm = L->off_eslot = L->off_slot = off;
  if (d.storage != PSFLIB_FP32) {
    off = align256(off + (size_t)ncols_pad * 4);  // exponent per column
    L->off_perm = off;
    off = align256(off + (size_t)ncols_pad * 4);  // slot -> column
    L->off_eslot = off;
    off = align256(off + (size_t)ncols_pad * 4);  // exponent per slot
    L->off_slot = off;
    off = align256(off + (size_t)ncols * 4);      // column -> slot
  }
  L->total = off;
  return L->total <= ((size_t)1 << 62);
}

}  // namespace psflib

extern "C" {

const char* psflib_status_string(psflib_status s) {
  // C callers may pass any int: read the bits as an int rather than load an
  // enumeration value outside the enumeration's range
  int v;
  memcpy(&v, &s, sizeof(v));
  switch (v) {
    case PSFLIB_OK: return "PSFLIB_OK";
    case PSFLIB_ERR_INVALID_ARG: return "PSFLIB_ERR_INVALID_ARG";
    case PSFLIB_ERR_RADII: return "PSFLIB_ERR_RADII";
    case PSFLIB_ERR_SIZE: return "PSFLIB_ERR_SIZE";
    case PSFLIB_ERR_UNSUPPORTED: return "PSFLIB_ERR_UNSUPPORTED";
    case PSFLIB_ERR_DEVICE: return "PSFLIB_ERR_DEVICE";
  }
  return "PSFLIB_ERR_UNKNOWN";
}

const char* psflib_last_error(void) { return g_last_error.c_str(); }

psflib_status psflib_library_bytes(const psflib_desc* desc, size_t* bytes) {
  psflib_status st = check_desc(desc);
  if (st != PSFLIB_OK) return st;
  if (!bytes) return fail(PSFLIB_ERR_INVALID_ARG, "bytes is NULL");
  psflib::Layout L;
  if (!psflib::compute_layout(*desc, &L)) return fail(PSFLIB_ERR_SIZE, "library size exceeds 2^62 bytes");
  *bytes = L.total;
  return PSFLIB_OK;
}

psflib_status psflib_build(const psflib_desc* desc, const float* d_cube, const double* h_radii,
                           void* d_lib, size_t lib_bytes, void* stream, psflib_handle** out) {
  psflib_status st = check_desc(desc);
  if (st != PSFLIB_OK) return st;
  if (!d_cube || !h_radii || !d_lib || !out)
    return fail(PSFLIB_ERR_INVALID_ARG, "d_cube, h_radii, d_lib and out must be non-NULL");
  if (((uintptr_t)d_lib & 255u) != 0) return fail(PSFLIB_ERR_INVALID_ARG, "d_lib must be 256-byte aligned");
  if (!aligned16(d_cube)) return fail(PSFLIB_ERR_INVALID_ARG, "d_cube must be 16-byte aligned");
  const int K = desc->n_psf;
  for (int k = 0; k < K; ++k) {
    if (!isfinite(h_radii[k])) return fail(PSFLIB_ERR_RADII, "radii must be finite");
    if (k > 0 && !(h_radii[k] > h_radii[k - 1]))
      return fail(PSFLIB_ERR_RADII, "radii must be strictly increasing");
  }
  psflib::Layout L;
  if (!psflib::compute_layout(*desc, &L)) return fail(PSFLIB_ERR_SIZE, "library size exceeds 2^62 bytes");
  if (lib_bytes < L.total)
    return fail(PSFLIB_ERR_SIZE, "library buffer too small: need " + std::to_string(L.total) +
                                     " bytes, got " + std::to_string(lib_bytes));
  const int storage = desc->storage;

  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;

  psflib_handle* h = new (std::nothrow) psflib_handle();
  if (!h) return fail(PSFLIB_ERR_DEVICE, "host allocation failed");
  h->desc = *desc;
  h->L = L;
  h->device = dev;
  h->lib = d_lib;
  h->radii.assign(h_radii, h_radii + K);

  // Workspace: radii | pmax | per-column geometry.
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  size_t off = 0;
  const size_t off_radii = off; off = align256(off + (size_t)K * 8);
  const size_t off_pmax = off;  off = align256(off + (size_t)K * 4);
  const size_t off_geo = off;   off = align256(off + (size_t)L.ncols_pad * sizeof(psflib::ColGeom));
  e = psflib::pool_alloc(&h->ws, off, dev, s);
  if (e != hipSuccess) {
    delete h;
    return device_fail(e, "workspace allocation");
  }
  char* ws = reinterpret_cast<char*>(h->ws);
  h->radii_dev = reinterpret_cast<double*>(ws + off_radii);
  h->pmax = reinterpret_cast<float*>(ws + off_pmax);
  h->geo = reinterpret_cast<psflib::ColGeom*>(ws + off_geo);

  char* lib = reinterpret_cast<char*>(d_lib);
  double* tau = reinterpret_cast<double*>(lib + L.off_tau);
  int32_t* exps = (storage == PSFLIB_FP32) ? nullptr : reinterpret_cast<int32_t*>(lib + L.off_exp);
  // Cubic-spline rotation: spline coefficients of the cube, then the
  // quarter-turn orbit build with a box of the coefficient pair staged per
  // tile.  Bilinear: the bucketed LDS build, the pair staged whole when it
  // fits the LDS, else a box of it per tile, read by the rotation-orbit
  // builds.  The gathers from pair-interleaved copies serve what those cannot
  // (bracket or column counts beyond the sort's bounds), and the 16-bit
  // libraries of PSFs larger than 256 x 256 whose scene side is not a
  // multiple of 8 (no rescale), which they write directly where the orbit
  // builds would stage a float32 copy.  The builds write float32 columns when
  // the flux-preserving rescale follows, or when a 16-bit library cannot be
  // written directly; the 16-bit forms then pack those columns in a last pass.
  const bool cubic = desc->rotate == PSFLIB_ROTATE_CUBIC;
  const bool flux = desc->flux == PSFLIB_FLUX_PRESERVE;
  const bool big16 = desc->n > 256 && storage != PSFLIB_FP32 && !flux && desc->N % 8 != 0;
  const bool lds = !big16 && (cubic ? psflib::build_cubic_orbit_supported(desc->n, K, desc->N)
                                    : psflib::build_lds_supported(desc->n, K, desc->N));
  // Flux-preserving orbit builds take two passes (the plain build's column
  // sums, then the build with each column scaled as it is stored) instead of
  // rewriting the library.  16-bit libraries are written directly in bracket
  // order: by quarter-turn orbits when N is a multiple of 8 (bilinear or
  // cubic, rescaled or not), else (bilinear, not rescaled) column by column
  // when the pair fits the LDS; the other 16-bit builds go through float32
  // columns and a packing pass (natural order)
  const bool flux_orbit =
      flux && lds && (cubic || psflib::build_orbit_flux_supported(desc->n, K, desc->N));
  const bool plain16 = storage != PSFLIB_FP32 && lds && (!flux || flux_orbit);
  const bool orbit16 = plain16 && (cubic ? psflib::build_cubic_orbit16_supported(desc->n, K, desc->N)
                                         : psflib::build_orbit16_supported(desc->n, K, desc->N));
  const bool direct16 =
      orbit16 || (plain16 && !flux && !cubic && psflib::build_lds16_supported(desc->n, K, L.ncols));
  const bool stage32 = storage != PSFLIB_FP32 && (lds || flux) && !direct16;
  const size_t spline_bytes = cubic ? align256(psflib::spline_scratch_bytes(K, desc->n)) : 0;
  const size_t path_bytes =
      spline_bytes + align256(orbit16 || flux_orbit ? psflib::build_orbit_scratch_bytes(K, desc->N, desc->n)
                              : direct16 ? psflib::build_lds16_scratch_bytes(K, L.ncols)
                              : cubic && lds ? psflib::build_orbit_scratch_bytes(K, desc->N, desc->n)
                              : lds    ? psflib::build_lds_scratch_bytes(K, desc->N, desc->n)
                              : cubic  ? 0
                                       : (size_t)((K > 1) ? (K - 1) : 1) * (size_t)L.M * 8);
  const size_t stage_bytes = align256(stage32 ? (size_t)L.ncols * (size_t)L.M * 4 : 0);
  const size_t sums_bytes =
      align256(flux ? (size_t)K * 8 : 0) + align256(flux_orbit ? (size_t)L.ncols * 4 : 0);
  const size_t tmp_bytes = path_bytes + stage_bytes + sums_bytes;
  void* tmp = nullptr;
  // on failure: wait for what this build enqueued (on its own stream), then
  // release its memory
  auto bail = [&](hipError_t err, const char* what) {
    psflib_status r = device_fail(err, what);
    if (tmp) (void)hipFreeAsync(tmp, s);
    (void)hipStreamSynchronize(s);
    (void)psflib::pool_release(h->ws, dev);
    delete h;
    return r;
  };
  e = hipMemcpyAsync(h->radii_dev, h->radii.data(), (size_t)K * 8, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return bail(e, "hipMemcpyAsync(radii)");
  e = psflib::pool_alloc(&tmp, tmp_bytes, dev, s);
  if (e != hipSuccess) { tmp = nullptr; return bail(e, "scratch allocation (build)"); }
  char* tp = reinterpret_cast<char*>(tmp);
  void* path_tmp = tp;
  float* A32 = stage32 ? reinterpret_cast<float*>(tp + path_bytes) : reinterpret_cast<float*>(d_lib);
  double* sums = flux ? reinterpret_cast<double*>(tp + path_bytes + stage_bytes) : nullptr;
  float* colscale = flux_orbit ? reinterpret_cast<float*>(tp + path_bytes + stage_bytes +
                                                          align256((size_t)K * 8))
                               : nullptr;
  // the format the build kernel writes, and where
  const int bstore = stage32 ? PSFLIB_FP32 : storage;
  void* bdst = stage32 ? reinterpret_cast<void*>(A32) : d_lib;
  if (cubic) {
    // the 16-bit exponent bound takes the largest |coefficient| per PSF
    e = psflib::launch_spline_pairs(d_cube, K, desc->n, path_tmp,
                                    storage != PSFLIB_FP32 ? h->pmax : nullptr, s);
    if (e != hipSuccess) return bail(e, "spline coefficient kernels");
  } else if (storage != PSFLIB_FP32) {
    e = psflib::launch_cube_max(d_cube, K, L.M, h->pmax, s);
    if (e != hipSuccess) return bail(e, "cube_max kernel");
  }
  e = psflib::launch_geometry(desc->N, desc->scene_pixscale, h->radii_dev, K, desc->interp,
                              desc->oob, h->pmax, storage != PSFLIB_FP32, h->geo, L.ncols_pad,
                              exps, s);
  if (e != hipSuccess) return bail(e, "geometry kernel");
  const float* cpairs = cubic ? psflib::spline_pairs_of(path_tmp, K, desc->n) : nullptr;
  void* otmp = tp + spline_bytes;  // the orbit builds' scratch
  int32_t* perm = reinterpret_cast<int32_t*>(lib + L.off_perm);
  int32_t* eslot = reinterpret_cast<int32_t*>(lib + L.off_eslot);
  int32_t* slot_of = reinterpret_cast<int32_t*>(lib + L.off_slot);
  if (flux_orbit) {
    // pass 1: the plain build's column sums, nothing stored
    e = psflib::launch_psf_sums(d_cube, K, L.M, sums, s);
    if (e != hipSuccess) return bail(e, "psf sums kernel");
    float* none = reinterpret_cast<float*>(d_lib);  // not written in this pass
    e = cubic ? psflib::launch_build_cubic_orbit(cpairs, K, h->geo, desc->n, desc->N, L.M, none, tau,
                                                 otmp, psflib::kOrbitSumsOnly, nullptr, s)
              : psflib::launch_build_orbit_sums(d_cube, K, h->geo, desc->n, desc->N, L.M, none, tau,
                                                otmp, s);
    if (e != hipSuccess) return bail(e, "flux column-sum pass");
    e = psflib::launch_flux_scale(h->geo, K, sums, h->pmax, L.ncols, tau, colscale, exps,
                                  storage != PSFLIB_FP32, s);
    if (e != hipSuccess) return bail(e, "flux scale kernel");
    // pass 2: the build, each column scaled as it is stored
    if (orbit16)
      e = cubic ? psflib::launch_build_cubic_orbit16(storage, cpairs, K, h->geo, desc->n, desc->N, L.M,
                                                     perm, eslot, slot_of, d_lib, tau, otmp,
                                                     colscale, s)
                : psflib::launch_build_orbit16(storage, d_cube, K, h->geo, desc->n, desc->N, L.M,
                                               perm, eslot, slot_of, d_lib, tau, otmp, colscale, s);
    else
      e = cubic ? psflib::launch_build_cubic_orbit(cpairs, K, h->geo, desc->n, desc->N, L.M,
                                                   reinterpret_cast<float*>(bdst), tau, otmp,
                                                   psflib::kOrbitScaled, colscale, s)
                : psflib::launch_build_orbit_scaled(d_cube, K, h->geo, desc->n, desc->N, L.M, colscale,
                                                    reinterpret_cast<float*>(bdst), tau, otmp, s);
    if (e != hipSuccess) return bail(e, "flux-preserving orbit build kernels");
  } else if (cubic && orbit16) {
    e = psflib::launch_build_cubic_orbit16(storage, psflib::spline_pairs_of(path_tmp, K, desc->n), K,
                                           h->geo, desc->n, desc->N, L.M,
                                           reinterpret_cast<int32_t*>(lib + L.off_perm),
                                           reinterpret_cast<int32_t*>(lib + L.off_eslot),
                                           reinterpret_cast<int32_t*>(lib + L.off_slot), d_lib, tau,
                                           tp + spline_bytes, nullptr, s);
    if (e != hipSuccess) return bail(e, "16-bit cubic orbit build kernels");
  } else if (cubic && lds) {
    e = psflib::launch_build_cubic_orbit(psflib::spline_pairs_of(path_tmp, K, desc->n), K, h->geo,
                                         desc->n, desc->N, L.M, reinterpret_cast<float*>(bdst), tau,
                                         tp + spline_bytes, psflib::kOrbitPlain, nullptr, s);
    if (e != hipSuccess) return bail(e, "cubic orbit build kernels");
  } else if (cubic) {
    e = psflib::launch_build_cubic(bstore, psflib::spline_pairs_of(path_tmp, K, desc->n), h->geo,
                                   desc->n, L.M, L.ncols, L.ncols_pad, bdst, tau, s);
    if (e != hipSuccess) return bail(e, "cubic build kernel");
  } else if (orbit16) {
    e = psflib::launch_build_orbit16(storage, d_cube, K, h->geo, desc->n, desc->N, L.M,
                                     reinterpret_cast<int32_t*>(lib + L.off_perm),
                                     reinterpret_cast<int32_t*>(lib + L.off_eslot),
                                     reinterpret_cast<int32_t*>(lib + L.off_slot), d_lib, tau,
                                     path_tmp, nullptr, s);
    if (e != hipSuccess) return bail(e, "16-bit orbit build kernels");
  } else if (direct16) {
    e = psflib::launch_build_lds16(storage, d_cube, K, h->geo, desc->n, L.M, L.ncols, L.ncols_pad,
                                   exps, reinterpret_cast<int32_t*>(lib + L.off_perm),
                                   reinterpret_cast<int32_t*>(lib + L.off_eslot),
                                   reinterpret_cast<int32_t*>(lib + L.off_slot), d_lib, tau,
                                   path_tmp, s);
    if (e != hipSuccess) return bail(e, "16-bit LDS build kernels");
  } else if (lds) {
    e = psflib::launch_build_lds(d_cube, K, h->geo, desc->n, desc->N, L.M,
                                 reinterpret_cast<float*>(bdst), tau, path_tmp, s);
    if (e != hipSuccess) return bail(e, "LDS build kernels");
  } else {
    e = psflib::launch_pair_cube(d_cube, K, L.M, reinterpret_cast<float*>(path_tmp), s);
    if (e != hipSuccess) return bail(e, "pair_cube kernel");
    e = psflib::launch_build(bstore, reinterpret_cast<const float*>(path_tmp), h->geo, desc->n,
                             L.M, L.ncols, L.ncols_pad, bdst, tau, s);
    if (e != hipSuccess) return bail(e, "build kernel");
  }
  if (flux && !flux_orbit) {
    e = psflib::launch_psf_sums(d_cube, K, L.M, sums, s);
    if (e != hipSuccess) return bail(e, "psf sums kernel");
    e = psflib::launch_flux_rescale(reinterpret_cast<float*>(bdst), h->geo, K, sums, h->pmax, L.M,
                                    L.ncols, tau, exps, storage != PSFLIB_FP32, s);
    if (e != hipSuccess) return bail(e, "flux rescale kernel");
  }
  if (stage32) {
    e = psflib::launch_pack16(storage, A32, h->geo, L.M, L.ncols, L.ncols_pad, d_lib, s);
    if (e != hipSuccess) return bail(e, "16-bit packing kernel");
  }
  if (storage != PSFLIB_FP32 && !direct16) {
    // natural column order: slot s holds column s
    e = psflib::launch_identity_order(reinterpret_cast<int32_t*>(lib + L.off_perm),
                                      reinterpret_cast<int32_t*>(lib + L.off_eslot),
                                      reinterpret_cast<int32_t*>(lib + L.off_slot), exps, L.ncols,
                                      L.ncols_pad, s);
    if (e != hipSuccess) return bail(e, "column order kernel");
  }
  e = hipFreeAsync(tmp, s);
  if (e != hipSuccess) { tmp = nullptr; return bail(e, "hipFreeAsync(build scratch)"); }
  tmp = nullptr;
  e = h->ws_uses.note(s);
  if (e != hipSuccess) return bail(e, "hipEventRecord(build)");
  *out = h;
  return PSFLIB_OK;
}

namespace {

// One split-K product (S = A Z, or G = A^T g when `adjoint`) with its
// partial sums in `partial` (at least the launcher's partial count).
hipError_t launch_product(const psflib_handle* h, bool adjoint, const float* in, float* out,
                          float* partial, hipStream_t s) {
  const psflib::Cols16 cx = psflib::cols16_of(h);
  if (adjoint)
    return psflib::launch_adjoint(h->desc.storage, h->lib, cx, in, h->L.M, h->L.ncols,
                                  h->L.ncols_pad, partial, out, s);
  return psflib::launch_matvec(h->desc.storage, h->lib, cx, in, h->L.M, h->L.ncols,
                               h->L.ncols_pad, partial, out, s);
}

// Temporary device memory of one call (split-K partial sums, packed scenes,
// reduction blocks).  Outside stream capture it is the calling stream's
// buffer: one per (device, stream), kept like the pool's blocks until the
// process ends and grown on demand.  Calls on one stream run in order, so
// every call on that stream (whatever its handle) can reuse the buffer, and
// calls on different streams never share one.  The lock is held over the
// call's launches, so a call from another host thread on the same stream
// cannot slip its kernels in between them.  This adds nothing to the stream
// per call (a stream-ordered free per call adds a marker: ~3 us between
// kernels).  Under capture the memory is allocated from the pool inside the
// graph instead, so every graph owns its own.
struct StreamBuffer {
  int dev;
  hipStream_t s;
  void* p;
  size_t bytes;
};
std::mutex g_sb_mu;
std::vector<StreamBuffer> g_sb;

class CallScratch {
 public:
  hipError_t acquire(int dev, hipStream_t s, size_t bytes) {
    s_ = s;
    if (bytes == 0) return hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusNone) {
      pooled_ = true;
      return psflib::pool_alloc(&p_, bytes, dev, s);
    }
    lock_ = std::unique_lock<std::mutex>(g_sb_mu);
    StreamBuffer* slot = nullptr;
    for (auto& sb : g_sb)
      if (sb.dev == dev && sb.s == s) slot = &sb;
    if (slot && slot->bytes >= bytes) {
      p_ = slot->p;
      return hipSuccess;
    }
    size_t want = (size_t)1 << 20;  // grow in powers of two from 1 MiB
    while (want < bytes) want <<= 1;
    e = psflib::pool_alloc(&p_, want, dev, s);
    if (e != hipSuccess) {
      p_ = nullptr;
      return e;
    }
    if (slot) {
      // the smaller buffer goes back to the pool after the work queued on s
      e = hipFreeAsync(slot->p, s);
      slot->p = p_;
      slot->bytes = want;
    } else {
      g_sb.push_back(StreamBuffer{dev, s, p_, want});
    }
    return e;
  }
  void* ptr() const { return p_; }
  // after the call's launches
  hipError_t release() {
    hipError_t e = hipSuccess;
    if (pooled_ && p_) e = hipFreeAsync(p_, s_);
    pooled_ = false;
    p_ = nullptr;
    if (lock_.owns_lock()) lock_.unlock();
    return e;
  }
  ~CallScratch() { (void)release(); }

 private:
  std::unique_lock<std::mutex> lock_;
  void* p_ = nullptr;
  bool pooled_ = false;
  hipStream_t s_ = nullptr;
};

psflib_status product(const psflib_handle* h, bool adjoint, const float* in, float* out,
                      hipStream_t s) {
  const int64_t floats =
      adjoint ? psflib::adjoint_partial_floats(h->desc.storage, h->L.M, h->L.ncols, h->L.ncols_pad)
              : psflib::matvec_partial_floats(h->desc.storage, h->L.M, h->L.ncols, h->L.ncols_pad);
  CallScratch cs;
  hipError_t e = cs.acquire(h->device, s, (size_t)floats * 4);
  if (e != hipSuccess) return device_fail(e, "partial-sum buffer");
  e = launch_product(h, adjoint, in, out, reinterpret_cast<float*>(cs.ptr()), s);
  const hipError_t e2 = cs.release();
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? PSFLIB_OK : device_fail(e, adjoint ? "adjoint kernels" : "matvec kernels");
}

}  // namespace

psflib_status psflib_apply(const psflib_handle* h, const float* d_scene, float* d_image, void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (!d_scene || !d_image) return fail(PSFLIB_ERR_INVALID_ARG, "d_scene and d_image must be non-NULL");
  if (!aligned16(d_scene) || !aligned16(d_image))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_scene and d_image must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  return product(h, false, d_scene, d_image, reinterpret_cast<hipStream_t>(stream));
}

psflib_status psflib_apply_noalloc(const psflib_handle* h, const float* d_scene, float* d_image,
                                   void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (!d_scene || !d_image) return fail(PSFLIB_ERR_INVALID_ARG, "d_scene and d_image must be non-NULL");
  if (!aligned16(d_scene) || !aligned16(d_image))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_scene and d_image must be 16-byte aligned");
  const int64_t floats =
      psflib::matvec_partial_floats(h->desc.storage, h->L.M, h->L.ncols, h->L.ncols_pad);
  if ((uint64_t)floats * 4 > psflib::kNoAllocScratchBytes)
    return fail(PSFLIB_ERR_SIZE, "psflib_apply_noalloc: this library needs " +
                                     std::to_string((uint64_t)floats * 4) +
                                     " bytes of partial sums, more than the fixed scratch of " +
                                     std::to_string(psflib::kNoAllocScratchBytes) + " bytes");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  void* part = nullptr;
  hipError_t e = psflib::noalloc_scratch(h->device, &part);
  if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress(scratch)");
  e = launch_product(h, false, d_scene, d_image, reinterpret_cast<float*>(part),
                     reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "matvec kernels");
  return PSFLIB_OK;
}

psflib_status psflib_apply_adjoint(const psflib_handle* h, const float* d_g, float* d_scene_grad,
                                   void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (!d_g || !d_scene_grad) return fail(PSFLIB_ERR_INVALID_ARG, "d_g and d_scene_grad must be non-NULL");
  if (!aligned16(d_g) || !aligned16(d_scene_grad))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_g and d_scene_grad must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  return product(h, true, d_g, d_scene_grad, reinterpret_cast<hipStream_t>(stream));
}

psflib_status psflib_apply_batched(const psflib_handle* h, const float* d_scenes, float* d_images,
                                   int32_t B, void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (B < 0) return fail(PSFLIB_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0) return PSFLIB_OK;
  if (!d_scenes || !d_images) return fail(PSFLIB_ERR_INVALID_ARG, "d_scenes and d_images must be non-NULL");
  if (!aligned16(d_scenes) || !aligned16(d_images))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_scenes and d_images must be 16-byte aligned");
  // one scene: the matvec streams the library faster than a one-scene product
  if (B == 1) return psflib_apply(h, d_scenes, d_images, stream);
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t bytes = psflib::batched_scratch_bytes(h->desc.storage, h->L.M, h->L.ncols, h->L.ncols_pad, B);
  CallScratch cs;
  hipError_t e = cs.acquire(h->device, s, bytes);
  if (e != hipSuccess) return device_fail(e, "scratch buffer (batched)");
  e = psflib::launch_batched(h->desc.storage, h->lib, psflib::cols16_of(h), d_scenes, d_images,
                             h->L.M, h->L.ncols, h->L.ncols_pad, B, cs.ptr(), bytes, s);
  const hipError_t e2 = cs.release();
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return device_fail(e, "batched kernels");
  return PSFLIB_OK;
}

psflib_status psflib_column_sums(const psflib_handle* h, double* d_tau, void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (!d_tau) return fail(PSFLIB_ERR_INVALID_ARG, "d_tau must be non-NULL");
  if (!aligned16(d_tau)) return fail(PSFLIB_ERR_INVALID_ARG, "d_tau must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  const char* lib = reinterpret_cast<const char*>(h->lib);
  hipError_t e = hipMemcpyAsync(d_tau, lib + h->L.off_tau, (size_t)h->L.ncols * 8,
                                hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "hipMemcpyAsync(tau)");
  return PSFLIB_OK;
}

psflib_status psflib_get_columns(const psflib_handle* h, const int32_t* d_cols, int32_t count,
                                 float* d_out, void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (count < 0) return fail(PSFLIB_ERR_INVALID_ARG, "count must be >= 0");
  if (count == 0) return PSFLIB_OK;
  if (count > 65535) return fail(PSFLIB_ERR_INVALID_ARG, "count must be <= 65535");
  if (!d_cols || !d_out) return fail(PSFLIB_ERR_INVALID_ARG, "d_cols and d_out must be non-NULL");
  if (!aligned16(d_cols) || !aligned16(d_out))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_cols and d_out must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipError_t e = psflib::launch_get_columns(h->desc.storage, h->lib, psflib::cols16_of(h), d_cols, count, h->L.M,
                                            h->L.ncols, d_out, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "get_columns kernel");
  return PSFLIB_OK;
}

psflib_status psflib_get_exponents(const psflib_handle* h, int32_t* d_exp, void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (h->desc.storage == PSFLIB_FP32)
    return fail(PSFLIB_ERR_UNSUPPORTED, "FP32 storage has no exponents");
  if (!d_exp) return fail(PSFLIB_ERR_INVALID_ARG, "d_exp must be non-NULL");
  if (!aligned16(d_exp)) return fail(PSFLIB_ERR_INVALID_ARG, "d_exp must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  const char* lib = reinterpret_cast<const char*>(h->lib);
  hipError_t e = hipMemcpyAsync(d_exp, lib + h->L.off_exp, (size_t)h->L.ncols * 4,
                                hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "hipMemcpyAsync(exponents)");
  return PSFLIB_OK;
}

psflib_status psflib_get_geometry(const psflib_handle* h, double* d_geom, int32_t* d_k, void* stream) {
  psflib_status st = check_handle(h);
  if (st != PSFLIB_OK) return st;
  if (!d_geom && !d_k) return PSFLIB_OK;
  if (!aligned16(d_geom) || !aligned16(d_k))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_geom and d_k must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = psflib::launch_export_geometry(h->geo, h->L.ncols, d_geom, d_k, s);
  if (e != hipSuccess) return device_fail(e, "export_geometry kernel");
  e = h->ws_uses.note(s);  // the export reads the workspace
  if (e != hipSuccess) return device_fail(e, "hipEventRecord(geometry export)");
  return PSFLIB_OK;
}

static psflib_status check_model_args(int32_t N, double S, double rmax, const void* a,
                                      const void* b) {
  if (N < 1 || N > kMaxScene) return fail(PSFLIB_ERR_INVALID_ARG, "N must be in [1, 46340]");
  if (!(S > 0.0) || !isfinite(S)) return fail(PSFLIB_ERR_INVALID_ARG, "scene_pixscale must be finite and > 0");
  if (isnan(rmax)) return fail(PSFLIB_ERR_INVALID_ARG, "rmax must not be NaN");
  if (!a || !b) return fail(PSFLIB_ERR_INVALID_ARG, "device pointers must be non-NULL");
  if (!aligned16(a) || !aligned16(b)) return fail(PSFLIB_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
  return PSFLIB_OK;
}

// psflib_render_disk_grad and psflib_chi2 are not run under stream capture
// (a captured fit chain faulted the GPU once, cause not found): refused
// before anything is enqueued.
static psflib_status refuse_capture(hipStream_t s, const char* what) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return device_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(PSFLIB_ERR_UNSUPPORTED, std::string(what) + " cannot be captured in a graph");
  return PSFLIB_OK;
}

psflib_status psflib_render_disk(int32_t N, double scene_pixscale, double rmax,
                                 const double* d_theta, float* d_scene, void* stream) {
  psflib_status st = check_model_args(N, scene_pixscale, rmax, d_theta, d_scene);
  if (st != PSFLIB_OK) return st;
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipError_t e = psflib::launch_render_disk(N, scene_pixscale, rmax, d_theta, d_scene,
                                            reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "render_disk kernel");
  return PSFLIB_OK;
}

psflib_status psflib_render_disk_grad(int32_t N, double scene_pixscale, double rmax,
                                      const double* d_theta, const float* d_dscene,
                                      double* d_dtheta, void* stream) {
  psflib_status st = check_model_args(N, scene_pixscale, rmax, d_theta, d_dscene);
  if (st != PSFLIB_OK) return st;
  if (!d_dtheta) return fail(PSFLIB_ERR_INVALID_ARG, "d_dtheta must be non-NULL");
  if (!aligned16(d_dtheta)) return fail(PSFLIB_ERR_INVALID_ARG, "d_dtheta must be 16-byte aligned");
  st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = refuse_capture(s, "psflib_render_disk_grad");
  if (st != PSFLIB_OK) return st;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  CallScratch cs;
  e = cs.acquire(dev, s, psflib::render_disk_grad_scratch_bytes(N));
  if (e != hipSuccess) return device_fail(e, "scratch buffer (disk gradient)");
  e = psflib::launch_render_disk_grad(N, scene_pixscale, rmax, d_theta, d_dscene, d_dtheta,
                                      cs.ptr(), s);
  const hipError_t e2 = cs.release();
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return device_fail(e, "render_disk_grad kernels");
  return PSFLIB_OK;
}

psflib_status psflib_chi2(int64_t M, double K, const float* d_image, const double* d_data,
                          const double* d_var, double* d_loss, float* d_grad, void* stream) {
  if (M < 1 || M > ((int64_t)1 << 36)) return fail(PSFLIB_ERR_INVALID_ARG, "M must be in [1, 2^36]");
  if (!isfinite(K)) return fail(PSFLIB_ERR_INVALID_ARG, "K must be finite");
  if (!d_image || !d_data || !d_var || !d_loss)
    return fail(PSFLIB_ERR_INVALID_ARG, "d_image, d_data, d_var and d_loss must be non-NULL");
  if (!aligned16(d_image) || !aligned16(d_data) || !aligned16(d_var) || !aligned16(d_loss) ||
      (d_grad && !aligned16(d_grad)))
    return fail(PSFLIB_ERR_INVALID_ARG, "device arrays must be 16-byte aligned");
  psflib_status st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = refuse_capture(s, "psflib_chi2");
  if (st != PSFLIB_OK) return st;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  CallScratch cs;
  e = cs.acquire(dev, s, psflib::chi2_scratch_bytes(M));
  if (e != hipSuccess) return device_fail(e, "scratch buffer (chi-square)");
  e = psflib::launch_chi2(M, K, d_image, d_data, d_var, d_loss, d_grad, cs.ptr(), s);
  const hipError_t e2 = cs.release();
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return device_fail(e, "chi-square kernels");
  return PSFLIB_OK;
}

psflib_status psflib_probe_hbm_read(const void* d_buf, size_t bytes, int32_t workgroups,
                                    int32_t unroll, int32_t slice, float* d_sink, void* stream) {
  if (!d_buf || !d_sink) return fail(PSFLIB_ERR_INVALID_ARG, "d_buf and d_sink must be non-NULL");
  if (!aligned16(d_buf) || !aligned16(d_sink))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_buf and d_sink must be 16-byte aligned");
  if (workgroups < 1 || workgroups > 65536)
    return fail(PSFLIB_ERR_INVALID_ARG, "workgroups must be in [1, 65536]");
  if (unroll != 4 && unroll != 8 && unroll != 16)
    return fail(PSFLIB_ERR_INVALID_ARG, "unroll must be 4, 8 or 16");
  psflib_status st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipError_t e = psflib::launch_probe_hbm_read(d_buf, bytes, workgroups, unroll, slice != 0,
                                               d_sink, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "HBM read probe");
  return PSFLIB_OK;
}

psflib_status psflib_probe_mfma(int32_t kind, int32_t iters, int32_t workgroups, float* d_sink,
                                void* stream) {
  if (kind < 0 || kind > 2) return fail(PSFLIB_ERR_INVALID_ARG, "kind must be 0, 1 or 2");
  if (iters < 1) return fail(PSFLIB_ERR_INVALID_ARG, "iters must be >= 1");
  if (workgroups < 1 || workgroups > 65536)
    return fail(PSFLIB_ERR_INVALID_ARG, "workgroups must be in [1, 65536]");
  if (!d_sink || !aligned16(d_sink))
    return fail(PSFLIB_ERR_INVALID_ARG, "d_sink must be non-NULL and 16-byte aligned");
  psflib_status st = psflib::check_pending_error();
  if (st != PSFLIB_OK) return st;
  hipError_t e = psflib::launch_probe_mfma(kind, iters, workgroups, d_sink,
                                           reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "MFMA probe");
  return PSFLIB_OK;
}

void psflib_destroy(psflib_handle* h) {
  if (!h) return;
  // wait for this handle's own uses of its workspace (not for the device)
  h->ws_uses.wait_all();
  (void)psflib::pool_release(h->ws, h->device);
  delete h;
}

}  // extern "C"
