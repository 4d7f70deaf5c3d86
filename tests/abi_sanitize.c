/* Host-side driver for the sanitizer build of the C ABI (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code only).  Every call below fails
 * validation before any device work -- a NULL handle, a NULL, misaligned or
 * undersized buffer, a bad enum, bad radii -- or touches no device at all, so
 * the driver never reaches a GPU and runs the same with or without one.  It
 * exercises the argument checks, the layout arithmetic (including sizes near
 * the 2^62 limit) and the error-message paths. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "psflib.h"

static int failures = 0;

#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static psflib_desc desc(int32_t n, int32_t K, int32_t N, int32_t storage) {
  psflib_desc d;
  memset(&d, 0, sizeof(d));
  d.n = n;
  d.n_psf = K;
  d.N = N;
  d.interp = PSFLIB_INTERP_LINEAR;
  d.scene_pixscale = 0.5;
  d.oob = PSFLIB_OOB_CLAMP;
  d.storage = storage;
  d.rotate = PSFLIB_ROTATE_BILINEAR;
  d.flux = PSFLIB_FLUX_NONE;
  return d;
}

int main(void) {
  /* never dereferenced: every call using them fails validation first */
  void* fake = (void*)(uintptr_t)(1u << 20);
  void* fake_odd = (void*)((uintptr_t)(1u << 20) + 4);
  float sink_host[4];

  for (int s = -1; s <= 6; ++s) EXPECT(psflib_status_string((psflib_status)s) != NULL);
  EXPECT(psflib_last_error() != NULL);

  /* sizes: valid layouts, every storage form, the extremes */
  size_t bytes = 0;
  for (int st = 0; st < 3; ++st) {
    psflib_desc d = desc(128, 64, 128, st);
    EXPECT(psflib_library_bytes(&d, &bytes) == PSFLIB_OK && bytes > (size_t)128 * 128 * 128 * 128);
    d = desc(1, 1, 1, st);
    EXPECT(psflib_library_bytes(&d, &bytes) == PSFLIB_OK && bytes > 0);
    d = desc(8192, 2, 46340, st);
    EXPECT(psflib_library_bytes(&d, &bytes) == PSFLIB_OK);
  }
  psflib_desc d = desc(16, 3, 16, PSFLIB_FP32);
  EXPECT(psflib_library_bytes(NULL, &bytes) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_library_bytes(&d, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(strlen(psflib_last_error()) > 0);
  {
    psflib_desc b = d; b.n = 0;            EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.n = 8193;                     EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.N = 46341;                    EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.n_psf = 0;                    EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.scene_pixscale = NAN;         EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.scene_pixscale = -1.0;        EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.scene_pixscale = INFINITY;    EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.interp = 9;                   EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.oob = -3;                     EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.storage = 7;                  EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.rotate = 5;                   EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
    b = d; b.flux = 2;                     EXPECT(psflib_library_bytes(&b, &bytes) == PSFLIB_ERR_INVALID_ARG);
  }

  /* build: argument checks, then radii, then the buffer size */
  size_t need = 0;
  EXPECT(psflib_library_bytes(&d, &need) == PSFLIB_OK);
  double good[3] = {0.0, 1.0, 2.0}, dup[3] = {0.0, 1.0, 1.0}, dec[3] = {0.0, 2.0, 1.0};
  double nan3[3] = {0.0, NAN, 2.0}, inf3[3] = {0.0, 1.0, INFINITY};
  psflib_handle* h = NULL;
  EXPECT(psflib_build(NULL, fake, good, fake, need, NULL, &h) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, NULL, good, fake, need, NULL, &h) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, fake, NULL, fake, need, NULL, &h) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, fake, good, NULL, need, NULL, &h) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, fake, good, fake, need, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, fake, good, fake_odd, need, NULL, &h) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, fake_odd, good, fake, need, NULL, &h) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_build(&d, fake, dup, fake, need, NULL, &h) == PSFLIB_ERR_RADII);
  EXPECT(psflib_build(&d, fake, dec, fake, need, NULL, &h) == PSFLIB_ERR_RADII);
  EXPECT(psflib_build(&d, fake, nan3, fake, need, NULL, &h) == PSFLIB_ERR_RADII);
  EXPECT(psflib_build(&d, fake, inf3, fake, need, NULL, &h) == PSFLIB_ERR_RADII);
  EXPECT(psflib_build(&d, fake, good, fake, need - 1, NULL, &h) == PSFLIB_ERR_SIZE);
  EXPECT(strstr(psflib_last_error(), "too small") != NULL);
  EXPECT(h == NULL);

  /* calls on a NULL handle */
  EXPECT(psflib_apply(NULL, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_apply_noalloc(NULL, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_apply_adjoint(NULL, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_apply_batched(NULL, fake, fake, 3, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_column_sums(NULL, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_get_columns(NULL, fake, 1, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_get_exponents(NULL, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_get_geometry(NULL, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  psflib_destroy(NULL);

  /* grouped plans */
  psflib_grouped* g = NULL;
  const psflib_handle* libs[1] = {NULL};
  int32_t los[1] = {0};
  const float* sc[1] = {(const float*)fake};
  float* im[1] = {(float*)fake};
  EXPECT(psflib_grouped_create(NULL, 1, los, sc, im, 1, 0, NULL, &g) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_grouped_create(libs, 0, los, sc, im, 1, 0, NULL, &g) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_grouped_create(libs, 1, los, sc, im, 1, 0, NULL, &g) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_grouped_create(libs, 1, NULL, sc, im, 1, 0, NULL, &g) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_grouped_create(libs, 1, los, sc, im, -1, 0, NULL, &g) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_grouped_run(NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  int64_t chunk = 0;
  float tuned = 0.0f;
  EXPECT(psflib_grouped_chunk(NULL, &chunk, &tuned) == PSFLIB_ERR_INVALID_ARG);
  int32_t rows = 0;
  EXPECT(psflib_grouped_shape(NULL, &chunk, &rows, &tuned) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_grouped_set_shape(NULL, 0, 256, NULL) == PSFLIB_ERR_INVALID_ARG);
  psflib_grouped_destroy(NULL);

  /* fitting model */
  EXPECT(psflib_render_disk(0, 0.5, 8.0, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk(46341, 0.5, 8.0, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk(8, -0.5, 8.0, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk(8, 0.5, NAN, fake, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk(8, 0.5, 8.0, NULL, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk(8, 0.5, 8.0, fake_odd, fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk_grad(8, 0.5, 8.0, fake, fake, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_render_disk_grad(8, 0.5, 8.0, fake, fake, fake_odd, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_chi2(0, 1.0, (const float*)fake, fake, fake, (double*)fake, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_chi2(16, NAN, (const float*)fake, fake, fake, (double*)fake, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_chi2(16, 1.0, NULL, fake, fake, (double*)fake, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_chi2(16, 1.0, (const float*)fake, fake, fake, NULL, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_chi2(16, 1.0, (const float*)fake, fake_odd, fake, (double*)fake, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);

  /* probes */
  EXPECT(psflib_probe_hbm_read(NULL, 1 << 20, 64, 8, 0, (float*)fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_hbm_read(fake, 1 << 20, 0, 8, 0, (float*)fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_hbm_read(fake, 1 << 20, 64, 3, 0, (float*)fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_hbm_read(fake_odd, 1 << 20, 64, 8, 1, (float*)fake, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_mfma(3, 10, 64, sink_host, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_mfma(1, 0, 64, sink_host, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_mfma(1, 10, 70000, sink_host, NULL) == PSFLIB_ERR_INVALID_ARG);
  EXPECT(psflib_probe_mfma(1, 10, 64, NULL, NULL) == PSFLIB_ERR_INVALID_ARG);

  if (failures) {
    fprintf(stderr, "abi_sanitize: %d failed expectations\n", failures);
    return 1;
  }
  printf("abi_sanitize ok\n");
  return 0;
}
