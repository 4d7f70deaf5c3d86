/*
 * psflib -- field-dependent PSF operator on AMD Instinct MI355X (gfx950).
 *
 * Implements the method of Milani & Douglas, "Faster imaging simulation
 * through complex systems: a coronagraphic example" (arXiv 2106.09122):
 *
 *   Sec. 2, Eqs. (2)-(3)  the library build: every scene pixel (field point)
 *                         gets the off-axis PSF interpolated in offset from a
 *                         datacube of PSFs sampled along +x and rotated to the
 *                         field point's position angle;
 *   Sec. 3, Eqs. (4)-(6)  the library matrix A = [I_1 ... I_{N^2}] (n^2 rows,
 *                         one column per scene pixel) and the simulated image
 *                         S = A Z.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers named d_* are HIP device memory; h_* are host memory.  The
 *    caller owns every buffer passed in, including the library buffer.
 *    Device arrays must be 16-byte aligned (the library buffer 256-byte), as
 *    hipMalloc and torch allocations are: kernels use 16-byte vector
 *    accesses.  A misaligned array is rejected with PSFLIB_ERR_INVALID_ARG.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call that touches the device is stream-ordered and returns without
 *    waiting for the GPU.
 *  - Outputs are overwritten, never accumulated into.
 *  - Scene pixel (row p, col q) of an N x N scene is j = p*N + q; image pixel
 *    (row a, col b) of the n x n image is i = a*n + b (row-major).  The optical
 *    axis is at ((n-1)/2, (n-1)/2) of every PSF and at ((N-1)/2, (N-1)/2) of
 *    the scene; x runs along columns and y along rows.
 *  - Radii and the scene pixel scale share one angular unit (any unit).  The
 *    PSF pixel scale is not an input: the rotation depends only on the angle.
 *  - Every call returns a status.  Arguments are validated before anything is
 *    enqueued, so a call that fails validation has enqueued nothing.  Errors
 *    raised by the HIP runtime are returned as PSFLIB_ERR_DEVICE; so is a
 *    runtime error still pending on the calling thread when a call starts (a
 *    fault of earlier asynchronous work, or an earlier failed runtime call),
 *    which is reported before anything is enqueued and then cleared.
 *    psflib_last_error() gives a human-readable message for the last failing
 *    call on the calling thread.
 *  - After psflib_build returns, a handle is read-only: psflib_apply,
 *    psflib_apply_adjoint, psflib_apply_batched and the read-back calls may
 *    run concurrently on different streams, and from different host threads,
 *    with one handle.  No two streams share temporary device memory: the
 *    temporaries of psflib_apply, psflib_apply_adjoint, psflib_apply_batched
 *    and psflib_render_disk_grad (split-K partial sums, packed scenes) live in
 *    one buffer per stream, taken from a pool the library keeps per device,
 *    grown on demand and shared, in stream order, by every call on that
 *    stream.  Under stream capture psflib_apply, psflib_apply_adjoint and
 *    psflib_apply_batched allocate their temporaries from the pool inside
 *    the graph instead, so each graph owns its own (tested: replays equal
 *    the eager results bitwise).  psflib_render_disk_grad and psflib_chi2
 *    return PSFLIB_ERR_UNSUPPORTED, enqueuing nothing, on a capturing stream:
 *    a captured fit chain faulted the GPU once, cause not found.
 *    Work that uses the library must be ordered after the build on the
 *    build's stream (same stream, or an event).
 *  - Device memory the library allocates for itself comes from that pool and
 *    is kept for reuse until the process ends (the per-stream buffers too:
 *    as large as the largest temporaries a call on that stream needed).
 */
#ifndef PSFLIB_H
#define PSFLIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSFLIB_OK = 0,
  PSFLIB_ERR_INVALID_ARG = 1, /* null pointer, bad enum, non-positive size, bad scale */
  PSFLIB_ERR_RADII = 2,       /* radii not finite or not strictly increasing */
  PSFLIB_ERR_SIZE = 3,        /* size overflow, or a buffer too small */
  PSFLIB_ERR_UNSUPPORTED = 4, /* valid request this library does not provide */
  PSFLIB_ERR_DEVICE = 5       /* HIP runtime error */
} psflib_status;

/* Radial interpolation of the PSF datacube (Sec. 2: linear or nearest). */
typedef enum { PSFLIB_INTERP_LINEAR = 0, PSFLIB_INTERP_NEAREST = 1 } psflib_interp;

/* Offsets r > radii[K-1]: CLAMP holds the last sampled PSF; ZERO gives an
 * all-zero column.  Offsets r < radii[0] always hold the first PSF. */
typedef enum { PSFLIB_OOB_CLAMP = 0, PSFLIB_OOB_ZERO = 1 } psflib_oob;

/* Storage of the library matrix.
 *  FP32       A as float, column-major: column j is the n*n floats of the
 *             flattened PSF I_j at element offset j*n*n (the layout of Eq. (5)).
 *  BF16_POW2  A_ij = M_ij * 2^e_j with M in bfloat16 and one int32 exponent
 *  FP16_POW2  per column (IEEE binary16 for FP16_POW2).  e_j makes the largest
 *             value the column can reach, (1-w) max P_k + w max P_{k+1}, land
 *             in [2^14, 2^15) after scaling, so binary16 neither overflows nor
 *             loses the column's faint wings to underflow.  Mantissas are
 *             stored by slot, in groups of 8 slots: element i of slot s sits
 *             at ((s/8)*n*n + i)*8 + s%8, so one 16-byte load holds row i of
 *             8 slots (the operand shape of the matrix cores).  Slot s holds
 *             column perm[s]; the build picks the order so that one workgroup
 *             can write whole 16-byte groups: for N a multiple of 8 (either
 *             rotation, with or without the flux rescale) slots 32b + 8k + u
 *             hold the k-th quarter turn about the star of the u-th of the
 *             b-th eight base columns (one quadrant, sorted by radial
 *             bracket); for other N, bilinear columns without the rescale
 *             whose PSF pair fits the LDS (n <= 141) are sorted by bracket;
 *             otherwise the natural order (slot j = column j).  The slot
 *             order is part of the library buffer (see psflib_library_bytes);
 *             psflib_get_columns reads columns by index whatever the order.
 *             Products accumulate in float32. */
typedef enum { PSFLIB_FP32 = 0, PSFLIB_BF16_POW2 = 1, PSFLIB_FP16_POW2 = 2 } psflib_storage;

/* Exponent e_j of an identically zero column in the 16-bit forms (its
 * mantissas are all zero; any finite value times 2^e_j underflows to 0, so a
 * scene value at such a column never sets the scene's scale). */
#define PSFLIB_ZERO_COLUMN_EXPONENT (-16384)

/* Interpolation of the rotation step (Sec. 2, the rotate() call).
 *  BILINEAR  four-neighbour bilinear sampling of the radially interpolated
 *            PSF Q, neighbours outside the n x n frame counting as zero.
 *  CUBIC     the cubic B-spline interpolating Q extended by zeros (the
 *            interpolation order the paper's rotate() uses by default): the
 *            spline coefficients of Q padded by 12 zero pixels per side (exact
 *            recursive filter, mirror boundary at the padded edge), sampled
 *            with the 4 x 4 cubic B-spline weights; coefficients beyond the
 *            padded array count as zero.  Entries can be slightly negative
 *            (spline overshoot); the 16-bit exponent bound then uses the
 *            largest |coefficient| of each sampled PSF in place of its largest
 *            value. */
typedef enum { PSFLIB_ROTATE_BILINEAR = 0, PSFLIB_ROTATE_CUBIC = 1 } psflib_rotate;

/* Column normalisation.
 *  NONE      columns are the rotated PSFs as sampled (the default; the column
 *            sums tau_j are reported by psflib_column_sums).
 *  PRESERVE  column j is rescaled so that it sums to the flux of the radially
 *            interpolated PSF before rotation, (1-w) sum(P_k) + w sum(P_{k+1}):
 *            the part of the PSF that the rotation carries out of the frame
 *            (and the spline's overshoot) no longer changes the total.  A
 *            column that sums to zero is left as is.  Each entry is the
 *            unscaled float32 entry times the column's float32 scale,
 *            rounded once; the 16-bit forms round that value, with the column
 *            exponent taken from the rescaled bound. */
typedef enum { PSFLIB_FLUX_NONE = 0, PSFLIB_FLUX_PRESERVE = 1 } psflib_flux;

typedef struct {
  int32_t n;             /* PSF side = image side (pixels); the image has n*n pixels */
  int32_t n_psf;         /* K >= 1 sampled off-axis PSFs, sources on +x */
  int32_t N;             /* scene side (pixels); the library has N*N columns */
  int32_t interp;        /* psflib_interp */
  double scene_pixscale; /* S > 0, in the unit of the radii (Eqs. (2)-(3)) */
  int32_t oob;           /* psflib_oob */
  int32_t storage;       /* psflib_storage */
  int32_t rotate;        /* psflib_rotate */
  int32_t flux;          /* psflib_flux */
} psflib_desc;

typedef struct psflib_handle psflib_handle;

/* Human-readable name of a status code (static storage). */
const char* psflib_status_string(psflib_status s);

/* Message describing the last failing call made on this thread (static,
 * thread-local storage; empty if none). */
const char* psflib_last_error(void);

/* Bytes the caller must allocate for the library buffer of `desc`: the matrix
 * (n^2 x N^2 entries in the chosen storage, with the 16-bit forms padded to a
 * multiple of 64 slots), followed by the per-column float64 column sums and,
 * for the 16-bit forms, four int32 arrays: the exponent per column, the
 * column per slot, the exponent per slot and the slot per column (each part
 * starting 256-byte aligned).  The matrix is the paper's
 * library of Sec. 3 (one flattened n x n PSF per scene pixel, Eq. (5)), whose
 * stored size Table 2 lists (n^2 N^2 float64 values there).  Host-only: no
 * device call.  Fails with PSFLIB_ERR_SIZE if the size does not fit in size_t
 * or exceeds 2^62. */
psflib_status psflib_library_bytes(const psflib_desc* desc, size_t* bytes);

/* Build the interpolated PSF library (Sec. 2; Eqs. (4)-(5)).
 *   d_cube   float32 [K][n][n] off-axis PSFs (k, row, col), source of PSF k at
 *            offset h_radii[k] on +x; values must be finite.  Read only during
 *            the build (the caller may free it once the stream passes the build).
 *   h_radii  float64 [K], finite and strictly increasing (copied before return).
 *   d_lib    library buffer of at least psflib_library_bytes() bytes, 256-byte
 *            aligned; written by the build and read by every later call.
 *   out      receives a new handle (host object) on success; it refers to
 *            d_lib, which must outlive it.  Free it with psflib_destroy().
 * Column j is, for field point (x_j, y_j) = ((q-(N-1)/2) S, (p-(N-1)/2) S),
 * r = sqrt(x^2+y^2), (cos, sin) = (x/r, y/r) ((1, 0) at r = 0): the PSF
 * interpolated to offset r, Q = (1-w) P_k + w P_{k+1}, rotated about the array
 * centre so that +x turns to the position angle (output pixel at offset u from
 * the centre samples Q at R(-theta) u), bilinearly with zero padding.
 * Takes the handle's device workspace (per-column geometry) and temporary
 * build buffers from the library's device pool, stream-ordered on `stream`. */
psflib_status psflib_build(const psflib_desc* desc, const float* d_cube, const double* h_radii,
                           void* d_lib, size_t lib_bytes, void* stream, psflib_handle** out);

/* Simulated image S = A Z (Sec. 3, Eq. (6)).
 *   d_scene  float32 [N*N] scene (flattened row-major, Sec. 3).
 *   d_image  float32 [n*n] output image.
 * Float32 accumulation in a fixed order (results are bitwise reproducible).
 * The split-K partial sums (a few MiB) sit in the buffer of `stream` (see
 * the conventions above). */
psflib_status psflib_apply(const psflib_handle* h, const float* d_scene, float* d_image, void* stream);

/* ---- Allocation-free apply -------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture that must not record allocations, tight serving loops, harnesses
 * that forbid hipMalloc.  The same product as psflib_apply (same kernels,
 * same summation order, so the image is bitwise equal), with the split-K
 * partial sums in a fixed device array of PSFLIB_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends; the call
 * allocates and frees nothing.
 *   The array is shared by every psflib_apply_noalloc call on that GPU and
 * keeps the last call's contents (nothing in it needs clearing: every
 * partial is written before it is read).  Calls that overlap on one GPU --
 * on different streams, or in graph replays running at once -- race on it
 * and give wrong images: order them (one stream, or events).
 *   Fails with PSFLIB_ERR_SIZE, before enqueuing anything, if the library needs
 * more partial sums than the array holds.  FP32 libraries need at most 4 MiB;
 * 16-bit ones at most max(4 MiB, ceil(N*N / 4096) * n*n * 4 bytes), which
 * can pass 8 MiB only when n*n*N*N > 2^32 (16-bit libraries of more than
 * 8 GiB, e.g. n = 128 with N >= 1024). */
#define PSFLIB_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
psflib_status psflib_apply_noalloc(const psflib_handle* h, const float* d_scene, float* d_image,
                                   void* stream);

/* Adjoint G = A^T g of the simulation S = A Z (Sec. 3, Eq. (6)): the
 * gradient of <g, A Z> with respect to the scene Z, which a retrieval of
 * scene parameters from simulated images needs (Sec. 5 plans such a
 * retrieval; the paper does not define the adjoint itself).
 *   d_g           float32 [n*n] image-space vector.
 *   d_scene_grad  float32 [N*N] output.
 * Float32 accumulation in a fixed order.  Partial sums (PSFs larger than
 * 128 x 128 only) are kept as in psflib_apply. */
psflib_status psflib_apply_adjoint(const psflib_handle* h, const float* d_g, float* d_scene_grad,
                                   void* stream);

/* Images of B scenes at once (Sec. 5: simulating many scenes at once):
 * d_images[b] = A d_scenes[b] for b < B.
 *   d_scenes  float32 [B][N*N];  d_images  float32 [B][n*n];  B >= 0.
 * FP32 storage runs float32 matrix-core products; the 16-bit forms round each
 * scene to the storage format with a per-scene power-of-two scale (so the
 * scaled scene spans [2^14, 2^15) at its largest) and run 16-bit matrix-core
 * products with float32 accumulation.  B = 1 runs psflib_apply instead (the
 * matvec streams the library faster).  Temporaries (packed scenes, K-split
 * partial images; up to ~100 MiB at 128 x 128 with 1024 scenes per pass) sit
 * in the buffer of `stream` (see the conventions above). */
psflib_status psflib_apply_batched(const psflib_handle* h, const float* d_scenes, float* d_images,
                                   int32_t B, void* stream);

/* Column sums tau_j = sum_i A_ij (float64 [N*N]), computed during the build
 * from the float32 values (before 16-bit rounding): the throughput of each
 * library PSF, by which a user can normalise the columns in the ways Sec. 3
 * leaves open (the library itself is not normalised). */
psflib_status psflib_column_sums(const psflib_handle* h, double* d_tau, void* stream);

/* Copy `count` library columns, dequantised to float32, into d_out
 * [count][n*n]; d_cols is a device int32 array of column indices in [0, N*N)
 * (an index outside that range yields a column of zeros; it is never used to
 * address the library). */
psflib_status psflib_get_columns(const psflib_handle* h, const int32_t* d_cols, int32_t count,
                                 float* d_out, void* stream);

/* Per-column exponents e_j (int32 [N*N]) of the 16-bit forms: column j is
 * stored as mantissas M_ij = A_ij * 2^-e_j; an identically zero column has
 * e_j = PSFLIB_ZERO_COLUMN_EXPONENT, so that a scene value at that column,
 * scaled by 2^e_j, is exactly 0 (it multiplies only zeros).
 * PSFLIB_ERR_UNSUPPORTED for FP32 storage. */
psflib_status psflib_get_exponents(const psflib_handle* h, int32_t* d_exp, void* stream);

/* Per-column geometry the build used (Sec. 2, Eqs. (2)-(3) and the radial
 * interpolation step): d_geom float64 [N*N][4] = (r, cos theta, sin theta, w)
 * and d_k int32 [N*N] = k, the lower radial sample (Q = (1-w) P_k + w P_{k+1}),
 * or -1 for a column that is identically zero (PSFLIB_OOB_ZERO beyond the
 * last sample).  Either output pointer may be NULL. */
psflib_status psflib_get_geometry(const psflib_handle* h, double* d_geom, int32_t* d_k, void* stream);

/* ---- Grouped simulation --------------------------------------------------
 * Many scenes, each simulated with its own library (libraries of different
 * sizes or wavelengths), as one graph launch (Sec. 5: simulating many
 * complex scenes at once).  A plan lists work tiles over every (library,
 * group of up to 16 of its scenes, row block, column chunk); a persistent
 * kernel streams each library once per scene group from HBM and multiplies
 * it with the group's scenes on the matrix cores; when a library is cut into
 * several chunks a second kernel adds the chunk partials in a fixed order
 * (bitwise reproducible).  The scene groups
 * are packed into the matrix-core operand at the start of every run.  All
 * launches are captured in a HIP graph.
 *   h_libs          host array of nlibs built handles; all share one storage
 *                   form and device, and must outlive the plan.
 *   h_lib_of_scene  host int32 [B]: the library of each scene.
 *   h_scenes        host array of B device pointers, scene b float32 [N_L^2]
 *                   of its library L; h_images: B device pointers, image b
 *                   float32 [n_L^2].  The pointers are fixed into the plan:
 *                   refill the buffers and run again; do not free them first.
 *   autotune        non-zero: time each candidate tile shape on this plan
 *                   (rows per item and chunk length, or whole columns per
 *                   item; running the graph, which writes the images) and keep
 *                   the fastest; the choice is cached per plan signature (the
 *                   storage and every scene's library size) for the process.
 *                   Zero: use the cached or default choice.
 * Synchronises `stream` (libraries built on it must be complete) and takes
 * the plan's device tables and partials from the library's device pool.  FP32 plans
 * take libraries with n*n <= 2^25 (n <= 5792; PSFLIB_ERR_UNSUPPORTED beyond). */
typedef struct psflib_grouped psflib_grouped;
psflib_status psflib_grouped_create(const psflib_handle* const* h_libs, int32_t nlibs,
                                    const int32_t* h_lib_of_scene, const float* const* h_scenes,
                                    float* const* h_images, int32_t B, int32_t autotune,
                                    void* stream, psflib_grouped** out);

/* Run the plan: one hipGraphLaunch on `stream`. */
psflib_status psflib_grouped_run(const psflib_grouped* g, void* stream);

/* The plan's chunk length (columns for FP32, 8-column groups for 16-bit; 0:
 * each item covers every column of its library) and, if it was autotuned, the
 * measured time of one run in ms (else 0). */
psflib_status psflib_grouped_chunk(const psflib_grouped* g, int64_t* chunk, float* tuned_ms);

/* The plan's tile shape: chunk length as psflib_grouped_chunk, rows per work
 * item (`rows` may be NULL; FP32 plans use 256, 16-bit plans 256, 128 or 64)
 * and the autotuned time (`tuned_ms` may be NULL). */
psflib_status psflib_grouped_shape(const psflib_grouped* g, int64_t* chunk, int32_t* rows,
                                   float* tuned_ms);

/* Rebuild the plan with a given tile shape instead of the tuned one: `chunk`
 * 8-column groups (16-bit, a multiple of 8) or columns (FP32, a multiple of
 * 16) per item, 0 for every column of the library in one item; `rows` per
 * item, 64, 128 or 256 for 16-bit plans and 256 for FP32 (else
 * PSFLIB_ERR_INVALID_ARG).  Waits for the plan's
 * earlier runs; synchronises `stream`.  The images are unchanged until the
 * next run.  Not to be called while another thread runs or destroys the
 * same plan. */
psflib_status psflib_grouped_set_shape(psflib_grouped* g, int64_t chunk, int32_t rows, void* stream);

/* Free the plan.  Waits on the host for the plan's own launches (events
 * recorded by psflib_grouped_run on each stream it ran on), not for other
 * work on the device.  NULL is ignored. */
void psflib_grouped_destroy(psflib_grouped* g);

/* ---- Fitting model -------------------------------------------------------
 * A smooth parametric exozodi disk on the scene grid of Eqs. (2)-(3), the
 * model that is fitted through the operator (Sec. 5 plans the retrieval of
 * disk parameters from simulated images; these two calls supply the model and
 * its gradient, psflib_apply_adjoint the operator's).
 *   d_theta  float64 [5] in device memory: (incl [rad], r0, width, gamma, flux)
 *   Z_j = flux (rho/r0)^gamma exp(-(rho - r0)^2 / (2 width^2)),
 *   rho = sqrt(x^2 + (y / cos incl)^2); Z_j = 0 where rho = 0 or where the
 *   pixel's sky radius exceeds rmax.  Evaluated in float64.
 * N in [1, 46340], S > 0 and finite, rmax not NaN. */
psflib_status psflib_render_disk(int32_t N, double scene_pixscale, double rmax,
                                 const double* d_theta, float* d_scene, void* stream);

/* d_dtheta[k] = sum_j d_dscene[j] * dZ_j/dtheta_k (float64 [5]), accumulated in
 * float64 in a fixed order (per-workgroup trees, then their sums in block
 * order), so repeated calls give identical results.  Uses N*N/256 * 40 bytes
 * of temporaries in the buffer of `stream` (see the conventions above). */
psflib_status psflib_render_disk_grad(int32_t N, double scene_pixscale, double rmax,
                                      const double* d_theta, const float* d_dscene,
                                      double* d_dtheta, void* stream);

/* The misfit the retrieval of Sec. 5 minimises, for Gaussian errors with a
 * per-pixel variance (e.g. photon noise of the simulated counts):
 *   L = sum_i (K S_i - D_i)^2 / var_i   and   dL/dS_i = 2 K (K S_i - D_i) / var_i,
 * K the exposure scale from image units to counts.  d_image float32 [M] (a
 * simulated image), d_data and d_var float64 [M] (var_i > 0), all in device
 * memory; M in [1, 2^36], K finite.  d_loss float64 [1] receives L, summed in
 * float64 in a fixed order (per-workgroup trees, then their sums in block
 * order: repeated calls give identical results); d_grad float32 [M] receives
 * dL/dS (the input of psflib_apply_adjoint), or NULL to skip it.  Uses M/256
 * * 8 bytes of temporaries in the buffer of `stream`.  With psflib_render_disk,
 * psflib_apply, psflib_apply_adjoint and psflib_render_disk_grad this gives
 * the loss of a disk model and its gradient without host arithmetic. */
psflib_status psflib_chi2(int64_t M, double K, const float* d_image, const double* d_data,
                          const double* d_var, double* d_loss, float* d_grad, void* stream);

/* ---- Measurement probes ---------------------------------------------------
 * Not part of the method: they measure, on the part itself, the ceilings the
 * products are compared against (the paper times its simulation against CPU
 * hardware, Table 4; here the reference points are the GPU's own memory and
 * matrix-core rates).
 *
 * psflib_probe_hbm_read: one kernel that streams `bytes` (rounded down to a
 * multiple of 16) of the device buffer d_buf with 16-byte non-temporal
 * loads over `workgroups` workgroups of 256 threads with `unroll` (4, 8 or
 * 16) loads in flight per thread, and sums what it reads.  slice = 0: the
 * workgroups stride over the buffer together (4 KiB runs w, w + grid, ...);
 * slice != 0: each workgroup streams its own contiguous 1/workgroups of it.
 * Rate = bytes / kernel time.  d_sink: float32 [workgroups], written only for
 * an impossible sum (it keeps the loads alive). */
psflib_status psflib_probe_hbm_read(const void* d_buf, size_t bytes, int32_t workgroups,
                                    int32_t unroll, int32_t slice, float* d_sink, void* stream);

/* psflib_probe_mfma: `workgroups` workgroups of 4 waves; every wave runs
 * `iters` rounds of 4 independent matrix-core products on register operands:
 * kind 0 = v_mfma_f32_32x32x2f32 (4096 flop each), 1 = ..._32x32x16_bf16,
 * 2 = ..._32x32x16_f16 (32768 flop each).  Rate = workgroups * 4 * iters * 4
 * * flop / kernel time.  d_sink as above. */
psflib_status psflib_probe_mfma(int32_t kind, int32_t iters, int32_t workgroups, float* d_sink,
                                void* stream);

/* Release the handle and its workspace.  Waits on the host for the handle's
 * own uses of its workspace (the build and psflib_get_geometry, by events
 * recorded on their streams), not for other work on the device; the caller
 * must not destroy a handle while calls that use it are still queued.  NULL
 * is ignored. */
void psflib_destroy(psflib_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PSFLIB_H */
