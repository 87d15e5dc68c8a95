/*
 * libjpet — list-mode MLEM reconstruction for the two-strip J-PET detector on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is that of P. Bialas et al., "GPU accelerated image reconstruction in a
 * two-strip J-PET tomograph" (arXiv:1502.07478):
 *   - events are the triples (z_u, z_d, dl) of the Setup section (Eq. 1),
 *   - the per-pixel sensitivity is Eq. 4,
 *   - the event kernel P(e|i) is Eq. 7 with the vectors of Eq. 8-11 and the C^-1 of
 *     Eq. 12: diagonal as the paper assumes, or with its off-diagonal gamma, and with
 *     sigma_z optionally depending on the event's hit positions,
 *   - it is evaluated over the pixel centres inside the 3-sigma ellipse of each event
 *     (Sec. 3, last paragraph; bounding box of App. B),
 *   - one iteration is the two-pass scheme of the implementation listing (Sec. 4):
 *     D_j = sum_i P_ji rho_i, then rho_l P_jl / D_j is accumulated into the new image,
 *     which is divided by the sensitivity (Eq. 3; Eq. 5 when no sensitivity is given).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units are millimetres.  The detector strips lie at y = +R (upper) and y = -R (lower) and
 * span z in [-L/2, L/2].  Images are float32, row-major [n_y][n_z]; pixel (i, k) is the
 * square of side `pixel` centred at
 *     y_i = (i + 1/2 - n_y/2) * pixel,   z_k = (k + 1/2 - n_z/2) * pixel.
 * Events are float32 [n][3] rows (z_u, z_d, dl) (array of structures, 12 bytes each).
 *
 * Memory: every array argument is DEVICE memory on the current HIP device, owned by the
 * caller, unless the argument says "host".  The library allocates no device memory in
 * any entry point below; scratch space is the caller's workspace.  It keeps no pointer
 * after a call returns, except in a batched graph (jpet_mlem_batched_graph_create), whose
 * captured launches hold the batch's pointers and whose instantiation is the HIP runtime's.
 *
 * Streams: `stream` is a hipStream_t (NULL = the legacy default stream).  Work is enqueued
 * asynchronously; outputs are valid once the stream has been synchronised, except that an
 * entry point given a non-NULL host `stats` pointer synchronises the stream before it
 * returns.  Calls that share a workspace must be ordered (same stream, or synchronised);
 * calls with distinct workspaces are independent and the library is reentrant.
 *
 * Errors: every entry point returns 0 (JPET_OK) or a negative code.  Arguments are fully
 * validated before anything is enqueued or written; on a validation error nothing is
 * written.  There are no C++ exceptions across this interface.
 */
#ifndef JPET_H
#define JPET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JPET_ABI_VERSION 3

enum jpet_status {
  JPET_OK = 0,
  JPET_EINVAL = -1,     /* a required pointer is NULL, a count is negative, flags are unknown */
  JPET_EDOMAIN = -2,    /* geometry out of domain (see jpet_geometry); log-likelihood is -inf */
  JPET_EWORKSPACE = -3, /* workspace NULL or smaller than the size query returned */
  JPET_EHIP = -4,       /* a HIP runtime call failed; jpet_last_hip_error() has its code */
  JPET_ENOTSUP = -5     /* valid request that this build does not implement */
};

/* Detector, resolution and pixel grid.  All members are read by value; the struct is
 * host memory.  Domain (else JPET_EDOMAIN): R, L, sigma_z, sigma_dl, pixel finite and > 0;
 * 0 < n_y, n_z <= 32768; n_y * pixel / 2 < R (every pixel centre lies between the strips);
 * kernel_variant in {0, 1}; 0 <= sigma_z_edge <= 1; gamma finite with
 * 2 gamma^2 < sigma_z,max^-2 sigma_dl^-2, sigma_z,max = sigma_z (1 + sigma_z_edge) (C^-1 of Eq. 12
 * positive definite for every event); plan 0 or a code listed by jpet_mlem_plan_candidates for
 * this geometry (a malformed code is JPET_EINVAL, one that does not fit JPET_EDOMAIN). */
typedef struct jpet_geometry {
  double R;              /* strip half-separation: strips at y = +R and y = -R (Setup, Eq. 1) */
  double L;              /* strip length; strips span z in [-L/2, L/2] (Eq. 4) */
  double sigma_z;        /* resolution of z_u and z_d (Eq. 12) */
  double sigma_dl;       /* resolution of dl (Eq. 12) */
  double gamma;          /* off-diagonal element of C^-1 (Eq. 12): C^-1 = [[u, 0, g], [0, u, -g],
                            [g, -g, w]], u = sigma_z^-2, w = sigma_dl^-2, in mm^-2 */
  double pixel;          /* pixel pitch, the same along y and z */
  int32_t n_y;           /* number of pixel rows (y) */
  int32_t n_z;           /* number of pixel columns (z) */
  int32_t kernel_variant;/* third component of a (Eq. 9): 0 as printed, 1 twice that (the
                            exact derivative of dl with respect to the emission angle) */
  int32_t plan;          /* launch plan of the event pass: 0 lets the library's cost model choose;
                            otherwise a plan code from jpet_mlem_plan_candidates (e.g. the one an
                            autotuner timed fastest).  It changes how the work is laid out, not
                            what is computed: results agree to FP32 rounding.  The workspace size,
                            preparation and iterations of one event list must use the same value. */
  double sigma_z_edge;   /* sigma_z depending on the hit positions (Sec. 3, after Eq. 12): an event
                            with measured hits z_u, z_d takes, in both z slots of C^-1 and in its
                            3-sigma ellipse, sigma_z (1 + sigma_z_edge * zeta) with
                            zeta = ((2 z_u / L)^2 + (2 z_d / L)^2) / 2, so sigma_z at the strip
                            centre rising by the fraction sigma_z_edge at its ends; 0: constant.
                            The log-likelihood entry points take 0 only (else JPET_ENOTSUP). */
} jpet_geometry;

/* Per-call counters (host memory).  An event is valid when its three numbers are finite,
 * |z_u| <= L/2, |z_d| <= L/2 and at least one pixel centre of the grid lies inside its
 * 3-sigma ellipse; other events are dropped (counted, not an error).  A valid event whose
 * denominator D is 0 (the current image vanishes on its ellipse) is skipped by the update
 * and counted in n_zero_denominator (value for the last iteration). */
typedef struct jpet_stats {
  int64_t n_events;
  int64_t n_valid;
  int64_t n_dropped;
  int64_t n_zero_denominator;
  int64_t n_pairs;             /* (valid event, in-ellipse pixel) pairs per iteration */
  int64_t n_kappa_nonpositive; /* in-ellipse pairs whose Eq. 7 denominator term is <= 0 (P := 0) */
  int64_t n_unplaced_rows;     /* ellipse rows the binned event pass could not place in its
                                  workgroup's region (last iteration); always 0 unless the
                                  library is faulty -- such rows are skipped, not written */
} jpet_stats;

/* Flags for jpet_mlem_iterate and jpet_loglik_grad. */
#define JPET_WS_PREPARED 1u /* the workspace already holds jpet_mlem_prepare's output for
                               exactly this geometry, event array and event count (for
                               jpet_loglik_grad: prepared with the mask's sigmas); skip that step */
/* Work splits of the event pass for comparison (jpet_mlem_iterate, jpet_mlem_backproject; at most
 * one of them): one wavefront per event (a lane per ellipse row), or one thread per event, the
 * granularity of the paper's GPU "thread" variant (Sec. 4, Table 1).  Both read the image and add
 * to the accumulators in global memory; the result equals the planned pass's to rounding. */
#define JPET_PASS_WAVE_PER_EVENT 2u
#define JPET_PASS_THREAD_PER_EVENT 4u
/* jpet_loglik_grad: the log-likelihood value alone (out3[1] and out3[2] are set to NaN and
 * grad_rho must be NULL): one forward pass forming the denominators, with none of the
 * back-projection or derivative work, e.g. for the function evaluations of a line search. */
#define JPET_LOGLIK_VALUE_ONLY 8u

/* Text for a status code (static storage, never NULL). */
const char* jpet_strerror(int status);

/* The hipError_t of the last failed HIP call made by this thread inside the library
 * (0 if none). */
int jpet_last_hip_error(void);

/* ABI version compiled into the library (JPET_ABI_VERSION). */
int jpet_abi_version(void);

/* Sensitivity image, Eq. 4: for each pixel centre (y, z) the fraction of in-plane emission
 * directions, uniform in angle, whose line meets both strips:
 *   s = (atan(min((L/2 - z)/(R - y), (L/2 + z)/(R + y)))
 *        - atan(max(-(L/2 + z)/(R - y), (z - L/2)/(R + y)))) / pi, clamped at 0.
 * Evaluated in double precision and rounded to float.
 *   s_out: device float [n_y * n_z], written entirely. */
int jpet_sensitivity(const jpet_geometry* g, float* s_out, void* stream);

/* Direct-reconstruction image (Eq. 2): for every valid event (finite, |z_u| and |z_d| <= L/2) the
 * point (y~, z~) of Eq. 2 in double precision, counted in the pixel that contains it (pixel index
 * floor(y~ / pixel + n_y / 2), likewise for z); points outside the grid are not counted.  A
 * diagnostic image and a possible MLEM starting image.
 *   events: device float [n][3]; img: device float [n_y*n_z], overwritten with the counts. */
int jpet_direct_image(const jpet_geometry* g, const float* events, int64_t n, float* img, void* stream);

/* Bytes of workspace that jpet_mlem_prepare / jpet_mlem_iterate / jpet_mlem_backproject need for
 * n_events events on this geometry (host output *bytes).  The workspace is any device
 * allocation of at least that size, aligned to 256 bytes.
 * Every entry point takes at most 2^31 - 1 events per call (else JPET_EINVAL): event positions
 * and bin offsets are 32-bit on the device.  Longer lists are processed in pieces with
 * jpet_mlem_backproject and jpet_mlem_update. */
int jpet_mlem_workspace_size(const jpet_geometry* g, int64_t n_events, size_t* bytes);

/* Iteration-invariant per-event work, done once per event list: direct reconstruction (Eq. 2),
 * the 3-sigma ellipse's pixel rows (App. B) and validity, and the spatial ordering of events
 * used by the event pass.  Writes only the workspace.
 *   events: device float [n][3]; 0 <= n <= 2^31 - 1. */
int jpet_mlem_prepare(const jpet_geometry* g, const float* events, int64_t n, void* ws, size_t ws_bytes,
                      void* stream);

/* n_iter list-mode MLEM iterations (Sec. 4 listing, Eq. 3) in place on rho.
 *   events: device float [n][3]
 *   s:      device float [n_y*n_z] sensitivity (e.g. from jpet_sensitivity), or NULL for the
 *           Eq. 5 form in which no sensitivity is applied (s = 1 everywhere)
 *   rho:    device float [n_y*n_z], the current image on entry, the image after n_iter
 *           iterations on return.  rho must be finite and >= 0.  Pixels with s = 0 are set to 0.
 *   n_iter >= 0; flags: 0 or JPET_WS_PREPARED, optionally with one of the JPET_PASS_* comparison
 *   work splits; stats: host, nullable (synchronises if given).
 * One iteration: for every valid event j, D_j = sum_{i in ellipse} P_ji rho_i; for D_j > 0 the
 * values rho_l P_jl / D_j are summed into the new image; then rho_l = sum / s_l (s_l > 0) or 0. */
int jpet_mlem_iterate(const jpet_geometry* g, const float* events, int64_t n, const float* s, float* rho,
                      int32_t n_iter, void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats,
                      void* stream);

/* One event pass of jpet_mlem_iterate without the pixel update, for event lists processed in
 * pieces (chunks of one acquisition that share the current image): for every valid event j with
 * D_j = sum_{i in ellipse} P_ji rho_i > 0, adds round(2^32 rho_l P_jl / D_j) to acc_l for every
 * pixel l of its ellipse (the accumulator of the Sec. 4 listing in 2^-32 fixed point).
 *   events, n, rho, ws, ws_bytes, flags, stats: as for jpet_mlem_iterate (rho is only read)
 *   acc:  device uint64 [n_y*n_z], added to; start it at 0 (e.g. after jpet_mlem_update or a
 *         memset).  Integer sums make the result independent of the order of calls and events.
 *         Up to 2^32 events' contributions fit before a pixel can overflow.
 * stats counts this call's events. */
int jpet_mlem_backproject(const jpet_geometry* g, const float* events, int64_t n, const float* rho, uint64_t* acc,
                          void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream);

/* The forward sums of the MLEM event pass: runs the pass of jpet_mlem_iterate (same plan and
 * kernel, with the same workspace rules and flags) on the image rho and writes each event's
 * denominator D_j = sum_{i in ellipse} P_ji rho_i (Sec. 4 listing, first loop; the denominator of
 * Eq. 3), P including its constant factor, as that pass forms it (FP32 terms, double-precision
 * sum of per-wavefront partials), rounded to float.  Dropped events get 0.  The pass's
 * back-projection goes to the workspace's accumulator and is discarded.
 *   D_out: device float [n], written entirely.  stats: as for jpet_mlem_iterate. */
int jpet_mlem_denominators(const jpet_geometry* g, const float* events, int64_t n, const float* rho, float* D_out,
                           void* ws, size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream);

/* The pixel update of Eq. 3 (Eq. 5 with s NULL) from an accumulator filled by
 * jpet_mlem_backproject:  rho_l = acc_l 2^-32 / s_l where s_l > 0, else 0 (s NULL: acc_l 2^-32);
 * then acc_l = 0.
 *   s: device float [n_y*n_z] or NULL; acc: device uint64 [n_y*n_z]; rho: device float, written. */
int jpet_mlem_update(const jpet_geometry* g, const float* s, uint64_t* acc, float* rho, void* stream);

/* Poisson list-mode log-likelihood of the image and its gradient (the objective whose EM step
 * is Eq. 3):
 *   l = sum_{valid j} log(D_j / pi) - sum_l s_l rho_l,     D_j = sum_{i in ellipse_j} P_ji rho_i
 *   dl/drho_l = sum_j P_jl / D_j - s_l
 *   dl/dsigma_z, dl/dsigma_dl: derivatives of l through P (Eq. 7) with the ellipse mask held
 *   fixed.  The mask is the 3-sigma ellipse at (sigma_mask[0], sigma_mask[1]) (host double[2],
 *   nullable = the geometry's sigmas); the kernel uses the geometry's sigmas.
 *   out3:     device double[3] = { l, dl/dsigma_z, dl/dsigma_dl }, sums in double precision
 *   grad_rho: device float [n_y*n_z] or NULL
 *   D_out:    device float [n] per-event D_j (0 for dropped events) or NULL
 *   s:        as for jpet_mlem_iterate (NULL = 1)
 * When a valid event has D_j = 0 the device value l is -inf; if stats is given (the call then
 * synchronises) the call also returns JPET_EDOMAIN in that case.
 * The workspace is sized by jpet_loglik_workspace_size (its layout differs from the MLEM one).
 * flags = JPET_WS_PREPARED reuses the preparation of an earlier jpet_loglik_grad call on the same
 * workspace with the same geometry, mask, events and count; it is refused (JPET_EINVAL) when
 * sigma_mask differs from the geometry's sigmas, because the prepared kernel constants belong to
 * the sigmas the workspace was prepared with.
 * Both log-likelihood entry points return JPET_ENOTSUP for a geometry with sigma_z_edge != 0 (the
 * log-likelihood is defined here for one sigma_z shared by all events). */
/* Bytes of workspace jpet_loglik_grad needs for n_events events (host output *bytes); the layout
 * follows the mask (sigma_mask as for jpet_loglik_grad, nullable). */
int jpet_loglik_workspace_size(const jpet_geometry* g, const double* sigma_mask, int64_t n_events, size_t* bytes);

int jpet_loglik_grad(const jpet_geometry* g, const double* sigma_mask, const float* events, int64_t n,
                     const float* s, const float* rho, double* out3, float* grad_rho, float* D_out, void* ws,
                     size_t ws_bytes, uint32_t flags, jpet_stats* stats, void* stream);

/* Batched reconstruction: many independent list-mode MLEM problems (each with its own geometry,
 * resolution, event list, sensitivity and image) advanced together (one MLEM iteration of each is
 * the Sec. 4 listing with Eq. 3).  Instances that fit the binned pass are grouped into classes by
 * kernel configuration (register cache, wavefronts per workgroup, workgroups per CU, region row
 * pitch); per iteration each class is one launch with one workgroup per workgroup item of its
 * instances, the items in order of decreasing size.  The classes are shared by the caller's stream
 * and a second stream of the library's (one per device, default priority, created by the first
 * batched call and kept until the process ends), forked from and joined back into the caller's
 * stream within each iteration, so one class's last workgroups overlap another's work.  Instances
 * that fit only the generic pass get their own launches.  A plan named in an instance's jpet_geometry.plan must be one the batched pass can run:
 * 32-bit accumulators (else JPET_EDOMAIN); plan 0 takes the cost model's cheapest such plan.  Each instance's result is that of jpet_mlem_iterate on it
 * alone with the same plan, to FP32 rounding of the denominators.
 * Host struct; pointers as for jpet_mlem_iterate. */
typedef struct jpet_instance {
  jpet_geometry g;
  const float* events; /* device float [n][3] */
  int64_t n;           /* >= 0 */
  const float* s;      /* device float [n_y*n_z] sensitivity, or NULL (Eq. 5) */
  float* rho;          /* device float [n_y*n_z]: the image, updated in place */
} jpet_instance;

/* Workspace bytes for the batch (host output).  inst: host array of count instances,
 * 0 <= count <= 65535. */
int jpet_mlem_batched_workspace_size(const jpet_instance* inst, int32_t count, size_t* bytes);

/* Per-event preparation of every instance (as jpet_mlem_prepare) into the batched workspace. */
int jpet_mlem_batched_prepare(const jpet_instance* inst, int32_t count, void* ws, size_t ws_bytes, void* stream);

/* n_iter MLEM iterations of every instance, in place on each rho.  flags: 0 or JPET_WS_PREPARED
 * (the workspace holds jpet_mlem_batched_prepare's output for the same instance array: same
 * geometries, event pointers and counts).  stats: host array of count entries, or NULL; entry k
 * describes instance k (the call then synchronises).  Instances must not share rho arrays. */
int jpet_mlem_batched_iterate(const jpet_instance* inst, int32_t count, int32_t n_iter, void* ws, size_t ws_bytes,
                              uint32_t flags, jpet_stats* stats, void* stream);

/* The same n_iter iterations captured once into a HIP graph (a reset, the batched passes, any
 * generic passes and the update per iteration, all kernels), for repeated launches with no host
 * work.  Creating the graph prepares the instances (unless JPET_WS_PREPARED) and writes the batch's
 * instance table and work list into the workspace on stream, in stream order, before capturing;
 * each launch then runs n_iter iterations on the images as they are at that point in the stream.
 * The instance array's device pointers, the workspace and the event lists must stay valid and
 * unchanged while the graph exists; a later jpet_mlem_batched_iterate or a graph of another
 * instance array on the same workspace rewrites the table (create the graph again after it).
 * The graph object is host memory and runtime state of the library's, released by
 * jpet_mlem_batched_graph_destroy.  n_iter >= 1; *out (host) receives the graph. */
typedef struct jpet_batched_graph jpet_batched_graph;
int jpet_mlem_batched_graph_create(const jpet_instance* inst, int32_t count, int32_t n_iter, void* ws,
                                   size_t ws_bytes, uint32_t flags, void* stream, jpet_batched_graph** out);
/* Enqueues one launch of the graph (n_iter iterations) on stream. */
int jpet_mlem_batched_graph_launch(jpet_batched_graph* graph, void* stream);
/* Releases the graph (NULL is allowed); it must not be executing. */
int jpet_mlem_batched_graph_destroy(jpet_batched_graph* graph);

/* jpet_mlem_iterate without a caller workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid allocation).  The workspace
 * is a device array of JPET_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from the
 * first call on that GPU until the process ends; the call allocates nothing.  Arguments and
 * results are those of jpet_mlem_iterate, except:
 *   - flags must be 0 (else JPET_EINVAL): every call prepares its events, and runs the planned
 *     event pass;
 *   - a geometry and event count whose workspace (jpet_mlem_workspace_size) exceeds
 *     JPET_NOALLOC_SCRATCH_BYTES returns JPET_EWORKSPACE before anything is enqueued (about
 *     300k events at 400 x 400 px of 2 mm, 500k at 64 x 64 px of 4 mm);
 *   - all calls on one GPU share its array, which keeps the last call's contents: calls that
 *     overlap on one GPU (different streams or threads without ordering between them) race and
 *     give undefined results.  Order them on one stream or synchronise between them. */
#define JPET_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)
int jpet_mlem_iterate_noalloc(const jpet_geometry* g, const float* events, int64_t n, const float* s, float* rho,
                              int32_t n_iter, uint32_t flags, jpet_stats* stats, void* stream);

/* Launch shape the library picks for jpet_mlem_iterate on this geometry and event count
 * (diagnostics and tuning reports).  Host output. */
typedef struct jpet_launch_info {
  int32_t binned;        /* 1: binned LDS event pass; 0: generic one-wavefront-per-event pass */
  int32_t tile_rows;     /* rows of a bin's tile core */
  int32_t tile_cols;     /* sheared columns of a bin's tile core */
  int32_t halo_rows;     /* rows added above and below the core */
  int32_t halo_cols;     /* columns added on each side of the core */
  int32_t t_bins;        /* bins along tan(theta~); 1 = no shear */
  int32_t bins;          /* total bins */
  int32_t waves;         /* wavefronts per workgroup */
  int32_t row_cache;     /* pixels of a row held in registers between the two passes */
  int32_t events_per_batch;
  int32_t events_per_workgroup;
  int32_t accumulator_bits; /* 64: 2^-32 fixed-point LDS accumulators; 32: 2^-accumulator_shift
                               ones, the shift set by the events per workgroup so that no slot can
                               overflow (faster LDS atomics, smaller regions); the image
                               accumulator is 64-bit in 2^-32 units either way */
  double t_bin_width;    /* width of a tan(theta~) bin */
  int64_t lds_bytes;     /* dynamic LDS per workgroup */
  int64_t max_workgroups;/* launch grid of the event pass */
  int32_t plan;          /* the plan's code (what jpet_geometry.plan would name to get this plan) */
  int32_t workgroups_per_cu; /* resident workgroups per CU the LDS region is sized for (0: generic) */
  int32_t accumulator_shift; /* 32-bit accumulators: units of 2^-accumulator_shift counts; 0 for 64-bit
                                ones (2^-32 units) */
  int32_t row_segments;  /* 1: a thread holds a whole ellipse row; 2: rows longer than row_cache
                            pixels are split in two, one thread each */
} jpet_launch_info;

int jpet_mlem_launch_info(const jpet_geometry* g, int64_t n_events, jpet_launch_info* info);

/* Launch plans that fit the geometry for n_events events, sorted by the library's cost-model
 * figure (ascending: the first is the one plan 0 selects).  pass: 0 for the MLEM event pass, 1 for
 * the log-likelihood pass (whose plans use 64-bit accumulators only; sigma_mask as for
 * jpet_loglik_grad, nullable).  g->plan is ignored.  Writes up to cap codes (and, if model_cost is
 * not NULL, their figures) to the host arrays and the number of fitting plans to *count (host).
 * A geometry whose ellipses fit no binned plan lists the generic pass's code (3) alone. */
int jpet_mlem_plan_candidates(const jpet_geometry* g, int32_t pass, const double* sigma_mask, int64_t n_events,
                              int32_t* codes, double* model_cost, int32_t cap, int32_t* count);

/* Autotuning support: the time of the MLEM event pass under each of the named plans, measured
 * on the caller's events and image (an autotuner lists plans with jpet_mlem_plan_candidates, times
 * them here and names the fastest in jpet_geometry.plan).  For each code: the events are prepared
 * with that plan into the workspace, one pass runs untimed, then reps passes are timed with HIP
 * events on stream; ms_out[k] (host) receives the mean milliseconds per pass, or -1 when the plan
 * does not fit.  The passes' back-projections go to the workspace and are discarded; rho is only
 * read.  Synchronises the stream.  The workspace must hold jpet_mlem_tune_workspace_size bytes
 * (the largest of the codes' workspaces); g->plan is ignored.
 *   events: device float [n][3]; rho: device float [n_y*n_z]; codes: host int32 [ncodes]; reps >= 1 */
int jpet_mlem_tune_workspace_size(const jpet_geometry* g, int64_t n_events, const int32_t* codes, int32_t ncodes,
                                  size_t* bytes);
int jpet_mlem_tune(const jpet_geometry* g, const float* events, int64_t n, const float* rho, const int32_t* codes,
                   int32_t ncodes, int32_t reps, void* ws, size_t ws_bytes, double* ms_out, void* stream);

/* Kernel timing.  While enabled (enable != 0), every launch of the MLEM event pass made by
 * jpet_mlem_iterate and jpet_mlem_backproject, and every iteration's group of event-pass launches
 * made by jpet_mlem_batched_iterate, is bracketed by a pair of HIP events recorded on the caller's stream (the
 * stream the kernel runs on).  jpet_profile_read waits for the recorded events, writes the
 * number of timed launches and their summed duration in milliseconds (host outputs, nullable)
 * and forgets them.  Disabling also forgets unread timings.  Process-wide, thread-safe; the
 * events are host-side objects, no device memory is allocated. */
int jpet_profile_enable(int enable);
int jpet_profile_read(int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* JPET_H */
