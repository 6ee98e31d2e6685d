/*
 * mfa_dvr.h -- C ABI of the MI355X (gfx950) MFA direct volume renderer.
 *
 * The library ray-casts a multivariate functional approximation (MFA): a
 * non-rational tensor-product B-spline volume given by a degree and a
 * clamped knot vector per axis and a grid of control points (Sect. 2.3 of
 * "MFA-DVR: direct volume rendering of MFA models").  Rendering follows
 * Sect. 3.1 and Algorithm 1: one ray per pixel, constant-distance samples
 * between the first and last sample inside the volume, normalisation to
 * the unit cube, the value query, the transfer function, the gradient
 * query with Phong shading, front-to-back compositing and early ray
 * termination.  All work runs in HIP kernels on the GPU.
 *
 * Conventions common to every entry point:
 *  - Return value: MFA_OK (0) or a negative mfa_status.  On error nothing
 *    is enqueued, output buffers are untouched, and mfa_last_error()
 *    describes the failure.
 *  - Host pointers inside descriptors (knots, control points, transfer
 *    function table) are owned by the caller and are only read during the
 *    call; the caller may free them as soon as the call returns.
 *  - Device pointers (images, points, values, gradients, counters) are
 *    owned by the caller, must be device memory of the context's GPU, and
 *    must stay valid until the work enqueued on the given stream has
 *    completed.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Render and
 *    evaluation calls are asynchronous on that stream.
 *  - A context is used by one host thread at a time.  Work it enqueues on
 *    different streams may run concurrently: every stream has its own
 *    planning space for mfa_render and mfa_render_curvature and its own
 *    ordering space for point queries (a batch is the exception: see
 *    mfa_batch_render).
 */
#ifndef MFA_DVR_H
#define MFA_DVR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mfa_status;
#define MFA_OK 0
#define MFA_ERR_INVALID (-1) /* bad argument: sizes, camera, TF, step, pointers */
#define MFA_ERR_MODEL (-2)   /* malformed model descriptor */
#define MFA_ERR_NOMEM (-3)   /* device memory or the context budget exhausted */
#define MFA_ERR_DEVICE (-4)  /* HIP runtime error (including an earlier fault) */
#define MFA_ERR_HANDLE (-5)  /* unknown context, model, batch or ticket handle */
#define MFA_ERR_TIMEOUT (-6) /* mfa_server_wait: the request has not finished yet */

/* Storage precision of the control points on the device.  Basis functions
 * and all accumulation are FP32 in either case. */
#define MFA_STORE_F32 0
#define MFA_STORE_BF16 1 /* FP64 -> FP32 -> BF16, each step round-to-nearest-even */
#define MFA_STORE_F16 2  /* FP64 -> FP32 -> IEEE binary16, each step RNE; |rounded| <= 65504 */

#define MFA_CAMERA_ORTHO 0
#define MFA_CAMERA_PERSP 1

#define MFA_MAX_DEGREE 4
#define MFA_MAX_TF 4096
#define MFA_MAX_CURV_TF 64

/* MFA model (Sect. 2.3): per axis a degree p in [1, MFA_MAX_DEGREE], n >= p+1
 * control points and a knot vector of n+p+1 FP64 values that is
 * non-decreasing and clamped (p+1 zeros first, p+1 ones last; interior
 * knots in (0,1) with multiplicity <= p).  Control points are FP64, finite,
 * x fastest: P[i,j,k] = ctrl[i + n0*(j + n1*k)].  The model maps the box
 * [lo, hi] (lo < hi per axis) affinely onto the unit parameter cube.
 * With `weights` (finite, > 0, same layout) the model is rational: the
 * field is sum N N N w P / sum N N N w, its gradient by the quotient rule;
 * the device stores the homogeneous values w*P and w in the storage
 * precision.  Rational models are rendered by the global-memory ray caster
 * (the brick kernels are non-rational only).  Without weights (null) every
 * weight is 1, which is how the paper uses the method. */
typedef struct mfa_model_desc {
  int32_t degree[3];
  int32_t store; /* MFA_STORE_F32, MFA_STORE_BF16 or MFA_STORE_F16 */
  int64_t n_ctrl[3];
  const double* knots[3];
  const double* ctrl;
  double lo[3];
  double hi[3];
  const double* weights; /* nullable: rational weights, n0*n1*n2 FP64 > 0, layout of ctrl */
} mfa_model_desc;

/* Fixed-point ray-cast camera (Sect. 3.1): one ray through the centre of
 * every pixel, row 0 at the top of the image.  F = unit(target - eye),
 * R = unit(F x up), V = R x F.
 *  - MFA_CAMERA_ORTHO: origin eye + a*half_w*R + b*half_h*V, direction F;
 *  - MFA_CAMERA_PERSP: origin eye, direction
 *    unit(F + a*tan(fov/2)*(W/H)*R + b*tan(fov/2)*V),
 *  with a = 2(c+1/2)/W - 1 and b = 1 - 2(r+1/2)/H for column c, row r.
 * fov_y_deg is the vertical field of view in (0, 180). */
typedef struct mfa_camera {
  int32_t kind;
  int32_t width;
  int32_t height;
  int32_t reserved;
  double eye[3];
  double target[3];
  double up[3];
  double fov_y_deg;
  double ortho_half_w;
  double ortho_half_h;
} mfa_camera;

/* Transfer function (Algorithm 1: colour and opacity transfer functions),
 * as one RGBA table of n entries (2 <= n <= MFA_MAX_TF), host memory,
 * linearly interpolated over [v_lo, v_hi] (v_lo < v_hi); values outside
 * the range clamp to the end entries.  Entries are finite, and every
 * opacity (the fourth value of an entry) lies in [0, 1]; otherwise
 * MFA_ERR_INVALID. */
typedef struct mfa_tf {
  int32_t n;
  int32_t reserved;
  const float* rgba; /* n*4 floats */
  double v_lo;
  double v_hi;
} mfa_tf;

/* Sampling, shading and termination (Sect. 3.1, Algorithm 1).
 *  step       constant world-space distance between samples (> 0);
 *             a ray with entry/exit parameters t0 < t1 takes
 *             floor((t1 - t0)/step) samples at t0 + (s + 1/2)*step;
 *  ert_alpha  early ray termination: a ray stops once its accumulated
 *             opacity exceeds this value, tested after compositing a
 *             sample; >= 1 disables termination;
 *  shading    0: unshaded colour; 1: Phong from the analytic gradient,
 *             c' = min(1, (ka + kd*|n.l|)*c + ks*max(0, r.v)^shininess),
 *             n = g / max(|g|, 1e-6), r = 2(n.l)n - l, v = -ray direction;
 *  headlight  1: l = -F (light along the view axis); 0: l = light_dir
 *             (normalised by the library);
 *  shininess  integer exponent in [0, 256]. */
typedef struct mfa_render_params {
  double step;
  double ert_alpha;
  int32_t shading;
  int32_t shininess;
  int32_t headlight;
  int32_t reserved;
  double ka;
  double kd;
  double ks;
  double light_dir[3];
} mfa_render_params;

typedef struct mfa_ctx mfa_ctx;

/* Create a context bound to HIP device `device`.  Errors: MFA_ERR_INVALID
 * (null ctx_out), MFA_ERR_DEVICE (no such device / HIP failure). */
mfa_status mfa_create(int32_t device, mfa_ctx** ctx_out);

/* Synchronise the device, free every model and internal buffer, and
 * destroy the context.  Null is accepted and ignored. */
mfa_status mfa_destroy(mfa_ctx* ctx);

/* Cap the device bytes that the context's models may occupy (0 = only the
 * device's free memory limits uploads).  Errors: MFA_ERR_HANDLE,
 * MFA_ERR_INVALID (negative). */
mfa_status mfa_set_memory_budget(mfa_ctx* ctx, int64_t bytes);

/* Validate, convert and upload an MFA model (Sect. 3: the encoded model is
 * the renderer's input).  Control points are rounded to the storage
 * precision (RNE); per-span knot differences and their reciprocals are
 * tabulated in FP32 for the basis recursion.  No gradient table is built:
 * gradients are evaluated on demand (Sect. 3.1).  Synchronous: the model
 * is resident and immutable when the call returns; *model_out receives a
 * handle > 0.  Errors: MFA_ERR_MODEL (see mfa_model_desc), MFA_ERR_NOMEM,
 * MFA_ERR_DEVICE, MFA_ERR_HANDLE, MFA_ERR_INVALID (null pointers, more
 * than 2^31 bytes of control points). */
mfa_status mfa_model_upload(mfa_ctx* ctx, const mfa_model_desc* desc, int64_t* model_out);

/* Release a model after synchronising the device.  Errors: MFA_ERR_HANDLE,
 * MFA_ERR_INVALID (the model is used by a live batch). */
mfa_status mfa_model_free(mfa_ctx* ctx, int64_t model);

/* Device bytes held by a model.  Errors: MFA_ERR_HANDLE, MFA_ERR_INVALID. */
mfa_status mfa_model_bytes(mfa_ctx* ctx, int64_t model, int64_t* bytes_out);

/* Render an image (Algorithm 1) into rgba_dev: width*height*4 FP32,
 * row-major, row 0 at the top, premultiplied (C_r, C_g, C_b, A).  A ray
 * that misses the box yields (0,0,0,0).  If samples_dev is not null it
 * receives (overwritten, one int64) the number of samples composited over
 * the whole image, early-terminated rays counting up to and including
 * their last sample.  Asynchronous on `stream`.  Not for HIP graph
 * capture: a call may allocate and copy (planning space, a new transfer
 * function), and consecutive frames on a stream share planning state that a
 * replayed graph would not advance; capture batches (mfa_batch_render)
 * instead.  Errors: MFA_ERR_INVALID (camera, TF or parameters, null
 * rgba_dev), MFA_ERR_HANDLE, MFA_ERR_DEVICE. */
mfa_status mfa_render(mfa_ctx* ctx, int64_t model, const mfa_camera* camera, const mfa_tf* tf,
                      const mfa_render_params* params, float* rgba_dev, int64_t* samples_dev,
                      void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Renders
 * exactly as mfa_render (same kernels, bit-identical image and count) but
 * calls no hipMalloc/hipFree and no allocating routine: the transfer
 * function copy and the tile-planning space live in one fixed device array
 * of 4 MiB per GPU, reserved by the library until the process ends (its
 * address is looked up by mfa_create).  The transfer function is copied
 * from host memory on `stream` before the call returns.  Limits: at most
 * 507,904 launch slots (one per 8x8-pixel super-tile, grouped per XCD);
 * images up to about 5600 x 5600 pixels fit, larger ones are refused with
 * MFA_ERR_INVALID and a message naming the limit.  Every call on a GPU
 * shares that GPU's array and each call clears what must start at zero:
 * calls that overlap on one GPU (another stream, another context or host
 * thread) race and may corrupt each other's images; order them on one
 * stream.  No kernel timing is recorded.  Errors: as mfa_render, plus
 * MFA_ERR_INVALID for an image beyond the limit. */
mfa_status mfa_render_noalloc(mfa_ctx* ctx, int64_t model, const mfa_camera* camera,
                              const mfa_tf* tf, const mfa_render_params* params, float* rgba_dev,
                              int64_t* samples_dev, void* stream);

/* Curvature transfer function: an m x m RGBA table (2 <= m <=
 * MFA_MAX_CURV_TF) over [k_lo, k_hi] x [k_lo, k_hi] of the two principal
 * curvatures k1 >= k2, entry (i2, i1) at rgba[4 (i2 m + i1)] (k1 along a
 * row), bilinearly interpolated with clamping.  Host memory, copied before
 * the call returns; opacities in [0, 1]. */
typedef struct mfa_curvature_tf {
  int32_t m;
  int32_t reserved;
  const float* rgba; /* m*m*4 floats */
  double k_lo;
  double k_hi;
} mfa_curvature_tf;

/* Render with a curvature transfer function, the use the model's analytic
 * second derivatives serve (Sect. 3.1: the representation gives all
 * derivatives together).  As mfa_render, except per sample: the value
 * table gives an opacity; the principal curvatures of the isosurface
 * through the sample, the two tangential eigenvalues of P H P / |g| (H the
 * world Hessian, g the world gradient, P = I - n n^T, n = g / |g|; 0 where
 * |g|^2 < 1e-12; a sphere around lower values has k1 = k2 = 1/r), index
 * the curvature table, whose colour becomes the sample's colour and whose
 * opacity multiplies the value table's; then Phong shading if enabled.
 * Up to degree 3 the LDS-brick ray caster renders it (like mfa_render,
 * with second derivatives); degree-4 models, or transfer functions that
 * leave too little LDS for bricks, use one lane per ray with global-memory
 * gathers.  The curvature table is read from global memory (cached).
 * Errors: as mfa_render,
 * plus MFA_ERR_INVALID for a malformed curvature table and MFA_ERR_MODEL
 * for a rational model. */
mfa_status mfa_render_curvature(mfa_ctx* ctx, int64_t model, const mfa_camera* camera,
                                const mfa_tf* tf, const mfa_curvature_tf* curvature,
                                const mfa_render_params* params, float* rgba_dev,
                                int64_t* samples_dev, void* stream);

/* One request of a render batch: the arguments of one mfa_render call. */
typedef struct mfa_render_request {
  int64_t model;
  const mfa_camera* camera;
  const mfa_tf* tf;
  const mfa_render_params* params;
  float* rgba_dev;      /* width*height*4 FP32, caller-owned device memory */
  int64_t* samples_dev; /* nullable; one int64 of device memory */
} mfa_render_request;

/* Prepare a batch of n render requests, each the problem of Algorithm 1
 * for its own model, camera, transfer function and parameters (different
 * models, image sizes and views may be mixed).  Every request is checked
 * as mfa_render checks it; the output buffers (images and counters) of a
 * batch must not overlap.  The call copies what the requests point to
 * (cameras, tables, parameters), uploads the per-request kernel records
 * and planning space to device memory (counted against the memory budget)
 * and returns synchronously; the caller's host structures may be freed at
 * once.  The output pointers are bound to the batch.  The models stay in
 * use until the batch is freed (mfa_model_free refuses them meanwhile).
 * *batch_out receives a handle > 0.  Errors: MFA_ERR_INVALID (n outside
 * [1, 65536], null pointers, overlapping outputs, or any request that
 * mfa_render would reject; the message names the request), MFA_ERR_HANDLE,
 * MFA_ERR_NOMEM, MFA_ERR_DEVICE. */
mfa_status mfa_batch_create(mfa_ctx* ctx, const mfa_render_request* reqs, int32_t n,
                            int64_t* batch_out);

/* Render every request of a batch on `stream`, asynchronously: per kernel
 * variant one work estimate and ordering pass over the tiles of all its
 * requests, longest first, and one ray-casting launch over them.  Each
 * image equals the image of mfa_render for the same request bit for bit.
 * The call only enqueues kernels (no allocation, copy or fill), so it can
 * be captured in a HIP graph and replayed.  A batch must not be rendered
 * on two streams at once (its planning space is shared).  Errors:
 * MFA_ERR_HANDLE, MFA_ERR_DEVICE. */
mfa_status mfa_batch_render(mfa_ctx* ctx, int64_t batch, void* stream);

/* Synchronise the device and release a batch.  Errors: MFA_ERR_HANDLE,
 * MFA_ERR_DEVICE. */
mfa_status mfa_batch_free(mfa_ctx* ctx, int64_t batch);

/* Result of mfa_autotune. */
typedef struct mfa_tune_result {
  float round_spans; /* chosen round length: knot spans along the fastest axis per lane */
  int32_t candidates; /* configurations timed */
  float best_ms;      /* median kernel time of the chosen configuration */
  float default_ms;   /* median kernel time of the default (3 spans, 4 lanes per ray) */
  int32_t lanes_per_ray; /* chosen lanes per ray: 1, 2 or 4 */
} mfa_tune_result;

/* Autotuner of the ray caster for one model: renders the given request
 * (into rgba_dev, which it overwrites) with each candidate configuration,
 * every combination of a round length (1.5, 2, 3, 4 and 6 knot spans per
 * lane's round of samples; a round's control points are staged in LDS
 * once) and a number of lanes sharing one ray (4, 2 or 1: a wave renders a
 * 4x4, 8x4 or 8x8-pixel tile), one warm-up and `repeats` timed launches
 * each, all candidates interleaved and enqueued back to back on `stream`
 * (the call returns after synchronising it), and keeps the configuration
 * with the smallest median kernel time for every later render of the model
 * (single frames, batches prepared afterwards, servers; curvature renders
 * keep four lanes per ray).  The LDS budget is fixed by the kernels'
 * occupancy.  Results of later renders change only by rounding (the FP32
 * sample stepping restarts from FP64 at each round, and each lane sums its
 * own samples).  out may be null.  Errors: MFA_ERR_HANDLE, MFA_ERR_INVALID
 * (the request, or repeats outside [1, 1000]), MFA_ERR_DEVICE. */
mfa_status mfa_autotune(mfa_ctx* ctx, int64_t model, const mfa_camera* camera, const mfa_tf* tf,
                        const mfa_render_params* params, float* rgba_dev, int32_t repeats,
                        void* stream, mfa_tune_result* out);

/* Set the ray caster's configuration for a model by hand (what
 * mfa_autotune chooses): round_spans in [0.5, 16] knot spans per lane's
 * round, lanes_per_ray 1, 2 or 4.  Applies to renders prepared after the
 * call.  Errors: MFA_ERR_HANDLE, MFA_ERR_INVALID. */
mfa_status mfa_model_set_tuning(mfa_ctx* ctx, int64_t model, float round_spans,
                                int32_t lanes_per_ray);

/* ----------------------------------------------------------------------
 * Serving: a render server with continuous batching.
 *
 * A worker thread owned by the server takes submitted requests in arrival
 * order and launches them as batches (as mfa_batch_render does) on up to
 * `streams` concurrent slots.  Whenever a slot is free, every queued
 * request that fits is admitted into one batch: at most `max_batch`
 * requests, and, when max_bytes > 0, only while the device bytes of the
 * requests in flight (their images and their share of the batch records
 * and planning space) stay within max_bytes.  Requests that arrive while
 * others run therefore start as soon as a slot frees up, and their work
 * overlaps the tail of the running batches on the device.  Every image
 * equals the image of mfa_render for the same request bit for bit.
 *
 * While a server exists its context must be used through the server only
 * (upload models before creating it; free them after destroying it).
 * mfa_server_submit and mfa_server_wait may be called from any host
 * thread.  A request's output buffers must stay valid and untouched until
 * its ticket has been waited for.
 * ---------------------------------------------------------------------- */
typedef struct mfa_server_config {
  int32_t streams;   /* concurrent batches, 1..8 (0 = 2) */
  int32_t max_batch; /* requests per batch, 1..65536 (0 = 256) */
  int64_t max_bytes; /* device-byte budget of requests in flight (0 = none) */
} mfa_server_config;

typedef struct mfa_request_info {
  int32_t status;     /* MFA_OK, or the error of a failed request */
  int32_t batch_size; /* requests in the batch that rendered it */
  int64_t submit_ns;  /* host steady-clock times: submission, */
  int64_t launch_ns;  /* admission into a launched batch, */
  int64_t done_ns;    /* completion seen by the worker */
  int32_t deferred;   /* 1 if max_bytes held it back while a launch slot was free */
  int32_t reserved;
} mfa_request_info;

typedef struct mfa_server mfa_server;

/* Start a server on a context (cfg may be null for the defaults).
 * Errors: MFA_ERR_HANDLE, MFA_ERR_INVALID (config out of range),
 * MFA_ERR_DEVICE. */
mfa_status mfa_server_create(mfa_ctx* ctx, const mfa_server_config* cfg, mfa_server** server_out);

/* Queue one request (checked as mfa_render checks it; everything it points
 * to is copied) and return its ticket (> 0).  Errors: MFA_ERR_HANDLE,
 * MFA_ERR_INVALID (any request mfa_render would reject, or the server is
 * shutting down), MFA_ERR_NOMEM (the request alone exceeds max_bytes). */
mfa_status mfa_server_submit(mfa_server* server, const mfa_render_request* req,
                             int64_t* ticket_out);

/* Wait up to timeout_us microseconds (< 0: without limit) for a request to
 * finish; on completion fill *info (nullable), forget the ticket and
 * return the request's status.  Errors: MFA_ERR_TIMEOUT (not finished; the
 * ticket stays valid), MFA_ERR_HANDLE (unknown or already waited-for
 * ticket; of several threads waiting for one ticket, one receives the
 * record and the others this), MFA_ERR_DEVICE (the request failed on the
 * device). */
mfa_status mfa_server_wait(mfa_server* server, int64_t ticket, int64_t timeout_us,
                           mfa_request_info* info);

/* Finish every queued and running request, stop the worker and release the
 * server.  Null is accepted and ignored. */
mfa_status mfa_server_destroy(mfa_server* server);

/* Kernel timing for measurement.  While enabled, every mfa_render and
 * mfa_render_curvature call records a pair of HIP events on its stream
 * immediately around the ray-casting kernel (after the per-frame tile planning), so that the
 * kernel's own duration can be read back; at most 65536 launches are
 * recorded, later ones are not.  Enabling or disabling discards what was
 * recorded.  Errors: MFA_ERR_HANDLE. */
mfa_status mfa_kernel_timing(mfa_ctx* ctx, int32_t enable);

/* Wait for the recorded events and write the kernel durations in
 * milliseconds, in call order, to ms_host (host memory of `cap` floats,
 * owned by the caller; only the first `cap` are written).  *count receives
 * the number of recorded launches.  The record is then cleared; recording
 * stays as it was.  Errors: MFA_ERR_HANDLE, MFA_ERR_INVALID (null count,
 * cap < 0, null ms_host with cap > 0), MFA_ERR_DEVICE. */
mfa_status mfa_kernel_times(mfa_ctx* ctx, float* ms_host, int64_t cap, int64_t* count);

/* Measured FP32 fused multiply-add rate of the context's device, the
 * attainable ceiling of the FP32 vector roofline without packed FP32: a
 * micro-loop of eight independent FMA chains per lane on 16 workgroups of
 * 256 threads per compute unit, timed with HIP events on the null stream.
 * Synchronous; writes TFLOP/s (2 flops per FMA) to *tflops.  Errors:
 * MFA_ERR_HANDLE, MFA_ERR_INVALID (null tflops), MFA_ERR_NOMEM,
 * MFA_ERR_DEVICE. */
mfa_status mfa_measure_fma_peak(mfa_ctx* ctx, double* tflops);

/* Value and world-space gradient queries (Algorithm 1: value query and
 * gradient query, all three derivatives at once) at n world points
 * xyz_dev (n*3 FP64, point-major).  Points outside the box are clamped to
 * it.  value_dev: n FP32; grad_dev: n*3 FP32 or null for value only.
 * n = 0 is a no-op.  Asynchronous on `stream`.  From 2^16 points on (for
 * models whose gathers would miss the caches), the points are sorted on
 * the device by bin (a 16^3 grid over the box, in Morton order; no sort
 * when they arrive in that order) and each bin is evaluated from its
 * control points staged in LDS, or, for rational models and models whose
 * bins need more than 64 KiB of LDS, gathered in bin order; results stay in
 * the caller's order and equal those of a direct query bit for bit.  This
 * uses 12 bytes of device memory per point in the stream's scratch, kept
 * until the context is destroyed; if it cannot be allocated, the points
 * are evaluated in the given order.
 * Errors: MFA_ERR_INVALID (n < 0, null buffers with n > 0), MFA_ERR_HANDLE,
 * MFA_ERR_DEVICE. */
mfa_status mfa_eval_points(mfa_ctx* ctx, int64_t model, int64_t n, const double* xyz_dev,
                           float* value_dev, float* grad_dev, void* stream);

/* Value, world gradient and world Hessian at n world points.  The model's
 * derivatives of every order are analytic (Sect. 3.1: the representation
 * gives all derivatives together); the second derivatives are what
 * curvature-based transfer functions take.  Same points, value and
 * gradient buffers and clamping as mfa_eval_points (grad_dev may be null);
 * hess_dev: n*6 FP32 per point, d2f/dx2, d2f/dy2, d2f/dz2, d2f/dxdy,
 * d2f/dxdz, d2f/dydz in world units, caller-owned device memory.  At a knot
 * the span on its right is used (one-sided second derivatives where the
 * model is only C^1 there).  Non-rational models only.  Errors:
 * MFA_ERR_INVALID (n < 0, null buffers with n > 0), MFA_ERR_MODEL
 * (rational model), MFA_ERR_HANDLE, MFA_ERR_DEVICE. */
mfa_status mfa_eval_hessian(mfa_ctx* ctx, int64_t model, int64_t n, const double* xyz_dev,
                            float* value_dev, float* grad_dev, float* hess_dev, void* stream);

/* Host-only validation, callable without a GPU; the same checks that
 * mfa_model_upload and mfa_render run before touching the device. */
mfa_status mfa_validate_model(const mfa_model_desc* desc);
mfa_status mfa_validate_render(const mfa_camera* camera, const mfa_tf* tf,
                               const mfa_render_params* params);

/* Message of the last failed call on this host thread (empty if none).
 * Valid until the next library call on the same thread. */
const char* mfa_last_error(void);

/* Library version string. */
const char* mfa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MFA_DVR_H */
