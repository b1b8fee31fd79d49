/*
 * fdtd.h -- C ABI of the MI355X (gfx950) second-order acoustic FDTD + CPML library.
 *
 * Operation (paper, section "Model" and section "CPML Boundary Layers"):
 * each call of fdtd_step advances every shot of a context by
 *
 *     u^{n+1} = 2 u^n - u^{n-1} + m * sum_d Lt_d(u^n) + m * f^n,   m = v^2 dt^2,
 *
 * where Lt_d is the radius-4 (eighth-order) central second derivative along
 * axis d, replaced inside the absorbing layer by the CFS/Roden-Gedney
 * stretched operator applied twice: psi_d <- b psi_d + a D1_d u^n,
 * eta_d = kinv D2_d u^n + dkinv D1_d u^n + D1_d psi_d,
 * zeta_d <- b zeta_d + a eta_d, Lt_d = kinv eta_d + zeta_d, with
 * b = exp(-(sigma/kappa + alpha) dt), a = sigma (b-1) / (kappa (sigma + kappa alpha))
 * and cubic sigma/kappa grading (sigma_max = -(q+1) v_ref ln R / (2 L h), q = 3,
 * kappa_max = 5, alpha_max = 0.05 sigma_max by default).
 * Faces outside the grid are zero Dirichlet, or "ghost" faces that are
 * filled by an on-device pack/unpack of the opposite face every s steps with
 * depth g = 4 s (one GPU's share of the paper's pencil-yz layout, section
 * "Multi-GPU Decomposition and Halo Exchange", with the enlarged ghost regions
 * of the same section; the loopback makes that axis periodic).
 *
 * Conventions of every entry point:
 *  - Return value: FDTD_OK (0) or a negative fdtd_status.  Nothing throws
 *    across this boundary; fdtd_last_error() gives a message for the context.
 *  - Arrays are x-fastest: element (i, j, k) of an nx*ny*nz array is at
 *    i + nx*(j + ny*k).
 *  - Pointers named *_dev are device pointers (hipMalloc'd or from a device
 *    tensor).  The caller owns them; the library only borrows them and never
 *    frees them.  The library never allocates device memory on the data
 *    path: all of its state lives in the caller-provided workspace.
 *  - All GPU work is ordered on the stream given to fdtd_create; no entry
 *    point synchronises unless stated.  Inside a step the library forks part
 *    of the work onto a second stream of its own (created by
 *    fdtd_bind_workspace) and joins it back before the step ends, with
 *    events, so the caller's stream still sees every step complete in order.
 *  - One host thread per context at a time.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_ctx fdtd_ctx;

enum fdtd_status {
    FDTD_OK = 0,
    FDTD_EINVAL = -1,        /* bad argument, shape, index or layer width       */
    FDTD_EUNSTABLE = -2,     /* dt above the leapfrog stability limit           */
    FDTD_ESTATE = -3,        /* call out of order (no workspace, no model, ...) */
    FDTD_ENOMEM = -4,        /* workspace or buffer too small                   */
    FDTD_EHIP = -5,          /* a HIP runtime call failed                       */
    FDTD_ENONFINITE = -6,    /* non-finite value found by fdtd_check_finite     */
    FDTD_EUNSUPPORTED = -7   /* valid request the library does not implement    */
};

enum fdtd_storage { FDTD_F32 = 0, FDTD_F16 = 1, FDTD_BF16 = 2 };
enum fdtd_face { FDTD_FACE_DIRICHLET = 0, FDTD_FACE_GHOST = 1 };
enum fdtd_variant {
    FDTD_VARIANT_AUTO = 0,   /* z-march (or the tuned choice, see fdtd_autotune);
                                naive for a single-shot context below 150^3 points */
    FDTD_VARIANT_NAIVE = 1,  /* one thread per point, all layer logic inline       */
    FDTD_VARIANT_ZMARCH = 2, /* LDS-staged xy tiles, z-marching register queue      */
    FDTD_VARIANT_TBLOCK = 3  /* tblock_k steps per launch (temporal blocking)       */
};

/* One shot (one independent grid).  Zero-valued optional fields take the
 * default shown. */
typedef struct {
    int32_t n[3];            /* nx, ny, nz (points, >= 9 each)                     */
    double h[3];             /* spacing per axis, metres (> 0)                     */
    double dt;               /* time step, seconds (> 0)                           */
    int32_t cpml[6];         /* layer width per face -x,+x,-y,+y,-z,+z (0 = none)  */
    int32_t face[6];         /* FDTD_FACE_DIRICHLET or FDTD_FACE_GHOST; ghost faces
                                come in pairs on y and/or z and carry no layer     */
    int32_t exchange_every;  /* s in {1,2,4} for ghost faces; ghost depth 4 s (0->1)*/
    double R;                /* target reflection, default 1e-8                    */
    double kappa_max;        /* default 5                                          */
    double alpha_frac;       /* alpha_max / sigma_max, default 0.05                */
    double v_ref;            /* velocity in sigma_max; 0 -> max of the model       */
    int32_t storage;         /* fdtd_storage of u^n, u^{n-1} (arithmetic is FP32)  */
    int32_t variant;         /* fdtd_variant                                       */
    int32_t tblock_k;        /* steps per launch for FDTD_VARIANT_TBLOCK (2 or 4)  */
    double field_scale;      /* power-of-two storage scale, 0 -> automatic for
                                16-bit storage, 1 for FP32                         */
} fdtd_shot_config;

/* Create a context for nshots shots on hip_stream (a hipStream_t, may be NULL
 * for the null stream).  Validates every shot (EINVAL for bad shapes, layers
 * wider than half an axis, bad faces, a field plane above 64 MiB (e.g.
 * more than about 4000 x 4000 FP32 points) or above 2 GiB / (W + 12) with W
 * the larger of 32 and the widest z layer + 4 (about 46 MiB with layers up
 * to 28 cells), or a layer array above 1 GiB, which the kernels' 32-bit
 * offsets cannot address; EUNSTABLE is checked at
 * fdtd_set_velocity, once the velocity is known).  *out receives the context
 * (host memory owned by the library; free with fdtd_destroy). */
int fdtd_create(const fdtd_shot_config *shots, int32_t nshots, void *hip_stream, fdtd_ctx **out);

/* Bytes of device workspace the context needs (fields, model, layer memory,
 * profiles, exchange buffers).  256-byte aligned sub-buffers. */
int fdtd_workspace_size(const fdtd_ctx *ctx, size_t *bytes);

/* Hand the context a device workspace of at least fdtd_workspace_size bytes.
 * Borrowed: the caller keeps it alive until fdtd_destroy and frees it.
 * Zeroes the wavefields and layer memory (enqueued on the stream). */
int fdtd_bind_workspace(fdtd_ctx *ctx, void *dev_ptr, size_t bytes);

/* Set the velocity model of one shot from a dense float32 [nz][ny][nx] device
 * array (m/s, > 0).  Computes m = v^2 dt^2, the layer profiles (FP64 on the
 * host, rounded once to FP32) and checks stability:
 * vmax dt sqrt(sum_d 6.50159 / h_d^2) <= 2, else FDTD_EUNSTABLE.
 * Synchronises the stream once (to read vmax). */
int fdtd_set_velocity(fdtd_ctx *ctx, int32_t shot, const float *v_dev);

/* Point source of one shot at node (i, j, k): from step n on, u^{n+1} gains
 * m * amplitude * wavelet_dev[n] / (hx hy hz) at that node (n < nt; zero after).
 * wavelet_dev: float32[nt] device array, borrowed (read by every step; keep
 * it alive and unchanged while stepping).  With 16-bit storage and an
 * automatic scale, this call copies the wavelet to the host once to choose
 * the power-of-two storage scale (synchronises).  Replaces any previous
 * source. */
int fdtd_inject_source(fdtd_ctx *ctx, int32_t shot, int32_t i, int32_t j, int32_t k,
                       const float *wavelet_dev, int32_t nt, float amplitude);

/* Receivers of one shot: ijk_dev is int32[nrec][3] (i, j, k) on the device,
 * borrowed until replaced.  Indices are validated on the host copy. */
int fdtd_set_receivers(fdtd_ctx *ctx, int32_t shot, const int32_t *ijk_dev, int32_t nrec);

/* Register float32 traces_dev[nt_capacity][nrec]: every later step n (counted
 * from the last fdtd_reset) writes row n with u^{n+1} at the receivers, while
 * n < nt_capacity.  NULL stops recording. */
int fdtd_record_receivers(fdtd_ctx *ctx, int32_t shot, float *traces_dev, int32_t nt_capacity);

/* Advance all shots by nsteps (asynchronous on the stream).  ESTATE if no
 * workspace is bound or a shot has no velocity.  With ghost faces the step
 * count must keep the exchange schedule (any count is accepted; exchanges
 * happen whenever the step counter is a multiple of s). */
int fdtd_step(fdtd_ctx *ctx, int32_t nsteps);

/* Same as fdtd_step, but the nsteps launches are captured once into a HIP
 * graph (kept in the context, keyed by nsteps and the step phase) and
 * replayed with one launch. */
int fdtd_step_graph(fdtd_ctx *ctx, int32_t nsteps);

/* Copy a wavefield of one shot to a dense float32 [nz][ny][nx] device array
 * (storage scale removed).  which: 0 = u^n (latest), 1 = u^{n-1}. */
int fdtd_get_field(fdtd_ctx *ctx, int32_t shot, int32_t which, float *dst_dev);

/* Overwrite a wavefield of one shot from a dense float32 [nz][ny][nx] device
 * array (for initial conditions).  which as in fdtd_get_field.  With 16-bit
 * storage the state is kept as (u^n, d^n = u^n - u^{n-1}): set u^n first,
 * then u^{n-1}. */
int fdtd_set_field(fdtd_ctx *ctx, int32_t shot, int32_t which, const float *src_dev);

/* Zero wavefields and layer memory and the step counter; keep model,
 * source and receivers. */
int fdtd_reset(fdtd_ctx *ctx);

/* Steps taken since the last fdtd_reset. */
int fdtd_get_step(const fdtd_ctx *ctx, int64_t *step);

/* Resume support.  The full state of every shot of the context (u^n, u^{n-1}
 * or, with 16-bit storage, d^n, and the layer memory psi, zeta, in the
 * library's own padded layout) and the step count, as one blob of
 * fdtd_state_size bytes in caller device memory (256-byte aligned pointers
 * are not required).  fdtd_save_state enqueues the copy on the stream;
 * fdtd_load_state restores a blob saved by a context created with the same
 * shot configurations (EINVAL for a blob of another configuration or storage,
 * checked from its header; it synchronises once to read the header), after
 * which stepping continues bit for bit as it would have from the saved step
 * (receiver rows are still indexed by the step count).  Model, source,
 * receivers and plans are not part of the blob. */
int fdtd_state_size(const fdtd_ctx *ctx, size_t *bytes);
int fdtd_save_state(fdtd_ctx *ctx, void *dst_dev, size_t bytes);
int fdtd_load_state(fdtd_ctx *ctx, const void *src_dev, size_t bytes);

/* Synchronise and scan the wavefields of every shot; FDTD_ENONFINITE if any
 * NaN or Inf is present. */
int fdtd_check_finite(fdtd_ctx *ctx);

/* NaN/Inf sentinel (failure detection; the paper has none).  With every > 0,
 * fdtd_step scans the newest wavefield level of every shot after each step
 * whose count is a multiple of `every`, into a sticky device flag, and when a
 * call enqueued a scan it synchronises once at its end and returns
 * FDTD_ENONFINITE if the flag is set; fdtd_step_graph scans once after each
 * graph launch instead.  every = 0 turns it off (the default).  The flag is
 * cleared by this call and by fdtd_reset.  EINVAL for every < 0, ESTATE
 * without a bound workspace. */
int fdtd_set_sentinel(fdtd_ctx *ctx, int32_t every);

/* Size in bytes of the device buffer fdtd_adjoint needs for one shot with
 * checkpoints every `every` steps over nt steps (checkpoints, two segments of
 * recomputed levels, adjoint state with a ring of up to 17 adjoint levels,
 * the receivers grouped by location, and the tables of a sweep over all
 * shots of this context).  It depends on the shot's receiver count: set the receivers
 * first (fdtd_adjoint returns ENOMEM if they outgrew the buffer since). */
int fdtd_adjoint_workspace_size(const fdtd_ctx *ctx, int32_t shot, int32_t every, int32_t nt, size_t *bytes);

/* Register the adjoint buffer of one shot and the checkpoint interval.  While
 * registered, fdtd_step saves the full state (u^n, u^{n-1}, psi, zeta) of
 * that shot every `every` steps from step 0.  every = 0 stops saving. */
int fdtd_set_checkpointing(fdtd_ctx *ctx, int32_t shot, int32_t every, void *buf_dev, size_t bytes);

/* Model gradient of J for one shot after a forward run of nt steps from
 * reset with checkpointing on: resid_dev is dJ/dtraces, float32 [nt][nrec];
 * grad_v_dev (float64 [nz][ny][nx], overwritten) receives dJ/dv.  Reverse-time
 * sweep of the exact transposed step with segment recomputation from the
 * checkpoints; the layer profiles (v_ref) and dt are held fixed.  Leaves the
 * forward state of this shot undefined (call fdtd_reset before stepping); the
 * step count and the other shots' states are kept, so that after one batched
 * forward run every shot's adjoint can be taken in turn. */
int fdtd_adjoint(fdtd_ctx *ctx, int32_t shot, int32_t nt, const float *resid_dev, double *grad_v_dev);

/* Model gradients of every shot of the context in one reverse sweep (the
 * batched form of fdtd_adjoint: each pass of a reverse step is one launch over
 * all shots, and the segments are recomputed by the batched forward step).
 * resid_dev and grad_v_dev are host arrays of one device pointer per shot, in
 * shot order, with fdtd_adjoint's layouts.  Every shot needs checkpointing
 * registered with the same interval (EINVAL otherwise) and a buffer sized by
 * fdtd_adjoint_workspace_size of this context.  Each gradient equals, bit for
 * bit, the one fdtd_adjoint gives for that shot.  Leaves the forward states
 * undefined; keeps the step count. */
int fdtd_adjoint_batch(fdtd_ctx *ctx, int32_t nt, const float *const *resid_dev, double *const *grad_v_dev);

/* Time candidate kernel shapes / temporal-block depths for every shot on
 * this device and keep the fastest per shape bucket; results are merged into
 * the JSON cache at cache_path (NULL = no file).  Synchronises; leaves the
 * wavefields reset. */
int fdtd_autotune(fdtd_ctx *ctx, const char *cache_path);

/* Fix the kernel plan of one shot by hand (what fdtd_autotune chooses):
 * variant (naive / z-march / temporal blocking), z-march tile height
 * (tile_ry 1, 2, 4 or 8: tiles of 8*tile_ry rows), x points per lane
 * (tile_cols 1: tiles 64 wide; 2: tiles 128 wide with paired loads, tile_ry
 * 1, 2 or 4), z-chunk length (16..4096 planes per workgroup) and temporal
 * depth (2 or 4, temporal blocking only).  Results do not depend on the plan
 * (same bits). */
int fdtd_set_plan(fdtd_ctx *ctx, int32_t shot, int32_t variant, int32_t tile_ry, int32_t zchunk, int32_t tblock_k,
                  int32_t tile_cols);

/* Choice made for one shot: variant, tile height (tile_ry), temporal depth,
 * x points per lane (tile_cols).  Any output pointer may be NULL. */
int fdtd_get_plan(const fdtd_ctx *ctx, int32_t shot, int32_t *variant, int32_t *tile_ry, int32_t *tblock_k,
                  int32_t *tile_cols);

/* Storage scale of one shot (stored value = scale * u). */
int fdtd_get_scale(const fdtd_ctx *ctx, int32_t shot, double *scale);

/* Per-kernel timing for measurement: while enabled (eager fdtd_step only;
 * fdtd_step_graph returns FDTD_EUNSUPPORTED), every launch of the kernel
 * classes below is bracketed by HIP events on the context's stream, and the
 * kernels of a step run one after another (otherwise the interior update
 * runs on a second stream, concurrently with the psi pass and the band
 * kernels), so that each duration is the kernel's own.
 * fdtd_get_timing synchronises, returns the mean duration (ms) and count of
 * one class since timing was enabled, and keeps accumulating.
 * Classes: 0 = single-step update of the points outside the layer bands
 * (z-march kernel; the naive kernel updates every point), 1 = psi pre-pass,
 * 2 = receiver gather, 3 = ghost pack/unpack, 4 = update of the layer-band
 * points, 5 = temporal-blocking kernel (K steps of the interior box per
 * launch).  Enabling again clears the counters. */
int fdtd_set_timing(fdtd_ctx *ctx, int32_t enable);
int fdtd_get_timing(fdtd_ctx *ctx, int32_t kernel_class, double *mean_ms, int64_t *count);

/* Measurement: the streaming ceiling that the interior update is measured
 * against.  o[i] = a[i] + b[i] * c[i] over n float32 elements (three streams
 * read, one written: the interior update's mix of u^n, u^{n-1}, m in and
 * u^{n+1} out), 16 bytes per lane, a grid-stride loop over `blocks` blocks of
 * 256 threads with `unroll` (1, 2 or 4) independent 16-byte pieces per thread
 * in flight.  blocks = 0 selects one-shot blocks instead: each block of 256
 * threads streams 256 * unroll consecutive 16-byte pieces once and exits, its
 * stores carrying the non-temporal hint of the field stores.  All four arrays
 * are device arrays of n floats, 16-byte aligned, n a multiple of 4 (EINVAL
 * otherwise, and for blocks < 0).  Asynchronous on hip_stream. */
int fdtd_stream_probe(const float *a_dev, const float *b_dev, const float *c_dev, float *o_dev, size_t n,
                      int32_t blocks, int32_t unroll, void *hip_stream);

const char *fdtd_strerror(int status);
const char *fdtd_last_error(const fdtd_ctx *ctx);
void fdtd_destroy(fdtd_ctx *ctx);

/* Size of the device array that holds the state of fdtd_forward_static. */
#define FDTD_STATIC_BYTES ((size_t)256 << 20)

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): one complete forward run of one shot,
 * equivalent to fdtd_create + fdtd_bind_workspace + fdtd_set_velocity +
 * fdtd_inject_source + fdtd_set_receivers + fdtd_record_receivers +
 * fdtd_step(nt) + fdtd_get_field + fdtd_destroy, with the same kernels and
 * the same results bit for bit, except that the context's workspace is a
 * fixed array of FDTD_STATIC_BYTES (256 MiB) compiled into the library
 * instead of caller memory.  Each GPU the library runs on holds its own copy
 * of that array from the library's first use on it until the process ends.
 * The call allocates no device memory (no hipMalloc, no allocating library
 * routine; host bookkeeping only) and creates no stream: everything runs on
 * hip_stream, and the call synchronises that stream before it returns (it
 * cannot be captured into a graph).
 *   shot         the shot's configuration, as for fdtd_create (one shot).
 *   v_dev        float32 [nz][ny][nx] velocity (m/s), as for fdtd_set_velocity.
 *   src_i/j/k, wavelet_dev, nt, amplitude
 *                point source as for fdtd_inject_source; wavelet_dev may be
 *                NULL (no source).  nt is also the number of steps run.
 *   rec_ijk_dev  int32 [nrec][3] receiver nodes (device), nrec >= 0.
 *   traces_dev   float32 [nt][nrec] (device): row n receives u^{n+1} at the
 *                receivers (required when nrec > 0).
 *   u_final_dev  float32 [nz][ny][nx] (device) receiving u^{nt}, or NULL.
 * Errors: those of the calls it stands for (EINVAL, EUNSTABLE, ...), and
 * FDTD_ENOMEM when the shot's workspace (fdtd_workspace_size of the same
 * configuration) exceeds FDTD_STATIC_BYTES, e.g. FP32 grids above about
 * 250^3 points, checked before any GPU work; the reason is printed to stderr.
 * Every call on one GPU shares that GPU's array and overwrites what the
 * previous call left there (everything that must start at zero is cleared on
 * entry): calls that overlap on one GPU, from several host threads or on
 * several streams, race and must be serialised by the caller. */
int fdtd_forward_static(const fdtd_shot_config *shot, const float *v_dev, int32_t src_i, int32_t src_j,
                        int32_t src_k, const float *wavelet_dev, int32_t nt, float amplitude,
                        const int32_t *rec_ijk_dev, int32_t nrec, float *traces_dev, float *u_final_dev,
                        void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_H */
