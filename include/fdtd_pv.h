/*
 * fdtd_pv.h -- C ABI of the first-order acoustic pressure-velocity FDTD + CPML
 * path of the MI355X (gfx950) library (the paper's own formulation).
 *
 * Operation (paper, section "Model", subsection "First-Order Acoustic Model and
 * Discrete Update", and section "CPML Boundary Layers"): each call of
 * fdtd_pv_step advances, per step,
 *
 *     v_d <- v_d - lambda [ kinv_d delta_d p + psi_v,d ]      (d = x, y, z)
 *     p   <- p   - lambda sum_d [ kinv_d delta_d v_d + psi_p,d ]
 *
 * with the radius-4 central first derivative (delta f)_i = sum_l a_l
 * (f_{i+l} - f_{i-l}) at unit spacing, lambda the wave-update scaling of the
 * paper's parameter table (c dt / h; 0.05 there), and inside the layer of
 * axis d the memory variables advanced with the current derivative before
 * they are used: psi <- b psi + a delta f.  b, a and kinv = 1/kappa follow
 * the cubic profiles of the same section in the normalised units c = h = 1,
 * dt = lambda (sigma_max = -4 ln R / (2 L), kappa_max = 5,
 * alpha_max = 0.05 sigma_max by default); outside the layers kinv = 1 and
 * psi = 0.  The grid is surrounded by zeros.  A point source adds
 * lambda w^n to p at its node after the pressure stage of step n; receivers
 * record p after each step.
 *
 * Conventions are those of fdtd.h: FDTD_* status codes, x-fastest dense
 * arrays (element (i, j, k) of an nx*ny*nz array at i + nx*(j + ny*k)),
 * *_dev pointers are device memory owned by the caller and only borrowed,
 * all GPU work is ordered on the stream given at creation, no entry point
 * synchronises unless stated, one host thread per context at a time.
 */
#ifndef FDTD_PV_H
#define FDTD_PV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_pv_ctx fdtd_pv_ctx;

/* One grid.  Zero-valued optional fields take the default shown. */
typedef struct {
    int32_t n[3];            /* nx, ny, nz (points, 9 .. 32768 each)                    */
    int32_t cpml[6];         /* layer width per face -x,+x,-y,+y,-z,+z (0 = none); the
                                two layers of an axis together narrower than the axis  */
    double lambda;           /* wave-update scaling c dt / h, in (0, 0.66722]: at most
                                2 / (sqrt(3) max_theta 2 sum_l a_l sin(l theta))        */
    double R;                /* target reflection, default 1e-8                         */
    double kappa_max;        /* default 5                                               */
    double alpha_frac;       /* alpha_max / sigma_max, default 0.05                     */
    int32_t variant;         /* 1: one thread per point; 2: z-marching stages (LDS xy
                                planes, register queue along z); 0: 2 from 2^24
                                points up, else 1.  Both give the same bits.            */
} fdtd_pv_config;

/* Create a context on hip_stream (a hipStream_t, may be NULL).  EINVAL for a
 * bad shape, layer or a lambda <= 0; EUNSTABLE for a lambda above the
 * leapfrog's stability limit 2 / (sqrt(3) max s) = 0.667226..., with s the
 * symbol of the first derivative, s(theta) = 2 sum_l a_l sin(l theta)
 * (computed from the weights on the host).  *out receives host memory owned by the
 * library (free with fdtd_pv_destroy). */
int fdtd_pv_create(const fdtd_pv_config *cfg, void *hip_stream, fdtd_pv_ctx **out);

/* Bytes of device workspace: p, v_x, v_y, v_z and the six memory-variable
 * fields (each padded by 4 points on every side), and the profiles. */
int fdtd_pv_workspace_size(const fdtd_pv_ctx *ctx, size_t *bytes);

/* Hand the context a device workspace of at least fdtd_pv_workspace_size
 * bytes, 256-byte aligned (ENOMEM if smaller, EINVAL if misaligned).  Zeroes
 * every field and uploads the profiles; synchronises the stream. */
int fdtd_pv_bind_workspace(fdtd_pv_ctx *ctx, void *dev_ptr, size_t bytes);

/* Pressure from / to a dense FP32 nx*ny*nz device array (v is left as is). */
int fdtd_pv_set_pressure(fdtd_pv_ctx *ctx, const float *p_dev);
int fdtd_pv_get_pressure(fdtd_pv_ctx *ctx, float *p_dev);

/* Point source at node (i, j, k) with nt FP32 samples w_dev (borrowed until
 * the context is destroyed or the source replaced); the n-th step since the
 * workspace was bound (n = 0, 1, ...) adds lambda w[n] for n < nt.  EINVAL
 * outside the grid. */
int fdtd_pv_set_source(fdtd_pv_ctx *ctx, int32_t i, int32_t j, int32_t k, const float *w_dev, int32_t nt);

/* Receivers: nrec (i, j, k) triples in rec_dev (int32, device); after the
 * n-th step from this call on (n = 0, 1, ...) p at receiver r goes to
 * traces_dev[n * nrec + r] for n < cap.  Both arrays are borrowed.  EINVAL
 * for a receiver outside the grid (checked on the host: synchronises). */
int fdtd_pv_set_receivers(fdtd_pv_ctx *ctx, const int32_t *rec_dev, int32_t nrec, float *traces_dev, int32_t cap);

/* Advance nsteps steps (two kernels per step, plus the receiver gather). */
int fdtd_pv_step(fdtd_pv_ctx *ctx, int32_t nsteps);

/* Message of the last failed call on this context. */
const char *fdtd_pv_last_error(const fdtd_pv_ctx *ctx);

void fdtd_pv_destroy(fdtd_pv_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
