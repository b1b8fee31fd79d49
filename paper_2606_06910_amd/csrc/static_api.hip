// static_api.hip -- fdtd_forward_static: one complete forward run of one shot
// whose library state lives in a fixed device array of this library instead
// of a caller-provided workspace, for callers that cannot allocate device
// memory.  It drives the same orchestration and kernels as fdtd_step on a
// bound workspace, so its results are those of that path, bit for bit.
#include "../../include/fdtd.h"
#include "fdtd_host.hpp"

#include <cstdio>
#include <mutex>

// The context's whole workspace (fields, model, layer memory, profiles, work
// lists, exchange buffers, step counter).  Each GPU the library runs on holds
// its own copy until the process ends.  In host code this name is only a
// stand-in for the symbol: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[FDTD_STATIC_BYTES];

static std::mutex g_mu;
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];   // per device id, set once with that device current

// device address of the current device's copy of the array (looked up once per device)
static int scratch_ptr(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FDTD_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fprintf(stderr, "fdtd_forward_static: hipGetSymbolAddress: %s\n", hipGetErrorString(e));
            return FDTD_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FDTD_OK;
}

extern "C" int fdtd_forward_static(const fdtd_shot_config *shot, const float *v_dev, int32_t src_i, int32_t src_j,
                                   int32_t src_k, const float *wavelet_dev, int32_t nt, float amplitude,
                                   const int32_t *rec_ijk_dev, int32_t nrec, float *traces_dev, float *u_final_dev,
                                   void *hip_stream) {
    if (!shot || !v_dev || nt < 0 || nrec < 0 || (nrec > 0 && (!rec_ijk_dev || !traces_dev))) return FDTD_EINVAL;
    void *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    fdtd_ctx *ctx = nullptr;
    rc = fdtd_create(shot, 1, hip_stream, &ctx);
    if (rc) return rc;
    if (ctx->need > (size_t)FDTD_STATIC_BYTES) {
        fprintf(stderr, "fdtd_forward_static: the shot needs %zu bytes of device state; the static array holds %zu\n",
                ctx->need, (size_t)FDTD_STATIC_BYTES);
        fdtd_destroy(ctx);
        return FDTD_ENOMEM;
    }
    // everything on the caller's stream: no second stream is created
    ctx->single_stream = true;
    rc = fdtd_bind_workspace(ctx, base, (size_t)FDTD_STATIC_BYTES);
    if (!rc) rc = fdtd_set_velocity(ctx, 0, v_dev);
    if (!rc && wavelet_dev) rc = fdtd_inject_source(ctx, 0, src_i, src_j, src_k, wavelet_dev, nt, amplitude);
    if (!rc && nrec > 0) rc = fdtd_set_receivers(ctx, 0, rec_ijk_dev, nrec);
    if (!rc && nrec > 0 && nt > 0) rc = fdtd_record_receivers(ctx, 0, traces_dev, nt);
    if (!rc) rc = fdtd_step(ctx, nt);
    if (!rc && u_final_dev) rc = fdtd_get_field(ctx, 0, 0, u_final_dev);
    if (rc) fprintf(stderr, "fdtd_forward_static: %s\n", ctx->err.c_str());
    // the array is reused by the next call: let this run finish before it returns
    if (!rc && hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) rc = FDTD_EHIP;
    fdtd_destroy(ctx);
    return rc;
}
