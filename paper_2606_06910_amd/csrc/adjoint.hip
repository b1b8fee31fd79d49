// adjoint.hip -- reverse-time adjoint of the step and the model gradient.
#include "fdtd_host.hpp"
#include "fdtd_launch.hpp"

extern "C" {
int fdtd_adjoint_workspace_size(const fdtd_ctx *ctx, int32_t shot, int32_t every, int32_t nt, size_t *bytes) {
    (void)ctx; (void)shot; (void)every; (void)nt; (void)bytes;
    return FDTD_EUNSUPPORTED;
}
int fdtd_set_checkpointing(fdtd_ctx *ctx, int32_t shot, int32_t every, void *buf_dev, size_t bytes) {
    (void)ctx; (void)shot; (void)every; (void)buf_dev; (void)bytes;
    return FDTD_EUNSUPPORTED;
}
int fdtd_adjoint(fdtd_ctx *ctx, int32_t shot, int32_t nt, const float *resid_dev, double *grad_v_dev) {
    (void)ctx; (void)shot; (void)nt; (void)resid_dev; (void)grad_v_dev;
    return FDTD_EUNSUPPORTED;
}
int fdtd_autotune(fdtd_ctx *ctx, const char *cache_path) {
    (void)ctx; (void)cache_path;
    return FDTD_EUNSUPPORTED;
}
}
