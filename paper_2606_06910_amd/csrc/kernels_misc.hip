// kernels_misc.hip -- setup, conversion and ghost-exchange kernels (gfx950).
//
//  k_fill_zero       zero a byte range with 16-byte stores (used instead of a
//                    runtime memset so that captured work never contains one)
//  k_vel_to_m        m = v^2 dt^2 into the padded field layout, and max(v)
//  k_get_field/k_set_field  dense float32 <-> padded storage (scale applied)
//  k_copy_jobs       strided box copies: ghost-face pack into contiguous
//                    buffers and unpack into the opposite ghost rows (the
//                    loopback stands in for the neighbour of one GPU's
//                    pencil-yz share, paper section "Multi-GPU Decomposition
//                    and Halo Exchange")
//  k_finite          flag any NaN/Inf in a field
#include "fdtd_dev.hpp"

__global__ __launch_bounds__(256) void k_fill_zero(uint4 *p, size_t n16) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// grid: (ceil(nx/256), ny, nz)
__global__ __launch_bounds__(256) void k_vel_to_m(const float *__restrict__ v, float *__restrict__ m, int nx, int ny,
                                                 int P, int S, double dt2, unsigned int *__restrict__ vmax_bits) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    float vv = 0.0f;
    if (x < nx) {
        vv = v[((long)z * ny + y) * nx + x];
        m[(long)z * S + (long)y * P + x] = (float)((double)vv * (double)vv * dt2);
    }
    // block max of the bit patterns (v > 0, so float order == unsigned order)
    __shared__ unsigned int red[256];
    unsigned int b = __float_as_uint(fmaxf(vv, 0.0f));
    red[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(vmax_bits, red[0]);
}

// minimum of v (to reject v <= 0): grid as k_vel_to_m
__global__ __launch_bounds__(256) void k_vel_min(const float *__restrict__ v, int nx, int ny,
                                                unsigned int *__restrict__ bad) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    float vv = v[((long)blockIdx.z * ny + blockIdx.y) * nx + x];
    if (!(vv > 0.0f) || !isfinite(vv)) atomicOr(bad, 1u);
}

template <typename T>
__global__ __launch_bounds__(256) void k_get_field(const T *__restrict__ u, float *__restrict__ dst, int nx, int ny,
                                                  int P, int S, float inv_scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    dst[((long)z * ny + y) * nx + x] = Store<T>::ld(u + (long)z * S + (long)y * P + x) * inv_scale;
}

template <typename T>
__global__ __launch_bounds__(256) void k_set_field(T *__restrict__ u, const float *__restrict__ src, int nx, int ny,
                                                  int P, int S, float scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    Store<T>::st(u + (long)z * S + (long)y * P + x, src[((long)z * ny + y) * nx + x] * scale);
}

// 16-bit state (u^n, d^n): u^{n-1} = u^n - d^n
template <typename T>
__global__ __launch_bounds__(256) void k_get_prev(const T *__restrict__ u, const T *__restrict__ d, float *__restrict__ dst,
                                                 int nx, int ny, int P, int S, float inv_scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const long i = (long)blockIdx.z * S + (long)blockIdx.y * P + x;
    dst[((long)blockIdx.z * ny + blockIdx.y) * nx + x] = (Store<T>::ld(u + i) - Store<T>::ld(d + i)) * inv_scale;
}
template <typename T>
__global__ __launch_bounds__(256) void k_set_prev(const T *__restrict__ u, T *__restrict__ d, const float *__restrict__ src,
                                                 int nx, int ny, int P, int S, float scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const long i = (long)blockIdx.z * S + (long)blockIdx.y * P + x;
    Store<T>::st(d + i, Store<T>::ld(u + i) - src[((long)blockIdx.z * ny + blockIdx.y) * nx + x] * scale);
}

// One row of a job per group of lanes: `lanes` consecutive threads copy a row
// in vb-byte pieces (16-byte pieces for FP32 rows that allow them), a block
// takes 256 / lanes rows per pass and strides over the job's rows; the only
// index arithmetic is one 32-bit division per row.  grid: (row blocks, njobs)
template <typename V>
__device__ __forceinline__ void copy_row(const char *s, char *d, int nv, int tv, int lanes) {
    for (int v = tv; v < nv; v += lanes) ((V *)d)[v] = ((const V *)s)[v];
}
__global__ __launch_bounds__(256) void k_copy_jobs(const CopyJob *__restrict__ jobs) {
    const CopyJob j = jobs[blockIdx.y];
    const int nrows = j.ey * j.ez;
    const int nv = j.ex * j.esz / j.vb;            // pieces per row
    const int lanes = nv < 256 ? nv : 256;         // threads per row
    const int rp = 256 / lanes;                    // rows per block pass
    const int tr = (int)threadIdx.x / lanes, tv = (int)threadIdx.x - tr * lanes;
    if (tr >= rp) return;
    for (int r = (int)blockIdx.x * rp + tr; r < nrows; r += (int)gridDim.x * rp) {
        const int z = r / j.ey, y = r - z * j.ey;
        const char *s = (const char *)j.src + ((long)z * j.sz + (long)y * j.sy) * j.esz;
        char *d = (char *)j.dst + ((long)z * j.dz + (long)y * j.dy) * j.esz;
        switch (j.vb) {
        case 16: copy_row<uint4>(s, d, nv, tv, lanes); break;
        case 8: copy_row<uint2>(s, d, nv, tv, lanes); break;
        case 4: copy_row<uint32_t>(s, d, nv, tv, lanes); break;
        default: copy_row<uint16_t>(s, d, nv, tv, lanes); break;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_finite(const T *__restrict__ u, int nx, int ny, int P, int S,
                                               unsigned int *__restrict__ bad) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    float f = Store<T>::ld(u + (long)blockIdx.z * S + (long)blockIdx.y * P + x);
    if (!isfinite(f)) atomicOr(bad, 1u);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void fdtd_launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    size_t n16 = bytes / 16;
    if (n16 == 0) return;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint4 *)p, n16);
}
void fdtd_launch_vel_to_m(const float *v, float *m, int nx, int ny, int nz, int P, int S, double dt2,
                          unsigned int *vmax_bits, unsigned int *bad, hipStream_t st) {
    dim3 grid((nx + 255) / 256, ny, nz);
    hipLaunchKernelGGL(k_vel_min, grid, dim3(256), 0, st, v, nx, ny, bad);
    hipLaunchKernelGGL(k_vel_to_m, grid, dim3(256), 0, st, v, m, nx, ny, P, S, dt2, vmax_bits);
}
template <typename T>
static void gf(const void *u, float *dst, int nx, int ny, int nz, int P, int S, float inv, hipStream_t st) {
    hipLaunchKernelGGL(k_get_field<T>, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, st, (const T *)u, dst, nx, ny, P,
                       S, inv);
}
template <typename T>
static void sf(void *u, const float *src, int nx, int ny, int nz, int P, int S, float sc, hipStream_t st) {
    hipLaunchKernelGGL(k_set_field<T>, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, st, (T *)u, src, nx, ny, P, S,
                       sc);
}
template <typename T>
static void fin(const void *u, int nx, int ny, int nz, int P, int S, unsigned int *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_finite<T>, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, st, (const T *)u, nx, ny, P, S, bad);
}
#define MISC_DISPATCH(stor, F, ...)                                                                      \
    do {                                                                                                  \
        if ((stor) == 1) F<_Float16>(__VA_ARGS__);                                                        \
        else if ((stor) == 2) F<__bf16>(__VA_ARGS__);                                                     \
        else F<float>(__VA_ARGS__);                                                                       \
    } while (0)

void fdtd_launch_get_field(int stor, const void *u, float *dst, int nx, int ny, int nz, int P, int S, float inv,
                           hipStream_t st) {
    MISC_DISPATCH(stor, gf, u, dst, nx, ny, nz, P, S, inv, st);
}
void fdtd_launch_set_field(int stor, void *u, const float *src, int nx, int ny, int nz, int P, int S, float sc,
                           hipStream_t st) {
    MISC_DISPATCH(stor, sf, u, src, nx, ny, nz, P, S, sc, st);
}
void fdtd_launch_finite(int stor, const void *u, int nx, int ny, int nz, int P, int S, unsigned int *bad,
                        hipStream_t st) {
    MISC_DISPATCH(stor, fin, u, nx, ny, nz, P, S, bad, st);
}
template <typename T>
static void gp(const void *u, const void *d, float *dst, int nx, int ny, int nz, int P, int S, float inv, hipStream_t st) {
    hipLaunchKernelGGL(k_get_prev<T>, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, st, (const T *)u, (const T *)d, dst,
                       nx, ny, P, S, inv);
}
template <typename T>
static void sp(const void *u, void *d, const float *src, int nx, int ny, int nz, int P, int S, float sc, hipStream_t st) {
    hipLaunchKernelGGL(k_set_prev<T>, dim3((nx + 255) / 256, ny, nz), dim3(256), 0, st, (const T *)u, (T *)d, src, nx,
                       ny, P, S, sc);
}
void fdtd_launch_get_prev(int stor, const void *u, const void *d, float *dst, int nx, int ny, int nz, int P, int S,
                          float inv, hipStream_t st) {
    MISC_DISPATCH(stor, gp, u, d, dst, nx, ny, nz, P, S, inv, st);
}
void fdtd_launch_set_prev(int stor, const void *u, void *d, const float *src, int nx, int ny, int nz, int P, int S,
                          float sc, hipStream_t st) {
    MISC_DISPATCH(stor, sp, u, d, src, nx, ny, nz, P, S, sc, st);
}
void fdtd_launch_copy_jobs(const void *jobs, int njobs, long max_rows, hipStream_t st) {
    if (njobs <= 0 || max_rows <= 0) return;
    const unsigned gx = (unsigned)(max_rows < 1024 ? max_rows : 1024);
    hipLaunchKernelGGL(k_copy_jobs, dim3(gx, njobs), dim3(256), 0, st, (const CopyJob *)jobs);
}


// Streaming ceiling of the interior update's access mix: o = a + b * c over
// float4 lanes (three streams read, one written, 16 bytes per lane), a
// grid-stride loop with `unroll` independent float4 per thread in flight.
template <int U>
__global__ __launch_bounds__(256) void k_stream_probe(const float4 *__restrict__ a, const float4 *__restrict__ b,
                                                     const float4 *__restrict__ c, float4 *__restrict__ o, size_t n4) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n4; i += U * stride) {
        float4 x[U], y[U], z[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            x[k] = a[i + k * stride];
            y[k] = b[i + k * stride];
            z[k] = c[i + k * stride];
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            o[i + k * stride] = make_float4(fmaf(y[k].x, z[k].x, x[k].x), fmaf(y[k].y, z[k].y, x[k].y),
                                            fmaf(y[k].z, z[k].z, x[k].z), fmaf(y[k].w, z[k].w, x[k].w));
    }
    for (; i < n4; i += stride) {
        const float4 x = a[i], y = b[i], z = c[i];
        o[i] = make_float4(fmaf(y.x, z.x, x.x), fmaf(y.y, z.y, x.y), fmaf(y.z, z.z, x.z), fmaf(y.w, z.w, x.w));
    }
}
// The same mix in one-shot blocks: block i streams the 256 U consecutive
// float4 pieces from 256 U i on (thread t the pieces t, t + 256, ...) and
// exits; the stores carry the non-temporal hint, as the field stores do.
typedef float fdtd_v4f __attribute__((ext_vector_type(4)));
template <int U>
__global__ __launch_bounds__(256) void k_stream_chunk(const float4 *__restrict__ a, const float4 *__restrict__ b,
                                                     const float4 *__restrict__ c, float4 *__restrict__ o, size_t n4) {
    const size_t base = (size_t)blockIdx.x * 256 * U + threadIdx.x;
    float4 x[U], y[U], z[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const size_t i = base + (size_t)k * 256;
        if (i < n4) {
            x[k] = a[i];
            y[k] = b[i];
            z[k] = c[i];
        }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const size_t i = base + (size_t)k * 256;
        if (i < n4) {
            const fdtd_v4f r = {fmaf(y[k].x, z[k].x, x[k].x), fmaf(y[k].y, z[k].y, x[k].y),
                                fmaf(y[k].z, z[k].z, x[k].z), fmaf(y[k].w, z[k].w, x[k].w)};
            __builtin_nontemporal_store(r, (fdtd_v4f *)&o[i]);
        }
    }
}
void fdtd_launch_stream_probe(const float *a, const float *b, const float *c, float *o, size_t n4, int blocks,
                              int unroll, hipStream_t st) {
    const dim3 g((unsigned)blocks), t(256);
    const float4 *A = (const float4 *)a, *B = (const float4 *)b, *C = (const float4 *)c;
    if (blocks == 0) {
        const int u = unroll >= 4 ? 4 : (unroll == 2 ? 2 : 1);
        const dim3 gc((unsigned)((n4 + 256 * (size_t)u - 1) / (256 * (size_t)u)));
        if (u == 4) hipLaunchKernelGGL(k_stream_chunk<4>, gc, t, 0, st, A, B, C, (float4 *)o, n4);
        else if (u == 2) hipLaunchKernelGGL(k_stream_chunk<2>, gc, t, 0, st, A, B, C, (float4 *)o, n4);
        else hipLaunchKernelGGL(k_stream_chunk<1>, gc, t, 0, st, A, B, C, (float4 *)o, n4);
        return;
    }
    if (unroll >= 4) hipLaunchKernelGGL(k_stream_probe<4>, g, t, 0, st, A, B, C, (float4 *)o, n4);
    else if (unroll == 2) hipLaunchKernelGGL(k_stream_probe<2>, g, t, 0, st, A, B, C, (float4 *)o, n4);
    else hipLaunchKernelGGL(k_stream_probe<1>, g, t, 0, st, A, B, C, (float4 *)o, n4);
}

__global__ void k_set_int(int *p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}
void fdtd_launch_set_int(int *p, int v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, p, v);
}
