// kernels_step.hip -- one leapfrog step of the second-order acoustic FDTD + CPML on gfx950.
//
//  k_psi          layer-memory pre-pass: psi_d <- b psi_d + a D1_d u^n on every
//                 slab point (paper, section "CPML Boundary Layers": the memory
//                 variable recursion, updated before it is used).
//  k_update_naive one thread per grid point; all layer logic inline.
//  k_zmarch       xy tile (64 x 16*RY points) staged through LDS with a 4-cell
//                 halo, marching along z with a 9-plane register queue of u^n;
//                 4 consecutive x points per lane (16-byte loads).
//  k_record       receiver gather for every shot and the device step counter.
//
// All kernels evaluate a point with the shared functions of fdtd_dev.hpp, so
// the naive and z-marching variants give identical bits.
#include "fdtd_dev.hpp"

// ---------------------------------------------------------------------------
// compute box of a shot: x in [0,nx); y, z extended by `ext` on ghost axes
// ---------------------------------------------------------------------------
struct Box {
    int ylo, yhi, zlo, zhi;
};
__device__ __forceinline__ Box shot_box(const DevShot &s, int ext) {
    Box b;
    b.ylo = s.ghost[1] ? -ext : 0;
    b.yhi = s.ny + (s.ghost[1] ? ext : 0);
    b.zlo = s.ghost[2] ? -ext : 0;
    b.zhi = s.nz + (s.ghost[2] ? ext : 0);
    return b;
}

// ---------------------------------------------------------------------------
// psi pre-pass.  grid: (blocks over the largest slab, 3 axes, shots)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_psi(const DevShot *__restrict__ shots, int iu, int ext) {
    const DevShot &s = shots[blockIdx.z];
    const int d = blockIdx.y;
    const int lo = s.Llo[d], hi = s.Lhi[d];
    if (lo + hi == 0) return;
    Box bx = shot_box(s, ext);
    const int Ny = bx.yhi - bx.ylo, Nz = bx.zhi - bx.zlo;
    long count;
    if (d == 0) count = (long)s.LX * Ny * Nz;
    else if (d == 1) count = (long)s.nx * s.LY * Nz;
    else count = (long)s.nx * Ny * s.LZ;
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int x, y, z, k;
    if (d == 0) {
        int is = (int)(t % s.LX);
        long r = t / s.LX;
        y = bx.ylo + (int)(r % Ny);
        z = bx.zlo + (int)(r / Ny);
        x = is < lo ? is : s.nx - hi + (is - lo);
        k = x;
    } else if (d == 1) {
        x = (int)(t % s.nx);
        long r = t / s.nx;
        int js = (int)(r % s.LY);
        z = bx.zlo + (int)(r / s.LY);
        y = js < lo ? js : s.ny - hi + (js - lo);
        k = y;
    } else {
        x = (int)(t % s.nx);
        long r = t / s.nx;
        y = bx.ylo + (int)(r % Ny);
        int ks = (int)(r / Ny);
        z = ks < lo ? ks : s.nz - hi + (ks - lo);
        k = z;
    }
    const T *u = (const T *)s.u[iu];
    const long c = (long)z * s.S + (long)y * s.P + x;
    const long stride = d == 0 ? 1 : (d == 1 ? s.P : s.S);
    float fl[4], fh[4];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
        fl[l - 1] = Store<T>::ld(u + c - l * stride);
        fh[l - 1] = Store<T>::ld(u + c + l * stride);
    }
    float d1 = d1_axis(s.w1[d], fl, fh);
    float *p = &s.psi[d][psi_index(s, d, x, y, z)];
    *p = psi_update(prof_at(s, d, 0, k), *p, prof_at(s, d, 1, k), d1);
}

// ---------------------------------------------------------------------------
// naive update: one thread per point.  grid: (ceil(nx/64), ceil(Ny/4), Nz)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_update_naive(const DevShot *__restrict__ shots, int shot, Roles R,
                                                     const int *__restrict__ stepc) {
    const DevShot &s = shots[shot];
    Box bx = shot_box(s, R.ext);
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = bx.ylo + blockIdx.y * 4 + threadIdx.y;
    const int z = bx.zlo + blockIdx.z;
    if (x >= s.nx || y >= bx.yhi || z >= bx.zhi || in_box(R, x, y, z)) return;
    point_update_global<T>(s, (const T *)s.u[R.iu], (const T *)s.u[R.ium1], (T *)s.u[R.iout], x, y, z,
                           source_at(s, *stepc));
}

// ---------------------------------------------------------------------------
// z-marching update
// ---------------------------------------------------------------------------
__device__ __forceinline__ float comp(const float4 &v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}
__device__ __forceinline__ void set_comp(float4 &v, int k, float f) {
    if (k == 0) v.x = f;
    else if (k == 1) v.y = f;
    else if (k == 2) v.z = f;
    else v.w = f;
}

template <typename T, int RY> struct ZCtx {
    static constexpr int TY = 16 * RY;
    static constexpr int NROW = TY + 8;
    const DevShot *s;
    const T *u;         // u^n
    const T *um;        // u^{n-1} (FP32 storage)
    T *w;               // u^{n+1} out (FP32: may equal um, in-place step)
    T *sec;             // second state field: FP32 u^{n-1}, 16-bit d^n (updated in place)
    const Roles *R;     // roles and exclusion box
    const float *m;
    int x0, y0, x, tx, ty;
    int yhi;
    long rowoff[RY];    // y*P + x for own rows
    int halo_slot;      // LDS float4 index this thread fills, -1 if none
    long halo_off;      // element offset (within a plane) of that halo float4
    bool cpml_xy;       // tile touches an x or y band
    bool partial;       // tile's xy footprint overlaps the exclusion box only partly
    int zlo_band, zhi_band; // z band: z < zlo_band || z >= zhi_band
    int step;
    float src;
};

template <typename T, int RY, int PH>
__device__ __forceinline__ void zbody(ZCtx<T, RY> &C, float4 (&q)[9][RY], float4 *sm, int z) {
    constexpr int TY = ZCtx<T, RY>::TY;
    const DevShot &s = *C.s;
    auto slot = [](int o) { return (PH + 4 + o + 9) % 9; };
    const long pz = (long)z * s.S;
    // global loads for this plane
#pragma unroll
    for (int r = 0; r < RY; ++r) q[slot(4)][r] = Store<T>::ld4(C.u + pz + 4 * (long)s.S + C.rowoff[r]);
    float4 um1[RY], mv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        um1[r] = Store<T>::ld4(C.sec + pz + C.rowoff[r]);
        mv[r] = *(const float4 *)(C.m + pz + C.rowoff[r]);
    }
    float4 hv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (C.halo_slot >= 0) hv = Store<T>::ld4(C.u + pz + C.halo_off);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) sm[(4 + C.ty * RY + r) * 18 + 1 + C.tx] = q[slot(0)][r];
    if (C.halo_slot >= 0) sm[C.halo_slot] = hv;
    __syncthreads();
    // y column of this lane's float4: rows ty*RY .. ty*RY+RY+7 (centre rows from registers)
    float4 ycol[RY + 8];
#pragma unroll
    for (int j = 0; j < RY + 8; ++j) {
        if (j >= 4 && j < 4 + RY) ycol[j] = q[slot(0)][j - 4];
        else ycol[j] = sm[(C.ty * RY + j) * 18 + 1 + C.tx];
    }
    const bool cpml = C.cpml_xy || z < C.zlo_band || z >= C.zhi_band;
    const bool srcplane = (wrap_ghost(s, 2, z) == s.sz);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = C.y0 + C.ty * RY + r;
        const float4 L = sm[(4 + C.ty * RY + r) * 18 + C.tx];
        const float4 R = sm[(4 + C.ty * RY + r) * 18 + C.tx + 2];
        const float4 Cc = q[slot(0)][r];
        const float xa[12] = {L.x, L.y, L.z, L.w, Cc.x, Cc.y, Cc.z, Cc.w, R.x, R.y, R.z, R.w};
        float4 out, outd;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float xl[4], xh[4], yl[4], yh[4], zl[4], zh[4];
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                xl[l - 1] = xa[4 + k - l];
                xh[l - 1] = xa[4 + k + l];
                yl[l - 1] = comp(ycol[4 + r - l], k);
                yh[l - 1] = comp(ycol[4 + r + l], k);
                zl[l - 1] = comp(q[slot(-l)][r], k);
                zh[l - 1] = comp(q[slot(l)][r], k);
            }
            const float c = xa[4 + k];
            const float lt = lap_interior(s, c, xl, xh, yl, yh, zl, zh);
            const bool src = srcplane && C.x + k == s.sx && wrap_ghost(s, 1, y) == s.sy;
            const Upd u = time_update<T>(comp(mv[r], k), lt, c, comp(um1[r], k), src, C.src);
            set_comp(out, k, u.u);
            set_comp(outd, k, u.d);
        }
        if (y < C.yhi) {
            T *dst = C.w + pz + C.rowoff[r];
            T *dsd = C.sec + pz + C.rowoff[r];
            if (!cpml && !C.partial && C.x + 3 < s.nx) {
                Store<T>::st4(dst, out);
                if constexpr (IsInc<T>::v) Store<T>::st4(dsd, outd);
            } else {
                // band points are written by the layer pass (it still needs the old state there);
                // points of the exclusion box are left alone
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (C.x + k < s.nx && !(cpml && any_band(s, C.x + k, y, z)) &&
                        !(C.partial && in_box(*C.R, C.x + k, y, z))) {
                        Store<T>::st(dst + k, comp(out, k));
                        if constexpr (IsInc<T>::v) Store<T>::st(dsd + k, comp(outd, k));
                    }
            }
        }
    }
}

template <typename T, int RY>
__global__ __launch_bounds__(256) void k_zmarch(const DevShot *__restrict__ shots, const WorkItem *__restrict__ work,
                                               Roles R, int zchunk, const int *__restrict__ stepc) {
    constexpr int TY = 16 * RY;
    constexpr int NROW = TY + 8;
    __shared__ float4 sm[NROW * 18];
    const WorkItem wi = work[blockIdx.x];
    const DevShot &s = shots[wi.shot];
    const int ext = R.ext;
    Box bx = shot_box(s, ext);
    ZCtx<T, RY> C;
    C.s = &s;
    C.y0 = bx.ylo + wi.ty * TY;
    if (C.y0 >= bx.yhi) return;
    const int zb = bx.zlo + wi.zc * zchunk;
    if (zb >= bx.zhi) return;
    const int ze = min(zb + zchunk, bx.zhi);
    C.yhi = bx.yhi;
    C.u = (const T *)s.u[R.iu];
    C.um = (const T *)s.u[R.ium1];
    C.w = (T *)s.u[R.iout];
    C.sec = IsInc<T>::v ? (T *)s.dinc : (T *)s.u[R.ium1];
    C.R = &R;
    C.m = s.m;
    C.x0 = wi.tx * 64;
    C.tx = threadIdx.x & 15;
    C.ty = threadIdx.x >> 4;
    C.x = C.x0 + 4 * C.tx;
#pragma unroll
    for (int r = 0; r < RY; ++r) C.rowoff[r] = (long)(C.y0 + C.ty * RY + r) * s.P + C.x;
    // halo assignment: 2*TY x-halo float4s, then 8 rows x 16 float4 y-halo
    const int t = threadIdx.x;
    C.halo_slot = -1;
    C.halo_off = 0;
    if (t < 2 * TY) {
        int row = t >> 1, side = t & 1;
        C.halo_slot = (4 + row) * 18 + (side ? 17 : 0);
        C.halo_off = (long)(C.y0 + row) * s.P + (side ? C.x0 + 64 : C.x0 - 4);
    } else if (t < 2 * TY + 128) {
        int k = t - 2 * TY, r8 = k >> 4, col = k & 15;
        int lrow = r8 < 4 ? r8 : TY + r8;
        int gy = r8 < 4 ? C.y0 - 4 + r8 : C.y0 + TY + (r8 - 4);
        C.halo_slot = lrow * 18 + 1 + col;
        C.halo_off = (long)gy * s.P + C.x0 + 4 * col;
    }
    // tile/plane layer classification
    bool cx = false, cy = false;
    if (s.Llo[0] > 0 && C.x0 < s.Llo[0] + FDTD_R) cx = true;
    if (s.Lhi[0] > 0 && C.x0 + 63 >= s.nx - s.Lhi[0] - FDTD_R) cx = true;
    if (s.Llo[1] > 0 && C.y0 < s.Llo[1] + FDTD_R) cy = true;
    if (s.Lhi[1] > 0 && C.y0 + TY - 1 >= s.ny - s.Lhi[1] - FDTD_R) cy = true;
    C.cpml_xy = cx || cy;
    C.zlo_band = s.Llo[2] > 0 ? s.Llo[2] + FDTD_R : -(1 << 30);
    C.zhi_band = s.Lhi[2] > 0 ? s.nz - s.Lhi[2] - FDTD_R : (1 << 30);
    C.step = *stepc;
    C.src = source_at(s, C.step);

    // exclusion box: a tile whose valid xy footprint lies inside it skips the
    // planes it covers (two z segments); a tile overlapping it partly masks points
    const int fx1 = min(C.x0 + 64, s.nx), fy1 = min(C.y0 + TY, bx.yhi);
    const bool boxz = R.lo[2] < R.hi[2] && R.lo[2] < ze && R.hi[2] > zb;
    const bool ovxy = C.x0 < R.hi[0] && fx1 > R.lo[0] && C.y0 < R.hi[1] && fy1 > R.lo[1];
    const bool inxy = C.x0 >= R.lo[0] && fx1 <= R.hi[0] && C.y0 >= R.lo[1] && fy1 <= R.hi[1];
    int seg_a[2] = {zb, 0}, seg_b[2] = {ze, 0};
    int nseg = 1;
    C.partial = false;
    if (boxz && ovxy) {
        if (inxy) {
            seg_b[0] = min(ze, R.lo[2]);
            seg_a[1] = max(zb, R.hi[2]);
            seg_b[1] = ze;
            nseg = 2;
        } else {
            C.partial = true;
        }
    }

    // band points are the band kernel's: planes of the z band are skipped, and
    // a tile whose footprint lies inside the x or y band has nothing to do
    {
        int nlo[3], nhi[3];
        const int n3[3] = {s.nx, s.ny, s.nz};
        band_box(n3, s.Llo, s.Lhi, s.ghost, ext, 6, nlo, nhi);
        if (C.x0 >= nhi[0] || fx1 <= nlo[0] || C.y0 >= nhi[1] || fy1 <= nlo[1]) return;
        for (int sg = 0; sg < nseg; ++sg) {
            seg_a[sg] = max(seg_a[sg], nlo[2]);
            seg_b[sg] = min(seg_b[sg], nhi[2]);
        }
    }
    float4 q[9][RY];
    for (int sg = 0; sg < nseg; ++sg) {
        const int a = seg_a[sg], b = seg_b[sg];
        if (a >= b) continue;
#pragma unroll
        for (int o = -4; o < 4; ++o)
#pragma unroll
            for (int r = 0; r < RY; ++r) q[o + 4][r] = Store<T>::ld4(C.u + (long)(a + o) * s.S + C.rowoff[r]);
#pragma unroll
        for (int r = 0; r < RY; ++r) q[8][r] = make_float4(0.f, 0.f, 0.f, 0.f);

        for (int z = a; z < b; ++z) {
            switch ((z - a) % 9) {
            case 0: zbody<T, RY, 0>(C, q, sm, z); break;
            case 1: zbody<T, RY, 1>(C, q, sm, z); break;
            case 2: zbody<T, RY, 2>(C, q, sm, z); break;
            case 3: zbody<T, RY, 3>(C, q, sm, z); break;
            case 4: zbody<T, RY, 4>(C, q, sm, z); break;
            case 5: zbody<T, RY, 5>(C, q, sm, z); break;
            case 6: zbody<T, RY, 6>(C, q, sm, z); break;
            case 7: zbody<T, RY, 7>(C, q, sm, z); break;
            default: zbody<T, RY, 8>(C, q, sm, z); break;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// receivers of every shot, then advance the device step counter.  One block.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_record(const DevShot *__restrict__ shots, int nshots, Roles R,
                                                 int *__restrict__ stepc) {
    const int n = *stepc;
    for (int si = 0; si < nshots; ++si) {
        const DevShot &s = shots[si];
        if (s.traces == nullptr || n >= s.trace_cap) continue;
        const T *u = (const T *)s.u[R.iout];
        for (int r = threadIdx.x; r < s.nrec; r += blockDim.x) {
            const int32_t *q = s.rec + 3 * r;
            if (in_box(R, q[0], q[1], q[2])) continue;   // recorded by the temporal-blocking kernel
            long c = (long)q[2] * s.S + (long)q[1] * s.P + q[0];
            s.traces[(long)n * s.nrec + r] = Store<T>::ld(u + c) * s.inv_scale;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *stepc = n + 1;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename T>
static void launch_psi_t(const DevShot *d_shots, int nshots, long max_count, int iu, int ext, hipStream_t st) {
    if (max_count <= 0) return;
    dim3 grid((unsigned)((max_count + 255) / 256), 3, nshots);
    hipLaunchKernelGGL(k_psi<T>, grid, dim3(256), 0, st, d_shots, iu, ext);
}
template <typename T>
static void launch_naive_t(const DevShot *d_shots, int shot, int nx, int Ny, int Nz, const Roles &R,
                           const int *stepc, hipStream_t st) {
    dim3 grid((nx + 63) / 64, (Ny + 3) / 4, Nz);
    hipLaunchKernelGGL(k_update_naive<T>, grid, dim3(64, 4), 0, st, d_shots, shot, R, stepc);
}
template <typename T>
static void launch_zmarch_t(const DevShot *d_shots, const WorkItem *work, int nwork, int ry, const Roles &R,
                            int zchunk, const int *stepc, hipStream_t st) {
    if (nwork <= 0) return;
    switch (ry) {
    case 1:
        hipLaunchKernelGGL((k_zmarch<T, 1>), dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
        break;
    case 4:
        hipLaunchKernelGGL((k_zmarch<T, 4>), dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
        break;
    default:
        hipLaunchKernelGGL((k_zmarch<T, 2>), dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
        break;
    }
}
template <typename T>
static void launch_record_t(const DevShot *d_shots, int nshots, const Roles &R, int *stepc, hipStream_t st) {
    hipLaunchKernelGGL(k_record<T>, dim3(1), dim3(1024), 0, st, d_shots, nshots, R, stepc);
}

#define FDTD_DISPATCH(stor, F, ...)                                                                      \
    do {                                                                                                  \
        if ((stor) == 1) F<_Float16>(__VA_ARGS__);                                                        \
        else if ((stor) == 2) F<__bf16>(__VA_ARGS__);                                                     \
        else F<float>(__VA_ARGS__);                                                                       \
    } while (0)

void fdtd_launch_psi(int stor, const DevShot *d_shots, int nshots, long max_count, int iu, int ext,
                     hipStream_t st) {
    FDTD_DISPATCH(stor, launch_psi_t, d_shots, nshots, max_count, iu, ext, st);
}
void fdtd_launch_naive(int stor, const DevShot *d_shots, int shot, int nx, int Ny, int Nz, const Roles &R,
                       const int *stepc, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_naive_t, d_shots, shot, nx, Ny, Nz, R, stepc, st);
}
void fdtd_launch_zmarch(int stor, const DevShot *d_shots, const WorkItem *work, int nwork, int ry, const Roles &R,
                        int zchunk, const int *stepc, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_zmarch_t, d_shots, work, nwork, ry, R, zchunk, stepc, st);
}
void fdtd_launch_record(int stor, const DevShot *d_shots, int nshots, const Roles &R, int *stepc, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_record_t, d_shots, nshots, R, stepc, st);
}
