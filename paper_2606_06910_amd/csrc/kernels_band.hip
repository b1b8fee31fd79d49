// kernels_band.hip -- update of the layer-band points (gfx950).
//
// The band is the union of the absorbing-layer slabs and the 4-cell margin
// their psi derivative reaches (paper, section "CPML Boundary Layers": the
// stretched second derivative and its memory variables).  It is cut into six
// disjoint boxes (band_box); each box is tiled in 32 x 16 xy tiles that
// march along z.  Per tile and plane:
//   * the plane of u^n (tile plus a 4-cell halo) is staged in LDS for the x
//     and y neighbours; the z neighbours come from a per-thread register
//     queue of 9 planes;
//   * every owned point evaluates lap_point (the layer-aware Laplacian of
//     fdtd_dev.hpp, psi neighbours and zeta from the slab arrays) and the
//     time update, with the same operation order as the other kernels.
// Points outside every band are left to the interior kernels.
#include "fdtd_dev.hpp"

namespace {
constexpr int BTX = 32;               // tile width (x)
constexpr int BTY = 16;               // tile height (y): 8 thread rows x 2 points
constexpr int BLW = BTX + 2 * FDTD_R; // LDS row length
constexpr int BLH = BTY + 2 * FDTD_R; // LDS rows
constexpr int BHALO = 2 * FDTD_R * BTY + 2 * FDTD_R * BTX;   // 128 x-halo + 256 y-halo values
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_band(const DevShot *__restrict__ shots, const BandItem *__restrict__ work,
                                              Roles R, int zchunk, const int *__restrict__ stepc) {
    __shared__ float sm[BLH * BLW];
    const BandItem wi = work[blockIdx.x];
    const DevShot &s = shots[wi.shot];
    int blo[3], bhi[3];
    const int n3[3] = {s.nx, s.ny, s.nz};
    band_box(n3, s.Llo, s.Lhi, s.ghost, R.ext, wi.box, blo, bhi);
    const int x0 = blo[0] + wi.tx * BTX;
    const int y0 = blo[1] + wi.ty * BTY;
    const int za = blo[2] + wi.zc * zchunk;
    const int bx1 = bhi[0], by1 = bhi[1];
    if (x0 >= bx1 || y0 >= by1 || za >= bhi[2]) return;
    const int zb = min(za + zchunk, bhi[2]);

    const int lx = threadIdx.x & (BTX - 1);
    const int ly = threadIdx.x / BTX;   // 0..7, rows 2 ly and 2 ly + 1
    const int x = x0 + lx;
    const T *u = (const T *)s.u[R.iu];
    const T *um = (const T *)s.u[R.ium1];
    T *w = (T *)s.u[R.iout];
    const long S = s.S, P = s.P;
    long rowoff[2];
    rowoff[0] = (long)(y0 + 2 * ly) * P + x;
    rowoff[1] = rowoff[0] + P;

    // halo values this thread stages: items t and t + 256 of 384
    // (0..127: x halo, row r = i / 8, side (i / 4) & 1, offset i & 3;
    //  128..383: y halo, 8 rows of 32)
    int hslot[2];
    long hoff[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = threadIdx.x + 256 * k;
        hslot[k] = -1;
        hoff[k] = 0;
        if (i < 2 * FDTD_R * BTY) {
            const int r = i >> 3, side = (i >> 2) & 1, o = i & 3;
            const int col = side ? BTX + FDTD_R + o : o;
            hslot[k] = (FDTD_R + r) * BLW + col;
            hoff[k] = (long)(y0 + r) * P + (x0 - FDTD_R + col);
        } else if (i < BHALO) {
            const int j = i - 2 * FDTD_R * BTY, r8 = j / BTX, c = j % BTX;
            const int lrow = r8 < FDTD_R ? r8 : BTY + r8;
            hslot[k] = lrow * BLW + FDTD_R + c;
            hoff[k] = (long)(y0 - FDTD_R + lrow) * P + x0 + c;
        }
    }

    const float srcamp = source_at(s, *stepc);
    float q[9][2];
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
        for (int r = 0; r < 2; ++r) q[o][r] = Store<T>::ld(u + (long)(za - FDTD_R + o) * S + rowoff[r]);

#pragma unroll 1
    for (int z = za; z < zb; ++z) {
        const long pz = (long)z * S;
#pragma unroll
        for (int r = 0; r < 2; ++r) q[8][r] = Store<T>::ld(u + pz + FDTD_R * S + rowoff[r]);
        float hv[2] = {0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (hslot[k] >= 0) hv[k] = Store<T>::ld(u + pz + hoff[k]);
        __syncthreads();   // readers of the previous plane are done
#pragma unroll
        for (int r = 0; r < 2; ++r) sm[(FDTD_R + 2 * ly + r) * BLW + FDTD_R + lx] = q[4][r];
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (hslot[k] >= 0) sm[hslot[k]] = hv[k];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = y0 + 2 * ly + r;
            if (x < bx1 && y < by1 && !in_box(R, x, y, z)) {
                const int row = FDTD_R + 2 * ly + r, col = FDTD_R + lx;
                float xl[4], xh[4], yl[4], yh[4], zl[4], zh[4];
#pragma unroll
                for (int l = 1; l <= 4; ++l) {
                    xl[l - 1] = sm[row * BLW + col - l];
                    xh[l - 1] = sm[row * BLW + col + l];
                    yl[l - 1] = sm[(row - l) * BLW + col];
                    yh[l - 1] = sm[(row + l) * BLW + col];
                    zl[l - 1] = q[4 - l][r];
                    zh[l - 1] = q[4 + l][r];
                }
                const float c = q[4][r];
                const float lt = lap_point(s, x, y, z, c, xl, xh, yl, yh, zl, zh);
                const long off = pz + rowoff[r];
                T *sec = IsInc<T>::v ? (T *)s.dinc : (T *)um;
                const Upd up = time_update<T>(s.m[off], lt, c, Store<T>::ld(sec + off), is_source(s, x, y, z),
                                              srcamp);
                Store<T>::st(w + off, up.u);
                if constexpr (IsInc<T>::v) Store<T>::st(sec + off, up.d);
            }
        }
#pragma unroll
        for (int o = 0; o < 8; ++o)
#pragma unroll
            for (int r = 0; r < 2; ++r) q[o][r] = q[o + 1][r];
    }
}

template <typename T>
static void launch_band_t(const DevShot *d_shots, const BandItem *work, int nwork, const Roles &R, int zchunk,
                          const int *stepc, hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_band<T>, dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
}

void fdtd_launch_band(int stor, const DevShot *d_shots, const BandItem *work, int nwork, const Roles &R, int zchunk,
                      const int *stepc, hipStream_t st) {
    if (stor == 1) launch_band_t<_Float16>(d_shots, work, nwork, R, zchunk, stepc, st);
    else if (stor == 2) launch_band_t<__bf16>(d_shots, work, nwork, R, zchunk, stepc, st);
    else launch_band_t<float>(d_shots, work, nwork, R, zchunk, stepc, st);
}
