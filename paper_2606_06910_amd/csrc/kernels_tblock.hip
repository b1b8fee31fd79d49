// kernels_tblock.hip -- temporal blocking of the interior: K leapfrog steps per launch (gfx950).
//
// The single-GPU counterpart of the paper's enlarged ghost regions (section
// "Multi-GPU Decomposition and Halo Exchange"): a tile advances K steps on
// data held on chip, recomputing a halo that shrinks by the stencil radius
// (4) per step, instead of exchanging/reloading it every step.
//
// Geometry.  B is the box of points outside every layer band (FP32 storage,
// Dirichlet faces); B_j is B shrunk by 4 j.  Tiles cover B_K with cores of
// CX x CY points and a z chunk; stage j (level n+j) is computed on the tile's
// region R_j = core grown by 4 (K - j) in x, y and z.  Stage j runs 4 (j-1)
// planes behind stage 1 in the z march.  Level n+j is written where later
// work needs it: B_j \ B_{j+2} for j <= K-2, all of B_j for the last two
// levels.  The layer shell (everything outside B_j) is advanced afterwards,
// level by level, by the z-marching kernel with B_j as its exclusion box.
//
// On chip: every thread owns float4 columns of R_1 (the core first, then the
// rings outward), and keeps for each owned column a 9-plane register queue of
// every level that column advances (z neighbours, centre and the level below).
// The level-0 xy plane (R_0) and, for j < K, a 5-plane ring of level j over
// R_j live in LDS for the x/y neighbours.  Arithmetic per point is the
// interior formula of the other kernels (identical bits).
#include "fdtd_dev.hpp"

template <int K> struct TB;
template <> struct TB<2> {
    static constexpr int CX = 32, CY = 32;
};
template <> struct TB<4> {
    static constexpr int CX = 16, CY = 16;
};

template <int K> struct TBGeo {
    static constexpr int CX = TB<K>::CX, CY = TB<K>::CY;
    // margin of region R_j beyond the core (j = 0..K)
    static __host__ __device__ constexpr int a(int j) { return 4 * (K - j); }
    static __host__ __device__ constexpr int W4(int j) { return (CX + 2 * a(j)) / 4; }  // float4 columns per row
    static __host__ __device__ constexpr int H(int j) { return CY + 2 * a(j); }        // rows
    static __host__ __device__ constexpr int ncols(int j) { return W4(j) * H(j); }
    static constexpr int NT = 256;
    static_assert(ncols(1) <= 2 * NT, "R_1 must fit two columns per thread");
    static_assert(ncols(2) <= NT, "columns of R_2 must all be first slots");
    // LDS: level-0 plane over R_0, 5-plane rings of levels 1..K-1 over R_j
    static __host__ __device__ constexpr int ring_off(int j) {  // float4 offset of ring j (j >= 1)
        int o = ncols(0);
        for (int q = 1; q < j; ++q) o += 5 * ncols(q);
        return o;
    }
    static constexpr int LDS_F4 = ring_off(K);
};

// column index (cores first, rings outward) -> local f4 column (lx4 in units of 4 points
// relative to the core origin, may be negative), row ly, and the innermost stage jmax
template <int K>
__device__ __forceinline__ void col_of(int idx, int &lx, int &ly, int &jmax) {
    using G = TBGeo<K>;
    if (idx < G::ncols(K)) {
        lx = 4 * (idx % G::W4(K));
        ly = idx / G::W4(K);
        jmax = K;
        return;
    }
    idx -= G::ncols(K);
    for (int j = K - 1; j >= 1; --j) {
        const int aj = G::a(j), an = G::a(j + 1);
        const int w4 = G::W4(j);
        const int nrow = 2 * 4 * w4;          // 4 rows above and 4 below, full width
        const int nside = 2 * G::H(j + 1);    // one float4 left and right of the inner region
        if (idx < nrow) {
            const int r = idx / w4, c = idx % w4;
            ly = r < 4 ? -aj + r : G::CY + an + (r - 4);
            lx = -aj + 4 * c;
            jmax = j;
            return;
        }
        idx -= nrow;
        if (idx < nside) {
            const int r = idx >> 1;
            ly = -an + r;
            lx = (idx & 1) ? G::CX + an : -aj;
            jmax = j;
            return;
        }
        idx -= nside;
    }
    jmax = 0;  // not a column of R_1
    lx = ly = 0;
}

// halo of the level-0 plane: R_0 \ R_1 (4-wide ring), one float4 per index
template <int K> __device__ __forceinline__ bool halo_of(int idx, int &lx, int &ly) {
    using G = TBGeo<K>;
    const int a0 = G::a(0), a1 = G::a(1);
    const int w4 = G::W4(0);
    const int nrow = 2 * 4 * w4, nside = 2 * G::H(1);
    if (idx < nrow) {
        const int r = idx / w4, c = idx % w4;
        ly = r < 4 ? -a0 + r : G::CY + a1 + (r - 4);
        lx = -a0 + 4 * c;
        return true;
    }
    idx -= nrow;
    if (idx < nside) {
        ly = -a1 + (idx >> 1);
        lx = (idx & 1) ? G::CX + a1 : -a0;
        return true;
    }
    return false;
}

template <int K> __device__ __forceinline__ int lds_idx(int level, int slot5, int lx, int ly) {
    using G = TBGeo<K>;
    if (level == 0) return (ly + G::a(0)) * G::W4(0) + (lx + G::a(0)) / 4;
    return G::ring_off(level) + slot5 * G::ncols(level) + (ly + G::a(level)) * G::W4(level) + (lx + G::a(level)) / 4;
}

struct TBArgs {
    int blo[3], bhi[3];     // the box B (outside every band), x bounds multiples of 4
    int L[6];               // buffer index of level n-1 .. n+K: L[j+1] holds level n+j
    const int *rec_zs;      // receivers sorted by z: start offsets per plane [nz+1]
    const int *rec_ix;      // receiver indices in z order [nrec]
};

// level value at (column, component) from a float4
__device__ __forceinline__ float cmp4(const float4 &v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

template <int K> struct TBThread {
    int lx[2], ly[2], jm[2];   // owned columns (jm = 0: none)
    int gx[2], gy[2];          // global coordinates
    int hx, hy;                // halo float4 of the level-0 plane (hx = INT_MIN: none)
    bool has_halo;
};

// Is (x, y, z) inside B shrunk by 4 j?
__device__ __forceinline__ bool in_Bj(const TBArgs &A, int j, int x, int y, int z) {
    const int m = 4 * j;
    return x >= A.blo[0] + m && x < A.bhi[0] - m && y >= A.blo[1] + m && y < A.bhi[1] - m && z >= A.blo[2] + m &&
           z < A.bhi[2] - m;
}

template <int K, int PH>
__device__ __forceinline__ void tb_iter(const DevShot &s, const TBArgs &A, const TBThread<K> &T, float4 (&q0)[K][9],
                                        float4 (&q1)[9], float4 *sm, int i, int zlo_s1, int zhi_s1, int step0,
                                        int zb, int ze) {
    using G = TBGeo<K>;
    const float *mp = s.m;
    const float *u0 = (const float *)s.u[A.L[1]];   // level n
    const float *um = (const float *)s.u[A.L[0]];   // level n-1
    // slot of plane (i + o) in a 9-deep queue
    auto sl = [](int o) { return ((PH + o) % 9 + 9) % 9; };
    // 1. loads: level-0 plane i+4 for owned columns; halo of plane i
    const long pz4 = (long)(i + 4) * s.S;
    if (T.jm[0]) q0[0][sl(4)] = *(const float4 *)(u0 + pz4 + (long)T.gy[0] * s.P + T.gx[0]);
    if (T.jm[1]) q1[sl(4)] = *(const float4 *)(u0 + pz4 + (long)T.gy[1] * s.P + T.gx[1]);
    float4 hv = make_float4(0.f, 0.f, 0.f, 0.f);
    const int X0 = T.gx[0] - T.lx[0], Y0 = T.gy[0] - T.ly[0];   // core origin
    if (T.has_halo) hv = *(const float4 *)(u0 + (long)i * s.S + (long)(Y0 + T.hy) * s.P + X0 + T.hx);
    __syncthreads();
    // 2. level-0 plane i into LDS
    if (T.jm[0]) sm[lds_idx<K>(0, 0, T.lx[0], T.ly[0])] = q0[0][sl(0)];
    if (T.jm[1]) sm[lds_idx<K>(0, 0, T.lx[1], T.ly[1])] = q1[sl(0)];
    if (T.has_halo) sm[lds_idx<K>(0, 0, T.hx, T.hy)] = hv;
    __syncthreads();
    // 3. stages j = 1..K at plane p = i - 4 (j - 1)
#pragma unroll
    for (int j = 1; j <= K; ++j) {
        const int p = i - 4 * (j - 1);
        const int zlo = zb - G::a(j), zhi = ze + G::a(j);
        if (p < zlo || p >= zhi) continue;
        const float *ol = (const float *)s.u[A.L[j + 1]];
        const float src = source_at(s, step0 + j - 1);
#pragma unroll
        for (int sidx = 0; sidx < 2; ++sidx) {
            if (T.jm[sidx] < j) continue;
            if (sidx == 1 && j > 1) continue;      // second slots are ring-1 columns (stage 1 only)
            const int lx = T.lx[sidx], ly = T.ly[sidx];
            const int gx = T.gx[sidx], gy = T.gy[sidx];
            // level j-1 at plane p: centre, z neighbours (queue), x/y neighbours (LDS)
            float4 zq[9];
#pragma unroll
            for (int o = -4; o <= 4; ++o) {
                // level j-1 at plane p + o; its queue slot: plane (i - 4(j-2)) is the newest of level j-1
                const int so = sl(-4 * (j - 1) + o);
                zq[o + 4] = (sidx == 0) ? q0[j - 1][so] : q1[so];
            }
            const int slot5 = ((p % 5) + 5) % 5;
            const int lvl = j - 1;
            const float4 Lf = sm[lds_idx<K>(lvl, slot5, lx - 4, ly)];
            const float4 Rf = sm[lds_idx<K>(lvl, slot5, lx + 4, ly)];
            float4 yv[8];
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                yv[4 - l] = sm[lds_idx<K>(lvl, slot5, lx, ly - l)];
                yv[3 + l] = sm[lds_idx<K>(lvl, slot5, lx, ly + l)];
            }
            // level j-2 at plane p (u^{n-1} for j = 1 from memory)
            float4 prev;
            if (j == 1) prev = *(const float4 *)(um + (long)p * s.S + (long)gy * s.P + gx);
            else prev = q0[j - 2][sl(-4 * (j - 1))];   // level j-2 at plane p
            const float4 mv = *(const float4 *)(mp + (long)p * s.S + (long)gy * s.P + gx);
            const float4 c4 = zq[4];
            const float xa[12] = {Lf.x, Lf.y, Lf.z, Lf.w, c4.x, c4.y, c4.z, c4.w, Rf.x, Rf.y, Rf.z, Rf.w};
            float res[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float xl[4], xh[4], yl[4], yh[4], zl[4], zh[4];
#pragma unroll
                for (int l = 1; l <= 4; ++l) {
                    xl[l - 1] = xa[4 + k - l];
                    xh[l - 1] = xa[4 + k + l];
                    yl[l - 1] = cmp4(yv[4 - l], k);
                    yh[l - 1] = cmp4(yv[3 + l], k);
                    zl[l - 1] = cmp4(zq[4 - l], k);
                    zh[l - 1] = cmp4(zq[4 + l], k);
                }
                const float c = xa[4 + k];
                const float lt = lap_interior(s, c, xl, xh, yl, yh, zl, zh);
                const bool is_src = (p == s.sz && gy == s.sy && gx + k == s.sx);
                res[k] = time_update<float>(cmp4(mv, k), lt, c, cmp4(prev, k), is_src, src).u;
            }
            const float4 r4 = make_float4(res[0], res[1], res[2], res[3]);
            // hand the level on: queue (columns that advance further) and LDS ring (j < K)
            if (j < K) {
                if (sidx == 0 && T.jm[0] > j) q0[j][sl(-4 * (j - 1))] = r4;
                sm[lds_idx<K>(j, slot5, lx, ly)] = r4;
            }
            // write where later work reads it
            if (in_Bj(A, j, gx, gy, p)) {
                const bool keep = (j >= K - 1) || !in_Bj(A, j + 2, gx, gy, p);
                if (keep) *(float4 *)(ol + (long)p * s.S + (long)gy * s.P + gx) = r4;
                // receivers of this plane inside B_j
                if (s.traces != nullptr && step0 + j - 1 < s.trace_cap) {
                    for (int e = A.rec_zs[p]; e < A.rec_zs[p + 1]; ++e) {
                        const int r = A.rec_ix[e];
                        const int32_t *rq = s.rec + 3 * r;
                        if (rq[1] == gy && rq[0] >= gx && rq[0] < gx + 4)
                            s.traces[(long)(step0 + j - 1) * s.nrec + r] = cmp4(r4, rq[0] - gx) * s.inv_scale;
                    }
                }
            }
        }
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_tblock(const DevShot *__restrict__ shots, const WorkItem *__restrict__ work,
                                               TBArgs A, int zchunk, const int *__restrict__ stepc) {
    using G = TBGeo<K>;
    __shared__ float4 sm[G::LDS_F4];
    const WorkItem wi = work[blockIdx.x];
    const DevShot &s = shots[wi.shot];
    const int kx0 = A.blo[0] + 4 * K, kx1 = A.bhi[0] - 4 * K;
    const int ky0 = A.blo[1] + 4 * K, ky1 = A.bhi[1] - 4 * K;
    const int kz0 = A.blo[2] + 4 * K, kz1 = A.bhi[2] - 4 * K;
    const int X0 = kx0 + wi.tx * G::CX, Y0 = ky0 + wi.ty * G::CY;
    const int zb = kz0 + wi.zc * zchunk;
    if (X0 >= kx1 || Y0 >= ky1 || zb >= kz1) return;
    const int ze = min(zb + zchunk, kz1);
    TBThread<K> T;
#pragma unroll
    for (int sidx = 0; sidx < 2; ++sidx) {
        const int idx = threadIdx.x + 256 * sidx;
        if (idx < G::ncols(1)) {
            col_of<K>(idx, T.lx[sidx], T.ly[sidx], T.jm[sidx]);
        } else {
            T.lx[sidx] = T.ly[sidx] = 0;
            T.jm[sidx] = 0;
        }
        T.gx[sidx] = X0 + T.lx[sidx];
        T.gy[sidx] = Y0 + T.ly[sidx];
    }
    T.has_halo = halo_of<K>(threadIdx.x, T.hx, T.hy);
    if (!T.has_halo) T.hx = T.hy = 0;
    const int step0 = *stepc;
    const float *u0 = (const float *)s.u[A.L[1]];
    float4 q0[K][9], q1[9];
    const int i0 = zb - G::a(1);
    // prologue: level-0 planes i0-4 .. i0+3 (plane P lives in queue slot (P - i0) mod 9)
#pragma unroll
    for (int o = -4; o < 4; ++o) {
        const long pz = (long)(i0 + o) * s.S;
        const int so = (o + 9) % 9;
        if (T.jm[0]) q0[0][so] = *(const float4 *)(u0 + pz + (long)T.gy[0] * s.P + T.gx[0]);
        if (T.jm[1]) q1[so] = *(const float4 *)(u0 + pz + (long)T.gy[1] * s.P + T.gx[1]);
    }
    const int iend = ze + G::a(1);
    for (int i = i0; i < iend; ++i) {
        switch ((i - i0) % 9) {
        case 0: tb_iter<K, 0>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 1: tb_iter<K, 1>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 2: tb_iter<K, 2>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 3: tb_iter<K, 3>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 4: tb_iter<K, 4>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 5: tb_iter<K, 5>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 6: tb_iter<K, 6>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        case 7: tb_iter<K, 7>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        default: tb_iter<K, 8>(s, A, T, q0, q1, sm, i, 0, 0, step0, zb, ze); break;
        }
    }
}

// core size of the temporal-blocking tiles (host side needs it for the work list)
int fdtd_tblock_core(int K, int axis) {
    if (K == 4) return axis == 0 ? TB<4>::CX : TB<4>::CY;
    return axis == 0 ? TB<2>::CX : TB<2>::CY;
}

void fdtd_launch_tblock(const DevShot *d_shots, const WorkItem *work, int nwork, int K, const void *args, int zchunk,
                        const int *stepc, hipStream_t st) {
    if (nwork <= 0) return;
    const TBArgs &A = *(const TBArgs *)args;
    if (K == 4)
        hipLaunchKernelGGL(k_tblock<4>, dim3(nwork), dim3(256), 0, st, d_shots, work, A, zchunk, stepc);
    else
        hipLaunchKernelGGL(k_tblock<2>, dim3(nwork), dim3(256), 0, st, d_shots, work, A, zchunk, stepc);
}
