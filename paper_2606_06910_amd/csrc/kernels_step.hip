// kernels_step.hip -- one leapfrog step of the second-order acoustic FDTD + CPML on gfx950.
//
//  k_psi_y        layer-memory pre-pass of y: psi_y <- b psi_y + a D1_y u^n on
//                 every y-slab point (paper, section "CPML Boundary Layers": the
//                 memory variable recursion, updated before it is used), along
//                 y lines with a register queue.
//  k_psi          the same for x and z, for shots whose band kernel does not
//                 advance psi_x and psi_z itself.
//  k_update_naive one thread per grid point; all layer logic inline.
//  k_zmarch       points outside the layer bands: xy tile (64 x NW*RY points)
//                 staged through LDS with a 4-cell halo, marching along z with
//                 an 11-plane register queue of u^n; one x point per lane.
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
// psi pre-pass of x and z (shots whose band kernel does not advance them
// itself).  grid: (blocks over the largest slab, axes d0 .., shots)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_psi(const DevShot *__restrict__ shots, int iu, int ext, int d0) {
    typedef __attribute__((address_space(1))) const T gT;
    typedef __attribute__((address_space(1))) float gf;
    const DevShot &s = shots[blockIdx.z];
    const int d = d0 + (int)blockIdx.y;
    const int lo = s.Llo[d], hi = s.Lhi[d];
    if (lo + hi == 0 || d == 1 || s.fused) return;   // psi_y: k_psi_y
    const Box bx = shot_box(s, ext);
    const unsigned Ny = bx.yhi - bx.ylo, Nz = bx.zhi - bx.zlo;
    // slab points as (a fastest, b, c): x-slab (is, y, z), y-slab (x, js, z), z-slab (x, y, ks)
    const unsigned W = d == 0 ? (unsigned)s.LX : (unsigned)s.nx;
    const unsigned M = d == 1 ? (unsigned)s.LY : Ny;
    const unsigned N = d == 2 ? (unsigned)s.LZ : Nz;
    // workgroups go to the 8 XCDs in turn; give each XCD a contiguous range of
    // logical blocks (the grid is a multiple of 8), so that the u rows that
    // neighbouring slab rows share are read through one L2
    const unsigned per = gridDim.x >> 3;
    const unsigned lb = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    const unsigned t = lb * 256u + threadIdx.x;
    if (t >= W * M * N) return;
    const unsigned r = t / W, a = t - r * W;
    const unsigned c = r / M, b = r - c * M;
    int x, y, z, k;
    if (d == 0) {
        x = (int)a < lo ? (int)a : s.nx - hi + ((int)a - lo);
        y = bx.ylo + (int)b;
        z = bx.zlo + (int)c;
        k = x;
    } else if (d == 1) {
        x = (int)a;
        y = (int)b < lo ? (int)b : s.ny - hi + ((int)b - lo);
        z = bx.zlo + (int)c;
        k = y;
    } else {
        x = (int)a;
        y = bx.ylo + (int)b;
        z = (int)c < lo ? (int)c : s.nz - hi + ((int)c - lo);
        k = z;
    }
    gT *u = (gT *)s.u[iu] + ((long)z * s.S + (long)y * s.P + x);
    const long stride = d == 0 ? 1 : (d == 1 ? s.P : s.S);
    float fl[4], fh[4];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
        fl[l - 1] = (float)u[-l * stride];
        fh[l - 1] = (float)u[l * stride];
    }
    const float d1 = d1_axis(s.w1[d], fl, fh);
    gf *pp = (gf *)s.psi[d] + psi_index(s, d, x, y, z);
    *pp = psi_update(prof_at(s, d, 0, k), *pp, prof_at(s, d, 1, k), d1);
}

// psi_y pre-pass along y: one thread per (x, z) line and layer side walks the
// side's slab rows with a 9-row register queue of u^n, so that each u row is
// read once per line, not once per neighbour that uses it.  grid: (blocks
// over the largest nx * Nz, 2 sides, shots)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_psi_y(const DevShot *__restrict__ shots, int iu, int ext) {
    typedef __attribute__((address_space(1))) const T gT;
    typedef __attribute__((address_space(1))) float gf;
    const DevShot &s = shots[blockIdx.z];
    const int side = (int)blockIdx.y;
    const int L = side ? s.Lhi[1] : s.Llo[1];
    if (L == 0) return;
    const Box bx = shot_box(s, ext);
    const unsigned nx = (unsigned)s.nx, Nz = (unsigned)(bx.zhi - bx.zlo);
    // contiguous ranges of lines per XCD (as in k_psi)
    const unsigned per = gridDim.x >> 3;
    const unsigned lb = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    const unsigned t = lb * 256u + threadIdx.x;
    if (t >= nx * Nz) return;
    const int x = (int)(t % nx), z = bx.zlo + (int)(t / nx);
    const int y0 = side ? s.ny - s.Lhi[1] : 0;
    const long P = s.P;
    gT *u = (gT *)s.u[iu] + ((long)z * s.S + x);   // element (x, y, z) at u[y P]
    gf *pp = (gf *)s.psi[1] + psi_index(s, 1, x, y0, z);
    float w[5];
#pragma unroll
    for (int l = 0; l < 5; ++l) w[l] = s.w1[1][l];
    float q[9];   // q[o] = u(x, y - 4 + o, z)
#pragma unroll
    for (int o = 0; o < 8; ++o) q[o] = (float)u[(long)(y0 - 4 + o) * P];
    for (int j = 0; j < L; ++j) {
        const int y = y0 + j;
        q[8] = (float)u[(long)(y + 4) * P];
        float fl[4], fh[4];
#pragma unroll
        for (int l = 1; l <= 4; ++l) {
            fl[l - 1] = q[4 - l];
            fh[l - 1] = q[4 + l];
        }
        const float d1 = d1_axis(w, fl, fh);
        pp[(long)j * nx] = psi_update(prof_at(s, 1, 0, y), pp[(long)j * nx], prof_at(s, 1, 1, y), d1);
#pragma unroll
        for (int o = 0; o < 8; ++o) q[o] = q[o + 1];
    }
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
// z-marching update of the points outside the layer bands.
//
// A workgroup of NW waves owns an xy tile of 64 x TY points (TY = NW RY) and a
// z chunk.  Lane l of wave w owns column x0 + l, rows w RY .. w RY + RY - 1.
// Per thread, a register queue of u^n planes along z (the queue index is a
// compile-time phase, so the queue never moves between registers); the
// centre plane with a 4-cell halo goes to one of two LDS buffers (one
// barrier per plane); x neighbours and y neighbours outside the thread's own
// rows come from LDS, the others from registers.  Global loads run two planes
// ahead of their use: u^n (queue of 11 planes, z - 4 .. z + 6), and u^{n-1}
// (or d^n), m and the halo (two more planes held in registers).  Addresses
// are a uniform plane base plus a loop-invariant 32-bit offset per lane.
// ---------------------------------------------------------------------------
constexpr int ZQ = 11;   // queue planes: 9 of the stencil + 2 in flight
template <int NW, int RY> struct ZM {
    static constexpr int NT = 64 * NW;                     // threads
    static constexpr int TY = NW * RY;                     // tile rows
    static constexpr int LW = 64 + 2 * FDTD_R;             // LDS row length
    static constexpr int LH = TY + 2 * FDTD_R;             // LDS rows
    static constexpr int LB = LH * LW + 4;                 // one LDS buffer (+ a dummy slot)
    static constexpr int NH = 2 * FDTD_R * TY + 2 * FDTD_R * 64;   // halo values per plane
    static constexpr int HS = (NH + NT - 1) / NT;          // halo values per thread
};

template <typename T, int NW, int RY> struct ZCtx {
    Coef K;
    // byte bases such that element (x, y, z) of a field is at base + z * Sb + off(x, y)
    const char *u, *m;
    char *w, *sec;       // u^{n+1} out; FP32: u^{n-1} (may be w: in-place step), 16-bit: d^n (in place)
    uint32_t Sb, Smb;    // plane strides in bytes: field, m
    Rsrc ru, rm, rw, rs; // descriptors based at the current round's first plane
    uint32_t off[RY];             // own rows: u^n byte offsets within a plane (kBufSkip where not needed)
    uint32_t offs[RY], offm[RY];  // own rows: second-state / u^{n+1} and m offsets (kBufSkip off the box)
    uint32_t hoff[ZM<NW, RY>::HS];    // halo byte offsets (a lane without a halo value reads its own point)
    int hslot[ZM<NW, RY>::HS];        // halo LDS index (the dummy slot for a lane without one)
    float umc[RY], mc[RY];       // second state and m of plane z
    float um1[RY], m1[RY];       // the same of plane z + 1
    const Roles *R;
    int zlast;           // last plane the current segment's stencils read (segment end + 3)
    int x, y0, lane, r0; // column, tile origin row, lane, first own row (tile-local)
    int nlo[3], nhi[3];  // box of points outside every band
    int sx, sy, sz;      // source node
    bool full;           // tile inside the non-band box and clear of the exclusion box
    bool partial;        // tile overlaps the exclusion box partly
    bool src_tile;       // the source column lies in this tile (or a ghost image of it)
    float src;
};

// plane z = z0 + PH of a round that started at plane z0 (descriptors based at z0)
template <typename T, int NW, int RY, int PH>
__device__ __forceinline__ void zbody(ZCtx<T, NW, RY> &C, const DevShot &s, float (&q)[ZQ][RY],
                                      float (&hq)[ZQ][ZM<NW, RY>::HS], float *L, int z) {
    using G = ZM<NW, RY>;
    auto slot = [](int o) { return (PH + 4 + o + ZQ) % ZQ; };
    // loads ahead of their use: u^n and its halo plane z + 6 (the halo in step with the
    // neighbouring tiles' own rows, which they load as part of their u^n queue, so
    // that it is found in L2), u^{n-1} (or d^n) and m plane z + 2
    float umn[RY], mn[RY];
    {
        // (past the last plane the segment's stencils read, the u^n loads re-read
        // that last plane instead: no stencil of the segment uses the value, and
        // the plane offset stays inside the field, because the scalar offset of
        // a buffer load is not covered by the descriptor's range check)
        const uint32_t s6 = (uint32_t)(min(z + 6, C.zlast) - z + PH) * C.Sb;
        const uint32_t s2 = (PH + 2) * C.Sb, m2 = (PH + 2) * C.Smb;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[slot(6)][r] = Buf<T>::ld(C.ru, C.off[r], s6);
#pragma unroll
        for (int k = 0; k < G::HS; ++k) hq[slot(6)][k] = Buf<T>::ld(C.ru, C.hoff[k], s6);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            umn[r] = Buf<T>::ldnt(C.rs, C.offs[r], s2);
            mn[r] = Buf<float>::ldnt(C.rm, C.offm[r], m2);
        }
    }
    // centre plane to LDS
#pragma unroll
    for (int r = 0; r < RY; ++r) L[(FDTD_R + C.r0 + r) * G::LW + FDTD_R + C.lane] = q[slot(0)][r];
#pragma unroll
    for (int k = 0; k < G::HS; ++k) L[C.hslot[k]] = hq[slot(0)][k];
    __syncthreads();
    const bool srcplane = C.src_tile && wrap_ghost(s, 2, z) == C.sz;
    const uint32_t s0 = PH * C.Sb;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = C.y0 + C.r0 + r;
        const float *row = L + (FDTD_R + C.r0 + r) * G::LW + FDTD_R + C.lane;
        float xl[4], xh[4], yl[4], yh[4], zl[4], zh[4];
#pragma unroll
        for (int l = 1; l <= 4; ++l) {
            xl[l - 1] = row[-l];
            xh[l - 1] = row[l];
            yl[l - 1] = r - l >= 0 ? q[slot(0)][r - l >= 0 ? r - l : 0] : row[-l * G::LW];
            yh[l - 1] = r + l < RY ? q[slot(0)][r + l < RY ? r + l : 0] : row[l * G::LW];
            zl[l - 1] = q[slot(-l)][r];
            zh[l - 1] = q[slot(l)][r];
        }
        const float c = q[slot(0)][r];
        const float lt = lap_interior(C.K, c, xl, xh, yl, yh, zl, zh);
        const bool src = srcplane && C.x == C.sx && wrap_ghost(s, 1, y) == C.sy;
        const Upd up = time_update<T>(C.mc[r], lt, c, C.umc[r], src, C.src);
        const bool ok = C.full || (C.x >= C.nlo[0] && C.x < C.nhi[0] && y >= C.nlo[1] && y < C.nhi[1] &&
                                   !(C.partial && in_box(*C.R, C.x, y, z)));
        // (a masked point's store takes an out-of-range offset: no branch per row)
        const uint32_t so = ok ? C.offs[r] : kBufSkip;
        Buf<T>::st(C.rw, so, s0, up.u);
        if constexpr (IsInc<T>::v) Buf<T>::st(C.rs, so, s0, up.d);
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        C.umc[r] = C.um1[r];
        C.um1[r] = umn[r];
        C.mc[r] = C.m1[r];
        C.m1[r] = mn[r];
    }
}

template <typename T, int NW, int RY>
__global__ __launch_bounds__(64 * NW) void k_zmarch(const DevShot *__restrict__ shots, const WorkItem *__restrict__ work,
                                                    Roles R, int zchunk, const int *__restrict__ stepc) {
    using G = ZM<NW, RY>;
    __shared__ float sm[2 * G::LB];
    const WorkItem wi = work[blockIdx.x];
    const DevShot &s = shots[wi.shot];
    const int ext = R.ext;
    const Box bx = shot_box(s, ext);
    ZCtx<T, NW, RY> C;
    const int x0 = wi.tx * 64;
    C.y0 = bx.ylo + wi.ty * G::TY;
    if (C.y0 >= bx.yhi) return;
    const int zb = bx.zlo + wi.zc * zchunk;
    if (zb >= bx.zhi) return;
    const int ze = min(zb + zchunk, bx.zhi);
    const int n3[3] = {s.nx, s.ny, s.nz};
    band_box(n3, s.Llo, s.Lhi, s.ghost, ext, 6, C.nlo, C.nhi);
    const int fx1 = min(x0 + 64, s.nx), fy1 = min(C.y0 + G::TY, bx.yhi);
    // a tile whose footprint lies inside the band has nothing to do (the band kernel's points)
    if (x0 >= C.nhi[0] || fx1 <= C.nlo[0] || C.y0 >= C.nhi[1] || fy1 <= C.nlo[1]) return;

    // exclusion box: a tile whose footprint lies inside it skips the planes it
    // covers (two z segments); a tile overlapping it partly masks points
    const bool boxz = R.lo[2] < R.hi[2] && R.lo[2] < ze && R.hi[2] > zb;
    const bool ovxy = x0 < R.hi[0] && fx1 > R.lo[0] && C.y0 < R.hi[1] && fy1 > R.lo[1];
    const bool inxy = x0 >= R.lo[0] && fx1 <= R.hi[0] && C.y0 >= R.lo[1] && fy1 <= R.hi[1];
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
    for (int sg = 0; sg < nseg; ++sg) {   // planes of the z band are the band kernel's
        seg_a[sg] = max(seg_a[sg], C.nlo[2]);
        seg_b[sg] = min(seg_b[sg], C.nhi[2]);
    }
    C.full = !C.partial && x0 >= C.nlo[0] && x0 + 64 <= C.nhi[0] && C.y0 >= C.nlo[1] && C.y0 + G::TY <= C.nhi[1];

    C.K = load_coef(s);
    const long P = s.P, esz = sizeof(T);
    const long lead = (long)s.fy * P + FDTD_R;     // elements before (x = -4, y = -fy) within a plane
    C.Sb = (uint32_t)((long)s.S * esz);
    C.Smb = (uint32_t)((long)s.S * 4);
    C.u = (const char *)s.u[R.iu] - lead * esz;
    C.w = (char *)s.u[R.iout] - lead * esz;
    C.sec = (char *)(IsInc<T>::v ? s.dinc : s.u[R.ium1]) - lead * esz;
    C.m = (const char *)s.m - lead * 4;
    C.R = &R;
    C.lane = threadIdx.x & 63;
    C.r0 = (threadIdx.x >> 6) * RY;
    C.x = x0 + C.lane;
    C.sx = s.sx;
    C.sy = s.sy;
    C.sz = s.sz;
    // the source column (or a ghost image of it) in this tile?
    {
        bool iny = false;
        for (int o = -1; o <= 1; ++o) {
            if (o != 0 && !s.ghost[1]) continue;
            const int yy = s.sy + o * s.ny;
            iny = iny || (yy >= C.y0 && yy < C.y0 + G::TY);
        }
        C.src_tile = s.wav != nullptr && s.sx >= x0 && s.sx < x0 + 64 && iny;
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const long e = (long)(C.y0 + C.r0 + r + s.fy) * P + C.x + FDTD_R;
        // loads a lane does not need read nothing (an offset past the descriptor's
        // range reads zero without touching memory): u^n only within 4 points of
        // the non-band box, the second state and m only inside it
        const int y = C.y0 + C.r0 + r;
        const bool nu = C.x >= C.nlo[0] - FDTD_R && C.x < C.nhi[0] + FDTD_R && y >= C.nlo[1] - FDTD_R &&
                        y < C.nhi[1] + FDTD_R;
        const bool ns = C.x >= C.nlo[0] && C.x < C.nhi[0] && y >= C.nlo[1] && y < C.nhi[1];
        C.off[r] = nu ? (uint32_t)(e * esz) : kBufSkip;
        C.offs[r] = ns ? (uint32_t)(e * esz) : kBufSkip;
        C.offm[r] = ns ? (uint32_t)(e * 4) : kBufSkip;
    }
    // halo: values 0 .. 8 TY - 1 are the x halo (row i / 8, column i % 8: 4 left, 4
    // right), then 8 rows of 64 (4 above, 4 below the tile)
#pragma unroll
    for (int k = 0; k < G::HS; ++k) {
        const int i = threadIdx.x + G::NT * k;
        C.hslot[k] = G::LH * G::LW;     // dummy
        C.hoff[k] = kBufSkip;
        if (i < 2 * FDTD_R * G::TY) {
            const int row = i >> 3, c8 = i & 7;
            const int col = c8 < 4 ? c8 : 64 + c8;     // LDS column
            C.hslot[k] = (FDTD_R + row) * G::LW + col;
            const int hx = x0 - FDTD_R + col, hy = C.y0 + row;
            if (hx >= C.nlo[0] - FDTD_R && hx < C.nhi[0] + FDTD_R && hy >= C.nlo[1] - FDTD_R && hy < C.nhi[1] + FDTD_R)
                C.hoff[k] = (uint32_t)(((long)(hy + s.fy) * P + hx + FDTD_R) * esz);
        } else if (i < G::NH) {
            const int j = i - 2 * FDTD_R * G::TY, r8 = j >> 6, c = j & 63;
            const int lrow = r8 < FDTD_R ? r8 : G::TY + r8;
            C.hslot[k] = lrow * G::LW + FDTD_R + c;
            const int hx = x0 + c, hy = C.y0 - FDTD_R + lrow;
            if (hx >= C.nlo[0] - FDTD_R && hx < C.nhi[0] + FDTD_R && hy >= C.nlo[1] - FDTD_R && hy < C.nhi[1] + FDTD_R)
                C.hoff[k] = (uint32_t)(((long)(hy + s.fy) * P + hx + FDTD_R) * esz);
        }
    }
    C.src = source_at(s, *stepc);

    float q[ZQ][RY], hq[ZQ][G::HS];
    int it = 0;
    for (int sg = 0; sg < nseg; ++sg) {
        const int a = seg_a[sg], b = seg_b[sg];
        if (a >= b) continue;
        C.zlast = b + FDTD_R - 1;
        {
            // planes a - 4 .. a + 5 (phase 0: slot o + 4); plane a + 6 is the first body's
            const Rsrc ru = make_rsrc(C.u + (long)(a - 4) * C.Sb);
#pragma unroll
            for (int o = -4; o < 6; ++o)
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    q[o + 4][r] = Buf<T>::ld(ru, C.off[r], (uint32_t)(min(a + o, C.zlast) - a + 4) * C.Sb);
            const Rsrc rs = make_rsrc(C.sec + (long)a * C.Sb);
            const Rsrc rm = make_rsrc(C.m + (long)a * C.Smb);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                q[ZQ - 1][r] = 0.0f;
                C.umc[r] = Buf<T>::ldnt(rs, C.offs[r], 0);
                C.mc[r] = Buf<float>::ldnt(rm, C.offm[r], 0);
                C.um1[r] = Buf<T>::ldnt(rs, C.offs[r], C.Sb);
                C.m1[r] = Buf<float>::ldnt(rm, C.offm[r], C.Smb);
            }
            // halo of planes a .. a + 5 (slots 4 .. 9)
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int k = 0; k < G::HS; ++k)
                    hq[o + 4][k] = Buf<T>::ld(ru, C.hoff[k], (uint32_t)(min(a + o, C.zlast) - a + 4) * C.Sb);
        }
        for (int z0 = a; z0 < b; z0 += ZQ) {
            C.ru = make_rsrc(C.u + (long)z0 * C.Sb);
            C.rs = make_rsrc(C.sec + (long)z0 * C.Sb);
            C.rm = make_rsrc(C.m + (long)z0 * C.Smb);
            C.rw = make_rsrc(C.w + (long)z0 * C.Sb);
            const int n = b - z0;
#define ZSTEP(PH)                                                                 \
    if (n > PH) {                                                                 \
        zbody<T, NW, RY, PH>(C, s, q, hq, sm + (it & 1) * G::LB, z0 + PH);        \
        ++it;                                                                     \
    }
            ZSTEP(0) ZSTEP(1) ZSTEP(2) ZSTEP(3) ZSTEP(4) ZSTEP(5)
            ZSTEP(6) ZSTEP(7) ZSTEP(8) ZSTEP(9) ZSTEP(10)
#undef ZSTEP
        }
    }
}

// ---------------------------------------------------------------------------
// z-march with two x points per lane.  The same scheme as k_zmarch, on tiles
// of 128 x TY points: lane l of wave w owns columns x0 + 2l and x0 + 2l + 1 of
// rows w RY .. w RY + RY - 1, and every global load and LDS access moves the
// pair at once (8 bytes per lane for FP32, 4 for 16-bit storage), so a point
// costs half the load instructions of the one-column kernel.  Rows start on
// 64-element boundaries and tiles at multiples of 128, so every pair's element
// offset is even and its load aligned.  Each point goes through the same arithmetic as
// every other variant, so the bits are the same.
// ---------------------------------------------------------------------------
template <int NW, int RY> struct ZM2 {
    static constexpr int NT = 64 * NW;                     // threads
    static constexpr int TY = NW * RY;                     // tile rows
    static constexpr int LW = 128 + 2 * FDTD_R;            // LDS row length
    static constexpr int LH = TY + 2 * FDTD_R;             // LDS rows
    static constexpr int LB = LH * LW + 8;                 // one LDS buffer (+ a dummy pair)
    static constexpr int NHX = 4 * TY;                     // x-halo pairs: 2 left and 2 right per row
    static constexpr int NH = NHX + 2 * FDTD_R * 64;       // + 8 halo rows of 64 pairs
    static constexpr int HS = (NH + NT - 1) / NT;          // halo pairs per thread
};

template <typename T, int NW, int RY> struct ZCtx2 {
    Coef K;
    const char *u, *m;
    char *w, *sec;
    uint32_t Sb, Smb;
    Rsrc ru, rm, rw, rs;
    uint32_t off[RY];             // own pair: u^n byte offset (kBufSkip when neither point needs it)
    uint32_t offs[RY], offm[RY];  // own pair: second-state / u^{n+1} and m offsets (kBufSkip off the box)
    uint32_t hoff[ZM2<NW, RY>::HS];
    int hslot[ZM2<NW, RY>::HS];   // LDS index of the halo pair (even; the dummy pair for a lane without one)
    float2 umc[RY], mc[RY];       // second state and m of plane z
    float2 um1[RY], m1[RY];       // the same of plane z + 1
    const Roles *R;
    int zlast;
    int x, y0, lane, r0;          // first column of the lane's pair, tile origin row, lane, first own row
    int nlo[3], nhi[3];
    int sx, sy, sz;
    bool full, partial, src_tile;
    float src;
};

template <typename T, int NW, int RY>
__device__ __forceinline__ bool zm2_ok(const ZCtx2<T, NW, RY> &C, int x, int y, int z) {
    return C.full || (x >= C.nlo[0] && x < C.nhi[0] && y >= C.nlo[1] && y < C.nhi[1] &&
                      !(C.partial && in_box(*C.R, x, y, z)));
}

template <typename T, int NW, int RY, int PH>
__device__ __forceinline__ void zbody2(ZCtx2<T, NW, RY> &C, const DevShot &s, float2 (&q)[ZQ][RY],
                                       float2 (&hq)[ZQ][ZM2<NW, RY>::HS], float *L, int z) {
    using G = ZM2<NW, RY>;
    auto slot = [](int o) { return (PH + 4 + o + ZQ) % ZQ; };
    float2 umn[RY], mn[RY];
    {
        // u^n and its halo of plane z + 6 (clamped to the segment's last read plane,
        // whose value no stencil of the segment then uses), second state and m of z + 2
        const uint32_t s6 = (uint32_t)(min(z + 6, C.zlast) - z + PH) * C.Sb;
        const uint32_t s2 = (PH + 2) * C.Sb, m2 = (PH + 2) * C.Smb;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[slot(6)][r] = Buf2<T>::ld(C.ru, C.off[r], s6);
#pragma unroll
        for (int k = 0; k < G::HS; ++k) hq[slot(6)][k] = Buf2<T>::ld(C.ru, C.hoff[k], s6);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            umn[r] = Buf2<T>::ld(C.rs, C.offs[r], s2);
            mn[r] = Buf2<float>::ld(C.rm, C.offm[r], m2);
        }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) *(float2 *)&L[(FDTD_R + C.r0 + r) * G::LW + FDTD_R + 2 * C.lane] = q[slot(0)][r];
#pragma unroll
    for (int k = 0; k < G::HS; ++k) *(float2 *)&L[C.hslot[k]] = hq[slot(0)][k];
    __syncthreads();
    const bool srcplane = C.src_tile && wrap_ghost(s, 2, z) == C.sz;
    const uint32_t s0 = PH * C.Sb;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = C.y0 + C.r0 + r;
        const float *row = L + (FDTD_R + C.r0 + r) * G::LW + FDTD_R + 2 * C.lane;
        const float2 cen = q[slot(0)][r];
        const float2 pm4 = *(const float2 *)(row - 4), pm2 = *(const float2 *)(row - 2);
        const float2 pp2 = *(const float2 *)(row + 2), pp4 = *(const float2 *)(row + 4);
        float2 ylo[4], yhi[4], zlo[4], zhi[4];
#pragma unroll
        for (int l = 1; l <= 4; ++l) {
            ylo[l - 1] = r - l >= 0 ? q[slot(0)][r - l >= 0 ? r - l : 0] : *(const float2 *)(row - l * G::LW);
            yhi[l - 1] = r + l < RY ? q[slot(0)][r + l < RY ? r + l : 0] : *(const float2 *)(row + l * G::LW);
            zlo[l - 1] = q[slot(-l)][r];
            zhi[l - 1] = q[slot(l)][r];
        }
        float yl[4], yh[4], zl[4], zh[4];
        // column 0 of the pair
        const float xl0[4] = {pm2.y, pm2.x, pm4.y, pm4.x}, xh0[4] = {cen.y, pp2.x, pp2.y, pp4.x};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            yl[l] = ylo[l].x;
            yh[l] = yhi[l].x;
            zl[l] = zlo[l].x;
            zh[l] = zhi[l].x;
        }
        const float lt0 = lap_interior(C.K, cen.x, xl0, xh0, yl, yh, zl, zh);
        // column 1
        const float xl1[4] = {cen.x, pm2.y, pm2.x, pm4.y}, xh1[4] = {pp2.x, pp2.y, pp4.x, pp4.y};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            yl[l] = ylo[l].y;
            yh[l] = yhi[l].y;
            zl[l] = zlo[l].y;
            zh[l] = zhi[l].y;
        }
        const float lt1 = lap_interior(C.K, cen.y, xl1, xh1, yl, yh, zl, zh);
        const bool srow = srcplane && wrap_ghost(s, 1, y) == C.sy;
        const Upd u0 = time_update<T>(C.mc[r].x, lt0, cen.x, C.umc[r].x, srow && C.x == C.sx, C.src);
        const Upd u1 = time_update<T>(C.mc[r].y, lt1, cen.y, C.umc[r].y, srow && C.x + 1 == C.sx, C.src);
        // (a masked point's store takes an out-of-range offset)
        const uint32_t so0 = zm2_ok(C, C.x, y, z) ? C.offs[r] : kBufSkip;
        const uint32_t so1 = zm2_ok(C, C.x + 1, y, z) ? C.offs[r] + (uint32_t)sizeof(T) : kBufSkip;
        Buf<T>::st(C.rw, so0, s0, u0.u);
        Buf<T>::st(C.rw, so1, s0, u1.u);
        if constexpr (IsInc<T>::v) {
            Buf<T>::st(C.rs, so0, s0, u0.d);
            Buf<T>::st(C.rs, so1, s0, u1.d);
        }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        C.umc[r] = C.um1[r];
        C.um1[r] = umn[r];
        C.mc[r] = C.m1[r];
        C.m1[r] = mn[r];
    }
}

template <typename T, int NW, int RY>
__global__ __launch_bounds__(64 * NW) void k_zmarch2(const DevShot *__restrict__ shots,
                                                     const WorkItem *__restrict__ work, Roles R, int zchunk,
                                                     const int *__restrict__ stepc) {
    using G = ZM2<NW, RY>;
    __shared__ float sm[2 * G::LB];
    const WorkItem wi = work[blockIdx.x];
    const DevShot &s = shots[wi.shot];
    const int ext = R.ext;
    const Box bx = shot_box(s, ext);
    ZCtx2<T, NW, RY> C;
    const int x0 = wi.tx * 128;
    C.y0 = bx.ylo + wi.ty * G::TY;
    if (C.y0 >= bx.yhi) return;
    const int zb = bx.zlo + wi.zc * zchunk;
    if (zb >= bx.zhi) return;
    const int ze = min(zb + zchunk, bx.zhi);
    const int n3[3] = {s.nx, s.ny, s.nz};
    band_box(n3, s.Llo, s.Lhi, s.ghost, ext, 6, C.nlo, C.nhi);
    const int fx1 = min(x0 + 128, s.nx), fy1 = min(C.y0 + G::TY, bx.yhi);
    if (x0 >= C.nhi[0] || fx1 <= C.nlo[0] || C.y0 >= C.nhi[1] || fy1 <= C.nlo[1]) return;

    const bool boxz = R.lo[2] < R.hi[2] && R.lo[2] < ze && R.hi[2] > zb;
    const bool ovxy = x0 < R.hi[0] && fx1 > R.lo[0] && C.y0 < R.hi[1] && fy1 > R.lo[1];
    const bool inxy = x0 >= R.lo[0] && fx1 <= R.hi[0] && C.y0 >= R.lo[1] && fy1 <= R.hi[1];
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
    for (int sg = 0; sg < nseg; ++sg) {
        seg_a[sg] = max(seg_a[sg], C.nlo[2]);
        seg_b[sg] = min(seg_b[sg], C.nhi[2]);
    }
    C.full = !C.partial && x0 >= C.nlo[0] && x0 + 128 <= C.nhi[0] && C.y0 >= C.nlo[1] && C.y0 + G::TY <= C.nhi[1];

    C.K = load_coef(s);
    const long P = s.P, esz = sizeof(T);
    const long lead = (long)s.fy * P + FDTD_R;     // elements before (x = -4, y = -fy) within a plane
    C.Sb = (uint32_t)((long)s.S * esz);
    C.Smb = (uint32_t)((long)s.S * 4);
    C.u = (const char *)s.u[R.iu] - lead * esz;
    C.w = (char *)s.u[R.iout] - lead * esz;
    C.sec = (char *)(IsInc<T>::v ? s.dinc : s.u[R.ium1]) - lead * esz;
    C.m = (const char *)s.m - lead * 4;
    C.R = &R;
    C.lane = threadIdx.x & 63;
    C.r0 = (threadIdx.x >> 6) * RY;
    C.x = x0 + 2 * C.lane;
    C.sx = s.sx;
    C.sy = s.sy;
    C.sz = s.sz;
    {
        bool iny = false;
        for (int o = -1; o <= 1; ++o) {
            if (o != 0 && !s.ghost[1]) continue;
            const int yy = s.sy + o * s.ny;
            iny = iny || (yy >= C.y0 && yy < C.y0 + G::TY);
        }
        C.src_tile = s.wav != nullptr && s.sx >= x0 && s.sx < x0 + 128 && iny;
    }
    // a pair is loaded when either of its points needs the value
    auto need = [&](int hx, int hy, int m) {
        return hx + 1 >= C.nlo[0] - m && hx < C.nhi[0] + m && hy >= C.nlo[1] - m && hy < C.nhi[1] + m;
    };
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = C.y0 + C.r0 + r;
        const long e = (long)(y + s.fy) * P + C.x + FDTD_R;
        C.off[r] = need(C.x, y, FDTD_R) ? (uint32_t)(e * esz) : kBufSkip;
        C.offs[r] = need(C.x, y, 0) ? (uint32_t)(e * esz) : kBufSkip;
        C.offm[r] = need(C.x, y, 0) ? (uint32_t)(e * 4) : kBufSkip;
    }
    // halo pairs: 0 .. 4 TY - 1 the x halo (row i / 4: pairs at columns -4, -2 and
    // 128, 130 of the tile), then 8 rows of 64 pairs (4 above, 4 below the tile)
#pragma unroll
    for (int k = 0; k < G::HS; ++k) {
        const int i = threadIdx.x + G::NT * k;
        C.hslot[k] = G::LH * G::LW;     // dummy pair
        C.hoff[k] = kBufSkip;
        if (i < G::NHX) {
            const int row = i >> 2, k4 = i & 3;
            const int col = k4 < 2 ? 2 * k4 : 128 + 2 * k4;     // LDS column
            C.hslot[k] = (FDTD_R + row) * G::LW + col;
            const int hx = x0 - FDTD_R + col, hy = C.y0 + row;
            if (need(hx, hy, FDTD_R)) C.hoff[k] = (uint32_t)(((long)(hy + s.fy) * P + hx + FDTD_R) * esz);
        } else if (i < G::NH) {
            const int j = i - G::NHX, r8 = j >> 6, c = j & 63;
            const int lrow = r8 < FDTD_R ? r8 : G::TY + r8;
            C.hslot[k] = lrow * G::LW + FDTD_R + 2 * c;
            const int hx = x0 + 2 * c, hy = C.y0 - FDTD_R + lrow;
            if (need(hx, hy, FDTD_R)) C.hoff[k] = (uint32_t)(((long)(hy + s.fy) * P + hx + FDTD_R) * esz);
        }
    }
    C.src = source_at(s, *stepc);

    float2 q[ZQ][RY], hq[ZQ][G::HS];
    int it = 0;
    for (int sg = 0; sg < nseg; ++sg) {
        const int a = seg_a[sg], b = seg_b[sg];
        if (a >= b) continue;
        C.zlast = b + FDTD_R - 1;
        {
            const Rsrc ru = make_rsrc(C.u + (long)(a - 4) * C.Sb);
#pragma unroll
            for (int o = -4; o < 6; ++o)
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    q[o + 4][r] = Buf2<T>::ld(ru, C.off[r], (uint32_t)(min(a + o, C.zlast) - a + 4) * C.Sb);
            const Rsrc rs = make_rsrc(C.sec + (long)a * C.Sb);
            const Rsrc rm = make_rsrc(C.m + (long)a * C.Smb);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                q[ZQ - 1][r] = make_float2(0.0f, 0.0f);
                C.umc[r] = Buf2<T>::ld(rs, C.offs[r], 0);
                C.mc[r] = Buf2<float>::ld(rm, C.offm[r], 0);
                C.um1[r] = Buf2<T>::ld(rs, C.offs[r], C.Sb);
                C.m1[r] = Buf2<float>::ld(rm, C.offm[r], C.Smb);
            }
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int k = 0; k < G::HS; ++k)
                    hq[o + 4][k] = Buf2<T>::ld(ru, C.hoff[k], (uint32_t)(min(a + o, C.zlast) - a + 4) * C.Sb);
        }
        for (int z0 = a; z0 < b; z0 += ZQ) {
            C.ru = make_rsrc(C.u + (long)z0 * C.Sb);
            C.rs = make_rsrc(C.sec + (long)z0 * C.Sb);
            C.rm = make_rsrc(C.m + (long)z0 * C.Smb);
            C.rw = make_rsrc(C.w + (long)z0 * C.Sb);
            const int n = b - z0;
#define ZSTEP2(PH)                                                                \
    if (n > PH) {                                                                 \
        zbody2<T, NW, RY, PH>(C, s, q, hq, sm + (it & 1) * G::LB, z0 + PH);       \
        ++it;                                                                     \
    }
            ZSTEP2(0) ZSTEP2(1) ZSTEP2(2) ZSTEP2(3) ZSTEP2(4) ZSTEP2(5)
            ZSTEP2(6) ZSTEP2(7) ZSTEP2(8) ZSTEP2(9) ZSTEP2(10)
#undef ZSTEP2
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
static void launch_psi_t(const DevShot *d_shots, int nshots, long max_count, int iu, int ext, int d0, int nd,
                         hipStream_t st) {
    if (max_count <= 0 || nd <= 0) return;
    dim3 grid((unsigned)((max_count + 255) / 256 + 7) / 8 * 8, nd, nshots);
    hipLaunchKernelGGL(k_psi<T>, grid, dim3(256), 0, st, d_shots, iu, ext, d0);
}
template <typename T>
static void launch_psi_y_t(const DevShot *d_shots, int nshots, long max_lines, int iu, int ext, hipStream_t st) {
    if (max_lines <= 0) return;
    dim3 grid((unsigned)((max_lines + 255) / 256 + 7) / 8 * 8, 2, nshots);
    hipLaunchKernelGGL(k_psi_y<T>, grid, dim3(256), 0, st, d_shots, iu, ext);
}
template <typename T>
static void launch_naive_t(const DevShot *d_shots, int shot, int nx, int Ny, int Nz, const Roles &R,
                           const int *stepc, hipStream_t st) {
    dim3 grid((nx + 63) / 64, (Ny + 3) / 4, Nz);
    hipLaunchKernelGGL(k_update_naive<T>, grid, dim3(64, 4), 0, st, d_shots, shot, R, stepc);
}
template <typename T>
static void launch_zmarch_t(const DevShot *d_shots, const WorkItem *work, int nwork, int ry, int cols, const Roles &R,
                            int zchunk, const int *stepc, hipStream_t st) {
    if (nwork <= 0) return;
    if (cols == 2) {
        // plan rows ry = 1, 2, 4: tiles of 128 x 8 ry points; (waves, rows per thread) = (4, 2), (8, 2), (16, 2)
        switch (ry) {
        case 1:
            hipLaunchKernelGGL((k_zmarch2<T, 4, 2>), dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
            break;
        case 4:
            hipLaunchKernelGGL((k_zmarch2<T, 16, 2>), dim3(nwork), dim3(1024), 0, st, d_shots, work, R, zchunk, stepc);
            break;
        default:
            hipLaunchKernelGGL((k_zmarch2<T, 8, 2>), dim3(nwork), dim3(512), 0, st, d_shots, work, R, zchunk, stepc);
            break;
        }
        return;
    }
    // plan rows ry = 1, 2, 4, 8: tiles of 64 x 8 ry points; (waves, rows per thread)
    // = (4, 2), (4, 4), (8, 4), (16, 4)
    switch (ry) {
    case 1:
        hipLaunchKernelGGL((k_zmarch<T, 4, 2>), dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
        break;
    case 4:
        hipLaunchKernelGGL((k_zmarch<T, 8, 4>), dim3(nwork), dim3(512), 0, st, d_shots, work, R, zchunk, stepc);
        break;
    case 8:
        hipLaunchKernelGGL((k_zmarch<T, 16, 4>), dim3(nwork), dim3(1024), 0, st, d_shots, work, R, zchunk, stepc);
        break;
    default:
        hipLaunchKernelGGL((k_zmarch<T, 4, 4>), dim3(nwork), dim3(256), 0, st, d_shots, work, R, zchunk, stepc);
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

void fdtd_launch_psi(int stor, const DevShot *d_shots, int nshots, long max_count, int iu, int ext, int d0, int nd,
                     hipStream_t st) {
    FDTD_DISPATCH(stor, launch_psi_t, d_shots, nshots, max_count, iu, ext, d0, nd, st);
}
void fdtd_launch_psi_y(int stor, const DevShot *d_shots, int nshots, long max_lines, int iu, int ext, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_psi_y_t, d_shots, nshots, max_lines, iu, ext, st);
}
void fdtd_launch_naive(int stor, const DevShot *d_shots, int shot, int nx, int Ny, int Nz, const Roles &R,
                       const int *stepc, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_naive_t, d_shots, shot, nx, Ny, Nz, R, stepc, st);
}
void fdtd_launch_zmarch(int stor, const DevShot *d_shots, const WorkItem *work, int nwork, int ry, int cols,
                        const Roles &R, int zchunk, const int *stepc, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_zmarch_t, d_shots, work, nwork, ry, cols, R, zchunk, stepc, st);
}
void fdtd_launch_record(int stor, const DevShot *d_shots, int nshots, const Roles &R, int *stepc, hipStream_t st) {
    FDTD_DISPATCH(stor, launch_record_t, d_shots, nshots, R, stepc, st);
}
