// kernels_band.hip -- update of the layer-band points (gfx950).
//
// The band is the union of the absorbing-layer slabs and the 4-cell margin
// their psi derivative reaches (paper, section "CPML Boundary Layers": the
// stretched second derivative and its memory variables).  It is cut into six
// disjoint boxes (band_box) of three kinds, each a specialisation of one
// tile routine (one launch covers the tiles of all kinds):
//   kind 0, boxes 0/1: z band (x, y band at the edges);
//   kind 1, boxes 2/3: y band (x band at the edges), z outside its band;
//   kind 2, boxes 4/5: x band only.
// Boxes are tiled in BAND_TX x BAND_TY columns and chunks of planes.  A thread
// owns a column and walks its planes with a register queue of u^n (and, for
// kind 0, of psi_z) along z; x and y neighbours are buffer loads (L1/L2).
// The layer data of the thread's x and y coordinates are set up once, those
// of each plane are uniform (scalar).  The arithmetic is lap_point's,
// operation for operation, so the bits equal the naive kernel's.  Points
// outside every band are left to the interior kernels.
#include "fdtd_dev.hpp"

namespace {
// layer data of one coordinate along one axis
struct AxisPt {
    float b, a, kinv, dkinv;
    int band, slab;
    int pos;              // slab position of the coordinate (slab points)
    int npos[8];          // slab positions of the neighbours c-1..c-4, c+1..c+4; the zero slot
                          // (slab width) where a neighbour lies outside [0, n) or the slabs
};
__device__ __forceinline__ void axis_point(const DevShot &s, int d, int c, AxisPt &A) {
    const int n = coord_n(s, d), lo = s.Llo[d], hi = s.Lhi[d];
    const bool band = in_band(c, n, lo, hi);
    const bool slab = band && in_slab(c, n, lo, hi);
    A.band = band;
    A.slab = slab;
    A.pos = slab ? slab_pos(c, n, lo, hi) : 0;
    A.b = band ? prof_at(s, d, 0, c) : 0.0f;
    A.a = band ? prof_at(s, d, 1, c) : 0.0f;
    A.kinv = band ? prof_at(s, d, 2, c) : 0.0f;
    A.dkinv = band ? prof_at(s, d, 3, c) : 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int cn = j < 4 ? c - (j + 1) : c + (j - 3);
        const bool ok = band && cn >= 0 && cn < n && in_slab(cn, n, lo, hi);
        A.npos[j] = ok ? slab_pos(cn, n, lo, hi) : lo + hi;
    }
}
}  // namespace

// Tile of one band box.  With FUSE (DevShot::fused) the tile also advances the
// layer memory of x and z itself, psi <- b psi + a D1 u^n with the D1 u^n its
// own stencil already forms, instead of reading the psi pass's result:
//  * psi_x: every x-slab point of a row lies in the same tile row (band_xtiles
//    gives the high x band a tile of its own), so a lane updates its own point
//    and takes its 8 neighbours from the other lanes of the row (ds_bpermute);
//  * psi_z (kind 0): a box holds a whole z slab and is walked in one pass, so
//    psi_z rides in the z queue: at plane z the lane advances psi_z at z + 4,
//    from a u^n queue that reaches z + 8.
// Each layer point is advanced once, by the tile that owns it, with the psi
// pass's operations, so the bits do not change.
template <typename T, int KIND, bool FUSE, int TY>
__device__ __forceinline__ void band_tile(const DevShot *__restrict__ shots, const BandItem wi, const Roles &R,
                                          int zchunk, const int *__restrict__ stepc, float *Lds) {
    constexpr int LB = band_lds(TY);
    constexpr bool HAS_Y = KIND <= 1, HAS_Z = KIND == 0;
    constexpr bool FZ = FUSE && HAS_Z;   // psi_z advanced in the z queue
    constexpr int QN = FZ ? 13 : 9;      // u^n queue: planes z - 4 .. z + QN - 5
    const DevShot &s = shots[wi.shot];
    int blo[3], bhi[3];
    const int n3[3] = {s.nx, s.ny, s.nz};
    band_box(n3, s.Llo, s.Lhi, s.ghost, R.ext, wi.box, blo, bhi);
    int x0, x1;
    band_xtiles(s.nx, s.Llo[0], s.Lhi[0], wi.box, blo[0], bhi[0], wi.tx, &x0, &x1);
    const int lx = (int)(threadIdx.x % BAND_TX), ly = (int)(threadIdx.x / BAND_TX);
    const int x = x0 + lx;
    const int yt = blo[1] + wi.ty * TY;   // first row of the tile
    const int y = yt + ly;
    // z boxes are walked whole (their tile list has one chunk), the others in chunks
    const int za = KIND == 0 ? blo[2] : blo[2] + wi.zc * zchunk;
    // the whole tile (uniform, barriers below): also the idle items that pad the
    // list (x0 past x1, a coordinate no layer data may be read at)
    if (za >= bhi[2] || yt >= bhi[1] || x0 >= x1) return;
    const int zb = KIND == 0 ? bhi[2] : min(za + zchunk, bhi[2]);
    // Every lane of the tile stages its u^n into the LDS plane, where the x and
    // y stencil taps of the points are read; lanes past the box end (act
    // false) compute nothing and store nothing.  A lane position outside the
    // rows and columns the field buffer holds reads zero (it is no tap of any
    // point of the box).
    const bool act = x < x1 && y < bhi[1];

    const Coef K = load_coef(s);
    float w1[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int l = 0; l < 5; ++l) w1[d][l] = s.w1[d][l];
    const float srcamp = source_at(s, *stepc);
    const bool src_col = x == s.sx && wrap_ghost(s, 1, y) == s.sy;
    const long P = s.P, S = s.S, esz = sizeof(T);
    const int fy = s.fy, fz = s.fz, nx = s.nx;

    // u^n, the second state and u^{n+1}: element (x + dx, y + dy, z') at
    //   base + (z' - za + 4) S esz [scalar] + vo + ((dy + 4) P + dx + 4) esz [lane]
    const long lead = (long)(za - 4) * S - (long)fy * P - 4;
    const Rsrc ru = make_rsrc((const char *)s.u[R.iu] + lead * esz);
    const Rsrc rw = make_rsrc((char *)s.u[R.iout] + lead * esz);
    const Rsrc rs = make_rsrc((char *)(IsInc<T>::v ? s.dinc : s.u[R.ium1]) + lead * esz);
    const Rsrc rm = make_rsrc((const char *)s.m + lead * 4);
    const uint32_t vo = (uint32_t)(((long)(y + fy - 4) * P + x) * esz);
    const uint32_t vc = vo + (uint32_t)((4 * P + 4) * esz);                 // the point itself
    const uint32_t vcm = (uint32_t)(((long)(y + fy) * P + x + 4) * 4);      // the point in m
    const uint32_t Sb = (uint32_t)(S * esz), Smb = (uint32_t)(S * 4);
    auto held = [&](int xp, int yp) { return xp >= -4 && xp < nx + 4 && yp >= -fy && yp < s.ny + fy; };
    auto lane_off = [&](int xp, int yp) -> uint32_t {
        return held(xp, yp) ? (uint32_t)(((long)(yp + fy) * P + xp + 4) * esz) : kBufSkip;
    };
    const uint32_t vcq = lane_off(x, y);             // the lane's u^n column (z queue, LDS plane)
    const uint32_t vca = act ? vc : kBufSkip;        // the point's own loads and stores
    const uint32_t vcma = act ? vcm : kBufSkip;
    // LDS slots (band_halo): the lane's own and its halo value(s), slot (c, r)
    // holding the point (x0 - 4 + c, yt - 4 + r)
    const int own = (ly + FDTD_R) * kBandLW + lx + FDTD_R;
    int hc1, hr1, hc2, hr2;
    band_halo((int)threadIdx.x, 0, TY, hc1, hr1);
    band_halo((int)threadIdx.x, 1, TY, hc2, hr2);
    const int hslot1 = hc1 >= 0 ? hr1 * kBandLW + hc1 : LB - 1;
    const uint32_t hoff1 = hc1 >= 0 ? lane_off(x0 - FDTD_R + hc1, yt - FDTD_R + hr1) : kBufSkip;
    const int hslot2 = hc2 >= 0 ? hr2 * kBandLW + hc2 : LB - 1;
    const uint32_t hoff2 = hc2 >= 0 ? lane_off(x0 - FDTD_R + hc2, yt - FDTD_R + hr2) : kBufSkip;

    AxisPt AX, AY;
    axis_point(s, 0, act ? x : x0, AX);
    if constexpr (HAS_Y) axis_point(s, 1, act ? y : yt, AY);
    // psi_d and zeta_d of an axis through one descriptor (zeta_d follows psi_d in the workspace)
    const Rsrc rpx = make_rsrc(s.psi[0]);
    const uint32_t zdx = (uint32_t)((const char *)s.zeta[0] - (const char *)s.psi[0]);
    // psi_x, zeta_x (psi_index layout): byte offset of (x', y) within a plane of
    // either layer block, plane stride Spx; a neighbour outside the slabs reads
    // zero through an out-of-range offset
    const int xlo = s.Llo[0], xhi = s.Lhi[0];
    const uint32_t Spx = (uint32_t)((long)s.PY * s.WX * 4);
    const uint32_t xhib = (uint32_t)((long)(s.nz + 2 * fz) * s.PY * s.WX * 4);
    const uint32_t vx_row = (uint32_t)((long)(y + fy) * s.WX * 4);
    auto xoff = [&](int xp) -> uint32_t {
        return xp < xlo ? vx_row + 4 * (uint32_t)xp : xhib + vx_row + 4 * (uint32_t)(xp - (nx - xhi));
    };
    uint32_t px_off[8], py_off[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        px_off[j] = act && AX.npos[j] != xlo + xhi ? xoff(j < 4 ? x - (j + 1) : x + (j - 3)) : kBufSkip;
    const uint32_t zx_off = act && AX.slab ? xoff(x) : kBufSkip;
    // FUSE: source lanes of the 8 x neighbours within the wave and the mask of
    // those inside the x slabs (all of them lie in this tile row); whether the
    // tile reaches the x band at all (uniform)
    int xsrc[8];
    unsigned xvalid = 0;
    bool xedge = false;
    if constexpr (FUSE) {
        const int lane = (int)(threadIdx.x & 63);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int off = j < 4 ? -(j + 1) : j - 3;
            xsrc[j] = ((lane + off) & 63) * 4;
            xvalid |= (AX.npos[j] != xlo + xhi) ? (1u << j) : 0u;
        }
        int a, b, e0, e1;
        band_range_x(nx, s.Llo[0], s.Lhi[0], a, b, e0, e1);
        xedge = x0 < a || x1 > b;
    }
    Rsrc rpy = rpx, rpz = rpx, rpr = rpx;
    uint32_t zy_off = 0, Spy = 0, vz_col = 0, Spz = 0, zdy = 0, zdz = 0;
    if constexpr (HAS_Y) {
        rpy = make_rsrc(s.psi[1]);
        zdy = (uint32_t)((const char *)s.zeta[1] - (const char *)s.psi[1]);
#pragma unroll
        for (int j = 0; j < 8; ++j) py_off[j] = act ? 4 * (uint32_t)(AY.npos[j] * nx + x) : kBufSkip;
        zy_off = act ? 4 * (uint32_t)(AY.pos * nx + x) : kBufSkip;
        Spy = (uint32_t)((long)s.SY * nx * 4);
    }
    const int nz = s.nz, zlo = s.Llo[2], zhi = s.Lhi[2];
    if constexpr (HAS_Z) {
        rpz = make_rsrc(s.psi[2]);
        rpr = make_rsrc(s.prof);
        zdz = (uint32_t)((const char *)s.zeta[2] - (const char *)s.psi[2]);
        vz_col = act ? (uint32_t)(((long)(y + fy) * nx + x) * 4) : kBufSkip;
        Spz = (uint32_t)((long)s.PY * nx * 4);
    }
    // plane p of the z slabs (uniform condition)
    auto zslab = [&](int p) -> bool { return p >= 0 && p < nz && in_slab(p, nz, zlo, zhi); };
    // psi_z of plane p at the column, 0 outside the z slabs
    auto psi_z_at = [&](int p) -> float {
        if (!zslab(p)) return 0.0f;
        return Buf<float>::ld(rpz, vz_col, (uint32_t)slab_pos(p, nz, zlo, zhi) * Spz);
    };
    // z-axis profile f (0 b, 1 a, 2 kinv, 3 dkinv) at plane p: a load whose
    // value every lane shares (issued with the other loads of a plane), made
    // a scalar where it is used
    auto zprof_ld = [&](int f, int p) -> float {
        return Buf<float>::ld(rpr, 0, (uint32_t)(((8 + f) * s.nmax + p) * 4));
    };
    auto uni = [](float v) -> float {
        return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
    };
    // FZ: psi_z at plane p (a z-slab plane) advanced from the u^n queue entries
    // u(p - 4) .. u(p + 4) = qq[c - 4] .. qq[c + 4] and the profiles b, a there
    auto psi_z_new = [&](const float *qq, int c, float b, float a, float old) -> float {
        float fl[4], fh[4];
#pragma unroll
        for (int l = 1; l <= 4; ++l) {
            fl[l - 1] = qq[c - l];
            fh[l - 1] = qq[c + l];
        }
        return psi_update(b, old, a, d1_axis(w1[2], fl, fh));
    };
    auto psi_z_store = [&](int p, float v) {
        Buf<float>::st(rpz, vz_col, (uint32_t)slab_pos(p, nz, zlo, zhi) * Spz, v);
    };

    // z queues at the column: q[o] = u(x, y, z - 4 + o); pq[o] = psi_z at z - 4 + o (0 outside its slab)
    float q[QN], pq[9];
#pragma unroll
    for (int o = 0; o < QN - 1; ++o) q[o] = Buf<T>::ld(ru, vcq, o * Sb);
    if constexpr (FZ) {
        // planes za - 4 .. za - 1 lie outside the z slabs (the host enables FUSE
        // only when the two z boxes share no layer point); za .. za + 3 are
        // advanced here from q (the box is at least 5 planes deep)
        // (every load first, then the arithmetic, then the stores)
        float old[4], pb[4], pa[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            old[o] = psi_z_at(za + o);
            pb[o] = zslab(za + o) ? zprof_ld(0, za + o) : 0.0f;
            pa[o] = zslab(za + o) ? zprof_ld(1, za + o) : 0.0f;
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            pq[o] = 0.0f;
            pq[o + 4] = zslab(za + o) ? psi_z_new(q, o + 4, uni(pb[o]), uni(pa[o]), old[o]) : 0.0f;
        }
#pragma unroll
        for (int o = 0; o < 4; ++o)
            if (zslab(za + o)) psi_z_store(za + o, pq[o + 4]);
    } else if constexpr (HAS_Z) {
#pragma unroll
        for (int o = 0; o < 8; ++o) pq[o] = psi_z_at(za - 4 + o);
    }

    // loads of one plane
    struct PL {
        float xl[4], xh[4], yl[4], yh[4];
        float qn, second, mm;         // u^n at the queue head, second state, m
        float px[8], zx, py[8], zy;   // psi_x / psi_y neighbours, zeta_x / zeta_y
        float pxo;                    // FUSE: psi_x of the point before its update
        float pqn, zz;                // psi_z four planes ahead (FZ: before its update), zeta_z
        float zpr[4], zb4, za4;       // z profiles at the plane; FZ: b, a four planes ahead
    };
    auto load = [&](int z, PL &p) {
        const uint32_t pz = (uint32_t)(z - za + 4) * Sb;
        // FZ: the head u(z + 8) is needed only while z + 4 is a grid plane (it may lie past the frame)
        const uint32_t vq = (!FZ || z + 4 < nz) ? vcq : kBufSkip;
        p.qn = Buf<T>::ld(ru, vq, pz + (QN - 5) * Sb);
        p.second = Buf<T>::ld(rs, vca, pz);
        p.mm = Buf<float>::ld(rm, vcma, (uint32_t)(z - za + 4) * Smb);
        // (a y neighbour outside the slabs reads the zero slot of its row)
        const uint32_t sox = (uint32_t)(z + fz) * Spx;
        if constexpr (FUSE) {
            if (AX.slab) {
                p.pxo = Buf<float>::ld(rpx, zx_off, sox);
                p.zx = Buf<float>::ld(rpx, zx_off, sox + zdx);
            }
        } else if (AX.band) {
#pragma unroll
            for (int j = 0; j < 8; ++j) p.px[j] = Buf<float>::ld(rpx, px_off[j], sox);
            if (AX.slab) p.zx = Buf<float>::ld(rpx, zx_off, sox + zdx);
        }
        if constexpr (HAS_Y) {
            if (AY.band) {
                const uint32_t soy = (uint32_t)(z + fz) * Spy;
#pragma unroll
                for (int j = 0; j < 8; ++j) p.py[j] = Buf<float>::ld(rpy, py_off[j], soy);
                if (AY.slab) p.zy = Buf<float>::ld(rpy, zy_off, soy + zdy);
            }
        }
        if constexpr (HAS_Z) {
            p.pqn = psi_z_at(z + 4);
            if (zslab(z)) p.zz = Buf<float>::ld(rpz, vz_col, (uint32_t)slab_pos(z, nz, zlo, zhi) * Spz + zdz);
            if (in_band(z, nz, zlo, zhi)) {
#pragma unroll
                for (int f = 0; f < 4; ++f) p.zpr[f] = zprof_ld(f, z);
            }
            if constexpr (FZ) {
                if (zslab(z + 4)) {
                    p.zb4 = zprof_ld(0, z + 4);
                    p.za4 = zprof_ld(1, z + 4);
                }
            }
        }
    };
    auto compute = [&](int z, PL &p) {
        q[QN - 1] = p.qn;
        float zl[4], zh[4];
#pragma unroll
        for (int l = 1; l <= 4; ++l) {
            zl[l - 1] = q[4 - l];
            zh[l - 1] = q[4 + l];
        }
        const float c = q[4];
        if constexpr (FUSE) {
            // psi_x of the point, then its neighbours from the lanes of the row
            float pn = 0.0f;
            if (AX.slab) {
                pn = psi_update(AX.b, p.pxo, AX.a, d1_axis(w1[0], p.xl, p.xh));
                Buf<float>::st(rpx, zx_off, (uint32_t)(z + fz) * Spx, pn);
            }
            if (xedge) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float v = __builtin_bit_cast(
                        float, __builtin_amdgcn_ds_bpermute(xsrc[j], __builtin_bit_cast(int, pn)));
                    p.px[j] = (xvalid >> j) & 1u ? v : 0.0f;
                }
            }
        }
        float pl[3][4], ph[3][4], zo[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            pl[0][l] = p.px[l];
            ph[0][l] = p.px[4 + l];
            pl[1][l] = p.py[l];
            ph[1][l] = p.py[4 + l];
        }
        zo[0] = p.zx;
        zo[1] = p.zy;
        // layer data of plane z (uniform; every plane of a kind-0 box is in the z band)
        AxisPt AZ;
        AZ.band = 0;
        AZ.slab = 0;
        AZ.pos = 0;
        AZ.b = AZ.a = AZ.kinv = AZ.dkinv = 0.0f;
        if constexpr (HAS_Z) {
            if constexpr (FZ) {
                pq[8] = 0.0f;
                if (zslab(z + 4)) {
                    pq[8] = psi_z_new(q, 8, uni(p.zb4), uni(p.za4), p.pqn);
                    psi_z_store(z + 4, pq[8]);
                }
            } else {
                pq[8] = p.pqn;
            }
            AZ.band = in_band(z, nz, zlo, zhi);
            AZ.slab = AZ.band && in_slab(z, nz, zlo, zhi);
            AZ.pos = AZ.slab ? slab_pos(z, nz, zlo, zhi) : 0;
            if (AZ.band) {
                AZ.b = uni(p.zpr[0]);
                AZ.a = uni(p.zpr[1]);
                AZ.kinv = uni(p.zpr[2]);
                AZ.dkinv = uni(p.zpr[3]);
            }
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                pl[2][l - 1] = pq[4 - l];
                ph[2][l - 1] = pq[4 + l];
            }
            zo[2] = p.zz;
        }
        // arithmetic of lap_point (every point of a z or y box lies in a band; an x box
        // also holds points of no band, between the x band and the whole-tile bound)
        const float *lo[3] = {p.xl, p.yl, zl};
        const float *hi[3] = {p.xh, p.yh, zh};
        const AxisPt *A3[3] = {&AX, &AY, &AZ};
        const bool bnd[3] = {(bool)AX.band, HAS_Y && AY.band, HAS_Z && AZ.band};
        const bool slb[3] = {(bool)AX.slab, HAS_Y && AY.slab, HAS_Z && AZ.slab};
        float L[3], zn[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float d2 = d2_axis(K.w2[d], c, lo[d], hi[d]);
            if (!bnd[d]) {
                L[d] = d2;
                continue;
            }
            const float d1 = d1_axis(w1[d], lo[d], hi[d]);
            const float dpsi = d1_axis(w1[d], pl[d], ph[d]);
            L[d] = cpml_axis(d2, d1, dpsi, A3[d]->kinv, A3[d]->dkinv, A3[d]->a, A3[d]->b, slb[d], zo[d], &zn[d]);
        }
        float lt = (L[0] + L[1]) + L[2];
        if constexpr (KIND == 2) {
            if (!bnd[0]) lt = lap_interior(K, c, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
        }
        const bool src = src_col && wrap_ghost(s, 2, z) == s.sz;
        const Upd up = time_update<T>(p.mm, lt, c, p.second, src, srcamp);
        if (act && !in_box(R, x, y, z)) {
            const uint32_t pz = (uint32_t)(z - za + 4) * Sb;
            Buf<T>::st(rw, vc, pz, up.u);
            if constexpr (IsInc<T>::v) Buf<T>::st(rs, vc, pz, up.d);
            if (slb[0]) Buf<float>::st(rpx, zx_off, (uint32_t)(z + fz) * Spx + zdx, zn[0]);
            if constexpr (HAS_Y)
                if (slb[1]) Buf<float>::st(rpy, zy_off, (uint32_t)(z + fz) * Spy + zdy, zn[1]);
            if constexpr (HAS_Z)
                if (slb[2]) Buf<float>::st(rpz, vz_col, (uint32_t)AZ.pos * Spz + zdz, zn[2]);
        }
#pragma unroll
        for (int o = 0; o < QN - 1; ++o) q[o] = q[o + 1];
        if constexpr (HAS_Z) {
#pragma unroll
            for (int o = 0; o < 8; ++o) pq[o] = pq[o + 1];
        }
    };

    // per plane: stage the lane's u^n (the queue centre) and the halo values
    // loaded one plane earlier into one of two LDS planes, issue the plane's
    // other loads and the next plane's halo, then one barrier and the taps
    float h1 = Buf<T>::ld(ru, hoff1, 4 * Sb), h2 = Buf<T>::ld(ru, hoff2, 4 * Sb);
    PL A;
    int buf = 0;
#pragma unroll 1
    for (int z = za; z < zb; ++z) {
        float *Lp = Lds + buf * LB;
        Lp[own] = q[4];
        Lp[hslot1] = h1;
        Lp[hslot2] = h2;
        load(z, A);
        // (plane z + 1 lies inside the field's frame planes even when z + 1 = zb)
        const uint32_t zn1 = (uint32_t)(z + 1 - za + 4) * Sb;
        h1 = Buf<T>::ld(ru, hoff1, zn1);
        h2 = Buf<T>::ld(ru, hoff2, zn1);
        __syncthreads();
#pragma unroll
        for (int l = 1; l <= 4; ++l) {
            A.xl[l - 1] = Lp[own - l];
            A.xh[l - 1] = Lp[own + l];
            A.yl[l - 1] = Lp[own - l * kBandLW];
            A.yh[l - 1] = Lp[own + l * kBandLW];
        }
        compute(z, A);
        buf ^= 1;
    }
}

// one launch for the tiles of all three kinds (a workgroup's kind is that of
// its box), so that they run side by side without extra streams; tiles of TY rows
template <typename T, int TY>
__global__ __launch_bounds__(BAND_TX *TY) void k_band(const DevShot *__restrict__ shots,
                                                     const BandItem *__restrict__ work, Roles R, int zchunk,
                                                     const int *__restrict__ stepc) {
    __shared__ float Lds[2 * band_lds(TY)];
    const BandItem wi = work[blockIdx.x];
    const int kind = wi.box >> 1;
    if (shots[wi.shot].fused) {
        if (kind == 0) band_tile<T, 0, true, TY>(shots, wi, R, zchunk, stepc, Lds);
        else if (kind == 1) band_tile<T, 1, true, TY>(shots, wi, R, zchunk, stepc, Lds);
        else band_tile<T, 2, true, TY>(shots, wi, R, zchunk, stepc, Lds);
    } else {
        if (kind == 0) band_tile<T, 0, false, TY>(shots, wi, R, zchunk, stepc, Lds);
        else if (kind == 1) band_tile<T, 1, false, TY>(shots, wi, R, zchunk, stepc, Lds);
        else band_tile<T, 2, false, TY>(shots, wi, R, zchunk, stepc, Lds);
    }
}

template <typename T>
static void launch_band_t(const DevShot *d_shots, const BandItem *work, int nwork, const Roles &R, int zchunk,
                          const int *stepc, int ty, hipStream_t st) {
    if (nwork <= 0) return;
    if (ty == BAND_TY_TALL)
        hipLaunchKernelGGL((k_band<T, BAND_TY_TALL>), dim3(nwork), dim3(BAND_TX * BAND_TY_TALL), 0, st, d_shots, work,
                           R, zchunk, stepc);
    else
        hipLaunchKernelGGL((k_band<T, BAND_TY>), dim3(nwork), dim3(BAND_TX * BAND_TY), 0, st, d_shots, work, R,
                           zchunk, stepc);
}

void fdtd_launch_band(int stor, const DevShot *d_shots, const BandItem *work, int nwork, const Roles &R, int zchunk,
                      const int *stepc, int ty, hipStream_t st) {
    if (stor == 1) launch_band_t<_Float16>(d_shots, work, nwork, R, zchunk, stepc, ty, st);
    else if (stor == 2) launch_band_t<__bf16>(d_shots, work, nwork, R, zchunk, stepc, ty, st);
    else launch_band_t<float>(d_shots, work, nwork, R, zchunk, stepc, ty, st);
}
