// fdtd_api.hip -- the C ABI (include/fdtd.h): validation, workspace layout,
// FP64 layer profiles, step orchestration, HIP graphs, ghost exchange tables,
// checkpoints, adjoint driver and autotuner.
//
// Profiles follow the paper's section "CPML Boundary Layers": node-based
// layer coordinate rho in [0,1] (1 at the outermost node, step 1/L), cubic
// grading sigma = sigma_max rho^3, kappa = 1 + (kappa_max - 1) rho^3,
// alpha = alpha_max (1 - rho), sigma_max = -(q+1) v_ref ln(R) / (2 L h) with
// q = 3, b = exp(-(sigma/kappa + alpha) dt), a = sigma (b-1)/(kappa (sigma +
// kappa alpha)), and d(1/kappa)/dx from the same grading.  They are computed
// in double precision here and rounded once to float for the kernels.
#include "../../include/fdtd.h"
#include "fdtd_launch.hpp"
#include "fdtd_host.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

// central weights of order 8: second derivative c0..c4 and first derivative d1..d4
static const double kC2[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
static const double kC1[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static int roundup(int x, int m) { return (x + m - 1) / m * m; }

#define FAIL(ctx, code, ...)                                                                                 \
    do {                                                                                                      \
        char _b[512];                                                                                         \
        snprintf(_b, sizeof _b, __VA_ARGS__);                                                                 \
        if (ctx) (ctx)->err = _b;                                                                             \
        return (code);                                                                                        \
    } while (0)
#define HIPCHK(ctx, expr)                                                                                     \
    do {                                                                                                      \
        hipError_t _e = (expr);                                                                               \
        if (_e != hipSuccess) FAIL(ctx, FDTD_EHIP, "%s: %s", #expr, hipGetErrorString(_e));                   \
    } while (0)

// ---------------------------------------------------------------------------
// layout and planning
// ---------------------------------------------------------------------------
static void plan_shot(ShotH &s) {
    const fdtd_shot_config &c = s.c;
    s.nx = c.n[0];
    s.ny = c.n[1];
    s.nz = c.n[2];
    s.gy = c.face[2] == FDTD_FACE_GHOST;
    s.gz = c.face[4] == FDTD_FACE_GHOST;
    s.s = (s.gy || s.gz) ? std::max(1, (int)c.exchange_every) : 1;
    s.g = 4 * s.s;
    s.fy = s.gy ? s.g : 4;
    s.fz = s.gz ? s.g : 4;
    s.esz = c.storage == FDTD_F32 ? 4 : 2;
    s.P = roundup(s.nx + 4, s.esz == 4 ? 64 : 128);
    s.PY = s.ny + 2 * s.fy;
    s.S = s.PY * s.P;
    for (int d = 0; d < 3; ++d) {
        s.Llo[d] = c.cpml[2 * d];
        s.Lhi[d] = c.cpml[2 * d + 1];
    }
    s.elems = (size_t)kOFF + (size_t)(s.nz + 2 * s.fz) * s.S + (size_t)(kTYMAX + 16) * s.P + 128;
    s.LX = s.Llo[0] + s.Lhi[0];
    s.LY = s.Llo[1] + s.Lhi[1];
    s.LZ = s.Llo[2] + s.Lhi[2];
    s.WX = std::max(s.Llo[0], s.Lhi[0]);
    s.SY = s.LY ? s.LY + 1 : 0;
    s.SZ = s.LZ ? s.LZ + 1 : 0;
    s.psi_elems[0] = (size_t)2 * (s.nz + 2 * s.fz) * s.PY * s.WX;
    s.psi_elems[1] = (size_t)(s.nz + 2 * s.fz) * s.SY * s.nx;
    s.psi_elems[2] = (size_t)s.SZ * s.PY * s.nx;
    s.nmax = std::max(s.nx, std::max(s.ny, s.nz));
    s.variant = c.variant == FDTD_VARIANT_AUTO ? FDTD_VARIANT_ZMARCH : c.variant;
    // default z-march plan (measured with the psi and band kernels running
    // beside it: 384^3 to 768^3 and the 1024 x 384 x 384 pencil at s = 1, 2,
    // 4).  The z-march's workgroups each hold a CU for the whole step, so their
    // number W sets how the 256 CUs are shared with the band kernel: aim at
    // W = 0.75 * 256 * (fraction of points outside the bands), never above 256
    // (a CU holding two z-march workgroups runs them at half speed and the
    // step waits for it).  Among tiles of 64 x 64, 64 x 32 and 64 x 16 points
    // (tile_ry 8, 4, 2) over 1..8 z chunks, the score |W - target| + 5 per
    // extra chunk + 20 for 64 x 16 tiles (more halo rows per point) is
    // lowest; ties go to the larger tile.
    {
        const int ext = s.g - 4;
        const int Ny = s.ny + (s.gy ? 2 * ext : 0), Nz = s.nz + (s.gz ? 2 * ext : 0);
        const int gh[3] = {0, s.gy, s.gz}, n3[3] = {s.nx, s.ny, s.nz};
        double inner = 1.0;
        for (int d = 0; d < 3; ++d) {
            // (the points outside the bands proper, on which the rule was measured)
            int a, b, e0, e1;
            band_range(n3[d], s.Llo[d], s.Lhi[d], gh[d], ext, a, b, e0, e1);
            inner *= (double)(b - a) / (double)(e1 - e0);
        }
        const double target = 0.75 * kCUs * inner;
        const long tx = (s.nx + 63) / 64;
        double best = 1e30;
        s.ry = 2;
        s.zchunk = std::min(std::max(32, (Nz + 15) / 16 * 16), 4096);
        for (int ry : {8, 4, 2}) {
            const long nxy = tx * ((Ny + 8 * ry - 1) / (8 * ry));
            for (int nc = 1; nc <= 8; ++nc) {
                int zc = (Nz + nc - 1) / nc;
                zc = std::min(std::max(32, (zc + 15) / 16 * 16), 4096);
                const long nch = (Nz + zc - 1) / zc;
                if (nch != nc) continue;   // that many chunks is not reachable
                const long W = nxy * nch;
                if (W > kCUs) continue;
                const double score = std::fabs((double)W - target) + 5.0 * (nch - 1) + (ry == 2 ? 20.0 : 0.0);
                if (score < best - 1e-9) {
                    best = score;
                    s.ry = ry;
                    s.zchunk = zc;
                }
            }
        }
    }
    s.tk = c.tblock_k > 1 ? c.tblock_k : 1;
    if (s.variant == FDTD_VARIANT_TBLOCK && s.tk < 2) s.tk = 2;
    // temporal blocking: four level buffers and the box B outside every band
    s.tb_bufs = s.variant == FDTD_VARIANT_TBLOCK;
    const int nn[3] = {s.nx, s.ny, s.nz};
    for (int d = 0; d < 3; ++d) {
        int lo, hi, e0, e1;   // the non-band range, as the band boxes and the z-march take it
        if (d == 0) band_range_x(nn[0], s.Llo[0], s.Lhi[0], lo, hi, e0, e1);
        else band_range(nn[d], s.Llo[d], s.Lhi[d], 0, 0, lo, hi, e0, e1);
        if (d == 0) {   // float4 columns: x bounds on multiples of 4
            lo = (lo + 3) / 4 * 4;
            hi = hi / 4 * 4;
        }
        s.blo[d] = lo;
        s.bhi[d] = std::max(lo, hi);
    }
}

static std::vector<WorkItem> tblock_tiles(const ShotH &s, int shot) {
    std::vector<WorkItem> v;
    const int K = s.tk;
    if (!s.tb_bufs || K < 2) return v;
    const int cx = fdtd_tblock_core(K, 0), cy = fdtd_tblock_core(K, 1);
    const int wx = s.bhi[0] - s.blo[0] - 8 * K, wy = s.bhi[1] - s.blo[1] - 8 * K, wz = s.bhi[2] - s.blo[2] - 8 * K;
    if (wx <= 0 || wy <= 0 || wz <= 0) return v;
    const int ntx = (wx + cx - 1) / cx, nty = (wy + cy - 1) / cy, ntz = (wz + s.tb_zchunk - 1) / s.tb_zchunk;
    for (int zc = 0; zc < ntz; ++zc)
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) v.push_back(WorkItem{shot, tx, ty, zc});
    return v;
}

static size_t tblock_capacity(const ShotH &s) {
    // the smallest core (K = 4) and z chunk bound the tile count
    if (!s.tb_bufs) return 0;
    const int cx = fdtd_tblock_core(4, 0), cy = fdtd_tblock_core(4, 1);
    return (size_t)((s.nx + cx - 1) / cx) * ((s.ny + cy - 1) / cy) * ((s.nz + s.tb_zchunk - 1) / s.tb_zchunk) + 8;
}

static int validate_shot(fdtd_ctx *ctx, const fdtd_shot_config &c, int i) {
    for (int d = 0; d < 3; ++d) {
        if (c.n[d] < 9) FAIL(ctx, FDTD_EINVAL, "shot %d: n[%d]=%d must be >= 9", i, d, c.n[d]);
        if (!(c.h[d] > 0)) FAIL(ctx, FDTD_EINVAL, "shot %d: h[%d] must be > 0", i, d);
    }
    if (!(c.dt > 0)) FAIL(ctx, FDTD_EINVAL, "shot %d: dt must be > 0", i);
    if ((long)c.n[0] * c.n[1] * c.n[2] > (1L << 30)) FAIL(ctx, FDTD_EUNSUPPORTED, "shot %d: grid too large", i);
    for (int f = 0; f < 6; ++f) {
        if (c.cpml[f] < 0) FAIL(ctx, FDTD_EINVAL, "shot %d: negative layer width", i);
        if (c.face[f] != FDTD_FACE_DIRICHLET && c.face[f] != FDTD_FACE_GHOST)
            FAIL(ctx, FDTD_EINVAL, "shot %d: face %d has an unknown type", i, f);
    }
    if (c.face[0] || c.face[1]) FAIL(ctx, FDTD_EINVAL, "shot %d: x faces cannot be ghost faces", i);
    for (int d = 1; d < 3; ++d) {
        if (c.face[2 * d] != c.face[2 * d + 1]) FAIL(ctx, FDTD_EINVAL, "shot %d: ghost faces come in pairs", i);
        if (c.face[2 * d] == FDTD_FACE_GHOST && (c.cpml[2 * d] || c.cpml[2 * d + 1]))
            FAIL(ctx, FDTD_EINVAL, "shot %d: ghost faces carry no absorbing layer", i);
    }
    for (int d = 0; d < 3; ++d) {
        if (2 * c.cpml[2 * d] >= c.n[d] || 2 * c.cpml[2 * d + 1] >= c.n[d])
            FAIL(ctx, FDTD_EINVAL, "shot %d: layer on axis %d must be narrower than half the axis", i, d);
    }
    bool ghost = c.face[2] || c.face[4];
    if (ghost) {
        int s = c.exchange_every ? c.exchange_every : 1;
        if (s != 1 && s != 2 && s != 4) FAIL(ctx, FDTD_EINVAL, "shot %d: exchange_every must be 1, 2 or 4", i);
        for (int d = 1; d < 3; ++d)
            if (c.face[2 * d] && c.n[d] < 4 * s)
                FAIL(ctx, FDTD_EINVAL, "shot %d: axis %d shorter than the ghost depth", i, d);
    }
    if (c.storage < 0 || c.storage > 2) FAIL(ctx, FDTD_EINVAL, "shot %d: unknown storage", i);
    const bool ghost_faces = c.face[2] || c.face[4];
    (void)ghost_faces;
    if (c.variant < 0 || c.variant > 3) FAIL(ctx, FDTD_EINVAL, "shot %d: unknown variant", i);
    if (c.variant == FDTD_VARIANT_TBLOCK && !(c.tblock_k == 2 || c.tblock_k == 4))
        FAIL(ctx, FDTD_EINVAL, "shot %d: tblock_k must be 2 or 4", i);
    if (c.variant == FDTD_VARIANT_TBLOCK && (c.storage != FDTD_F32 || ghost_faces))
        FAIL(ctx, FDTD_EINVAL, "shot %d: temporal blocking runs FP32 storage with Dirichlet faces", i);
    if (c.R < 0 || c.R >= 1 || c.kappa_max < 0 || c.alpha_frac < 0 || c.v_ref < 0)
        FAIL(ctx, FDTD_EINVAL, "shot %d: bad layer parameters", i);
    if (c.field_scale != 0) {
        int e;
        double mnt = frexp(c.field_scale, &e);
        if (!(c.field_scale > 0) || mnt != 0.5) FAIL(ctx, FDTD_EINVAL, "shot %d: field_scale must be a power of 2", i);
    }
    return FDTD_OK;
}

// XCD-aware order: hardware hands workgroup b to XCD (b mod 8); give each XCD a
// contiguous spatial range so that tiles sharing halos share an L2.
template <typename W> static W idle_item(const std::vector<W> &sp);
template <> WorkItem idle_item(const std::vector<WorkItem> &sp) {
    return WorkItem{sp.empty() ? 0 : sp[0].shot, 0, 1 << 20, 0};   // exits immediately
}
template <> BandItem idle_item(const std::vector<BandItem> &sp) {
    return BandItem{sp.empty() ? 0 : sp[0].shot, 0, 1 << 20, 0, 0, 0, 0, 0};
}
template <typename W> static std::vector<W> xcd_order(const std::vector<W> &sp) {
    const int X = 8;
    size_t N = (sp.size() + X - 1) / X * X;
    std::vector<W> out(N);
    size_t per = N / X;
    for (size_t w = 0; w < N; ++w) {
        size_t src = (w % X) * per + w / X;
        out[w] = src < sp.size() ? sp[src] : idle_item(sp);
    }
    return out;
}

// band-kernel tiles of a shot, for the largest compute box it uses (smaller
// boxes reuse the list; tiles past a box end exit at once)
static std::vector<BandItem> band_tiles(const ShotH &s, int shot, int ty) {
    const int ext = (s.gy || s.gz) ? s.g - 4 : 0;
    const int n3[3] = {s.nx, s.ny, s.nz}, gh[3] = {0, s.gy, s.gz};
    std::vector<BandItem> v;
    for (int b = 0; b < 6; ++b) {
        int lo[3], hi[3];
        band_box(n3, s.Llo, s.Lhi, gh, ext, b, lo, hi);
        const int wx = hi[0] - lo[0], wy = hi[1] - lo[1], wz = hi[2] - lo[2];
        if (wx <= 0 || wy <= 0 || wz <= 0) continue;
        // z boxes (b < 2) are walked whole; x tiles as band_xtiles cuts them
        int x0, x1;
        const int ntx = band_xtiles(s.nx, s.Llo[0], s.Lhi[0], b, lo[0], hi[0], 0, &x0, &x1);
        const int nzc = b < 2 ? 1 : (wz + kBandZ - 1) / kBandZ, nty = (wy + ty - 1) / ty;
        for (int zc = 0; zc < nzc; ++zc)
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < ntx; ++tx) v.push_back(BandItem{shot, b, tx, ty, zc, 0, 0, 0});
    }
    return v;
}
// (the shorter tiles give the longer list)
static size_t band_capacity(const ShotH &s) { return band_tiles(s, 0, BAND_TY).size() + 8; }

static std::vector<WorkItem> shot_tiles(const ShotH &s, int shot, int ry, int zchunk, int cols) {
    int ext = s.g - 4;
    int Ny = s.ny + (s.gy ? 2 * ext : 0);
    int Nz = s.nz + (s.gz ? 2 * ext : 0);
    int TY = 8 * ry;   // z-march tile rows: tiles of 64 cols x 8 ry points
    const int TX = 64 * cols;
    int ntx = (s.nx + TX - 1) / TX, nty = (Ny + TY - 1) / TY, ntz = (Nz + zchunk - 1) / zchunk;
    std::vector<WorkItem> v;
    v.reserve((size_t)ntx * nty * ntz);
    for (int zc = 0; zc < ntz; ++zc)
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) v.push_back(WorkItem{shot, tx, ty, zc});
    return v;
}

static size_t work_capacity(const ShotH &s) {
    int ext = s.g - 4;
    int Ny = s.ny + (s.gy ? 2 * ext : 0);
    int Nz = s.nz + (s.gz ? 2 * ext : 0);
    return (size_t)((s.nx + 63) / 64) * ((Ny + 7) / 8) * ((Nz + 15) / 16) + 8;
}

static long psi_count(const ShotH &s, int d, int ext) {
    int Ny = s.ny + (s.gy ? 2 * ext : 0);
    int Nz = s.nz + (s.gz ? 2 * ext : 0);
    if (d == 0) return (long)s.LX * Ny * Nz;
    if (d == 1) return (long)s.nx * s.LY * Nz;
    return (long)s.nx * Ny * s.LZ;
}

// Whether the band kernel advances psi_x and psi_z itself (DevShot::fused).
// It needs every x-layer point and the band points that read it in one tile
// row (each x band at most BAND_TX wide, and the two x bands far enough apart
// that neither reads the other's layer points), and likewise the two z boxes
// sharing no layer point.  Naive shots read every psi from the psi pass.
static bool shot_fused(const ShotH &s) {
    if (s.variant == FDTD_VARIANT_NAIVE) return false;
    const int lx = s.Llo[0], hx = s.Lhi[0], lz = s.Llo[2], hz = s.Lhi[2];
    if (lx + hx > 0 && (lx + FDTD_R > kBandTX || hx + FDTD_R > kBandTX || s.nx < lx + hx + 2 * FDTD_R)) return false;
    if (lz + hz > 0 && s.nz < lz + hz + 2 * FDTD_R) return false;
    return true;
}

// ---------------------------------------------------------------------------
// profiles (FP64)
// ---------------------------------------------------------------------------
static void layer_profile(const ShotH &s, int d, double vref, double *b, double *a, double *kinv, double *dkinv) {
    const fdtd_shot_config &c = s.c;
    const int n = d == 0 ? s.nx : (d == 1 ? s.ny : s.nz);
    const int lo = s.Llo[d], hi = s.Lhi[d];
    const double q = 3.0;
    const double R = c.R > 0 ? c.R : 1e-8;
    const double kmax = c.kappa_max > 0 ? c.kappa_max : 5.0;
    const double af = c.alpha_frac > 0 ? c.alpha_frac : 0.05;
    const double h = c.h[d];
    for (int i = 0; i < n; ++i) {
        int L = 0;
        double rho = 0.0, drho = 0.0;
        if (lo > 0 && i < lo) {
            L = lo;
            rho = (double)(lo - i) / lo;
            drho = -1.0 / (lo * h);
        } else if (hi > 0 && i >= n - hi) {
            L = hi;
            rho = (double)(i - (n - 1 - hi)) / hi;
            drho = 1.0 / (hi * h);
        }
        if (rho > 0) {
            const double sigma_max = -(q + 1.0) * vref * std::log(R) / (2.0 * L * h);
            const double r3 = rho * rho * rho;
            const double sigma = sigma_max * r3;
            const double kappa = 1.0 + (kmax - 1.0) * r3;
            const double alpha = af * sigma_max * (1.0 - rho);
            const double bb = std::exp(-(sigma / kappa + alpha) * c.dt);
            b[i] = bb;
            a[i] = sigma > 0 ? sigma * (bb - 1.0) / (kappa * (sigma + kappa * alpha)) : 0.0;
            kinv[i] = 1.0 / kappa;
            dkinv[i] = -(kmax - 1.0) * 3.0 * rho * rho * drho / (kappa * kappa);
        } else {
            b[i] = 0.0;
            a[i] = 0.0;
            kinv[i] = 1.0;
            dkinv[i] = 0.0;
        }
    }
}

// largest eigenvalue factor of -D2 for the radius-4 weights: -(c0 + 2 sum c_l (-1)^l)
static double d2_symbol_max() {
    double s = kC2[0];
    for (int l = 1; l <= 4; ++l) s += 2.0 * kC2[l] * ((l & 1) ? -1.0 : 1.0);
    return -s;
}

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
static char *wsp(fdtd_ctx *ctx, size_t off) { return ctx->ws + off; }

static void *field_origin(fdtd_ctx *ctx, const ShotH &s, size_t off) {
    return wsp(ctx, off) + origin_elems(s) * s.esz;
}
static float *m_origin(fdtd_ctx *ctx, const ShotH &s) {
    return (float *)(wsp(ctx, s.o_m) + origin_elems(s) * 4);
}

static void fill_desc(fdtd_ctx *ctx, int i) {
    ShotH &s = ctx->shots[i];
    DevShot &D = ctx->hdesc[i];
    memset(&D, 0, sizeof D);
    D.u[0] = field_origin(ctx, s, s.o_u[0]);
    D.u[1] = field_origin(ctx, s, s.o_u[1]);
    D.u[2] = s.tb_bufs ? field_origin(ctx, s, s.o_u[2]) : nullptr;
    D.u[3] = s.tb_bufs ? field_origin(ctx, s, s.o_u[3]) : nullptr;
    D.dinc = s.esz == 2 ? field_origin(ctx, s, s.o_d) : nullptr;
    D.m = m_origin(ctx, s);
    for (int d = 0; d < 3; ++d) {
        D.psi[d] = (float *)wsp(ctx, s.o_psi[d]);
        D.zeta[d] = (float *)wsp(ctx, s.o_zeta[d]);
    }
    D.prof = (const float *)wsp(ctx, s.o_prof);
    D.wav = s.has_src ? s.wav : nullptr;
    D.traces = s.traces;
    D.rec = s.rec;
    const double vol = s.c.h[0] * s.c.h[1] * s.c.h[2];
    D.src_scale = (float)((double)s.amp * s.scale / vol);
    D.inv_scale = (float)(1.0 / s.scale);
    D.src_nt = s.has_src ? s.src_nt : 0;
    D.sx = s.has_src ? s.sx : -(1 << 30);
    D.sy = s.has_src ? s.sy : -(1 << 30);
    D.sz = s.has_src ? s.sz : -(1 << 30);
    D.nrec = s.nrec;
    D.trace_cap = s.traces ? s.cap : 0;
    D.nx = s.nx;
    D.ny = s.ny;
    D.nz = s.nz;
    D.P = s.P;
    D.PY = s.PY;
    D.S = s.S;
    D.fy = s.fy;
    D.fz = s.fz;
    for (int d = 0; d < 3; ++d) {
        D.Llo[d] = s.Llo[d];
        D.Lhi[d] = s.Lhi[d];
    }
    D.LX = s.LX;
    D.LY = s.LY;
    D.LZ = s.LZ;
    D.WX = s.WX;
    D.SY = s.SY;
    D.SZ = s.SZ;
    D.nmax = s.nmax;
    D.ghost[0] = 0;
    D.ghost[1] = s.gy;
    D.ghost[2] = s.gz;
    D.fused = shot_fused(s) ? 1 : 0;
    double cc = 0;
    for (int d = 0; d < 3; ++d) {
        const double h = s.c.h[d];
        for (int l = 0; l <= 4; ++l) {
            D.w2[d][l] = (float)(kC2[l] / (h * h));
            D.w1[d][l] = (float)(kC1[l] / h);
        }
        // centre weight of the difference form (the nearest pair enters as f_{+-1} - f_c)
        D.w2[d][0] = (float)((kC2[0] + 2.0 * kC2[1]) / (h * h));
        cc += (kC2[0] + 2.0 * kC2[1]) / (h * h);
    }
    D.cc = (float)cc;
}

static int upload_desc(fdtd_ctx *ctx) {
    for (size_t i = 0; i < ctx->shots.size(); ++i) fill_desc(ctx, (int)i);
    HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, ctx->o_desc), ctx->hdesc.data(), sizeof(DevShot) * ctx->hdesc.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return FDTD_OK;
}

// largest piece (16, 8, 4 or 2 bytes, at least the element) that divides both
// row starts, every stride and the row length of a copy job, in bytes
static void set_copy_vec(CopyJob &j) {
    const uintptr_t bits = (uintptr_t)j.src | (uintptr_t)j.dst | (uintptr_t)(j.sy * j.esz) |
                           (uintptr_t)(j.sz * j.esz) | (uintptr_t)(j.dy * j.esz) | (uintptr_t)(j.dz * j.esz) |
                           (uintptr_t)(j.ex * j.esz);
    j.vb = j.esz;
    for (int vb : {16, 8, 4})
        if (vb > j.esz && (bits & (uintptr_t)(vb - 1)) == 0) {
            j.vb = vb;
            break;
        }
}

// ghost-exchange copy jobs (loopback): [parity][phase] with phases
// 0 pack-y, 1 unpack-y, 2 pack-z, 3 unpack-z
static void build_jobs(fdtd_ctx *ctx, int i, std::vector<CopyJob> (&jobs)[2][4], long (&maxe)[2][4]) {
    ShotH &s = ctx->shots[i];
    for (int p = 0; p < 2; ++p)
        for (int ph = 0; ph < 4; ++ph) {
            jobs[p][ph].clear();
            maxe[p][ph] = 0;
        }
    if (!s.gy && !s.gz) return;
    char *xb = wsp(ctx, s.o_xbuf);
    for (int p = 0; p < 2; ++p) {
        // fields: u^n depth g; u^{n-1} depth g-4; psi_x, zeta_x depth g-4
        struct F {
            char *org;      // origin (element (0,0,0) or slab (is=0,y=0,z=0))
            int esz, ex;    // element size, x extent
            long rowst, plst;
            int dep;
        };
        std::vector<F> fs;
        char *un = (char *)field_origin(ctx, s, s.o_u[p]);
        char *um = (char *)field_origin(ctx, s, s.esz == 2 ? s.o_d : s.o_u[p ^ 1]);
        fs.push_back(F{un, (int)s.esz, s.nx, (long)s.P, (long)s.S, s.g});
        if (s.g - 4 > 0) {
            fs.push_back(F{um, (int)s.esz, s.nx, (long)s.P, (long)s.S, s.g - 4});
            // x layer arrays: the two layers are blocks of their own (psi_index)
            for (int w = 0; w < 2; ++w)
                for (int side = 0; side < 2; ++side) {
                    const int ex = side == 0 ? s.Llo[0] : s.Lhi[0];
                    if (ex <= 0) continue;
                    char *base = wsp(ctx, w == 0 ? s.o_psi[0] : s.o_zeta[0]) +
                                 (size_t)side * (s.nz + 2 * s.fz) * s.PY * s.WX * 4;
                    char *org = base + ((size_t)s.fz * s.PY + s.fy) * s.WX * 4;
                    fs.push_back(F{org, 4, ex, (long)s.WX, (long)s.PY * s.WX, s.g - 4});
                }
        }
        // phase y
        size_t off = 0;
        if (s.gy) {
            for (auto &f : fs) {
                long face = (long)f.dep * s.nz * f.ex;  // elements per face
                for (int side = 0; side < 2; ++side) {
                    // side 0: owned rows [0,dep) -> ghost rows [ny, ny+dep)
                    // side 1: owned rows [ny-dep, ny) -> ghost rows [-dep, 0)
                    int ys = side == 0 ? 0 : s.ny - f.dep;
                    int yd = side == 0 ? s.ny : -f.dep;
                    char *buf = xb + off;
                    CopyJob pk{f.org + ((long)ys * f.rowst) * f.esz, buf, f.esz, f.ex, f.dep, s.nz,
                               f.rowst, f.plst, (long)f.ex, (long)f.ex * f.dep, 0};
                    CopyJob up{buf, f.org + ((long)yd * f.rowst) * f.esz, f.esz, f.ex, f.dep, s.nz,
                               (long)f.ex, (long)f.ex * f.dep, f.rowst, f.plst, 0};
                    set_copy_vec(pk);
                    set_copy_vec(up);
                    jobs[p][0].push_back(pk);
                    jobs[p][1].push_back(up);
                    maxe[p][0] = std::max(maxe[p][0], (long)f.dep * s.nz);
                    maxe[p][1] = std::max(maxe[p][1], (long)f.dep * s.nz);
                    off += align256(face * f.esz);
                }
            }
        }
        off = 0;
        if (s.gz) {
            for (auto &f : fs) {
                int dy = s.gy ? f.dep : 0;
                int Ny = s.ny + 2 * dy;
                long face = (long)f.dep * Ny * f.ex;
                for (int side = 0; side < 2; ++side) {
                    int zs = side == 0 ? 0 : s.nz - f.dep;
                    int zd = side == 0 ? s.nz : -f.dep;
                    char *buf = xb + off;
                    char *src = f.org + ((long)zs * f.plst - (long)dy * f.rowst) * f.esz;
                    char *dst = f.org + ((long)zd * f.plst - (long)dy * f.rowst) * f.esz;
                    CopyJob pk{src, buf, f.esz, f.ex, Ny, f.dep, f.rowst, f.plst, (long)f.ex, (long)f.ex * Ny, 0};
                    CopyJob up{buf, dst, f.esz, f.ex, Ny, f.dep, (long)f.ex, (long)f.ex * Ny, f.rowst, f.plst, 0};
                    set_copy_vec(pk);
                    set_copy_vec(up);
                    jobs[p][2].push_back(pk);
                    jobs[p][3].push_back(up);
                    maxe[p][2] = std::max(maxe[p][2], (long)Ny * f.dep);
                    maxe[p][3] = std::max(maxe[p][3], (long)Ny * f.dep);
                    off += align256(face * f.esz);
                }
            }
        }
    }
}

static size_t xbuf_bytes(const ShotH &s) {
    if (!s.gy && !s.gz) return 0;
    size_t by = 0, bz = 0;
    auto add = [&](int esz, int ex, int dep) {
        if (dep <= 0) return;
        if (s.gy) by += 2 * align256((size_t)dep * s.nz * ex * esz);
        if (s.gz) bz += 2 * align256((size_t)dep * (s.ny + (s.gy ? 2 * dep : 0)) * ex * esz);
    };
    add((int)s.esz, s.nx, s.g);
    add((int)s.esz, s.nx, s.g - 4);
    for (int w = 0; w < 2; ++w) {
        if (s.Llo[0] > 0) add(4, s.Llo[0], s.g - 4);
        if (s.Lhi[0] > 0) add(4, s.Lhi[0], s.g - 4);
    }
    return std::max(by, bz);
}

// ---------------------------------------------------------------------------
// per-kernel-class event timing
// ---------------------------------------------------------------------------
static hipEvent_t take_event(fdtd_ctx *ctx) {
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_used++];
}
static hipEvent_t tic(fdtd_ctx *ctx, hipStream_t st) {
    if (!ctx->timing) return nullptr;
    hipEvent_t e = take_event(ctx);
    if (e) (void)hipEventRecord(e, st);
    return e;
}
static void toc(fdtd_ctx *ctx, int cls, hipEvent_t start, hipStream_t st) {
    if (!ctx->timing || !start) return;
    hipEvent_t e = take_event(ctx);
    if (!e) return;
    (void)hipEventRecord(e, st);
    ctx->ev_pairs[cls].push_back(std::make_pair(start, e));
}
static hipEvent_t tic(fdtd_ctx *ctx) { return tic(ctx, ctx->stream); }
static void toc(fdtd_ctx *ctx, int cls, hipEvent_t start) { toc(ctx, cls, start, ctx->stream); }
// fold recorded pairs into the sums (synchronises) and recycle the events
static int drain_timing(fdtd_ctx *ctx) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < kTimingClasses; ++c) {
        for (auto &pr : ctx->ev_pairs[c]) {
            float ms = 0;
            HIPCHK(ctx, hipEventElapsedTime(&ms, pr.first, pr.second));
            ctx->t_sum[c] += ms;
            ctx->t_cnt[c] += 1;
        }
        ctx->ev_pairs[c].clear();
    }
    ctx->ev_used = 0;
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------
static void save_checkpoint(fdtd_ctx *ctx, int i, int k);

static int ghost_ext(const fdtd_ctx *ctx, long step) {
    for (const ShotH &s : ctx->shots)
        if (s.gy || s.gz) return 4 * (s.s - 1 - (int)(step % s.s));
    return 0;
}

static void enqueue_exchange(fdtd_ctx *ctx, int i) {
    ShotH &s = ctx->shots[i];
    const int p = ctx->iu;
    for (int ph = 0; ph < 4; ++ph) {
        if (s.njobs[p][ph] == 0) continue;
        fdtd_launch_copy_jobs(wsp(ctx, s.o_jobs[p][ph]), s.njobs[p][ph], s.jobmax[p][ph], ctx->stream);
    }
}

static Roles plain_roles(const fdtd_ctx *ctx, int ext) {
    Roles R;
    R.iu = ctx->iu;
    R.ium1 = ctx->ium1;
    R.iout = ctx->ium1;
    R.ext = ext;
    for (int d = 0; d < 3; ++d) R.lo[d] = R.hi[d] = 0;
    return R;
}

// psi pre-pass and update of one shot or of all shots (shot < 0).  The
// z-march of the points outside the bands runs on the side stream, forked
// from and joined back to the main one, concurrently with the psi pass and
// the band kernels: the two sets of points are disjoint and both read only
// u^n (and their own points' second state).  The band kernel covers the
// tiles of all three band kinds in one launch after the psi pass.  (One fork
// per step keeps a captured graph to two branches per step: graphs of many
// steps with more parallel branches have exhausted the HIP runtime's launch
// resources.)  Naive shots update every point after the psi pass, on the main
// stream.  With per-kernel timing enabled everything stays on the main
// stream, so that each timed duration is the kernel's own.
static void enqueue_psi_update(fdtd_ctx *ctx, int shot, const Roles &R) {
    const DevShot *dd = (const DevShot *)wsp(ctx, ctx->o_desc);
    int *stepc = (int *)wsp(ctx, ctx->o_stepc);
    const int stor = ctx->storage;
    const int ext = R.ext;
    const int lo = shot < 0 ? 0 : shot, hi = shot < 0 ? (int)ctx->shots.size() : shot + 1;
    const bool grouped = shot < 0 && !ctx->groups.empty();
    bool any_zm = false;
    for (int i = lo; i < hi; ++i) any_zm = any_zm || ctx->shots[i].variant != FDTD_VARIANT_NAIVE;
    hipStream_t side = ctx->stream;
    if (any_zm && ctx->side && !ctx->timing) {
        (void)hipEventRecord(ctx->ev_fork, ctx->stream);
        (void)hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
        side = ctx->side;
    }
    if (any_zm) {
        hipEvent_t t0 = tic(ctx, side);
        if (grouped) {
            const WorkItem *wa = (const WorkItem *)wsp(ctx, ctx->o_work_all);
            for (const auto &g : ctx->groups)
                fdtd_launch_zmarch(stor, dd, wa + g.off, g.nwork, g.ry, g.cols, R, g.zchunk, stepc, side);
        } else {
            for (int i = lo; i < hi; ++i) {
                const ShotH &s = ctx->shots[i];
                if (s.variant == FDTD_VARIANT_NAIVE) continue;
                fdtd_launch_zmarch(stor, dd, (const WorkItem *)wsp(ctx, s.o_work), s.nwork, s.ry, s.zcols, R, s.zchunk,
                                   stepc,
                                   side);
            }
        }
        toc(ctx, 0, t0, side);
    }
    // psi pass: psi_y along y lines; psi_x and psi_z of shots that are not
    // fused (the kernel skips the fused ones)
    bool all_fused = true;
    long maxc = 0, maxl = 0;
    for (int i = lo; i < hi; ++i) {
        const ShotH &si = ctx->shots[i];
        all_fused = all_fused && shot_fused(si);
        maxc = std::max(maxc, std::max(psi_count(si, 0, ext), psi_count(si, 2, ext)));
        if (si.LY > 0) maxl = std::max(maxl, (long)si.nx * (si.nz + (si.gz ? 2 * ext : 0)));
    }
    hipEvent_t t0 = tic(ctx);
    fdtd_launch_psi_y(stor, dd + lo, hi - lo, maxl, R.iu, ext, ctx->stream);
    if (!all_fused) fdtd_launch_psi(stor, dd + lo, hi - lo, maxc, R.iu, ext, 0, 3, ctx->stream);
    toc(ctx, 1, t0);
    if (any_zm) {
        t0 = tic(ctx);
        if (grouped) {
            fdtd_launch_band(stor, dd, (const BandItem *)wsp(ctx, ctx->o_band_all), ctx->nband_all, R, kBandZ, stepc,
                             ctx->band_ty, ctx->stream);
        } else {
            for (int i = lo; i < hi; ++i) {
                const ShotH &s = ctx->shots[i];
                if (s.variant == FDTD_VARIANT_NAIVE) continue;
                fdtd_launch_band(stor, dd, (const BandItem *)wsp(ctx, s.o_band), s.nband, R, kBandZ, stepc, ctx->band_ty,
                                 ctx->stream);
            }
        }
        toc(ctx, 4, t0);
    }
    for (int i = lo; i < hi; ++i) {
        const ShotH &s = ctx->shots[i];
        if (s.variant != FDTD_VARIANT_NAIVE) continue;
        const int Ny = s.ny + (s.gy ? 2 * ext : 0), Nz = s.nz + (s.gz ? 2 * ext : 0);
        t0 = tic(ctx);
        fdtd_launch_naive(stor, dd, i, s.nx, Ny, Nz, R, stepc, ctx->stream);
        toc(ctx, 0, t0);
    }
    if (side != ctx->stream) {
        (void)hipEventRecord(ctx->ev_join, side);
        (void)hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
    }
}

// one step of one shot (shot >= 0) or of every shot (shot < 0)
static void enqueue_step(fdtd_ctx *ctx, int shot) {
    const long n = ctx->step;
    int lo = shot < 0 ? 0 : shot, hi = shot < 0 ? (int)ctx->shots.size() : shot + 1;
    for (int i = lo; i < hi; ++i) {
        ShotH &s = ctx->shots[i];
        if (s.ck_every > 0 && ctx->saving && n % s.ck_every == 0 && n / s.ck_every < s.ck_count)
            save_checkpoint(ctx, i, (int)(n / s.ck_every));
        if ((s.gy || s.gz) && n % s.s == 0) {
            hipEvent_t t0 = tic(ctx);
            enqueue_exchange(ctx, i);
            toc(ctx, 3, t0);
        }
    }
    const int ext = ghost_ext(ctx, n);
    const DevShot *dd = (const DevShot *)wsp(ctx, ctx->o_desc);
    const Roles R = plain_roles(ctx, ext);
    enqueue_psi_update(ctx, shot, R);
    hipEvent_t t0 = tic(ctx);
    fdtd_launch_record(ctx->storage, dd + lo, hi - lo, R, (int *)wsp(ctx, ctx->o_stepc), ctx->stream);
    toc(ctx, 2, t0);
    std::swap(ctx->iu, ctx->ium1);
    ctx->step = n + 1;
}

// Temporal blocking applies to a single-shot context whose shot has the four
// level buffers, a non-empty B_K, and no checkpoint saving in progress.
static bool tblock_active(const fdtd_ctx *ctx) {
    if (ctx->shots.size() != 1) return false;
    const ShotH &s = ctx->shots[0];
    if (s.variant != FDTD_VARIANT_TBLOCK || !s.tb_bufs || s.tk < 2 || s.ntbwork <= 0) return false;
    if (s.ck_every > 0 && ctx->saving) return false;
    return true;
}

// K steps: the interior kernel on B, then the shell level by level outside B_j
static void enqueue_tblock(fdtd_ctx *ctx) {
    ShotH &s = ctx->shots[0];
    const int K = s.tk;
    const int A = ctx->iu, Bf = ctx->ium1;
    int spare[2], ns = 0;
    for (int b = 0; b < 4; ++b)
        if (b != A && b != Bf) spare[ns++] = b;
    // level n+j lives in Lv[j+1]: n-1 -> Bf, n -> A, odd j -> spare[0], even j -> spare[1]
    int Lv[6];
    Lv[0] = Bf;
    Lv[1] = A;
    for (int j = 1; j <= 4; ++j) Lv[j + 1] = (j & 1) ? spare[0] : spare[1];
    const DevShot *dd = (const DevShot *)wsp(ctx, ctx->o_desc);
    int *stepc = (int *)wsp(ctx, ctx->o_stepc);
    TBArgsHost a;
    for (int d = 0; d < 3; ++d) {
        a.blo[d] = s.blo[d];
        a.bhi[d] = s.bhi[d];
    }
    for (int j = 0; j < 6; ++j) a.L[j] = Lv[j];
    a.rec_zs = (const int *)wsp(ctx, s.o_reczs);
    a.rec_ix = (const int *)wsp(ctx, s.o_recix);
    hipEvent_t t0 = tic(ctx);
    fdtd_launch_tblock(dd, (const WorkItem *)wsp(ctx, s.o_tbwork), s.ntbwork, K, &a, s.tb_zchunk, stepc, ctx->stream);
    toc(ctx, 5, t0);
    for (int j = 1; j <= K; ++j) {
        Roles R;
        R.iu = Lv[j];
        R.ium1 = Lv[j - 1];
        R.iout = Lv[j + 1];
        R.ext = 0;
        for (int d = 0; d < 3; ++d) {
            R.lo[d] = s.blo[d] + 4 * j;
            R.hi[d] = s.bhi[d] - 4 * j;
        }
        enqueue_psi_update(ctx, 0, R);
        t0 = tic(ctx);
        fdtd_launch_record(ctx->storage, dd, 1, R, stepc, ctx->stream);
        toc(ctx, 2, t0);
    }
    ctx->iu = Lv[K + 1];
    ctx->ium1 = Lv[K];
    ctx->step += K;
}

// nsteps steps of every shot (temporal blocks where they apply)
// NaN/Inf sentinel: scan the newest level of every shot into the sticky flag
// (scratch slot 3), cleared only by fdtd_set_sentinel and fdtd_reset
static void enqueue_sentinel(fdtd_ctx *ctx) {
    unsigned int *flag = (unsigned int *)wsp(ctx, ctx->o_scratch) + 3;
    for (auto &s : ctx->shots)
        fdtd_launch_finite(ctx->storage, field_origin(ctx, s, s.o_u[ctx->iu]), s.nx, s.ny, s.nz, s.P, s.S, flag,
                           ctx->stream);
}

// nsteps steps; returns how many sentinel scans were enqueued (a scan follows
// each step whose count is a multiple of sentinel_every)
static int enqueue_steps(fdtd_ctx *ctx, int nsteps) {
    int k = 0, scans = 0;
    while (k < nsteps) {
        const long before = ctx->step;
        if (tblock_active(ctx) && nsteps - k >= ctx->shots[0].tk) {
            enqueue_tblock(ctx);
            k += ctx->shots[0].tk;
        } else {
            enqueue_step(ctx, -1);
            ++k;
        }
        const long e = ctx->sentinel_every;
        if (e > 0 && ctx->step / e != before / e) {
            enqueue_sentinel(ctx);
            ++scans;
        }
    }
    return scans;
}

// read the sentinel flag (synchronises the stream)
static int sentinel_check(fdtd_ctx *ctx) {
    unsigned int bad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&bad, (unsigned int *)wsp(ctx, ctx->o_scratch) + 3, 4, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad)
        FAIL(ctx, FDTD_ENONFINITE, "non-finite value in a wavefield at or before step %ld (sentinel every %d steps)",
             ctx->step, ctx->sentinel_every);
    return FDTD_OK;
}

static int ready(fdtd_ctx *ctx) {
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    for (size_t i = 0; i < ctx->shots.size(); ++i)
        if (!ctx->shots[i].vel_set) FAIL(ctx, FDTD_ESTATE, "shot %zu has no velocity model", i);
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// checkpoints: state k = (u^n, u^{n-1}, psi, zeta) before step k*every
// ---------------------------------------------------------------------------
size_t fdtd_state_bytes(const ShotH &s) {
    size_t b = 2 * align256(s.elems * s.esz);
    for (int d = 0; d < 3; ++d) b += 2 * align256(s.psi_elems[d] * 4);
    return b;
}

static void copy_state(fdtd_ctx *ctx, int i, char *ck, bool save) {
    ShotH &s = ctx->shots[i];
    size_t fb = s.elems * s.esz;
    // slot 0 of a checkpoint always holds u^n, slot 1 u^{n-1} (FP32) or d^n (16-bit)
    char *un = wsp(ctx, s.o_u[ctx->iu]);
    char *um = s.esz == 2 ? wsp(ctx, s.o_d) : wsp(ctx, s.o_u[ctx->ium1]);
    size_t off = 0;
    char *dsts[2] = {un, um};
    for (int k = 0; k < 2; ++k) {
        if (save) (void)hipMemcpyAsync(ck + off, dsts[k], fb, hipMemcpyDeviceToDevice, ctx->stream);
        else (void)hipMemcpyAsync(dsts[k], ck + off, fb, hipMemcpyDeviceToDevice, ctx->stream);
        off += align256(fb);
    }
    for (int d = 0; d < 3; ++d) {
        size_t pb = s.psi_elems[d] * 4;
        char *arr[2] = {wsp(ctx, s.o_psi[d]), wsp(ctx, s.o_zeta[d])};
        for (int k = 0; k < 2; ++k) {
            if (pb) {
                if (save) (void)hipMemcpyAsync(ck + off, arr[k], pb, hipMemcpyDeviceToDevice, ctx->stream);
                else (void)hipMemcpyAsync(arr[k], ck + off, pb, hipMemcpyDeviceToDevice, ctx->stream);
            }
            off += align256(pb);
        }
    }
}

static void save_checkpoint(fdtd_ctx *ctx, int i, int k) {
    ShotH &s = ctx->shots[i];
    copy_state(ctx, i, s.ck_buf + (size_t)k * fdtd_state_bytes(s), true);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fdtd_strerror(int st) {
    switch (st) {
    case FDTD_OK: return "ok";
    case FDTD_EINVAL: return "invalid argument";
    case FDTD_EUNSTABLE: return "time step above the stability limit";
    case FDTD_ESTATE: return "call out of order";
    case FDTD_ENOMEM: return "buffer too small";
    case FDTD_EHIP: return "HIP runtime error";
    case FDTD_ENONFINITE: return "non-finite value in a wavefield";
    case FDTD_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

const char *fdtd_last_error(const fdtd_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int fdtd_create(const fdtd_shot_config *shots, int32_t nshots, void *hip_stream, fdtd_ctx **out) {
    if (!out || !shots || nshots <= 0 || nshots > FDTD_MAXSHOTS) return FDTD_EINVAL;
    *out = nullptr;
    fdtd_ctx *ctx = new fdtd_ctx();
    ctx->stream = (hipStream_t)hip_stream;
    int ghost_s = 0;
    for (int i = 0; i < nshots; ++i) {
        int rc = validate_shot(ctx, shots[i], i);
        if (rc) {
            std::string e = ctx->err;
            delete ctx;
            fprintf(stderr, "fdtd_create: %s\n", e.c_str());
            return rc;
        }
        if (shots[i].storage != shots[0].storage) {
            delete ctx;
            return FDTD_EINVAL;
        }
        ShotH s;
        s.c = shots[i];
        plan_shot(s);
        // kernels address a field plane, and a layer array, with 32-bit offsets;
        // the band kernel reaches up to its z walk (a whole z box, or a chunk of
        // kBandZ planes) plus 12 planes from one descriptor
        const size_t walk = (size_t)std::max(kBandZ, std::max(s.Llo[2], s.Lhi[2]) + FDTD_R) + 12;
        bool big = (size_t)s.S * s.esz > ((size_t)1 << 26) || walk * s.S * s.esz >= ((size_t)1 << 31);
        for (int d = 0; d < 3; ++d) big = big || 2 * s.psi_elems[d] * 4 > ((size_t)1 << 31) - 4096;
        if (big) {
            delete ctx;
            fprintf(stderr, "fdtd_create: shot %d: a field plane above 64 MiB or 2 GiB / (z walk + 12 planes), "
                            "or a layer array above 1 GiB\n", i);
            return FDTD_EINVAL;
        }
        if (s.gy || s.gz) {
            if (ghost_s && ghost_s != s.s) {
                delete ctx;
                return FDTD_EINVAL;
            }
            ghost_s = s.s;
        }
        ctx->shots.push_back(s);
    }
    ctx->storage = shots[0].storage;
    // the automatic variant of a lone small shot is the naive kernel: below about
    // 150^3 points the z-march has too few tiles to fill the chip and the band
    // kernel's share is large (measured with graph steps: 64^3 14.0 k vs 4.5 k
    // Mpts/s, 128^3 38.2 k vs 30.4 k; 160^3 48.3 k vs 50.1 k).  Shots of a
    // batch share the grouped z-march and band launches and stay on the z-march.
    if (nshots == 1 && shots[0].variant == FDTD_VARIANT_AUTO) {
        ShotH &s0 = ctx->shots[0];
        if ((long)s0.nx * s0.ny * s0.nz < kSmallShot) s0.variant = FDTD_VARIANT_NAIVE;
    }
    // a batch whose single-shot plans would together hold more z-march
    // workgroups than there are CUs runs many small ones instead (64 x 8 tiles,
    // 64-plane chunks), balanced by their number: measured on 24 shots of
    // 96..288 points per axis, 110.2 k against 98.8 k Mpts/s (the autotuner
    // starts from here)
    if (nshots > 1) {
        long W = 0;
        for (const auto &sh : ctx->shots)
            if (sh.variant == FDTD_VARIANT_ZMARCH) W += (long)shot_tiles(sh, 0, sh.ry, sh.zchunk, sh.zcols).size();
        if (W > kCUs)
            for (auto &sh : ctx->shots) {
                sh.ry = 1;
                sh.zchunk = 64;
                sh.zcols = 1;
            }
    }
    for (auto &sh : ctx->shots)
        if (sh.tb_bufs && nshots != 1) {
            delete ctx;
            fprintf(stderr, "fdtd_create: temporal blocking needs a single-shot context\n");
            return FDTD_EINVAL;
        }
    // Band-kernel tile height: a lone large shot takes tiles of BAND_TY_TALL rows
    // (fewer, taller workgroups beside the z-march: the 512^3 step 0.715 ->
    // 0.695 ms), batches and small shots the shorter ones (their many small
    // boxes need the workgroups: the 24-shot batch is 18 % slower with tall tiles).
    ctx->band_ty = BAND_TY;
    if (nshots == 1 && (long)ctx->shots[0].nx * ctx->shots[0].ny * ctx->shots[0].nz >= (1L << 27))
        ctx->band_ty = BAND_TY_TALL;
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    ctx->o_stepc = take(256);
    ctx->o_scratch = take(256);
    ctx->o_desc = take(sizeof(DevShot) * nshots);
    size_t cap_all = 0;
    for (auto &s : ctx->shots) cap_all += work_capacity(s) + 8;
    ctx->o_work_all = take(sizeof(WorkItem) * cap_all);
    size_t band_all = 0;
    for (auto &s : ctx->shots) band_all += band_capacity(s);
    ctx->o_band_all = take(sizeof(BandItem) * band_all);
    for (auto &s : ctx->shots) {
        s.o_u[0] = take(s.elems * s.esz);
        s.o_u[1] = take(s.elems * s.esz);
        if (s.tb_bufs) {
            s.o_u[2] = take(s.elems * s.esz);
            s.o_u[3] = take(s.elems * s.esz);
            s.o_tbwork = take(sizeof(WorkItem) * tblock_capacity(s));
            s.o_reczs = take(sizeof(int) * (size_t)(s.nz + 1));
            s.o_recix = take(sizeof(int) * (size_t)kMaxRec);
        }
        s.o_d = s.esz == 2 ? take(s.elems * s.esz) : 0;   // 16-bit: increment field
        s.o_m = take(s.elems * 4);
        for (int d = 0; d < 3; ++d) {
            s.o_psi[d] = take(s.psi_elems[d] * 4);
            s.o_zeta[d] = take(s.psi_elems[d] * 4);
        }
        s.o_prof = take((size_t)3 * 4 * s.nmax * 4);
        s.o_work = take(sizeof(WorkItem) * work_capacity(s));
        s.o_band = take(sizeof(BandItem) * band_capacity(s));
        s.xbuf_bytes = xbuf_bytes(s);
        s.o_xbuf = take(s.xbuf_bytes);
        for (int p = 0; p < 2; ++p)
            for (int ph = 0; ph < 4; ++ph) s.o_jobs[p][ph] = take(sizeof(CopyJob) * 16);
    }
    ctx->need = off;
    ctx->hdesc.resize(nshots);
    *out = ctx;
    return FDTD_OK;
}

int fdtd_workspace_size(const fdtd_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return FDTD_EINVAL;
    *bytes = ctx->need;
    return FDTD_OK;
}

static int write_work_lists(fdtd_ctx *ctx) {
    std::map<std::array<int, 3>, std::vector<WorkItem>> byplan;
    std::vector<BandItem> band_all;
    for (size_t i = 0; i < ctx->shots.size(); ++i) {
        ShotH &s = ctx->shots[i];
        {
            std::vector<BandItem> bt = band_tiles(s, (int)i, ctx->band_ty);
            std::vector<BandItem> bw = xcd_order(bt);
            if (bw.size() > band_capacity(s)) FAIL(ctx, FDTD_EINVAL, "band list overflow");
            s.nband = (int)bw.size();
            if (!bw.empty())
                HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_band), bw.data(), sizeof(BandItem) * bw.size(),
                                           hipMemcpyHostToDevice, ctx->stream));
            if (s.variant != FDTD_VARIANT_NAIVE) band_all.insert(band_all.end(), bt.begin(), bt.end());
        }
        std::vector<WorkItem> sp = shot_tiles(s, (int)i, s.ry, s.zchunk, s.zcols);
        std::vector<WorkItem> w = xcd_order(sp);
        if (w.size() > work_capacity(s)) FAIL(ctx, FDTD_EINVAL, "work list overflow");
        s.nwork = (int)w.size();
        HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_work), w.data(), sizeof(WorkItem) * w.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (s.variant != FDTD_VARIANT_NAIVE) {
            auto &v = byplan[std::array<int, 3>{s.ry, s.zchunk, s.zcols}];
            v.insert(v.end(), sp.begin(), sp.end());
        }
        s.ntbwork = 0;
        if (s.tb_bufs) {
            std::vector<WorkItem> tb = tblock_tiles(s, (int)i);
            if (!tb.empty()) {
                std::vector<WorkItem> tw = xcd_order(tb);
                if (tw.size() > tblock_capacity(s)) FAIL(ctx, FDTD_EINVAL, "tile list overflow");
                s.ntbwork = (int)tw.size();
                HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_tbwork), tw.data(), sizeof(WorkItem) * tw.size(),
                                           hipMemcpyHostToDevice, ctx->stream));
                HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            }
        }
    }
    ctx->groups.clear();
    std::vector<WorkItem> all;
    for (auto &kv : byplan) {
        std::vector<WorkItem> wa = xcd_order(kv.second);
        fdtd_ctx::Group g{kv.first[0], kv.first[1], kv.first[2], all.size(), (int)wa.size()};
        ctx->groups.push_back(g);
        all.insert(all.end(), wa.begin(), wa.end());
    }
    ctx->nwork_all = (int)all.size();
    {
        std::vector<BandItem> bw = xcd_order(band_all);
        ctx->nband_all = (int)bw.size();
        if (!bw.empty())
            HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, ctx->o_band_all), bw.data(), sizeof(BandItem) * bw.size(),
                                       hipMemcpyHostToDevice, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (!all.empty()) {
        HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, ctx->o_work_all), all.data(), sizeof(WorkItem) * all.size(),
                                   hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return FDTD_OK;
}

static int zero_state(fdtd_ctx *ctx) {
    for (auto &s : ctx->shots) {
        fdtd_launch_fill_zero(wsp(ctx, s.o_u[0]), align256(s.elems * s.esz), ctx->stream);
        fdtd_launch_fill_zero(wsp(ctx, s.o_u[1]), align256(s.elems * s.esz), ctx->stream);
        if (s.esz == 2) fdtd_launch_fill_zero(wsp(ctx, s.o_d), align256(s.elems * s.esz), ctx->stream);
        if (s.tb_bufs)
            for (int b = 2; b < 4; ++b) fdtd_launch_fill_zero(wsp(ctx, s.o_u[b]), align256(s.elems * s.esz), ctx->stream);
        for (int d = 0; d < 3; ++d) {
            fdtd_launch_fill_zero(wsp(ctx, s.o_psi[d]), align256(s.psi_elems[d] * 4), ctx->stream);
            fdtd_launch_fill_zero(wsp(ctx, s.o_zeta[d]), align256(s.psi_elems[d] * 4), ctx->stream);
        }
    }
    fdtd_launch_set_int((int *)wsp(ctx, ctx->o_stepc), 0, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    ctx->iu = 0;
    ctx->ium1 = 1;
    ctx->step = 0;
    return FDTD_OK;
}

int fdtd_bind_workspace(fdtd_ctx *ctx, void *dev_ptr, size_t bytes) {
    if (!ctx || !dev_ptr) return FDTD_EINVAL;
    if (!ctx->side && !ctx->single_stream) {
        HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    }
    if (bytes < ctx->need) FAIL(ctx, FDTD_ENOMEM, "workspace of %zu bytes, need %zu", bytes, ctx->need);
    if (((uintptr_t)dev_ptr) & 255) FAIL(ctx, FDTD_EINVAL, "workspace must be 256-byte aligned");
    ctx->ws = (char *)dev_ptr;
    ctx->ws_bytes = bytes;
    fdtd_clear_graphs(ctx);
    // m and profiles start at zero too (frame of m must stay zero)
    for (auto &s : ctx->shots) {
        fdtd_launch_fill_zero(wsp(ctx, s.o_m), align256(s.elems * 4), ctx->stream);
        fdtd_launch_fill_zero(wsp(ctx, s.o_prof), align256((size_t)3 * 4 * s.nmax * 4), ctx->stream);
    }
    int rc = zero_state(ctx);
    if (rc) return rc;
    rc = write_work_lists(ctx);
    if (rc) return rc;
    for (size_t i = 0; i < ctx->shots.size(); ++i) {
        ShotH &s = ctx->shots[i];
        std::vector<CopyJob> jobs[2][4];
        long maxe[2][4];
        build_jobs(ctx, (int)i, jobs, maxe);
        for (int p = 0; p < 2; ++p)
            for (int ph = 0; ph < 4; ++ph) {
                if (jobs[p][ph].size() > 16) FAIL(ctx, FDTD_EINVAL, "too many exchange jobs");
                s.njobs[p][ph] = (int)jobs[p][ph].size();
                s.jobmax[p][ph] = maxe[p][ph];
                if (!jobs[p][ph].empty())
                    HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_jobs[p][ph]), jobs[p][ph].data(),
                                               sizeof(CopyJob) * jobs[p][ph].size(), hipMemcpyHostToDevice,
                                               ctx->stream));
            }
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return upload_desc(ctx);
}

int fdtd_set_velocity(fdtd_ctx *ctx, int32_t shot, const float *v_dev) {
    if (!ctx || !v_dev || shot < 0 || shot >= (int)ctx->shots.size()) return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "bind a workspace first");
    ShotH &s = ctx->shots[shot];
    unsigned int *scr = (unsigned int *)wsp(ctx, ctx->o_scratch);
    fdtd_launch_set_int((int *)scr, 0, ctx->stream);
    fdtd_launch_set_int((int *)(scr + 1), 0, ctx->stream);
    fdtd_launch_vel_to_m(v_dev, m_origin(ctx, s), s.nx, s.ny, s.nz, s.P, s.S, s.c.dt * s.c.dt, scr, scr + 1,
                         ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    unsigned int hv[2];
    HIPCHK(ctx, hipMemcpyAsync(hv, scr, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (hv[1]) FAIL(ctx, FDTD_EINVAL, "velocity must be finite and > 0");
    float vmax;
    memcpy(&vmax, &hv[0], 4);
    s.vmax = vmax;
    double lim = 0;
    for (int d = 0; d < 3; ++d) lim += d2_symbol_max() / (s.c.h[d] * s.c.h[d]);
    const double cfl = s.vmax * s.c.dt * std::sqrt(lim);
    if (cfl > 2.0) FAIL(ctx, FDTD_EUNSTABLE, "vmax dt sqrt(sum 6.50159/h^2) = %.6f > 2", cfl);
    s.vref = s.c.v_ref > 0 ? s.c.v_ref : s.vmax;
    std::vector<double> b(s.nmax), a(s.nmax), ki(s.nmax), dk(s.nmax);
    std::vector<float> prof((size_t)3 * 4 * s.nmax, 0.0f);
    for (int d = 0; d < 3; ++d) {
        layer_profile(s, d, s.vref, b.data(), a.data(), ki.data(), dk.data());
        int n = d == 0 ? s.nx : (d == 1 ? s.ny : s.nz);
        for (int i = 0; i < n; ++i) {
            prof[(size_t)(d * 4 + 0) * s.nmax + i] = (float)b[i];
            prof[(size_t)(d * 4 + 1) * s.nmax + i] = (float)a[i];
            prof[(size_t)(d * 4 + 2) * s.nmax + i] = (float)ki[i];
            prof[(size_t)(d * 4 + 3) * s.nmax + i] = (float)dk[i];
        }
    }
    HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_prof), prof.data(), prof.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (s.gy || s.gz) {
        // m is static: give the ghost rows/planes the opposite face's values once
        // (two phases, y then z spanning the y ghosts, so corners are filled too)
        float *mo = m_origin(ctx, s);
        std::vector<CopyJob> jy, jz;
        const int g = s.g;
        if (s.gy) {
            jy.push_back(CopyJob{mo, mo + (long)s.ny * s.P, 4, s.nx, g, s.nz, (long)s.P, (long)s.S, (long)s.P, (long)s.S,
                                 0});
            jy.push_back(CopyJob{mo + (long)(s.ny - g) * s.P, mo - (long)g * s.P, 4, s.nx, g, s.nz, (long)s.P, (long)s.S,
                                 (long)s.P, (long)s.S, 0});
        }
        if (s.gz) {
            const int dy = s.gy ? g : 0, Ny = s.ny + 2 * dy;
            float *b = mo - (long)dy * s.P;
            jz.push_back(CopyJob{b, b + (long)s.nz * s.S, 4, s.nx, Ny, g, (long)s.P, (long)s.S, (long)s.P, (long)s.S,
                                 0});
            jz.push_back(CopyJob{b + (long)(s.nz - g) * s.S, b - (long)g * s.S, 4, s.nx, Ny, g, (long)s.P, (long)s.S,
                                 (long)s.P, (long)s.S, 0});
        }
        for (auto *jobs : {&jy, &jz}) {
            if (jobs->empty()) continue;
            long mx = 0;
            for (auto &j : *jobs) {
                set_copy_vec(j);
                mx = std::max(mx, (long)j.ey * j.ez);
            }
            HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_jobs[0][0]), jobs->data(), sizeof(CopyJob) * jobs->size(),
                                       hipMemcpyHostToDevice, ctx->stream));
            fdtd_launch_copy_jobs(wsp(ctx, s.o_jobs[0][0]), (int)jobs->size(), mx, ctx->stream);
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        }
        // restore the exchange table that slot held
        std::vector<CopyJob> jobs[2][4];
        long maxe[2][4];
        build_jobs(ctx, shot, jobs, maxe);
        if (!jobs[0][0].empty())
            HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_jobs[0][0]), jobs[0][0].data(), sizeof(CopyJob) * jobs[0][0].size(),
                                       hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    s.vel_set = true;
    if (s.c.storage == FDTD_F32) s.scale = 1.0;
    else if (s.c.field_scale > 0) s.scale = s.c.field_scale;
    return upload_desc(ctx);
}

int fdtd_inject_source(fdtd_ctx *ctx, int32_t shot, int32_t i, int32_t j, int32_t k, const float *wavelet_dev,
                       int32_t nt, float amplitude) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size()) return FDTD_EINVAL;
    ShotH &s = ctx->shots[shot];
    if (!wavelet_dev || nt <= 0) FAIL(ctx, FDTD_EINVAL, "wavelet missing");
    if (i < 0 || i >= s.nx || j < 0 || j >= s.ny || k < 0 || k >= s.nz)
        FAIL(ctx, FDTD_EINVAL, "source (%d,%d,%d) outside the grid", i, j, k);
    if (s.c.storage != FDTD_F32 && s.c.field_scale == 0) {
        if (!s.vel_set) FAIL(ctx, FDTD_ESTATE, "16-bit storage: set the velocity before the source");
        std::vector<float> w(nt);
        HIPCHK(ctx, hipMemcpyAsync(w.data(), wavelet_dev, (size_t)nt * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        double wmax = 0;
        for (float x : w) wmax = std::max(wmax, (double)std::fabs(x));
        double inj = s.vmax * s.vmax * s.c.dt * s.c.dt * std::fabs((double)amplitude) * wmax /
                     (s.c.h[0] * s.c.h[1] * s.c.h[2]);
        double sc = inj > 0 ? std::exp2(std::round(std::log2(128.0 / inj))) : 1.0;
        s.scale = std::min(std::max(sc, std::exp2(-40.0)), std::exp2(40.0));
    }
    s.has_src = true;
    s.wav = wavelet_dev;
    s.src_nt = nt;
    s.amp = amplitude;
    s.sx = i;
    s.sy = j;
    s.sz = k;
    return upload_desc(ctx);
}

int fdtd_set_receivers(fdtd_ctx *ctx, int32_t shot, const int32_t *ijk_dev, int32_t nrec) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size() || nrec < 0) return FDTD_EINVAL;
    ShotH &s = ctx->shots[shot];
    if (nrec > 0) {
        if (!ijk_dev) return FDTD_EINVAL;
        std::vector<int32_t> h((size_t)nrec * 3);
        HIPCHK(ctx, hipMemcpyAsync(h.data(), ijk_dev, h.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int r = 0; r < nrec; ++r) {
            int i = h[3 * r], j = h[3 * r + 1], k = h[3 * r + 2];
            if (i < 0 || i >= s.nx || j < 0 || j >= s.ny || k < 0 || k >= s.nz)
                FAIL(ctx, FDTD_EINVAL, "receiver %d at (%d,%d,%d) outside the grid", r, i, j, k);
        }
    }
    s.rec = nrec > 0 ? ijk_dev : nullptr;
    s.nrec = nrec;
    if (s.tb_bufs && ctx->ws) {
        // receivers sorted by z for the temporal-blocking kernel
        if (nrec > kMaxRec) FAIL(ctx, FDTD_EINVAL, "at most %d receivers with temporal blocking", kMaxRec);
        std::vector<int32_t> h((size_t)nrec * 3);
        if (nrec > 0) {
            HIPCHK(ctx, hipMemcpyAsync(h.data(), ijk_dev, h.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        }
        std::vector<int> zs(s.nz + 1, 0), ix(std::max(nrec, 1));
        for (int r = 0; r < nrec; ++r) zs[h[3 * r + 2] + 1]++;
        for (int z = 0; z < s.nz; ++z) zs[z + 1] += zs[z];
        std::vector<int> fill(zs.begin(), zs.end() - 1);
        for (int r = 0; r < nrec; ++r) ix[fill[h[3 * r + 2]]++] = r;
        HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_reczs), zs.data(), zs.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(wsp(ctx, s.o_recix), ix.data(), ix.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    fdtd_clear_graphs(ctx);
    return upload_desc(ctx);
}

int fdtd_record_receivers(fdtd_ctx *ctx, int32_t shot, float *traces_dev, int32_t nt_capacity) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size()) return FDTD_EINVAL;
    ShotH &s = ctx->shots[shot];
    if (traces_dev && nt_capacity <= 0) return FDTD_EINVAL;
    s.traces = traces_dev;
    s.cap = traces_dev ? nt_capacity : 0;
    fdtd_clear_graphs(ctx);
    return upload_desc(ctx);
}

int fdtd_step(fdtd_ctx *ctx, int32_t nsteps) {
    if (!ctx || nsteps < 0) return FDTD_EINVAL;
    int rc = ready(ctx);
    if (rc) return rc;
    int done = 0, scans = 0;
    while (done < nsteps) {
        const int chunk = std::min(nsteps - done, 256);
        scans += enqueue_steps(ctx, chunk);
        done += chunk;
        if (ctx->timing && ctx->ev_used > 2000) {
            rc = drain_timing(ctx);
            if (rc) return rc;
        }
    }
    HIPCHK(ctx, hipGetLastError());
    return scans > 0 ? sentinel_check(ctx) : FDTD_OK;
}

int fdtd_set_sentinel(fdtd_ctx *ctx, int32_t every) {
    if (!ctx || every < 0) return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    ctx->sentinel_every = every;
    fdtd_launch_set_int((int *)wsp(ctx, ctx->o_scratch) + 3, 0, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return FDTD_OK;
}

int fdtd_set_timing(fdtd_ctx *ctx, int32_t enable) {
    if (!ctx) return FDTD_EINVAL;
    if (ctx->timing) {
        int rc = drain_timing(ctx);
        if (rc) return rc;
    }
    ctx->timing = enable != 0;
    for (int c = 0; c < kTimingClasses; ++c) {
        ctx->t_sum[c] = 0;
        ctx->t_cnt[c] = 0;
        ctx->ev_pairs[c].clear();
    }
    ctx->ev_used = 0;
    return FDTD_OK;
}

int fdtd_get_timing(fdtd_ctx *ctx, int32_t cls, double *mean_ms, int64_t *count) {
    if (!ctx || cls < 0 || cls >= kTimingClasses || !mean_ms || !count) return FDTD_EINVAL;
    int rc = drain_timing(ctx);
    if (rc) return rc;
    *count = ctx->t_cnt[cls];
    *mean_ms = ctx->t_cnt[cls] ? ctx->t_sum[cls] / ctx->t_cnt[cls] : 0.0;
    return FDTD_OK;
}

int fdtd_step_graph(fdtd_ctx *ctx, int32_t nsteps) {
    if (!ctx || nsteps < 0) return FDTD_EINVAL;
    int rc = ready(ctx);
    if (rc) return rc;
    if (ctx->timing) FAIL(ctx, FDTD_EUNSUPPORTED, "per-kernel timing needs eager stepping");
    if (nsteps == 0) return FDTD_OK;
    long period = 2;
    for (auto &s : ctx->shots) {
        period = std::max(period, (long)s.s * 2);
        if (s.ck_every > 0 && ctx->saving) period = std::max(period, (long)s.ck_every * 2);
    }
    // a graph embeds the checkpoint schedule only for its own start step
    bool ck = false;
    for (auto &s : ctx->shots) ck = ck || (s.ck_every > 0 && ctx->saving);
    if (tblock_active(ctx)) period = std::max(period, (long)ctx->shots[0].tk * 4);
    long phase = ck ? ctx->step : ctx->step % period;
    std::pair<long, long> key(nsteps, phase * 16 + ctx->iu * 4 + ctx->ium1);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        long step0 = ctx->step;
        int iu0 = ctx->iu, ium10 = ctx->ium1;
        // capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph is launched on the caller's
        if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t user = ctx->stream;
        ctx->stream = ctx->cap_stream;
        hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            ctx->stream = user;
            (void)hipGetLastError();
            FAIL(ctx, FDTD_EHIP, "graph capture: %s", hipGetErrorString(e));
        }
        const int sentinel = ctx->sentinel_every;
        ctx->sentinel_every = 0;   // graphs hold no scans: one scan follows each graph launch
        enqueue_steps(ctx, nsteps);
        ctx->sentinel_every = sentinel;
        const int end_iu = ctx->iu, end_ium1 = ctx->ium1;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->stream, &g);
        ctx->stream = user;
        ctx->step = step0;
        ctx->iu = iu0;
        ctx->ium1 = ium10;
        if (e != hipSuccess || !g) {
            (void)hipGetLastError();
            FAIL(ctx, FDTD_EHIP, "graph capture: %s", hipGetErrorString(e));
        }
        hipGraphExec_t ge;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) FAIL(ctx, FDTD_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        it = ctx->graphs.emplace(key, fdtd_ctx::GraphEntry{ge, end_iu, end_ium1}).first;
    }
    HIPCHK(ctx, hipGraphLaunch(it->second.exec, ctx->stream));
    ctx->step += nsteps;
    ctx->iu = it->second.end_iu;
    ctx->ium1 = it->second.end_ium1;
    if (ctx->sentinel_every > 0) {
        enqueue_sentinel(ctx);
        return sentinel_check(ctx);
    }
    return FDTD_OK;
}

int fdtd_get_field(fdtd_ctx *ctx, int32_t shot, int32_t which, float *dst_dev) {
    if (!ctx || !dst_dev || shot < 0 || shot >= (int)ctx->shots.size() || which < 0 || which > 1)
        return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    ShotH &s = ctx->shots[shot];
    if (which == 1 && s.esz == 2) {
        // 16-bit state holds d^n = u^n - u^{n-1}
        fdtd_launch_get_prev(ctx->storage, field_origin(ctx, s, s.o_u[ctx->iu]), field_origin(ctx, s, s.o_d),
                             dst_dev, s.nx, s.ny, s.nz, s.P, s.S, (float)(1.0 / s.scale), ctx->stream);
        HIPCHK(ctx, hipGetLastError());
        return FDTD_OK;
    }
    const void *u = field_origin(ctx, s, s.o_u[which ? ctx->ium1 : ctx->iu]);
    fdtd_launch_get_field(ctx->storage, u, dst_dev, s.nx, s.ny, s.nz, s.P, s.S, (float)(1.0 / s.scale), ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return FDTD_OK;
}

int fdtd_set_field(fdtd_ctx *ctx, int32_t shot, int32_t which, const float *src_dev) {
    if (!ctx || !src_dev || shot < 0 || shot >= (int)ctx->shots.size() || which < 0 || which > 1)
        return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    ShotH &s = ctx->shots[shot];
    if (which == 1 && s.esz == 2) {
        fdtd_launch_set_prev(ctx->storage, field_origin(ctx, s, s.o_u[ctx->iu]), field_origin(ctx, s, s.o_d),
                             src_dev, s.nx, s.ny, s.nz, s.P, s.S, (float)s.scale, ctx->stream);
        HIPCHK(ctx, hipGetLastError());
        return FDTD_OK;
    }
    void *u = field_origin(ctx, s, s.o_u[which ? ctx->ium1 : ctx->iu]);
    fdtd_launch_set_field(ctx->storage, u, src_dev, s.nx, s.ny, s.nz, s.P, s.S, (float)s.scale, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return FDTD_OK;
}

int fdtd_reset(fdtd_ctx *ctx) {
    if (!ctx) return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    fdtd_launch_set_int((int *)wsp(ctx, ctx->o_scratch) + 3, 0, ctx->stream);   // sentinel flag
    return zero_state(ctx);
}

int fdtd_get_step(const fdtd_ctx *ctx, int64_t *step) {
    if (!ctx || !step) return FDTD_EINVAL;
    *step = ctx->step;
    return FDTD_OK;
}

int fdtd_check_finite(fdtd_ctx *ctx) {
    if (!ctx) return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    unsigned int *scr = (unsigned int *)wsp(ctx, ctx->o_scratch);
    fdtd_launch_set_int((int *)(scr + 2), 0, ctx->stream);
    for (auto &s : ctx->shots)
        for (int k = 0; k < 2; ++k)
            fdtd_launch_finite(ctx->storage, field_origin(ctx, s, s.o_u[k]), s.nx, s.ny, s.nz, s.P, s.S, scr + 2,
                               ctx->stream);
    unsigned int bad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&bad, scr + 2, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad) FAIL(ctx, FDTD_ENONFINITE, "non-finite value in a wavefield");
    return FDTD_OK;
}

int fdtd_set_plan(fdtd_ctx *ctx, int32_t shot, int32_t variant, int32_t tile_ry, int32_t zchunk, int32_t tblock_k,
                  int32_t tile_cols) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size()) return FDTD_EINVAL;
    if (variant < 1 || variant > 3) FAIL(ctx, FDTD_EINVAL, "variant must be naive, z-march or temporal blocking");
    if (tile_ry != 1 && tile_ry != 2 && tile_ry != 4 && tile_ry != 8)
        FAIL(ctx, FDTD_EINVAL, "tile size must be 1, 2, 4 or 8 (64 x 8 tile_ry points)");
    if (zchunk < 16 || zchunk > 4096) FAIL(ctx, FDTD_EINVAL, "z chunk must be in [16, 4096]");
    if (tile_cols != 1 && tile_cols != 2) FAIL(ctx, FDTD_EINVAL, "tile_cols must be 1 or 2 (x points per lane)");
    if (tile_cols == 2 && tile_ry == 8) FAIL(ctx, FDTD_EINVAL, "two-column tiles are 128 x 8, 16 or 32 points");
    if (variant == FDTD_VARIANT_TBLOCK && tblock_k != 2 && tblock_k != 4) FAIL(ctx, FDTD_EINVAL, "tblock_k must be 2 or 4");
    ShotH &s = ctx->shots[shot];
    if (variant == FDTD_VARIANT_TBLOCK && !s.tb_bufs)
        FAIL(ctx, FDTD_EINVAL, "create the shot with the temporal-blocking variant to switch to it");
    s.variant = variant;
    s.ry = tile_ry;
    s.zchunk = zchunk;
    s.zcols = tile_cols;
    s.tk = variant == FDTD_VARIANT_TBLOCK ? tblock_k : 1;
    fdtd_clear_graphs(ctx);
    if (!ctx->ws) return FDTD_OK;
    const int rc = write_work_lists(ctx);
    if (rc) return rc;
    // the variant decides whether the band kernel advances psi_x and psi_z itself
    // (DevShot::fused), which the kernels read from the descriptor
    return upload_desc(ctx);
}

int fdtd_get_plan(const fdtd_ctx *ctx, int32_t shot, int32_t *variant, int32_t *tile_ry, int32_t *tblock_k,
                  int32_t *tile_cols) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size()) return FDTD_EINVAL;
    const ShotH &s = ctx->shots[shot];
    if (variant) *variant = s.variant;
    if (tile_ry) *tile_ry = s.ry;
    if (tile_cols) *tile_cols = s.zcols;
    if (tblock_k) *tblock_k = s.variant == FDTD_VARIANT_TBLOCK ? s.tk : 1;
    return FDTD_OK;
}

int fdtd_get_scale(const fdtd_ctx *ctx, int32_t shot, double *scale) {
    if (!ctx || !scale || shot < 0 || shot >= (int)ctx->shots.size()) return FDTD_EINVAL;
    *scale = ctx->shots[shot].scale;
    return FDTD_OK;
}

// saved-state blob: a header (256-byte aligned), then each shot's state in the checkpoint layout
struct StateHeader {
    char magic[8];       // "FDTDSTAT"
    int64_t step;
    int32_t nshots, storage;
    uint64_t shot_bytes[FDTD_MAXSHOTS];   // fdtd_state_bytes of each shot (identifies the layout)
};
static_assert(sizeof(StateHeader) <= 8 + 8 + 8 + 8 * FDTD_MAXSHOTS, "header layout");
static size_t state_blob_bytes(const fdtd_ctx *ctx) {
    size_t b = align256(sizeof(StateHeader));
    for (const ShotH &s : ctx->shots) b += fdtd_state_bytes(s);
    return b;
}

int fdtd_state_size(const fdtd_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return FDTD_EINVAL;
    *bytes = state_blob_bytes(ctx);
    return FDTD_OK;
}

int fdtd_save_state(fdtd_ctx *ctx, void *dst_dev, size_t bytes) {
    if (!ctx || !dst_dev) return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    if (bytes < state_blob_bytes(ctx)) FAIL(ctx, FDTD_ENOMEM, "state buffer of %zu bytes, need %zu", bytes,
                                            state_blob_bytes(ctx));
    StateHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, "FDTDSTAT", 8);
    h.step = ctx->step;
    h.nshots = (int32_t)ctx->shots.size();
    h.storage = ctx->storage;
    for (size_t i = 0; i < ctx->shots.size(); ++i) h.shot_bytes[i] = fdtd_state_bytes(ctx->shots[i]);
    static_assert(sizeof(StateHeader) <= sizeof(ctx->state_hdr), "header fits");
    memcpy(ctx->state_hdr, &h, sizeof h);   // kept in the context until the copy has run
    char *dst = (char *)dst_dev;
    HIPCHK(ctx, hipMemcpyAsync(dst, ctx->state_hdr, sizeof h, hipMemcpyHostToDevice, ctx->stream));
    size_t off = align256(sizeof(StateHeader));
    for (size_t i = 0; i < ctx->shots.size(); ++i) {
        copy_state(ctx, (int)i, dst + off, true);
        off += fdtd_state_bytes(ctx->shots[i]);
    }
    HIPCHK(ctx, hipGetLastError());
    return FDTD_OK;
}

int fdtd_load_state(fdtd_ctx *ctx, const void *src_dev, size_t bytes) {
    if (!ctx || !src_dev) return FDTD_EINVAL;
    if (!ctx->ws) FAIL(ctx, FDTD_ESTATE, "no workspace bound");
    if (bytes < state_blob_bytes(ctx)) FAIL(ctx, FDTD_EINVAL, "state buffer of %zu bytes, need %zu", bytes,
                                            state_blob_bytes(ctx));
    StateHeader h;
    HIPCHK(ctx, hipMemcpyAsync(&h, src_dev, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (memcmp(h.magic, "FDTDSTAT", 8) != 0) FAIL(ctx, FDTD_EINVAL, "not a saved state");
    if (h.nshots != (int32_t)ctx->shots.size() || h.storage != ctx->storage || h.step < 0)
        FAIL(ctx, FDTD_EINVAL, "saved state is of another context configuration");
    for (size_t i = 0; i < ctx->shots.size(); ++i)
        if (h.shot_bytes[i] != fdtd_state_bytes(ctx->shots[i]))
            FAIL(ctx, FDTD_EINVAL, "saved state of shot %zu has another layout", i);
    const char *src = (const char *)src_dev;
    size_t off = align256(sizeof(StateHeader));
    for (size_t i = 0; i < ctx->shots.size(); ++i) {
        copy_state(ctx, (int)i, (char *)src + off, false);
        off += fdtd_state_bytes(ctx->shots[i]);
    }
    ctx->step = h.step;
    fdtd_launch_set_int((int *)wsp(ctx, ctx->o_stepc), (int)h.step, ctx->stream);
    fdtd_clear_graphs(ctx);
    HIPCHK(ctx, hipGetLastError());
    return FDTD_OK;
}

int fdtd_stream_probe(const float *a_dev, const float *b_dev, const float *c_dev, float *o_dev, size_t n,
                      int32_t blocks, int32_t unroll, void *hip_stream) {
    if (!a_dev || !b_dev || !c_dev || !o_dev || n == 0 || (n & 3) || blocks < 0 || blocks > (1 << 20) ||
        n / 4 / 256 >= (1u << 31))
        return FDTD_EINVAL;
    if ((((uintptr_t)a_dev | (uintptr_t)b_dev | (uintptr_t)c_dev | (uintptr_t)o_dev) & 15) != 0) return FDTD_EINVAL;
    fdtd_launch_stream_probe(a_dev, b_dev, c_dev, o_dev, n / 4, blocks, unroll, (hipStream_t)hip_stream);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EHIP;
}

void fdtd_destroy(fdtd_ctx *ctx) {
    if (!ctx) return;
    fdtd_clear_graphs(ctx);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->adj_stream) (void)hipStreamDestroy(ctx->adj_stream);
    for (auto e : ctx->ev_adj)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// internal helpers used by the adjoint and autotuner translation units
// ---------------------------------------------------------------------------
char *fdtd_ws(fdtd_ctx *ctx, size_t off) { return wsp(ctx, off); }
void fdtd_enqueue_step_shot(fdtd_ctx *ctx, int shot) { enqueue_step(ctx, shot); }
void fdtd_restore_state(fdtd_ctx *ctx, int i, char *ck) { copy_state(ctx, i, ck, false); }
void *fdtd_field_origin(fdtd_ctx *ctx, const ShotH &s, size_t off) { return field_origin(ctx, s, off); }
float *fdtd_m_origin(fdtd_ctx *ctx, const ShotH &s) { return m_origin(ctx, s); }
int fdtd_rewrite_work(fdtd_ctx *ctx) { return write_work_lists(ctx); }
int fdtd_reupload(fdtd_ctx *ctx) { return upload_desc(ctx); }
int fdtd_ready(fdtd_ctx *ctx) { return ready(ctx); }
int fdtd_zero_state(fdtd_ctx *ctx) { return zero_state(ctx); }
void fdtd_set_copy_vec(CopyJob &j) { set_copy_vec(j); }
