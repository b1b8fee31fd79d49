// adjoint.hip -- reverse-time adjoint of the step and the velocity gradient (gfx950).
//
// The forward step is linear in (u^n, u^{n-1}, psi, zeta); its exact
// transpose, written in the same leapfrog shape with lambda^{n+1} (adjoint of
// u^{n+1}) and lambda^{n+2}, is, with Lbar = m lambda^{n+1}:
//   zeta_b  <- b (zeta_b + Lbar)                  (slab)
//   E_d      = kinv Lbar + a (zeta_b + Lbar)      (slab; Lbar elsewhere)
//   psit     = psi_b - D1_d E_d ;  F_d = a psit ;  psi_b <- b psit   (slab)
//   lambda^n = 2 lambda^{n+1} - lambda^{n+2}
//            + sum_d [ D2_d(kinv E_d) - D1_d(dkinv E_d) - D1_d(F_d) ]
// (D2 symmetric, D1 antisymmetric; outside band d the axis term is D2_d Lbar).
// The residual at the receivers is added to lambda^{n+1} first.  The model
// enters only through m = v^2 dt^2 multiplying (Lt u^n + f^n) = (u^{n+1} - 2u^n
// + u^{n-1}) / m, so dJ/dv = (2/v) sum_n lambda^{n+1} (u^{n+1} - 2u^n + u^{n-1}),
// accumulated in FP64.  Forward levels are recomputed per segment from
// checkpoints saved every `every` steps.
#include "fdtd_host.hpp"
#include "fdtd_launch.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

struct AdjArgs {
    const DevShot *s;        // forward descriptor (geometry, m, profiles, coefficients)
    float *lam;              // lambda^{n+1}   (origin-adjusted, FP32, forward layout)
    float *lamp;             // lambda^{n+2} in, lambda^n out
    float *psib[3], *zetab[3];          // compact slab layouts (as psi)
    float *E[3];             // origin-adjusted FP32 fields (band points; zero elsewhere)
    float *F[3];             // origin-adjusted FP32 fields (slab points; zero elsewhere)
    const int *band[3];      // band coordinates per axis
    int nband[3];
    const void *um, *u0, *up;   // forward u^{n-1}, u^n, u^{n+1} (storage type)
    float *Lb;               // Lbar = m lambda^{n+1} at every grid point (origin-adjusted; zero in the frame)
    double *G;               // dense accumulator sum lambda * (u^{n+1} - 2u^n + u^{n-1})
};

__device__ __forceinline__ long fidx(const DevShot &s, int x, int y, int z) {
    return (long)z * s.S + (long)y * s.P + x;
}

// residual injection: one thread per distinct receiver location, adding the
// residuals of the receivers there in receiver order (repeated receivers add
// up, with the rounding of a serial pass over the receivers).  gstart[g] ..
// gstart[g + 1] index ridx, the receivers of location g.
__global__ __launch_bounds__(256) void k_adj_resid(float *lam, const DevShot *sp, const float *resid_row,
                                                   const int *gstart, const int *ridx, int ngroups) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    const DevShot &s = *sp;
    const int k0 = gstart[g], k1 = gstart[g + 1];
    const int32_t *q = s.rec + 3 * ridx[k0];
    float *l = lam + fidx(s, q[0], q[1], q[2]);
    float v = *l;
    for (int k = k0; k < k1; ++k) v += resid_row[ridx[k]];
    *l = v;
}

// Lbar = m lambda^{n+1} once per point, so that the passes below read it
// instead of forming it at every stencil tap (the same product, so the same bits)
__global__ __launch_bounds__(256) void k_adj_lbar(AdjArgs a) {
    const DevShot &s = *a.s;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= s.nx) return;
    const long i = fidx(s, x, (int)blockIdx.y, (int)blockIdx.z);
    a.Lb[i] = s.m[i] * a.lam[i];
}

// pass 1 on band points of axis d = blockIdx.y: E_d and the zeta adjoint
__global__ __launch_bounds__(256) void k_adj_p1(AdjArgs a) {
    const DevShot &s = *a.s;
    const int d = (int)blockIdx.y;
    const int nb = a.nband[d];
    if (nb == 0) return;
    const int n1 = d == 0 ? s.ny : s.nx;          // the two other axes, fastest first
    const int n2 = d == 2 ? s.ny : s.nz;
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = (long)nb * n1 * n2;
    if (t >= total) return;
    int x, y, z, c;
    if (d == 0) {
        c = a.band[0][t % nb];
        long r = t / nb;
        x = c;
        y = (int)(r % n1);
        z = (int)(r / n1);
    } else if (d == 1) {
        x = (int)(t % n1);
        long r = t / n1;
        c = a.band[1][r % nb];
        y = c;
        z = (int)(r / nb);
    } else {
        x = (int)(t % n1);
        long r = t / n1;
        y = (int)(r % n2);
        c = a.band[2][r / n2];
        z = c;
    }
    const long i = fidx(s, x, y, z);
    const float lb = a.Lb[i];
    const int n = coord_n(s, d);
    float e = lb;
    if (in_slab(c, n, s.Llo[d], s.Lhi[d])) {
        float *zb = &a.zetab[d][psi_index(s, d, x, y, z)];
        const float zt = *zb + lb;
        e = fmaf(prof_at(s, d, 2, c), lb, prof_at(s, d, 1, c) * zt);
        *zb = prof_at(s, d, 0, c) * zt;
    }
    a.E[d][i] = e;
}

// pass 2 on slab points of axis d = blockIdx.y: psi adjoint and F_d = a (psi_b - D1 E_d)
__global__ __launch_bounds__(256) void k_adj_p2(AdjArgs a) {
    const DevShot &s = *a.s;
    const int d = (int)blockIdx.y;
    const int lo = s.Llo[d], hi = s.Lhi[d];
    if (lo + hi == 0) return;
    long count;
    if (d == 0) count = (long)s.LX * s.ny * s.nz;
    else if (d == 1) count = (long)s.nx * s.LY * s.nz;
    else count = (long)s.nx * s.ny * s.LZ;
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int x, y, z, k;
    if (d == 0) {
        int is = (int)(t % s.LX);
        long r = t / s.LX;
        y = (int)(r % s.ny);
        z = (int)(r / s.ny);
        x = is < lo ? is : s.nx - hi + (is - lo);
        k = x;
    } else if (d == 1) {
        x = (int)(t % s.nx);
        long r = t / s.nx;
        int js = (int)(r % s.LY);
        z = (int)(r / s.LY);
        y = js < lo ? js : s.ny - hi + (js - lo);
        k = y;
    } else {
        x = (int)(t % s.nx);
        long r = t / s.nx;
        y = (int)(r % s.ny);
        int ks = (int)(r / s.ny);
        z = ks < lo ? ks : s.nz - hi + (ks - lo);
        k = z;
    }
    const long i = fidx(s, x, y, z);
    const long stride = d == 0 ? 1 : (d == 1 ? s.P : s.S);
    float el[4], eh[4];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
        el[l - 1] = a.E[d][i - l * stride];
        eh[l - 1] = a.E[d][i + l * stride];
    }
    const long pi = psi_index(s, d, x, y, z);
    const float pt = a.psib[d][pi] - d1_axis(s.w1[d], el, eh);
    a.F[d][i] = prof_at(s, d, 1, k) * pt;
    a.psib[d][pi] = prof_at(s, d, 0, k) * pt;
}

// Pass 3 on every point: lambda^n and the gradient accumulation.  Along an
// axis d whose band the wave does not touch, the axis term is D2_d Lbar.  A
// wave that touches it evaluates the band form for all its lanes:
//   D2_d(K) - D1_d(dkinv E_d) - D1_d(F_d),  K = kinv E_d in the band, Lbar outside,
// with dkinv E_d and F_d zero outside the slab and every field zero outside
// the grid.  At a lane outside the band this is D2_d Lbar with the same bits
// (kinv = 1 and E_d = Lbar in the band outside the slab; the D1 terms are
// exact zeros), so the per-lane branch is not needed.  A wave is one y row of
// 64 x points (blockDim = 64 x 4), so the y and z tests are wave-uniform and
// the x test is taken per 64-point tile.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_p3(AdjArgs a, float inv_scale) {
    const DevShot &s = *a.s;
    const int x0 = blockIdx.x * 64;
    const int x = x0 + threadIdx.x;
    const int y = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * 4 + threadIdx.y));
    const int z = blockIdx.z;
    if (x >= s.nx || y >= s.ny) return;
    const int xe = min(x0 + 64, s.nx) - 1;   // last x of the tile
    const long i = fidx(s, x, y, z);
    const int cc[3] = {x, y, z};
    const long st[3] = {1, (long)s.P, (long)s.S};
    // the band of an axis is an interval at each end of the grid, so a tile meets it iff one of its end points lies in it
    const bool touch[3] = {in_band(x0, s.nx, s.Llo[0], s.Lhi[0]) || in_band(xe, s.nx, s.Llo[0], s.Lhi[0]),
                           in_band(y, s.ny, s.Llo[1], s.Lhi[1]), in_band(z, s.nz, s.Llo[2], s.Lhi[2])};
    float acc = fmaf(2.0f, a.lam[i], -a.lamp[i]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int n = coord_n(s, d);
        const int c = cc[d];
        float t;
        if (!touch[d]) {
            float lo[4], hi[4];
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                lo[l - 1] = a.Lb[i - l * st[d]];
                hi[l - 1] = a.Lb[i + l * st[d]];
            }
            t = d2_axis(s.w2[d], a.Lb[i], lo, hi);
        } else {
            const int lo_ = s.Llo[d], hi_ = s.Lhi[d];
            const float *pk = s.prof + (d * 4 + 2) * s.nmax, *pdk = s.prof + (d * 4 + 3) * s.nmax;
            const float *E = a.E[d], *F = a.F[d];
            // one tap at coordinate cq along d, element j: K and dkinv E_d
            auto tap = [&](int cq, long j, float &kv, float &dv) {
                const float e = E[j], lb = a.Lb[j];
                const int cl = min(max(cq, 0), n - 1);
                const bool ing = cq >= 0 && cq < n;
                kv = ing && in_band(cq, n, lo_, hi_) ? pk[cl] * e : (ing ? lb : 0.0f);
                dv = ing && in_slab(cq, n, lo_, hi_) ? pdk[cl] * e : 0.0f;
            };
            float kl[4], kh[4], dl[4], dh[4], fl[4], fh[4], kc, dc;
            tap(c, i, kc, dc);
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                const long im = i - l * st[d], ip = i + l * st[d];
                tap(c - l, im, kl[l - 1], dl[l - 1]);
                tap(c + l, ip, kh[l - 1], dh[l - 1]);
                fl[l - 1] = F[im];
                fh[l - 1] = F[ip];
            }
            t = d2_axis(s.w2[d], kc, kl, kh) - d1_axis(s.w1[d], dl, dh) - d1_axis(s.w1[d], fl, fh);
        }
        acc = acc + t;
    }
    // gradient: lambda^{n+1} (u^{n+1} - 2 u^n + u^{n-1})
    const double d2u = ((double)Store<T>::ld((const T *)a.up + i) - 2.0 * (double)Store<T>::ld((const T *)a.u0 + i) +
                        (double)Store<T>::ld((const T *)a.um + i)) * (double)inv_scale;
    const long gi = ((long)z * s.ny + y) * s.nx + x;
    a.G[gi] += (double)a.lam[i] * d2u;
    a.lamp[i] = acc;
}

// dJ/dv = 2 G dt / sqrt(m)  (v = sqrt(m) / dt)
__global__ __launch_bounds__(256) void k_adj_finish(const DevShot *sp, double *G, double dt) {
    const DevShot &s = *sp;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= s.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const long gi = ((long)z * s.ny + y) * s.nx + x;
    G[gi] = 2.0 * G[gi] * dt / sqrt((double)s.m[fidx(s, x, y, z)]);
}

__global__ __launch_bounds__(256) void k_zero_f64(double *p, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

#define AFAIL(ctx, code, ...)                                                                                \
    do {                                                                                                      \
        char _b[512];                                                                                         \
        snprintf(_b, sizeof _b, __VA_ARGS__);                                                                 \
        (ctx)->err = _b;                                                                                      \
        return (code);                                                                                        \
    } while (0)
#define AHIP(ctx, expr)                                                                                       \
    do {                                                                                                      \
        hipError_t _e = (expr);                                                                               \
        if (_e != hipSuccess) AFAIL(ctx, FDTD_EHIP, "%s: %s", #expr, hipGetErrorString(_e));                  \
    } while (0)

namespace {
struct AdjLayout {
    size_t ck = 0, seg = 0, lam = 0, lamp = 0, psib[3] = {}, zetab[3] = {}, F[3] = {}, E[3] = {}, band[3] = {};
    size_t gstart = 0, ridx = 0;   // receivers grouped by location (k_adj_resid)
    size_t lb = 0;                 // Lbar field
    size_t total = 0;
    int nck = 0;
};

static std::vector<int> band_coords(const ShotH &s, int d) {
    const int n = d == 0 ? s.nx : (d == 1 ? s.ny : s.nz);
    const int lo = s.Llo[d], hi = s.Lhi[d];
    std::vector<int> v;
    for (int c = 0; c < n; ++c)
        if ((lo > 0 && c < lo + FDTD_R) || (hi > 0 && c >= n - hi - FDTD_R)) v.push_back(c);
    return v;
}

static AdjLayout adj_layout(const ShotH &s, int every, int nt) {
    AdjLayout L;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += a256(b);
        return o;
    };
    L.nck = (nt + every - 1) / every;
    L.ck = take(fdtd_state_bytes(s) * (size_t)L.nck);
    L.seg = take(a256(s.elems * s.esz) * (size_t)(every + 2));
    L.lam = take(s.elems * 4);
    L.lamp = take(s.elems * 4);
    for (int d = 0; d < 3; ++d) {
        L.psib[d] = take(s.psi_elems[d] * 4);
        L.zetab[d] = take(s.psi_elems[d] * 4);
        L.F[d] = take((s.Llo[d] + s.Lhi[d]) > 0 ? s.elems * 4 : 0);
        L.E[d] = take((s.Llo[d] + s.Lhi[d]) > 0 ? s.elems * 4 : 0);
        L.band[d] = take((size_t)s.nmax * 4);
    }
    L.lb = take(s.elems * 4);
    L.gstart = take((size_t)(s.nrec + 1) * 4);
    L.ridx = take((size_t)std::max(s.nrec, 1) * 4);
    L.total = off;
    return L;
}
}  // namespace

static char *origin4(const ShotH &s, char *base) { return base + origin_elems(s) * 4; }
static char *origin_t(const ShotH &s, char *base) { return base + origin_elems(s) * s.esz; }

template <typename T>
static void launch_p3(const AdjArgs &a, const ShotH &s, float inv, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_p3<T>, dim3((s.nx + 63) / 64, (s.ny + 3) / 4, s.nz), dim3(64, 4), 0, st, a, inv);
}

extern "C" {

int fdtd_adjoint_workspace_size(const fdtd_ctx *ctx, int32_t shot, int32_t every, int32_t nt, size_t *bytes) {
    if (!ctx || !bytes || shot < 0 || shot >= (int)ctx->shots.size() || every <= 0 || nt <= 0) return FDTD_EINVAL;
    *bytes = adj_layout(ctx->shots[shot], every, nt).total;
    return FDTD_OK;
}

int fdtd_set_checkpointing(fdtd_ctx *ctx, int32_t shot, int32_t every, void *buf_dev, size_t bytes) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size() || every < 0) return FDTD_EINVAL;
    ShotH &s = ctx->shots[shot];
    fdtd_clear_graphs(ctx);
    if (every == 0) {
        s.ck_every = 0;
        s.ck_buf = nullptr;
        s.ck_bytes = 0;
        s.ck_count = 0;
        s.ck_nt = 0;
        return FDTD_OK;
    }
    if (!buf_dev) return FDTD_EINVAL;
    if (s.gy || s.gz) AFAIL(ctx, FDTD_EUNSUPPORTED, "the adjoint supports Dirichlet faces only");
    if (s.esz != 4) AFAIL(ctx, FDTD_EUNSUPPORTED, "the adjoint runs on FP32 fields");
    if (((uintptr_t)buf_dev) & 255) AFAIL(ctx, FDTD_EINVAL, "adjoint buffer must be 256-byte aligned");
    // capacity: the largest nt this buffer holds checkpoints for
    int nck = 0;
    while (adj_layout(s, every, (nck + 1) * every).total <= bytes && nck < (1 << 20)) ++nck;
    if (nck == 0) AFAIL(ctx, FDTD_ENOMEM, "adjoint buffer too small");
    s.ck_every = every;
    s.ck_count = nck;
    s.ck_nt = nck * every;
    s.ck_buf = (char *)buf_dev;
    s.ck_bytes = bytes;
    return FDTD_OK;
}

int fdtd_adjoint(fdtd_ctx *ctx, int32_t shot, int32_t nt, const float *resid_dev, double *grad_v_dev) {
    if (!ctx || shot < 0 || shot >= (int)ctx->shots.size() || nt <= 0 || !resid_dev || !grad_v_dev)
        return FDTD_EINVAL;
    if (!ctx->ws) AFAIL(ctx, FDTD_ESTATE, "no workspace bound");
    ShotH &s = ctx->shots[shot];
    if (s.ck_every <= 0 || !s.ck_buf) AFAIL(ctx, FDTD_ESTATE, "checkpointing is not set for shot %d", shot);
    if (nt > s.ck_nt) AFAIL(ctx, FDTD_ENOMEM, "adjoint buffer holds checkpoints for %d steps, asked %d", s.ck_nt, nt);
    if (ctx->step < nt) AFAIL(ctx, FDTD_ESTATE, "run the forward for %d steps first (at step %ld)", nt, ctx->step);
    if (!s.vel_set) AFAIL(ctx, FDTD_ESTATE, "no velocity model");
    const int every = s.ck_every;
    AdjLayout L = adj_layout(s, every, nt);
    if (L.total > s.ck_bytes)
        AFAIL(ctx, FDTD_ENOMEM, "adjoint buffer of %zu bytes, %zu needed (receivers set after sizing it?)", s.ck_bytes,
              L.total);
    char *B = s.ck_buf;
    hipStream_t st = ctx->stream;
    DevShot *dd = (DevShot *)fdtd_ws(ctx, ctx->o_desc);
    const DevShot *sp = dd + shot;

    // recomputation must not overwrite the recorded traces
    DevShot saved = ctx->hdesc[shot];
    ctx->hdesc[shot].traces = nullptr;
    ctx->hdesc[shot].trace_cap = 0;
    AHIP(ctx, hipMemcpyAsync(dd + shot, &ctx->hdesc[shot], sizeof(DevShot), hipMemcpyHostToDevice, st));
    AHIP(ctx, hipStreamSynchronize(st));

    // adjoint state to zero; band coordinate lists
    fdtd_launch_fill_zero(B + L.lam, a256(s.elems * 4), st);
    fdtd_launch_fill_zero(B + L.lamp, a256(s.elems * 4), st);
    fdtd_launch_fill_zero(B + L.lb, a256(s.elems * 4), st);
    AdjArgs a;
    memset(&a, 0, sizeof a);
    a.s = sp;
    a.lam = (float *)origin4(s, B + L.lam);
    a.lamp = (float *)origin4(s, B + L.lamp);
    a.Lb = (float *)origin4(s, B + L.lb);
    for (int d = 0; d < 3; ++d) {
        fdtd_launch_fill_zero(B + L.psib[d], a256(s.psi_elems[d] * 4), st);
        fdtd_launch_fill_zero(B + L.zetab[d], a256(s.psi_elems[d] * 4), st);
        a.psib[d] = (float *)(B + L.psib[d]);
        a.zetab[d] = (float *)(B + L.zetab[d]);
        if (s.Llo[d] + s.Lhi[d] > 0) {
            fdtd_launch_fill_zero(B + L.F[d], a256(s.elems * 4), st);
            a.F[d] = (float *)origin4(s, B + L.F[d]);
        }
        std::vector<int> bc = band_coords(s, d);
        a.nband[d] = (int)bc.size();
        if (!bc.empty()) {
            fdtd_launch_fill_zero(B + L.E[d], a256(s.elems * 4), st);
            a.E[d] = (float *)origin4(s, B + L.E[d]);
            AHIP(ctx, hipMemcpyAsync(B + L.band[d], bc.data(), bc.size() * 4, hipMemcpyHostToDevice, st));
            AHIP(ctx, hipStreamSynchronize(st));
            a.band[d] = (const int *)(B + L.band[d]);
        }
    }
    // receivers grouped by location, in first-appearance order; receiver order within a group
    int ngroups = 0;
    if (s.nrec > 0) {
        std::vector<int32_t> h((size_t)s.nrec * 3);
        AHIP(ctx, hipMemcpy(h.data(), s.rec, h.size() * 4, hipMemcpyDeviceToHost));
        std::vector<int> gstart, ridx;
        std::vector<std::vector<int>> members;
        std::map<std::array<int32_t, 3>, int> where;
        for (int r = 0; r < s.nrec; ++r) {
            const std::array<int32_t, 3> key{h[3 * r], h[3 * r + 1], h[3 * r + 2]};
            auto it = where.find(key);
            if (it == where.end()) {
                where[key] = (int)members.size();
                members.push_back({r});
            } else {
                members[it->second].push_back(r);
            }
        }
        for (auto &m : members) {
            gstart.push_back((int)ridx.size());
            ridx.insert(ridx.end(), m.begin(), m.end());
        }
        gstart.push_back((int)ridx.size());
        ngroups = (int)members.size();
        AHIP(ctx, hipMemcpyAsync(B + L.gstart, gstart.data(), gstart.size() * 4, hipMemcpyHostToDevice, st));
        AHIP(ctx, hipMemcpyAsync(B + L.ridx, ridx.data(), ridx.size() * 4, hipMemcpyHostToDevice, st));
        AHIP(ctx, hipStreamSynchronize(st));
    }
    const int *gstart_d = (const int *)(B + L.gstart), *ridx_d = (const int *)(B + L.ridx);
    const long N = (long)s.nx * s.ny * s.nz;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)std::min<long>((N + 255) / 256, 65536)), dim3(256), 0, st,
                       grad_v_dev, N);
    a.G = grad_v_dev;
    const size_t fb = a256(s.elems * s.esz);
    char *seg = B + L.seg;
    // the context's step count and level roles, restored on exit: the other shots
    // of the context keep their forward state, so that each shot's adjoint can
    // follow one batched forward run
    const long step_in = ctx->step;
    const int iu_in = ctx->iu, ium1_in = ctx->ium1;
    const bool was_saving = ctx->saving;
    ctx->saving = false;
    // largest per-axis thread counts of passes 1 (band points) and 2 (slab points)
    long p1_max = 0, p2_max = 0;
    for (int d = 0; d < 3; ++d) {
        const int n1 = d == 0 ? s.ny : s.nx, n2 = d == 2 ? s.ny : s.nz;
        p1_max = std::max(p1_max, (long)a.nband[d] * n1 * n2);
        if (s.Llo[d] + s.Lhi[d] > 0)
            p2_max = std::max(p2_max, d == 0 ? (long)s.LX * s.ny * s.nz
                                             : (d == 1 ? (long)s.nx * s.LY * s.nz : (long)s.nx * s.ny * s.LZ));
    }
    const int nck = (nt + every - 1) / every;
    const float inv_scale = (float)(1.0 / s.scale);
    int *stepc = (int *)fdtd_ws(ctx, ctx->o_stepc);
    for (int k = nck - 1; k >= 0; --k) {
        const int s0 = k * every, s1 = std::min(s0 + every, nt);
        // restore the state before step s0, then recompute the segment's levels
        fdtd_restore_state(ctx, shot, B + L.ck + (size_t)k * fdtd_state_bytes(s));
        fdtd_launch_set_int(stepc, s0, st);
        ctx->step = s0;
        AHIP(ctx, hipMemcpyAsync(seg + fb, fdtd_ws(ctx, s.o_u[ctx->iu]), s.elems * s.esz,
                                 hipMemcpyDeviceToDevice, st));
        AHIP(ctx, hipMemcpyAsync(seg, fdtd_ws(ctx, s.o_u[ctx->ium1]), s.elems * s.esz,
                                 hipMemcpyDeviceToDevice, st));
        for (int n = s0; n < s1; ++n) {
            fdtd_enqueue_step_shot(ctx, shot);
            AHIP(ctx, hipMemcpyAsync(seg + (size_t)(n - s0 + 2) * fb, fdtd_ws(ctx, s.o_u[ctx->iu]),
                                     s.elems * s.esz, hipMemcpyDeviceToDevice, st));
        }
        // reverse sweep over the segment
        for (int n = s1 - 1; n >= s0; --n) {
            if (ngroups > 0)
                hipLaunchKernelGGL(k_adj_resid, dim3((ngroups + 255) / 256), dim3(256), 0, st, a.lam, sp,
                                   resid_dev + (size_t)n * s.nrec, gstart_d, ridx_d, ngroups);
            hipLaunchKernelGGL(k_adj_lbar, dim3((s.nx + 255) / 256, s.ny, s.nz), dim3(256), 0, st, a);
            a.up = origin_t(s, seg + (size_t)(n - s0 + 2) * fb);
            a.u0 = origin_t(s, seg + (size_t)(n - s0 + 1) * fb);
            a.um = origin_t(s, seg + (size_t)(n - s0) * fb);
            if (p1_max > 0)   // the three axes in one launch (disjoint outputs)
                hipLaunchKernelGGL(k_adj_p1, dim3((unsigned)((p1_max + 255) / 256), 3), dim3(256), 0, st, a);
            if (p2_max > 0)
                hipLaunchKernelGGL(k_adj_p2, dim3((unsigned)((p2_max + 255) / 256), 3), dim3(256), 0, st, a);
            if (ctx->storage == FDTD_F16) launch_p3<_Float16>(a, s, inv_scale, st);
            else if (ctx->storage == FDTD_BF16) launch_p3<__bf16>(a, s, inv_scale, st);
            else launch_p3<float>(a, s, inv_scale, st);
            std::swap(a.lam, a.lamp);
        }
        AHIP(ctx, hipGetLastError());
    }
    hipLaunchKernelGGL(k_adj_finish, dim3((s.nx + 255) / 256, s.ny, s.nz), dim3(256), 0, st, sp, grad_v_dev,
                       s.c.dt);
    ctx->saving = was_saving;
    ctx->step = step_in;
    ctx->iu = iu_in;
    ctx->ium1 = ium1_in;
    fdtd_launch_set_int(stepc, (int)step_in, st);
    fdtd_clear_graphs(ctx);
    ctx->hdesc[shot] = saved;
    AHIP(ctx, hipMemcpyAsync(dd + shot, &ctx->hdesc[shot], sizeof(DevShot), hipMemcpyHostToDevice, st));
    AHIP(ctx, hipStreamSynchronize(st));
    AHIP(ctx, hipGetLastError());
    return FDTD_OK;
}

}  // extern "C"
