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
// The sweep runs on mu^n = m lambda^n, which is Lbar itself one step later:
//   mu^n = 2 mu^{n+1} - mu^{n+2} + m sum_d [ D2_d(K_d) - D1_d(W_d) ],
//   K_d = kinv E_d in the slab and mu^{n+1} elsewhere (kinv = 1, E_d = Lbar in
//   the rest of the band), W_d = dkinv E_d + F_d in the slab and 0 elsewhere.
// Away from every band this is the forward leapfrog applied to mu (D2 is
// symmetric).  The residual at the receivers enters lambda^{n+1}, i.e. m times
// it enters mu^{n+1}, first.  The model enters only through m = v^2 dt^2
// multiplying (Lt u^n + f^n) = (u^{n+1} - 2u^n + u^{n-1}) / m, so
// dJ/dv = (2/v) sum_n lambda^{n+1} (u^{n+1} - 2u^n + u^{n-1})
//       = 2 dt / (m sqrt(m)) sum_n mu^{n+1} (u^{n+1} - 2u^n + u^{n-1}),
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
    float *mu1;              // mu^{n+1} = m lambda^{n+1}  (origin-adjusted, FP32, forward layout)
    float *mu2;              // mu^{n+2} in, mu^n out
    float *psib[3], *zetab[3];          // compact slab layouts (as psi)
    float *E[3];             // origin-adjusted full-grid arrays, written at slab points of axis d only:
    float *K[3];             //   E_d, kinv E_d and W_d = dkinv E_d + a (psi_b - D1_d E_d);
    float *W[3];             //   W_d stays zero elsewhere
    const float *um, *u0, *up;   // forward u^{n-1}, u^n, u^{n+1} (FP32)
    double *G;               // dense accumulator sum mu^{n+1} (u^{n+1} - 2u^n + u^{n-1})
};

__device__ __forceinline__ long fidx(const DevShot &s, int x, int y, int z) {
    return (long)z * s.S + (long)y * s.P + x;
}

// residual injection: one thread per distinct receiver location; the residuals
// of the receivers there are summed in receiver order (repeated receivers add
// up) and m times the sum enters mu^{n+1}.  gstart[g] .. gstart[g + 1] index
// ridx, the receivers of location g.
__global__ __launch_bounds__(256) void k_adj_resid(float *mu, const DevShot *sp, const float *resid_row,
                                                   const int *gstart, const int *ridx, int ngroups) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    const DevShot &s = *sp;
    const int k0 = gstart[g], k1 = gstart[g + 1];
    const int32_t *q = s.rec + 3 * ridx[k0];
    const long i = fidx(s, q[0], q[1], q[2]);
    float r = 0.0f;
    for (int k = k0; k < k1; ++k) r += resid_row[ridx[k]];
    mu[i] = fmaf(s.m[i], r, mu[i]);
}

// slab point t of axis d: its coordinates and its coordinate along d
__device__ __forceinline__ bool slab_point(const DevShot &s, int d, long t, int &x, int &y, int &z, int &k) {
    const int lo = s.Llo[d], hi = s.Lhi[d];
    if (lo + hi == 0) return false;
    long count;
    if (d == 0) count = (long)s.LX * s.ny * s.nz;
    else if (d == 1) count = (long)s.nx * s.LY * s.nz;
    else count = (long)s.nx * s.ny * s.LZ;
    if (t >= count) return false;
    if (d == 0) {
        const int is = (int)(t % s.LX);
        const long r = t / s.LX;
        y = (int)(r % s.ny);
        z = (int)(r / s.ny);
        x = is < lo ? is : s.nx - hi + (is - lo);
        k = x;
    } else if (d == 1) {
        x = (int)(t % s.nx);
        const long r = t / s.nx;
        const int js = (int)(r % s.LY);
        z = (int)(r / s.LY);
        y = js < lo ? js : s.ny - hi + (js - lo);
        k = y;
    } else {
        x = (int)(t % s.nx);
        const long r = t / s.nx;
        y = (int)(r % s.ny);
        const int ks = (int)(r / s.ny);
        z = ks < lo ? ks : s.nz - hi + (ks - lo);
        k = z;
    }
    return true;
}

// whether coordinate c (possibly outside [0, n)) lies in a slab of the axis
__device__ __forceinline__ bool slab_in_grid(int c, int n, int lo, int hi) {
    return c >= 0 && c < n && in_slab(c, n, lo, hi);
}

// pass 1 on slab points of axis d = blockIdx.y: the zeta adjoint, E_d and K_d
__global__ __launch_bounds__(256) void k_adj_p1(AdjArgs a) {
    const DevShot &s = *a.s;
    const int d = (int)blockIdx.y;
    int x, y, z, k;
    if (!slab_point(s, d, (long)blockIdx.x * blockDim.x + threadIdx.x, x, y, z, k)) return;
    const long i = fidx(s, x, y, z);
    const float lb = a.mu1[i];
    float *zb = &a.zetab[d][psi_index(s, d, x, y, z)];
    const float kinv = prof_at(s, d, 2, k);
    const float zt = *zb + lb;
    const float e = fmaf(kinv, lb, prof_at(s, d, 1, k) * zt);
    *zb = prof_at(s, d, 0, k) * zt;
    a.E[d][i] = e;
    a.K[d][i] = kinv * e;
}

// pass 2 on slab points of axis d = blockIdx.y: the psi adjoint and
// W_d = dkinv E_d + a (psi_b - D1_d E_d), E_d being Lbar at the taps outside the slab
__global__ __launch_bounds__(256) void k_adj_p2(AdjArgs a) {
    const DevShot &s = *a.s;
    const int d = (int)blockIdx.y;
    int x, y, z, k;
    if (!slab_point(s, d, (long)blockIdx.x * blockDim.x + threadIdx.x, x, y, z, k)) return;
    const int n = coord_n(s, d), lo = s.Llo[d], hi = s.Lhi[d];
    const long i = fidx(s, x, y, z);
    const long stride = d == 0 ? 1 : (d == 1 ? s.P : s.S);
    const float *E = a.E[d];
    float el[4], eh[4];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
        const float *pl = slab_in_grid(k - l, n, lo, hi) ? E : a.mu1;
        const float *ph = slab_in_grid(k + l, n, lo, hi) ? E : a.mu1;
        el[l - 1] = pl[i - l * stride];
        eh[l - 1] = ph[i + l * stride];
    }
    const long pi = psi_index(s, d, x, y, z);
    const float pt = a.psib[d][pi] - d1_axis(s.w1[d], el, eh);
    a.W[d][i] = fmaf(prof_at(s, d, 3, k), E[i], prof_at(s, d, 1, k) * pt);
    a.psib[d][pi] = prof_at(s, d, 0, k) * pt;
}

// Pass 3 on every point: mu^n and the gradient accumulation.  Along an axis d
// whose band the wave does not touch, the axis term is D2_d mu^{n+1}.  A wave
// that touches it evaluates D2_d(K_d) - D1_d(W_d) for all its lanes, taking
// K_d from its array at slab taps and mu^{n+1} at the others.  At a lane
// outside the band no tap lies in the slab, so this is D2_d mu^{n+1} with the
// same bits (the W_d taps are exact zeros).  A wave is one y row of 64 x
// points (blockDim = 64 x 4), so the y and z tests are wave-uniform and the x
// test is taken per 64-point tile.
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
    const float c = a.mu1[i];
    float t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float lo[4], hi[4];
        if (!touch[d]) {
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                lo[l - 1] = a.mu1[i - l * st[d]];
                hi[l - 1] = a.mu1[i + l * st[d]];
            }
            t[d] = d2_axis(s.w2[d], c, lo, hi);
        } else {
            const int n = coord_n(s, d), Llo = s.Llo[d], Lhi = s.Lhi[d];
            const int k = cc[d];
            const float *Kd = a.K[d], *Wd = a.W[d];
            float wl[4], wh[4];
            const float kc = (slab_in_grid(k, n, Llo, Lhi) ? Kd : a.mu1)[i];
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                const long im = i - l * st[d], ip = i + l * st[d];
                lo[l - 1] = (slab_in_grid(k - l, n, Llo, Lhi) ? Kd : a.mu1)[im];
                hi[l - 1] = (slab_in_grid(k + l, n, Llo, Lhi) ? Kd : a.mu1)[ip];
                wl[l - 1] = Wd[im];
                wh[l - 1] = Wd[ip];
            }
            t[d] = d2_axis(s.w2[d], kc, lo, hi) - d1_axis(s.w1[d], wl, wh);
        }
    }
    const float out = leapfrog(s.m[i], (t[0] + t[1]) + t[2], c, a.mu2[i]);
    // gradient: mu^{n+1} (u^{n+1} - 2 u^n + u^{n-1})
    const double d2u = (((double)a.up[i] - 2.0 * (double)a.u0[i]) + (double)a.um[i]) * (double)inv_scale;
    const long gi = ((long)z * s.ny + y) * s.nx + x;
    a.G[gi] += (double)c * d2u;
    a.mu2[i] = out;
}

// dJ/dv = 2 G dt / (m sqrt(m))  (G sums mu = m lambda; v = sqrt(m) / dt)
__global__ __launch_bounds__(256) void k_adj_finish(const DevShot *sp, double *G, double dt) {
    const DevShot &s = *sp;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= s.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const long gi = ((long)z * s.ny + y) * s.nx + x;
    const double m = (double)s.m[fidx(s, x, y, z)];
    G[gi] = 2.0 * G[gi] * dt / (m * sqrt(m));
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
    size_t ck = 0, seg = 0, mu1 = 0, mu2 = 0, psib[3] = {}, zetab[3] = {}, E[3] = {}, K[3] = {}, W[3] = {};
    size_t gstart = 0, ridx = 0;   // receivers grouped by location (k_adj_resid)
    size_t total = 0;
    int nck = 0;
};

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
    L.mu1 = take(s.elems * 4);
    L.mu2 = take(s.elems * 4);
    for (int d = 0; d < 3; ++d) {
        const size_t full = (s.Llo[d] + s.Lhi[d]) > 0 ? s.elems * 4 : 0;
        L.psib[d] = take(s.psi_elems[d] * 4);
        L.zetab[d] = take(s.psi_elems[d] * 4);
        L.E[d] = take(full);
        L.K[d] = take(full);
        L.W[d] = take(full);
    }
    L.gstart = take((size_t)(s.nrec + 1) * 4);
    L.ridx = take((size_t)std::max(s.nrec, 1) * 4);
    L.total = off;
    return L;
}

// slab points of axis d (pass 1 and 2 launch one thread per point)
static long slab_count(const ShotH &s, int d) {
    if (s.Llo[d] + s.Lhi[d] == 0) return 0;
    if (d == 0) return (long)s.LX * s.ny * s.nz;
    if (d == 1) return (long)s.nx * s.LY * s.nz;
    return (long)s.nx * s.ny * s.LZ;
}
}  // namespace

static char *origin4(const ShotH &s, char *base) { return base + origin_elems(s) * 4; }

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

    // adjoint state to zero (W_d stays zero outside the slabs)
    fdtd_launch_fill_zero(B + L.mu1, a256(s.elems * 4), st);
    fdtd_launch_fill_zero(B + L.mu2, a256(s.elems * 4), st);
    AdjArgs a;
    memset(&a, 0, sizeof a);
    a.s = sp;
    a.mu1 = (float *)origin4(s, B + L.mu1);
    a.mu2 = (float *)origin4(s, B + L.mu2);
    for (int d = 0; d < 3; ++d) {
        fdtd_launch_fill_zero(B + L.psib[d], a256(s.psi_elems[d] * 4), st);
        fdtd_launch_fill_zero(B + L.zetab[d], a256(s.psi_elems[d] * 4), st);
        a.psib[d] = (float *)(B + L.psib[d]);
        a.zetab[d] = (float *)(B + L.zetab[d]);
        if (s.Llo[d] + s.Lhi[d] > 0) {
            fdtd_launch_fill_zero(B + L.E[d], a256(s.elems * 4), st);
            fdtd_launch_fill_zero(B + L.K[d], a256(s.elems * 4), st);
            fdtd_launch_fill_zero(B + L.W[d], a256(s.elems * 4), st);
            a.E[d] = (float *)origin4(s, B + L.E[d]);
            a.K[d] = (float *)origin4(s, B + L.K[d]);
            a.W[d] = (float *)origin4(s, B + L.W[d]);
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
    // largest per-axis thread count of passes 1 and 2 (slab points)
    long slab_max = 0;
    for (int d = 0; d < 3; ++d) slab_max = std::max(slab_max, slab_count(s, d));
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
                hipLaunchKernelGGL(k_adj_resid, dim3((ngroups + 255) / 256), dim3(256), 0, st, a.mu1, sp,
                                   resid_dev + (size_t)n * s.nrec, gstart_d, ridx_d, ngroups);
            a.up = (const float *)origin4(s, seg + (size_t)(n - s0 + 2) * fb);
            a.u0 = (const float *)origin4(s, seg + (size_t)(n - s0 + 1) * fb);
            a.um = (const float *)origin4(s, seg + (size_t)(n - s0) * fb);
            if (slab_max > 0) {   // the three axes in one launch each (disjoint outputs)
                hipLaunchKernelGGL(k_adj_p1, dim3((unsigned)((slab_max + 255) / 256), 3), dim3(256), 0, st, a);
                hipLaunchKernelGGL(k_adj_p2, dim3((unsigned)((slab_max + 255) / 256), 3), dim3(256), 0, st, a);
            }
            hipLaunchKernelGGL(k_adj_p3, dim3((s.nx + 63) / 64, (s.ny + 3) / 4, s.nz), dim3(64, 4), 0, st, a,
                               inv_scale);
            std::swap(a.mu1, a.mu2);
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
