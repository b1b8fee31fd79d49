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
//       = 2 dt / (m sqrt(m)) sum_n mu^{n+1} (e^{n+1} - e^n),  e^n = u^n - u^{n-1},
// accumulated in FP64.  Forward levels are recomputed per segment from
// checkpoints saved every `every` steps, and the increments e kept (FP32).
// The mu levels live in a ring of G + 1 slots (G <= 16 steps), so that
// the FP64 accumulator is read and written once per G reverse steps, by a
// pass over the last G levels, and not by every step.  One sweep covers one
// shot or every shot of the context: each pass is one launch over all of them.
#include "fdtd_host.hpp"
#include "fdtd_launch.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

// Adjoint state of one shot of a sweep (device array, one entry per shot).
struct AdjShot {
    DevShot s;               // the forward descriptor (geometry, m, profiles, coefficients)
    float *mu;               // ring slot 0 of the mu levels (origin-adjusted); mu^n is in slot n mod mslots
    long mstride;            // elements between ring slots
    int mslots;              // ring slots: G + 1
    float *psib[3], *zetab[3];          // compact slab layouts (as psi)
    float *E[3];             // origin-adjusted full-grid arrays, written at slab points of axis d only:
    float *K[3];             //   E_d, kinv E_d and W_d = dkinv E_d + a (psi_b - D1_d E_d);
    float *W[3];             //   W_d stays zero elsewhere
    const float *lev;        // increments e of the recomputed levels (FP32, origin-adjusted slot 0 of half 0)
    long lstride;            // elements between slots
    int nslot;               // slots per half: every + 1
    float inv_scale;         // 1 / storage scale of the fields
    double *G;               // dense accumulator sum mu^{n+1} (u^{n+1} - 2u^n + u^{n-1}), [nz][ny][nx]
    const float *resid;      // dJ/dtraces [nt][nrec]
    const int *gstart, *ridx;   // receivers grouped by location (k_adj_resid)
    int ngroups, nrec;
    int bbase, btx, bty;          // the gradient pass: first block, tiles along x and y
    int bbase2;                   // pass 3 (two planes per block): first block
};
// A block of passes 1, 2 or 3 finds its shot (and for 1, 2 its axis and first
// slab point) in a table indexed by block (scalar loads), not by searching.
struct SlabBlock {
    int shot_axis;   // shot of the sweep * 4 + axis
    int t0;          // first slab point of the block along that axis
};
// one reverse step n: mu^n goes to ring slot m0, mu^{n+1} and mu^{n+2} are in
// slots m1 and m2 (n, n + 1, n + 2 mod the ring size)
struct AdjStep {
    int n, m0, m1, m2;
};
// gradient pass over reverse steps n_lo .. n_lo + cnt - 1 of the segment that
// starts at step s0: e^n, e^{n+1} are in slots n - s0, n - s0 + 1 of half `half`
struct AdjGrad {
    int half, s0, n_lo, cnt;
};

__device__ __forceinline__ long fidx(const DevShot &s, int x, int y, int z) {
    return (long)z * s.S + (long)y * s.P + x;
}

__device__ __forceinline__ float *mu_slot(const AdjShot &a, int k) { return a.mu + (long)k * a.mstride; }

// residual injection: one thread per distinct receiver location of shot
// blockIdx.y; the residuals of the receivers there are summed in receiver
// order (repeated receivers add up) and m times the sum enters mu^{n+1}.
// gstart[g] .. gstart[g + 1] index ridx, the receivers of location g.
__global__ __launch_bounds__(256) void k_adj_resid(const AdjShot *__restrict__ A, AdjStep st) {
    const AdjShot &a = A[blockIdx.y];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.ngroups) return;
    const DevShot &s = a.s;
    const float *row = a.resid + (long)st.n * a.nrec;
    const int k0 = a.gstart[g], k1 = a.gstart[g + 1];
    const int32_t *q = s.rec + 3 * a.ridx[k0];
    const long i = fidx(s, q[0], q[1], q[2]);
    float r = 0.0f;
    for (int k = k0; k < k1; ++k) r += row[a.ridx[k]];
    float *mu = mu_slot(a, st.m1);
    mu[i] = fmaf(s.m[i], r, mu[i]);
}

// Increment e = u[q] - u[q ^ 1] of one shot's two level buffers (the newest
// level minus the one before) into a slot, over the grid: blockIdx.y is the
// shot, blocks stride over the rows.
struct DiffJob {
    const float *a, *b;   // origin-adjusted
    float *d;
    int nx, ny, nz, P;
    long S;
};
__global__ __launch_bounds__(256) void k_adj_diff(const DiffJob *__restrict__ jobs) {
    const DiffJob j = jobs[blockIdx.y];
    const int rows = j.ny * j.nz;
    for (int r = (int)blockIdx.x; r < rows; r += (int)gridDim.x) {
        const int z = r / j.ny, y = r - z * j.ny;
        const long o = (long)z * j.S + (long)y * j.P;
        // (non-temporal accesses: the levels are read once here, the increment only by the
        // gradient pass)
        for (int x = (int)threadIdx.x; x < j.nx; x += 256)
            __builtin_nontemporal_store(__builtin_nontemporal_load(&j.a[o + x]) - __builtin_nontemporal_load(&j.b[o + x]),
                                        &j.d[o + x]);
    }
}

// Passes 1 and 2 take one thread per slab point: a block holds 256 consecutive
// points of one shot's axis (the slab points of axis d in the order x fastest,
// then y, then z, with the coordinate along d running over the slab positions).
__device__ __forceinline__ bool slab_point(const AdjShot *__restrict__ A, const SlabBlock *__restrict__ blk, int &sh,
                                           int &d, int &x, int &y, int &z, int &k) {
    const SlabBlock b = blk[blockIdx.x];
    sh = b.shot_axis >> 2;
    d = b.shot_axis & 3;
    const DevShot &s = A[sh].s;
    const int lo = s.Llo[d], hi = s.Lhi[d];
    const int t = b.t0 + (int)threadIdx.x;
    if (d == 0) {
        const int is = t % s.LX, r = t / s.LX;
        y = r % s.ny;
        z = r / s.ny;
        x = is < lo ? is : s.nx - hi + (is - lo);
        k = x;
        return z < s.nz;
    }
    x = t % s.nx;
    const int r = t / s.nx;
    if (d == 1) {
        const int js = r % s.LY;
        z = r / s.LY;
        y = js < lo ? js : s.ny - hi + (js - lo);
        k = y;
    } else {
        y = r % s.ny;
        const int ks = r / s.ny;
        z = ks < lo ? ks : s.nz - hi + (ks - lo);
        k = z;
        return ks < s.LZ;
    }
    return z < s.nz;
}

// whether coordinate c (possibly outside [0, n)) lies in a slab of the axis
__device__ __forceinline__ bool slab_in_grid(int c, int n, int lo, int hi) {
    return c >= 0 && c < n && in_slab(c, n, lo, hi);
}

// pass 1 on slab points: the zeta adjoint, E_d and K_d
__global__ __launch_bounds__(256) void k_adj_p1(const AdjShot *__restrict__ A, const SlabBlock *__restrict__ blk,
                                                AdjStep st) {
    int sh, d, x, y, z, k;
    if (!slab_point(A, blk, sh, d, x, y, z, k)) return;
    const AdjShot &a = A[sh];
    const DevShot &s = a.s;
    const long i = fidx(s, x, y, z);
    const float lb = mu_slot(a, st.m1)[i];
    float *zb = &a.zetab[d][psi_index(s, d, x, y, z)];
    const float kinv = prof_at(s, d, 2, k);
    const float zt = *zb + lb;
    const float e = fmaf(kinv, lb, prof_at(s, d, 1, k) * zt);
    *zb = prof_at(s, d, 0, k) * zt;
    a.E[d][i] = e;
    a.K[d][i] = kinv * e;
}

// pass 2 on slab points: the psi adjoint and W_d = dkinv E_d + a (psi_b - D1_d E_d),
// E_d being Lbar = mu^{n+1} at the taps outside the slab
__global__ __launch_bounds__(256) void k_adj_p2(const AdjShot *__restrict__ A, const SlabBlock *__restrict__ blk,
                                                AdjStep st) {
    int sh, d, x, y, z, k;
    if (!slab_point(A, blk, sh, d, x, y, z, k)) return;
    const AdjShot &a = A[sh];
    const DevShot &s = a.s;
    const int n = coord_n(s, d), lo = s.Llo[d], hi = s.Lhi[d];
    const long i = fidx(s, x, y, z);
    const long stride = d == 0 ? 1 : (d == 1 ? s.P : s.S);
    const float *E = a.E[d], *mu1 = mu_slot(a, st.m1);
    float el[4], eh[4];
#pragma unroll
    for (int l = 1; l <= 4; ++l) {
        el[l - 1] = (slab_in_grid(k - l, n, lo, hi) ? E : mu1)[i - l * stride];
        eh[l - 1] = (slab_in_grid(k + l, n, lo, hi) ? E : mu1)[i + l * stride];
    }
    const long pi = psi_index(s, d, x, y, z);
    const float pt = a.psib[d][pi] - d1_axis(s.w1[d], el, eh);
    a.W[d][i] = fmaf(prof_at(s, d, 3, k), E[i], prof_at(s, d, 1, k) * pt);
    a.psib[d][pi] = prof_at(s, d, 0, k) * pt;
}

// The point of this thread in pass 3's and the gradient pass's block tiling
// (a block is a 64 x 4 tile of one plane of one shot, one y row per wave);
// false for threads past the grid.
struct TilePoint {
    int x, y, z, x0;
};
__device__ __forceinline__ bool tile_point(const AdjShot &a, int lb, TilePoint &p) {
    const DevShot &s = a.s;
    const int nxy = a.btx * a.bty;
    p.z = lb / nxy;
    const int r = lb - p.z * nxy;
    if (p.z >= s.nz) return false;
    const int by = r / a.btx, bx = r - by * a.btx;
    p.x0 = bx * 64;
    p.x = p.x0 + (int)(threadIdx.x & 63);
    p.y = __builtin_amdgcn_readfirstlane(by * 4 + (int)(threadIdx.x >> 6));
    return p.x < s.nx && p.y < s.ny;
}

// Pass 3 on every point: mu^n = 2 mu^{n+1} - mu^{n+2} + m sum_d t_d, each
// point taking its taps from memory.  Along an axis d whose band the wave does
// not touch, t_d = D2_d mu^{n+1}.  A wave that touches it evaluates
// D2_d(K_d) - D1_d(W_d) for all its lanes, taking K_d from its array at slab
// taps and mu^{n+1} at the others.  At a lane outside the band no tap lies in
// the slab, so this is D2_d mu^{n+1} with the same bits (the W_d taps are
// exact zeros).  The y and z tests are wave-uniform and the x test is taken
// per 64-point tile.  A block is a 64 x 4 tile of two consecutive planes: a
// thread loads its column of mu^{n+1} over the ten planes z0 - 4 .. z0 + 5
// once, for the z taps of both of its points.
__device__ __forceinline__ void p3_point(const AdjShot &a, const DevShot &s, const AdjStep &st, int x, int y, int z,
                                         bool tx, const float *col) {
    const long i = fidx(s, x, y, z);
    const int cc[3] = {x, y, z};
    const long stv[3] = {1, (long)s.P, (long)s.S};
    const bool touch[3] = {tx, in_band(y, s.ny, s.Llo[1], s.Lhi[1]), in_band(z, s.nz, s.Llo[2], s.Lhi[2])};
    const float *mu1 = mu_slot(a, st.m1);
    const float c = col[4];
    float t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float lo[4], hi[4];
        if (!touch[d]) {
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                lo[l - 1] = d == 2 ? col[4 - l] : mu1[i - l * stv[d]];
                hi[l - 1] = d == 2 ? col[4 + l] : mu1[i + l * stv[d]];
            }
            t[d] = d2_axis(s.w2[d], c, lo, hi);
        } else {
            const int n = coord_n(s, d), Llo = s.Llo[d], Lhi = s.Lhi[d];
            const int k = cc[d];
            const float *Kd = a.K[d], *Wd = a.W[d];
            float wl[4], wh[4];
            const float kc = (slab_in_grid(k, n, Llo, Lhi) ? Kd : mu1)[i];
#pragma unroll
            for (int l = 1; l <= 4; ++l) {
                const long im = i - l * stv[d], ip = i + l * stv[d];
                lo[l - 1] = (slab_in_grid(k - l, n, Llo, Lhi) ? Kd : mu1)[im];
                hi[l - 1] = (slab_in_grid(k + l, n, Llo, Lhi) ? Kd : mu1)[ip];
                wl[l - 1] = Wd[im];
                wh[l - 1] = Wd[ip];
            }
            t[d] = d2_axis(s.w2[d], kc, lo, hi) - d1_axis(s.w1[d], wl, wh);
        }
    }
    // non-temporal store, and loads for the streams read once (m, mu^{n+2}), as in the forward
    // step (3 smallest batched shots: 290 -> 285 us per reverse step with these and the
    // increments' and gradient pass's hints)
    __builtin_nontemporal_store(leapfrog(__builtin_nontemporal_load(&s.m[i]), (t[0] + t[1]) + t[2], c,
                                         __builtin_nontemporal_load(&mu_slot(a, st.m2)[i])),
                                &mu_slot(a, st.m0)[i]);
}

__global__ __launch_bounds__(256) void k_adj_p3(const AdjShot *__restrict__ A, const int *__restrict__ block_shot,
                                                AdjStep st) {
    const int b = (int)blockIdx.x;
    const AdjShot &a = A[block_shot[b]];
    const DevShot &s = a.s;
    const int lb = b - a.bbase2, nxy = a.btx * a.bty;
    const int z0 = 2 * (lb / nxy), r = lb - (lb / nxy) * nxy;
    if (z0 >= s.nz) return;
    const int by = r / a.btx, bx = r - by * a.btx;
    const int x0 = bx * 64;
    const int x = x0 + (int)(threadIdx.x & 63);
    const int y = __builtin_amdgcn_readfirstlane(by * 4 + (int)(threadIdx.x >> 6));
    if (x >= s.nx || y >= s.ny) return;
    // the band of an axis is an interval at each end of the grid, so a tile meets it iff one of its end points lies in it
    const bool tx = in_band(x0, s.nx, s.Llo[0], s.Lhi[0]) || in_band(min(x0 + 64, s.nx) - 1, s.nx, s.Llo[0], s.Lhi[0]);
    const bool two = z0 + 1 < s.nz;
    const float *mu1 = mu_slot(a, st.m1);
    const long i0 = fidx(s, x, y, z0);
    // planes z0 - 4 .. z0 + 4 lie in the field with its 4-plane frames; z0 + 5 only when z0 + 1 is a plane
    // (two planes per block: measured 282.5 -> 274.5 us per reverse step on the three smallest batched
    // shots; a loop over 2, 4 or 8 planes compiled to one wave less per SIMD and was slower)
    float col[10];
#pragma unroll
    for (int k = 0; k < 9; ++k) col[k] = mu1[i0 + (k - 4) * (long)s.S];
    col[9] = two ? mu1[i0 + 5 * (long)s.S] : 0.0f;
    p3_point(a, s, st, x, y, z0, tx, col);
    if (two) p3_point(a, s, st, x, y, z0 + 1, tx, col + 1);
}

// Gradient pass over cnt reverse steps, taken in the sweep's order (n from
// high to low): G += mu^{n+1} (e^{n+1} - e^n) / scale in FP64 at every point,
// reading the accumulator once.  Same block tiling as pass 3.
__global__ __launch_bounds__(256) void k_adj_grad(const AdjShot *__restrict__ A, const int *__restrict__ block_shot,
                                                  AdjGrad g) {
    const int b = (int)blockIdx.x;
    const AdjShot &a = A[block_shot[b]];
    const DevShot &s = a.s;
    TilePoint p;
    if (!tile_point(a, b - a.bbase, p)) return;
    const long i = fidx(s, p.x, p.y, p.z);
    const long gi = ((long)p.z * s.ny + p.y) * s.nx + p.x;
    const float *e = a.lev + (long)g.half * a.nslot * a.lstride + i;
    const double sc = (double)a.inv_scale;
    const int top = g.n_lo + g.cnt - 1;
    int ms = (top + 1) % a.mslots;   // ring slot of mu^{n+1}
    float ehi = e[(long)(top - g.s0 + 1) * a.lstride];
    double acc = a.G[gi];
#pragma unroll 4
    for (int n = top; n >= g.n_lo; --n) {
        const float elo = __builtin_nontemporal_load(&e[(long)(n - g.s0) * a.lstride]);   // read once
        const float c = __builtin_nontemporal_load(&mu_slot(a, ms)[i]);
        acc += (double)c * (((double)ehi - (double)elo) * sc);
        ehi = elo;
        ms = ms == 0 ? a.mslots - 1 : ms - 1;
    }
    a.G[gi] = acc;
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
// blocks of passes 1, 2 (slab points) and of pass 3 and the gradient pass of one shot
struct AdjCounts {
    long slab[3];   // slab points per axis
    int btx, bty;
    long slab_blocks() const {
        long b = 0;
        for (int d = 0; d < 3; ++d) b += (slab[d] + 255) / 256;
        return b;
    }
    long blocks(const ShotH &s) const { return (long)btx * bty * s.nz; }
    long blocks2(const ShotH &s) const { return (long)btx * bty * ((s.nz + 1) / 2); }
};
static AdjCounts adj_counts(const ShotH &s) {
    AdjCounts c;
    const int cx = (s.nx + 63) / 64;
    c.slab[0] = (long)s.LX * s.ny * s.nz;
    c.slab[1] = (long)s.nx * s.LY * s.nz;
    c.slab[2] = (long)s.nx * s.ny * s.LZ;
    c.btx = cx;
    c.bty = (s.ny + 3) / 4;
    return c;
}

struct AdjLayout {
    size_t ck = 0, seg = 0, mu = 0, psib[3] = {}, zetab[3] = {}, E[3] = {}, K[3] = {}, W[3] = {};
    size_t gstart = 0, ridx = 0;   // receivers grouped by location (k_adj_resid)
    // tables of a sweep over every shot of the context (those of a sweep's first shot are used):
    // AdjShot entries, increment jobs, checkpoint-restore jobs, the slab-pass and pass-3 block tables
    size_t tab = 0, jobs = 0, rjobs = 0, smap = 0, bmap = 0, bmap2 = 0;
    size_t total = 0;
    int nck = 0;   // checkpoint slots
};

// The regions sit at offsets fixed by the buffer's checkpoint capacity
// (nslots), never by the steps of one sweep: a sweep over fewer steps than
// the forward checkpointed must not place its state over later checkpoints.
// reverse steps per gradient pass (at most 16, a segment split evenly), and
// the mu ring that holds their levels
static int grad_chunk(int every) {
    const int passes = (every + 15) / 16;
    return (every + passes - 1) / passes;
}
static int mu_slots(int every) { return grad_chunk(every) + 1; }

static AdjLayout adj_layout(const fdtd_ctx *ctx, const ShotH &s, int every, int nslots) {
    AdjLayout L;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += a256(b);
        return o;
    };
    const size_t nctx = ctx->shots.size();
    long sblocks = 0, blocks = 0, blocks2 = 0;
    for (const ShotH &t : ctx->shots) {
        const AdjCounts c = adj_counts(t);
        sblocks += c.slab_blocks();
        blocks += c.blocks(t);
        blocks2 += c.blocks2(t);
    }
    L.nck = nslots;
    L.ck = take(fdtd_state_bytes(s) * (size_t)L.nck);
    L.seg = take(a256(s.elems * s.esz) * (size_t)(every + 1) * 2);   // two segments' increments
    L.mu = take(a256(s.elems * 4) * (size_t)mu_slots(every));   // the ring of mu levels
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
    L.tab = take(sizeof(AdjShot) * nctx);
    L.jobs = take(sizeof(DiffJob) * (size_t)(2 * (every + 1) * 2) * nctx);
    L.rjobs = take(sizeof(CopyJob) * (size_t)L.nck * 2 * 8 * nctx);
    L.smap = take(sizeof(SlabBlock) * (size_t)std::max(sblocks, 1L));
    L.bmap = take(sizeof(int) * (size_t)std::max(blocks, 1L));
    L.bmap2 = take(sizeof(int) * (size_t)std::max(blocks2, 1L));
    L.total = off;
    return L;
}

// A flat copy of `bytes` (a multiple of 256) as rows of 256 bytes, so that
// k_copy_jobs spreads it over many blocks.
static CopyJob flat_job(const void *src, void *dst, size_t bytes) {
    CopyJob c;
    c.src = src;
    c.dst = dst;
    c.esz = 4;
    c.ex = 64;
    c.ey = (int)(bytes / 256);
    c.ez = 1;
    c.sy = c.dy = 64;
    c.sz = c.dz = (long)c.ey * 64;
    fdtd_set_copy_vec(c);
    return c;
}
}  // namespace

static char *origin4(const ShotH &s, char *base) { return base + origin_elems(s) * 4; }

// One reverse sweep over the shots sh (one shot, or every shot of the context).
// The reverse sweep of segment k runs on the adjoint stream while the main
// stream restores checkpoint k - 1, recomputes its levels and keeps their
// increments in the other half of each increment buffer: the two touch
// disjoint memory (the forward state and one half, the adjoint state and the
// other half).  ev_adj[b] (ready): the increments of half b are written;
// ev_adj[2 + b] (free): the sweep that read half b is done.
static int adjoint_sweep(fdtd_ctx *ctx, const std::vector<int> &sh, int nt, const float *const *resid,
                         double *const *grad) {
    const int nsh = (int)sh.size(), nctx = (int)ctx->shots.size();
    if (!ctx->ws) AFAIL(ctx, FDTD_ESTATE, "no workspace bound");
    int every = 0;
    for (int q = 0; q < nsh; ++q) {
        const ShotH &s = ctx->shots[sh[q]];
        if (!resid[q] || !grad[q]) return FDTD_EINVAL;
        if (s.ck_every <= 0 || !s.ck_buf) AFAIL(ctx, FDTD_ESTATE, "checkpointing is not set for shot %d", sh[q]);
        if (q == 0) every = s.ck_every;
        else if (s.ck_every != every) AFAIL(ctx, FDTD_EINVAL, "the shots of one sweep need one checkpoint interval");
        if (nt > s.ck_nt)
            AFAIL(ctx, FDTD_ENOMEM, "shot %d: adjoint buffer holds checkpoints for %d steps, asked %d", sh[q], s.ck_nt,
                  nt);
        if (!s.vel_set) AFAIL(ctx, FDTD_ESTATE, "shot %d: no velocity model", sh[q]);
        const AdjLayout L = adj_layout(ctx, s, every, s.ck_count);
        if (L.total > s.ck_bytes)
            AFAIL(ctx, FDTD_ENOMEM, "shot %d: adjoint buffer of %zu bytes, %zu needed (receivers set after sizing it?)",
                  sh[q], s.ck_bytes, L.total);
    }
    if (ctx->step < nt) AFAIL(ctx, FDTD_ESTATE, "run the forward for %d steps first (at step %ld)", nt, ctx->step);
    hipStream_t st = ctx->stream;
    DevShot *dd = (DevShot *)fdtd_ws(ctx, ctx->o_desc);

    // recomputation must not overwrite the recorded traces
    std::vector<DevShot> saved(nsh);
    for (int q = 0; q < nsh; ++q) {
        saved[q] = ctx->hdesc[sh[q]];
        ctx->hdesc[sh[q]].traces = nullptr;
        ctx->hdesc[sh[q]].trace_cap = 0;
        AHIP(ctx, hipMemcpyAsync(dd + sh[q], &ctx->hdesc[sh[q]], sizeof(DevShot), hipMemcpyHostToDevice, st));
    }
    AHIP(ctx, hipStreamSynchronize(st));

    // adjoint state to zero (W_d stays zero outside the slabs), receiver
    // groups, the AdjShot table, the wave and block maps, the level-copy and
    // checkpoint-restore jobs
    const int nck = (nt + every - 1) / every;
    std::vector<AdjShot> tab(nsh);
    std::vector<DiffJob> jobs((size_t)2 * (every + 1) * 2 * nsh);
    std::vector<CopyJob> rjobs((size_t)nck * 2 * 8 * nsh);
    std::vector<SlabBlock> smap;
    std::vector<int> bmap, bmap2;
    int bbase = 0, bbase2 = 0, maxg = 0;
    long maxrows = 0, maxck = 0;
    for (int q = 0; q < nsh; ++q) {
        const ShotH &s = ctx->shots[sh[q]];
        const AdjLayout L = adj_layout(ctx, s, every, s.ck_count);
        char *B = s.ck_buf;
        AdjShot &a = tab[q];
        memset(&a, 0, sizeof a);
        a.s = ctx->hdesc[sh[q]];
        fdtd_launch_fill_zero(B + L.mu, a256(s.elems * 4) * (size_t)mu_slots(every), st);
        a.mu = (float *)origin4(s, B + L.mu);
        a.mstride = (long)(a256(s.elems * 4) / 4);
        a.mslots = mu_slots(every);
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
        const size_t fb = a256(s.elems * s.esz);
        a.lev = (const float *)origin4(s, B + L.seg);
        a.lstride = (long)(fb / 4);
        a.nslot = every + 1;
        a.inv_scale = (float)(1.0 / s.scale);
        a.G = grad[q];
        a.resid = resid[q];
        a.nrec = s.nrec;
        // receivers grouped by location, in first-appearance order; receiver order within a group
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
            a.ngroups = (int)members.size();
            AHIP(ctx, hipMemcpyAsync(B + L.gstart, gstart.data(), gstart.size() * 4, hipMemcpyHostToDevice, st));
            AHIP(ctx, hipMemcpyAsync(B + L.ridx, ridx.data(), ridx.size() * 4, hipMemcpyHostToDevice, st));
            AHIP(ctx, hipStreamSynchronize(st));
        }
        a.gstart = (const int *)(B + L.gstart);
        a.ridx = (const int *)(B + L.ridx);
        maxg = std::max(maxg, a.ngroups);
        // wave units of passes 1, 2 and blocks of pass 3
        const AdjCounts cnt = adj_counts(s);
        for (int d = 0; d < 3; ++d)
            for (long t0 = 0; t0 < cnt.slab[d]; t0 += 256) smap.push_back(SlabBlock{q * 4 + d, (int)t0});
        a.btx = cnt.btx;
        a.bty = cnt.bty;
        a.bbase = bbase;
        bbase += (int)cnt.blocks(s);
        bmap.insert(bmap.end(), (size_t)cnt.blocks(s), q);
        a.bbase2 = bbase2;
        bbase2 += (int)cnt.blocks2(s);
        bmap2.insert(bmap2.end(), (size_t)cnt.blocks2(s), q);
        // checkpoint restore of segment k with u^n going to level buffer iu: u^n,
        // u^{n-1}, then psi_d and zeta_d of each axis, as the checkpoint stores them
        for (int k = 0; k < nck; ++k)
            for (int iu = 0; iu < 2; ++iu) {
                const char *ck = B + L.ck + (size_t)k * fdtd_state_bytes(s);
                char *dst[8] = {fdtd_ws(ctx, s.o_u[iu]), fdtd_ws(ctx, s.o_u[iu ^ 1])};
                size_t len[8] = {a256(s.elems * s.esz), a256(s.elems * s.esz)};
                for (int d = 0; d < 3; ++d) {
                    dst[2 + 2 * d] = fdtd_ws(ctx, s.o_psi[d]);
                    dst[3 + 2 * d] = fdtd_ws(ctx, s.o_zeta[d]);
                    len[2 + 2 * d] = len[3 + 2 * d] = a256(s.psi_elems[d] * 4);
                }
                size_t off = 0;
                for (int f = 0; f < 8; ++f) {
                    CopyJob &c = rjobs[(((size_t)k * 2 + iu) * 8 + f) * nsh + q];
                    c = flat_job(ck + off, dst[f], len[f]);
                    maxck = std::max(maxck, (long)c.ey);
                    off += len[f];
                }
            }
        // increments: level buffer qb minus the other one into slot j of half b
        for (int b = 0; b < 2; ++b)
            for (int j = 0; j < every + 1; ++j)
                for (int qb = 0; qb < 2; ++qb) {
                    DiffJob &c = jobs[((size_t)(b * (every + 1) + j) * 2 + qb) * nsh + q];
                    c.a = (const float *)fdtd_field_origin(ctx, s, s.o_u[qb]);
                    c.b = (const float *)fdtd_field_origin(ctx, s, s.o_u[qb ^ 1]);
                    c.d = (float *)(origin4(s, B + L.seg) + ((size_t)b * (every + 1) + j) * fb);
                    c.nx = s.nx;
                    c.ny = s.ny;
                    c.nz = s.nz;
                    c.P = s.P;
                    c.S = s.S;
                }
        maxrows = std::max(maxrows, (long)s.ny * s.nz);
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)std::min<long>(((long)s.nx * s.ny * s.nz + 255) / 256, 65536)),
                           dim3(256), 0, st, grad[q], (long)s.nx * s.ny * s.nz);
    }
    const ShotH &s0h = ctx->shots[sh[0]];
    const AdjLayout L0 = adj_layout(ctx, s0h, every, s0h.ck_count);
    const AdjShot *tab_d = (const AdjShot *)(s0h.ck_buf + L0.tab);
    const DiffJob *jobs_d = (const DiffJob *)(s0h.ck_buf + L0.jobs);
    const CopyJob *rjobs_d = (const CopyJob *)(s0h.ck_buf + L0.rjobs);
    const SlabBlock *smap_d = (const SlabBlock *)(s0h.ck_buf + L0.smap);
    const int *bmap_d = (const int *)(s0h.ck_buf + L0.bmap);
    const int *bmap2_d = (const int *)(s0h.ck_buf + L0.bmap2);
    const unsigned nslab = (unsigned)smap.size();
    AHIP(ctx, hipMemcpyAsync((void *)tab_d, tab.data(), sizeof(AdjShot) * nsh, hipMemcpyHostToDevice, st));
    AHIP(ctx, hipMemcpyAsync((void *)jobs_d, jobs.data(), sizeof(DiffJob) * jobs.size(), hipMemcpyHostToDevice, st));
    AHIP(ctx, hipMemcpyAsync((void *)rjobs_d, rjobs.data(), sizeof(CopyJob) * rjobs.size(), hipMemcpyHostToDevice,
                             st));
    if (!smap.empty())
        AHIP(ctx, hipMemcpyAsync((void *)smap_d, smap.data(), sizeof(SlabBlock) * smap.size(), hipMemcpyHostToDevice,
                                 st));
    AHIP(ctx, hipMemcpyAsync((void *)bmap_d, bmap.data(), sizeof(int) * bmap.size(), hipMemcpyHostToDevice, st));
    AHIP(ctx, hipMemcpyAsync((void *)bmap2_d, bmap2.data(), sizeof(int) * bmap2.size(), hipMemcpyHostToDevice, st));
    AHIP(ctx, hipStreamSynchronize(st));
    // e of the newest level (in buffer qb) into slot j of half b, every shot in one launch
    auto store_increment = [&](int b, int j, int qb) {
        hipLaunchKernelGGL(k_adj_diff, dim3((unsigned)std::min<long>(maxrows, 2048), nsh), dim3(256), 0, st,
                           jobs_d + ((size_t)(b * (every + 1) + j) * 2 + qb) * nsh);
    };

    // the context's step count and level roles, restored on exit: the other shots
    // of the context keep their forward state
    const long step_in = ctx->step;
    const int iu_in = ctx->iu, ium1_in = ctx->ium1;
    const bool was_saving = ctx->saving;
    ctx->saving = false;
    const int step_shot = nsh == nctx ? -1 : sh[0];
    int *stepc = (int *)fdtd_ws(ctx, ctx->o_stepc);
    hipStream_t sa = st;
    if (!ctx->single_stream) {
        if (!ctx->adj_stream) {
            AHIP(ctx, hipStreamCreateWithFlags(&ctx->adj_stream, hipStreamNonBlocking));
            for (auto &e : ctx->ev_adj) AHIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        sa = ctx->adj_stream;
        AHIP(ctx, hipEventRecord(ctx->ev_adj[4], st));   // the set-up above, before any sweep
        AHIP(ctx, hipStreamWaitEvent(sa, ctx->ev_adj[4], 0));
    }
    const int M = mu_slots(every), chunk = grad_chunk(every);
    for (int k = nck - 1; k >= 0; --k) {
        const int s0 = k * every, s1 = std::min(s0 + every, nt);
        const int b = k & 1;
        if (sa != st && k + 2 <= nck - 1) AHIP(ctx, hipStreamWaitEvent(st, ctx->ev_adj[2 + b], 0));
        // restore the states before step s0 (one copy launch for every shot), then
        // recompute the segment's levels
        fdtd_launch_copy_jobs(rjobs_d + ((size_t)k * 2 + ctx->iu) * 8 * nsh, 8 * nsh, maxck, st);
        fdtd_launch_set_int(stepc, s0, st);
        ctx->step = s0;
        store_increment(b, 0, ctx->iu);   // e^{s0} = u^{s0} - u^{s0 - 1}
        for (int n = s0; n < s1; ++n) {
            fdtd_enqueue_step_shot(ctx, step_shot);
            store_increment(b, n - s0 + 1, ctx->iu);   // e^{n+1}
        }
        if (sa != st) {
            AHIP(ctx, hipEventRecord(ctx->ev_adj[b], st));
            AHIP(ctx, hipStreamWaitEvent(sa, ctx->ev_adj[b], 0));
        }
        // reverse sweep over the segment; after every `chunk` steps (and at the
        // segment's start) the gradient pass folds the steps since the last one
        // into G, while their mu^{n+1} are still in the ring (the ring holds the
        // chunk's cnt + 1 <= M levels n .. n + cnt)
        int top = s1 - 1;
        for (int n = s1 - 1; n >= s0; --n) {
            const AdjStep as{n, n % M, (n + 1) % M, (n + 2) % M};
            if (maxg > 0) hipLaunchKernelGGL(k_adj_resid, dim3((maxg + 255) / 256, nsh), dim3(256), 0, sa, tab_d, as);
            if (nslab > 0) {
                hipLaunchKernelGGL(k_adj_p1, dim3(nslab), dim3(256), 0, sa, tab_d, smap_d, as);
                hipLaunchKernelGGL(k_adj_p2, dim3(nslab), dim3(256), 0, sa, tab_d, smap_d, as);
            }
            hipLaunchKernelGGL(k_adj_p3, dim3((unsigned)bbase2), dim3(256), 0, sa, tab_d, bmap2_d, as);
            if (top - n + 1 == chunk || n == s0) {
                const AdjGrad ag{b, s0, n, top - n + 1};
                hipLaunchKernelGGL(k_adj_grad, dim3((unsigned)bbase), dim3(256), 0, sa, tab_d, bmap_d, ag);
                top = n - 1;
            }
        }
        if (sa != st) AHIP(ctx, hipEventRecord(ctx->ev_adj[2 + b], sa));
        AHIP(ctx, hipGetLastError());
    }
    if (sa != st) {
        AHIP(ctx, hipEventRecord(ctx->ev_adj[4], sa));
        AHIP(ctx, hipStreamWaitEvent(st, ctx->ev_adj[4], 0));
    }
    for (int q = 0; q < nsh; ++q) {
        const ShotH &s = ctx->shots[sh[q]];
        hipLaunchKernelGGL(k_adj_finish, dim3((s.nx + 255) / 256, s.ny, s.nz), dim3(256), 0, st, dd + sh[q], grad[q],
                           s.c.dt);
    }
    ctx->saving = was_saving;
    ctx->step = step_in;
    ctx->iu = iu_in;
    ctx->ium1 = ium1_in;
    fdtd_launch_set_int(stepc, (int)step_in, st);
    fdtd_clear_graphs(ctx);
    for (int q = 0; q < nsh; ++q) {
        ctx->hdesc[sh[q]] = saved[q];
        AHIP(ctx, hipMemcpyAsync(dd + sh[q], &ctx->hdesc[sh[q]], sizeof(DevShot), hipMemcpyHostToDevice, st));
    }
    AHIP(ctx, hipStreamSynchronize(st));
    AHIP(ctx, hipGetLastError());
    return FDTD_OK;
}

extern "C" {

int fdtd_adjoint_workspace_size(const fdtd_ctx *ctx, int32_t shot, int32_t every, int32_t nt, size_t *bytes) {
    if (!ctx || !bytes || shot < 0 || shot >= (int)ctx->shots.size() || every <= 0 || nt <= 0) return FDTD_EINVAL;
    *bytes = adj_layout(ctx, ctx->shots[shot], every, (nt + every - 1) / every).total;
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
    while (adj_layout(ctx, s, every, nck + 1).total <= bytes && nck < (1 << 20)) ++nck;
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
    return adjoint_sweep(ctx, std::vector<int>{shot}, nt, &resid_dev, &grad_v_dev);
}

int fdtd_adjoint_batch(fdtd_ctx *ctx, int32_t nt, const float *const *resid_dev, double *const *grad_v_dev) {
    if (!ctx || nt <= 0 || !resid_dev || !grad_v_dev) return FDTD_EINVAL;
    std::vector<int> sh(ctx->shots.size());
    for (size_t i = 0; i < sh.size(); ++i) sh[i] = (int)i;
    return adjoint_sweep(ctx, sh, nt, resid_dev, grad_v_dev);
}

}  // extern "C"
