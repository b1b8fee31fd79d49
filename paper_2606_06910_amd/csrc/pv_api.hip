// pv_api.hip -- the paper's first-order pressure-velocity FDTD + CPML on gfx950
// (paper, section "Model", subsection "First-Order Acoustic Model and Discrete
// Update", and section "CPML Boundary Layers").  The C ABI is declared in
// include/fdtd_pv.h.
//
//  k_pv_vel   velocity stage: v_d -= lambda (kinv_d delta_d p + psi_v,d), the
//             memory variable advanced first inside axis d's layer
//  k_pv_pres  pressure stage: p -= lambda sum_d (kinv_d delta_d v_d + psi_p,d),
//             then the point source
//  k_pv_vel_zm, k_pv_pres_zm  the same stages z-marching: register queue of
//             the z taps, x / y taps from an LDS plane (the default variant)
//  k_pv_rec   receiver gather
//
// Layout: every field x fastest with a zero frame of 4 points on each side
// (row pitch P >= nx + 4 so that x = -4 .. -1 reads the previous row's zero
// tail; 4 frame rows and planes on y and z), 256-byte aligned rows.  One
// thread per point; the neighbours of a stencil come through the caches.
#include "../../include/fdtd.h"
#include "../../include/fdtd_pv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

namespace {

constexpr int kR = 4;        // stencil radius
constexpr int kLead = 128;   // leading pad of every field (elements)
constexpr int kNF = 10;      // p, v_x, v_y, v_z, psi_v x3, psi_p x3
constexpr int kRY = 1;       // z-march: rows per thread
constexpr int kNW = 8;       // z-march: waves per workgroup
constexpr int kTY = kRY * kNW;          // tile rows (tile: 64 x kTY)
constexpr int kLW = 64 + 2 * kR;        // LDS row length with the x halo
constexpr int kLH = kTY + 2 * kR;       // LDS rows with the y halo
constexpr int kZC = 16;                 // z-march: planes per chunk (measured: 8 .. 64)

// central first-derivative weights of order 8 at unit spacing (a_1 .. a_4)
constexpr double kA1[kR + 1] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

struct PvArgs {
    float *p;
    float *v[3];
    float *psv[3];          // memory of the pressure derivatives (velocity stage)
    float *psp[3];          // memory of the velocity derivatives (pressure stage)
    const float *prof;      // [axis][b, a, kinv][nmax]
    const float *wav;       // source samples (or null)
    int n[3], lo[3], hi[3];
    int src[3];
    int nmax, wav_n, step;
    long P, S;              // row and plane pitch (elements)
    float lam;
    float w[kR + 1];
};

__device__ __forceinline__ bool pv_slab(int c, int n, int lo, int hi) {
    return (lo > 0 && c < lo) || (hi > 0 && c >= n - hi);
}

// delta_d f at element i: sum_l a_l (f_{i+l st} - f_{i-l st})
__device__ __forceinline__ float pv_delta(const float *__restrict__ f, long i, long st, const float *w) {
    float acc = w[1] * (f[i + st] - f[i - st]);
#pragma unroll
    for (int l = 2; l <= kR; ++l) acc = fmaf(w[l], f[i + l * st] - f[i - l * st], acc);
    return acc;
}

// kinv_d g + psi_d, psi_d <- b psi_d + a g first (inside the layer of axis d only)
__device__ __forceinline__ float pv_stretched(const PvArgs &g, int d, int c, float grad, float *psi, long i) {
    if (!pv_slab(c, g.n[d], g.lo[d], g.hi[d])) return grad;
    const float *pr = g.prof + (long)d * 3 * g.nmax;
    const float ps = fmaf(pr[c], psi[i], pr[g.nmax + c] * grad);
    psi[i] = ps;
    return fmaf(pr[2 * g.nmax + c], grad, ps);
}

// grid: (ceil(nx / 64), ceil(ny / 4), nz), block 64 x 4
__global__ __launch_bounds__(256) void k_pv_vel(PvArgs g) {
    const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y, z = blockIdx.z;
    if (x >= g.n[0] || y >= g.n[1]) return;
    const long i = (long)z * g.S + (long)y * g.P + x;
    const int c[3] = {x, y, z};
    const long st[3] = {1, g.P, g.S};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float t = pv_stretched(g, d, c[d], pv_delta(g.p, i, st[d], g.w), g.psv[d], i);
        g.v[d][i] = fmaf(-g.lam, t, g.v[d][i]);
    }
}

__global__ __launch_bounds__(256) void k_pv_pres(PvArgs g) {
    const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y, z = blockIdx.z;
    if (x >= g.n[0] || y >= g.n[1]) return;
    const long i = (long)z * g.S + (long)y * g.P + x;
    const int c[3] = {x, y, z};
    const long st[3] = {1, g.P, g.S};
    float div = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) div += pv_stretched(g, d, c[d], pv_delta(g.v[d], i, st[d], g.w), g.psp[d], i);
    float pn = fmaf(-g.lam, div, g.p[i]);
    if (g.wav && g.step < g.wav_n && x == g.src[0] && y == g.src[1] && z == g.src[2])
        pn = fmaf(g.lam, g.wav[g.step], pn);
    g.p[i] = pn;
}

// ---------------------------------------------------------------------------
// z-marching stages.  A workgroup of kNW waves owns a 64 x kTY xy tile and a
// chunk of kZC planes; lane l of wave w owns column x0 + l and rows
// w kRY .. w kRY + kRY - 1 (one row at kRY = 1: more resident waves beat
// more rows per thread).  The z taps come from a register queue of the
// field's planes z - 4 .. z + 4 (own rows), the x and y taps from the plane z
// staged in LDS with its halo (two buffers: one barrier per plane).  Every
// tap is summed in the order of pv_delta, so the results equal the
// one-thread-per-point kernels bit for bit.  Points outside the grid (tile
// overhang) compute on the zero frame and store nothing.
// grid: (ceil(nx / 64), ceil(ny / kTY), ceil(nz / kZC)), block 64 x kNW
// ---------------------------------------------------------------------------
__device__ __forceinline__ float zm_d(const float *w, float a1, float b1, float a2, float b2, float a3, float b3,
                                      float a4, float b4) {
    // sum_l w_l (a_l - b_l), a = f_{+l}, b = f_{-l}, in pv_delta's order
    float acc = w[1] * (a1 - b1);
    acc = fmaf(w[2], a2 - b2, acc);
    acc = fmaf(w[3], a3 - b3, acc);
    acc = fmaf(w[4], a4 - b4, acc);
    return acc;
}

// halo slots of a plane: x halo (4 columns each side, kTY rows), y halo (4 rows
// each side, 64 columns); 'xh' / 'yh' select which are staged
template <bool XH, bool YH> struct Halo {
    static constexpr int NX = XH ? 2 * kR * kTY : 0;
    static constexpr int NY = YH ? 2 * kR * 64 : 0;
    static constexpr int N = NX + NY;
    static constexpr int PER = (N + 64 * kNW - 1) / (64 * kNW);
};

constexpr long kNoHalo = -(1L << 62);   // halo slot without a value (reads as zero)

template <bool XH, bool YH>
__device__ __forceinline__ void halo_setup(int t, int x0, int y0, long P, long (&off)[Halo<XH, YH>::PER],
                                           int (&slot)[Halo<XH, YH>::PER]) {
    using H = Halo<XH, YH>;
#pragma unroll
    for (int k = 0; k < H::PER; ++k) {
        const int i = t + 64 * kNW * k;
        off[k] = kNoHalo;
        slot[k] = kLH * kLW;            // dummy slot
        if (i < H::NX) {
            const int row = i / (2 * kR), c8 = i % (2 * kR);
            const int lx = c8 < kR ? c8 - kR : 64 + (c8 - kR);
            slot[k] = (row + kR) * kLW + lx + kR;
            off[k] = (long)(y0 + row) * P + x0 + lx;
        } else if (i < H::N) {
            const int j = i - H::NX, r8 = j / 64, c = j % 64;
            const int ly = r8 < kR ? r8 - kR : kTY + (r8 - kR);
            slot[k] = (ly + kR) * kLW + c + kR;
            off[k] = (long)(y0 + ly) * P + x0 + c;
        }
    }
}

__global__ __launch_bounds__(64 * kNW) void k_pv_vel_zm(PvArgs g) {
    using H = Halo<true, true>;
    __shared__ float sm[2][kLH * kLW + 1];
    const int lane = threadIdx.x, wv = threadIdx.y, t = wv * 64 + lane;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kTY;
    const int za = blockIdx.z * kZC, zb = min(za + kZC, g.n[2]);
    const int x = x0 + lane;
    const long P = g.P, S = g.S;
    long hoff[H::PER];
    int hslot[H::PER];
    halo_setup<true, true>(t, x0, y0, P, hoff, hslot);
    float q[2 * kR + 1][kRY];     // p at z - 4 .. z + 4, own rows
    float hq[H::PER];             // halo of plane z
#pragma unroll
    for (int o = 0; o < 2 * kR + 1; ++o)
#pragma unroll
        for (int r = 0; r < kRY; ++r) q[o][r] = g.p[(long)(za - kR + o) * S + (long)(y0 + wv * kRY + r) * P + x];
#pragma unroll
    for (int k = 0; k < H::PER; ++k) hq[k] = hoff[k] != kNoHalo ? g.p[(long)za * S + hoff[k]] : 0.0f;
    float vc[3][kRY];             // v_d of plane z, own rows (read, updated, written back)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int r = 0; r < kRY; ++r) vc[d][r] = g.v[d][(long)za * S + (long)(y0 + wv * kRY + r) * P + x];
    int buf = 0;
    for (int z = za; z < zb; ++z) {
        float *L = sm[buf];
#pragma unroll
        for (int r = 0; r < kRY; ++r) L[(wv * kRY + r + kR) * kLW + lane + kR] = q[kR][r];
#pragma unroll
        for (int k = 0; k < H::PER; ++k) L[hslot[k]] = hq[k];
        // loads ahead: p plane z + 5 (own rows) and the halo of plane z + 1
        float nq[kRY], nh[H::PER];
#pragma unroll
        for (int r = 0; r < kRY; ++r)   // (the last frame plane is nz + 3; plane nz + 4 is never used)
            nq[r] = z + kR + 1 <= g.n[2] + kR - 1 ? g.p[(long)(z + kR + 1) * S + (long)(y0 + wv * kRY + r) * P + x]
                                                  : 0.0f;
#pragma unroll
        for (int k = 0; k < H::PER; ++k) nh[k] = hoff[k] != kNoHalo ? g.p[(long)(z + 1) * S + hoff[k]] : 0.0f;
        float vn[3][kRY];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int r = 0; r < kRY; ++r) vn[d][r] = g.v[d][(long)(z + 1) * S + (long)(y0 + wv * kRY + r) * P + x];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRY; ++r) {
            const int y = y0 + wv * kRY + r;
            const float *c = L + (wv * kRY + r + kR) * kLW + lane + kR;
            const float gx = zm_d(g.w, c[1], c[-1], c[2], c[-2], c[3], c[-3], c[4], c[-4]);
            const float gy = zm_d(g.w, c[kLW], c[-kLW], c[2 * kLW], c[-2 * kLW], c[3 * kLW], c[-3 * kLW],
                                  c[4 * kLW], c[-4 * kLW]);
            const float gz = zm_d(g.w, q[kR + 1][r], q[kR - 1][r], q[kR + 2][r], q[kR - 2][r], q[kR + 3][r],
                                  q[kR - 3][r], q[kR + 4][r], q[kR - 4][r]);
            if (x < g.n[0] && y < g.n[1]) {
                const long i = (long)z * S + (long)y * P + x;
                const int cc[3] = {x, y, z};
                const float gr[3] = {gx, gy, gz};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float tt = pv_stretched(g, d, cc[d], gr[d], g.psv[d], i);
                    g.v[d][i] = fmaf(-g.lam, tt, vc[d][r]);
                }
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int r = 0; r < kRY; ++r) vc[d][r] = vn[d][r];
#pragma unroll
        for (int o = 0; o < 2 * kR; ++o)
#pragma unroll
            for (int r = 0; r < kRY; ++r) q[o][r] = q[o + 1][r];
#pragma unroll
        for (int r = 0; r < kRY; ++r) q[2 * kR][r] = nq[r];
#pragma unroll
        for (int k = 0; k < H::PER; ++k) hq[k] = nh[k];
        buf ^= 1;
    }
}

__global__ __launch_bounds__(64 * kNW) void k_pv_pres_zm(PvArgs g) {
    using HX = Halo<true, false>;
    using HY = Halo<false, true>;
    __shared__ float sx[2][kLH * kLW + 1];   // v_x plane with its x halo
    __shared__ float sy[2][kLH * kLW + 1];   // v_y plane with its y halo
    const int lane = threadIdx.x, wv = threadIdx.y, t = wv * 64 + lane;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kTY;
    const int za = blockIdx.z * kZC, zb = min(za + kZC, g.n[2]);
    const int x = x0 + lane;
    const long P = g.P, S = g.S;
    long xoff[HX::PER], yoff[HY::PER];
    int xslot[HX::PER], yslot[HY::PER];
    halo_setup<true, false>(t, x0, y0, P, xoff, xslot);
    halo_setup<false, true>(t, x0, y0, P, yoff, yslot);
    float q[2 * kR + 1][kRY];     // v_z at z - 4 .. z + 4, own rows
#pragma unroll
    for (int o = 0; o < 2 * kR + 1; ++o)
#pragma unroll
        for (int r = 0; r < kRY; ++r) q[o][r] = g.v[2][(long)(za - kR + o) * S + (long)(y0 + wv * kRY + r) * P + x];
    float cx[kRY], cy[kRY], hx[HX::PER], hy[HY::PER];   // plane z of v_x, v_y (own rows and halo)
#pragma unroll
    for (int r = 0; r < kRY; ++r) {
        const long o = (long)za * S + (long)(y0 + wv * kRY + r) * P + x;
        cx[r] = g.v[0][o];
        cy[r] = g.v[1][o];
    }
#pragma unroll
    for (int k = 0; k < HX::PER; ++k) hx[k] = xoff[k] != kNoHalo ? g.v[0][(long)za * S + xoff[k]] : 0.0f;
#pragma unroll
    for (int k = 0; k < HY::PER; ++k) hy[k] = yoff[k] != kNoHalo ? g.v[1][(long)za * S + yoff[k]] : 0.0f;
    float pc[kRY];                // p of plane z, own rows
#pragma unroll
    for (int r = 0; r < kRY; ++r) pc[r] = g.p[(long)za * S + (long)(y0 + wv * kRY + r) * P + x];
    int buf = 0;
    for (int z = za; z < zb; ++z) {
        float *LX = sx[buf], *LY = sy[buf];
#pragma unroll
        for (int r = 0; r < kRY; ++r) {
            LX[(wv * kRY + r + kR) * kLW + lane + kR] = cx[r];
            LY[(wv * kRY + r + kR) * kLW + lane + kR] = cy[r];
        }
#pragma unroll
        for (int k = 0; k < HX::PER; ++k) LX[xslot[k]] = hx[k];
#pragma unroll
        for (int k = 0; k < HY::PER; ++k) LY[yslot[k]] = hy[k];
        // loads ahead: v_z plane z + 5, v_x / v_y / p plane z + 1 (own rows and halo)
        float nq[kRY], pn1[kRY];
#pragma unroll
        for (int r = 0; r < kRY; ++r) {
            const long o = (long)(y0 + wv * kRY + r) * P + x;
            nq[r] = z + kR + 1 <= g.n[2] + kR - 1 ? g.v[2][(long)(z + kR + 1) * S + o] : 0.0f;
            cx[r] = g.v[0][(long)(z + 1) * S + o];
            cy[r] = g.v[1][(long)(z + 1) * S + o];
            pn1[r] = g.p[(long)(z + 1) * S + o];
        }
#pragma unroll
        for (int k = 0; k < HX::PER; ++k) hx[k] = xoff[k] != kNoHalo ? g.v[0][(long)(z + 1) * S + xoff[k]] : 0.0f;
#pragma unroll
        for (int k = 0; k < HY::PER; ++k) hy[k] = yoff[k] != kNoHalo ? g.v[1][(long)(z + 1) * S + yoff[k]] : 0.0f;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRY; ++r) {
            const int y = y0 + wv * kRY + r;
            const int li = (wv * kRY + r + kR) * kLW + lane + kR;
            const float *ax = LX + li, *ay = LY + li;
            const float gx = zm_d(g.w, ax[1], ax[-1], ax[2], ax[-2], ax[3], ax[-3], ax[4], ax[-4]);
            const float gy = zm_d(g.w, ay[kLW], ay[-kLW], ay[2 * kLW], ay[-2 * kLW], ay[3 * kLW], ay[-3 * kLW],
                                  ay[4 * kLW], ay[-4 * kLW]);
            const float gz = zm_d(g.w, q[kR + 1][r], q[kR - 1][r], q[kR + 2][r], q[kR - 2][r], q[kR + 3][r],
                                  q[kR - 3][r], q[kR + 4][r], q[kR - 4][r]);
            if (x < g.n[0] && y < g.n[1]) {
                const long i = (long)z * S + (long)y * P + x;
                const int cc[3] = {x, y, z};
                const float gr[3] = {gx, gy, gz};
                float div = 0.0f;
#pragma unroll
                for (int d = 0; d < 3; ++d) div += pv_stretched(g, d, cc[d], gr[d], g.psp[d], i);
                float pn = fmaf(-g.lam, div, pc[r]);
                if (g.wav && g.step < g.wav_n && x == g.src[0] && y == g.src[1] && z == g.src[2])
                    pn = fmaf(g.lam, g.wav[g.step], pn);
                g.p[i] = pn;
            }
        }
#pragma unroll
        for (int o = 0; o < 2 * kR; ++o)
#pragma unroll
            for (int r = 0; r < kRY; ++r) q[o][r] = q[o + 1][r];
#pragma unroll
        for (int r = 0; r < kRY; ++r) {
            q[2 * kR][r] = nq[r];
            pc[r] = pn1[r];
        }
        buf ^= 1;
    }
}

__global__ __launch_bounds__(256) void k_pv_rec(const float *__restrict__ p, const int32_t *__restrict__ rec,
                                               int nrec, long P, long S, float *__restrict__ out) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nrec; r += gridDim.x * blockDim.x)
        out[r] = p[(long)rec[3 * r + 2] * S + (long)rec[3 * r + 1] * P + rec[3 * r]];
}

// dense (nz, ny, nx) <-> padded field; grid (ceil(nx / 256), ny, nz)
__global__ __launch_bounds__(256) void k_pv_copy(float *__restrict__ dst, const float *__restrict__ src, int nx,
                                                int ny, long P, long S, int to_padded) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const long dense = ((long)blockIdx.z * ny + blockIdx.y) * nx + x;
    const long pad = (long)blockIdx.z * S + (long)blockIdx.y * P + x;
    if (to_padded) dst[pad] = src[dense];
    else dst[dense] = src[pad];
}

__global__ __launch_bounds__(256) void k_pv_zero(uint4 *p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// FP64 layer coefficients of one axis in the normalised units (h = 1, c = 1,
// dt = lambda); rho is sampled at the nodes: 1 at the outermost, steps of 1/L,
// no memory from node L inward
void pv_profile(int n, int lo, int hi, double lam, double R, double kmax, double af, float *b, float *a, float *kinv) {
    for (int i = 0; i < n; ++i) {
        int L = 0;
        double rho = 0.0;
        if (lo > 0 && i < lo) {
            L = lo;
            rho = (double)(lo - i) / lo;
        } else if (hi > 0 && i >= n - hi) {
            L = hi;
            rho = (double)(i - (n - 1 - hi)) / hi;
        }
        if (rho > 0) {
            const double sigma_max = -4.0 * std::log(R) / (2.0 * L);
            const double r3 = rho * rho * rho;
            const double sigma = sigma_max * r3, kappa = 1.0 + (kmax - 1.0) * r3;
            const double alpha = af * sigma_max * (1.0 - rho);
            const double bb = std::exp(-(sigma / kappa + alpha) * lam);
            b[i] = (float)bb;
            a[i] = (float)(sigma * (bb - 1.0) / (kappa * (sigma + kappa * alpha)));
            kinv[i] = (float)(1.0 / kappa);
        } else {
            b[i] = 0.0f;
            a[i] = 0.0f;
            kinv[i] = 1.0f;
        }
    }
}

// Largest lambda for which the 3-D leapfrog of the two stages keeps every
// Fourier mode bounded.  A mode exp(i k.x) sees delta_d as i s(k_d) with
// s(theta) = 2 sum_l a_l sin(l theta); eliminating v gives
// p^{n+1} - 2 p^n + p^{n-1} = -lambda^2 S^2 p^n, S^2 = sum_d s(k_d)^2, which is
// bounded iff lambda^2 S^2 <= 4.  S^2 reaches 3 max(s)^2, so the limit is
// 2 / (sqrt(3) max s).  The maximum of s is found by a dense scan of
// [0, pi] refined by golden-section search around the best sample.
double pv_lambda_limit() {
    auto sym = [](double t) {
        double acc = 0.0;
        for (int l = 1; l <= kR; ++l) acc += 2.0 * kA1[l] * std::sin(l * t);
        return acc;
    };
    const int M = 4096;
    const double pi = 3.14159265358979323846;
    int best = 0;
    for (int i = 1; i <= M; ++i)
        if (sym(pi * i / M) > sym(pi * best / M)) best = i;
    double lo = pi * std::max(best - 1, 0) / M, hi = pi * std::min(best + 1, M) / M;
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int it = 0; it < 100; ++it) {
        const double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
        if (sym(c) > sym(d)) hi = d;
        else lo = c;
    }
    return 2.0 / (std::sqrt(3.0) * sym(0.5 * (lo + hi)));
}

}  // namespace

struct fdtd_pv_ctx {
    fdtd_pv_config c{};
    hipStream_t st = nullptr;
    std::string err;
    int n[3] = {}, lo[3] = {}, hi[3] = {};
    int nmax = 0;
    long P = 0, S = 0;
    size_t elems = 0, field_bytes = 0, prof_bytes = 0, total = 0;
    std::vector<float> prof;
    char *ws = nullptr;
    int src[3] = {-1, -1, -1};
    const float *wav = nullptr;
    int wav_n = 0;
    const int32_t *rec = nullptr;
    int nrec = 0;
    float *traces = nullptr;
    int cap = 0;
    long step = 0;       // steps since the workspace was bound (source sample index)
    long rec0 = 0;       // step at which the receivers were set (trace row 0)

    float *field(int f) const { return (float *)(ws + (size_t)f * field_bytes) + kLead + 4 * S + 4 * P; }
};

#define PVFAIL(ctx, code, ...)                                                                               \
    do {                                                                                                      \
        char _b[512];                                                                                         \
        snprintf(_b, sizeof _b, __VA_ARGS__);                                                                 \
        (ctx)->err = _b;                                                                                      \
        return (code);                                                                                        \
    } while (0)
#define PVHIP(ctx, expr)                                                                                      \
    do {                                                                                                      \
        hipError_t _e = (expr);                                                                               \
        if (_e != hipSuccess) PVFAIL(ctx, FDTD_EHIP, "%s: %s", #expr, hipGetErrorString(_e));                 \
    } while (0)

static PvArgs pv_args(const fdtd_pv_ctx *ctx) {
    PvArgs g;
    g.p = ctx->field(0);
    for (int d = 0; d < 3; ++d) {
        g.v[d] = ctx->field(1 + d);
        g.psv[d] = ctx->field(4 + d);
        g.psp[d] = ctx->field(7 + d);
        g.n[d] = ctx->n[d];
        g.lo[d] = ctx->lo[d];
        g.hi[d] = ctx->hi[d];
        g.src[d] = ctx->src[d];
    }
    g.prof = (const float *)(ctx->ws + (size_t)kNF * ctx->field_bytes);
    g.wav = ctx->wav;
    g.wav_n = ctx->wav_n;
    g.nmax = ctx->nmax;
    g.step = (int)ctx->step;
    g.P = ctx->P;
    g.S = ctx->S;
    g.lam = (float)ctx->c.lambda;
    for (int l = 0; l <= kR; ++l) g.w[l] = (float)kA1[l];
    return g;
}

extern "C" {

int fdtd_pv_create(const fdtd_pv_config *cfg, void *hip_stream, fdtd_pv_ctx **out) {
    if (!cfg || !out) return FDTD_EINVAL;
    *out = nullptr;
    for (int d = 0; d < 3; ++d) {
        const int n = cfg->n[d], lo = cfg->cpml[2 * d], hi = cfg->cpml[2 * d + 1];
        // (the per-point stages launch one workgroup row per plane: nz stays below the grid limit)
        if (n < 9 || n > (1 << 15) || lo < 0 || hi < 0 || lo + hi >= n) return FDTD_EINVAL;
    }
    if (!(cfg->lambda > 0.0)) return FDTD_EINVAL;
    if (cfg->lambda > pv_lambda_limit()) {
        fprintf(stderr, "fdtd_pv_create: lambda = %g above the stability limit %.6f\n", cfg->lambda,
                pv_lambda_limit());
        return FDTD_EUNSTABLE;
    }
    if (cfg->R < 0 || cfg->R >= 1 || cfg->kappa_max < 0 || cfg->alpha_frac < 0) return FDTD_EINVAL;
    if (cfg->variant < 0 || cfg->variant > 2) return FDTD_EINVAL;
    fdtd_pv_ctx *ctx = new fdtd_pv_ctx;
    ctx->c = *cfg;
    if (ctx->c.R == 0) ctx->c.R = 1e-8;
    if (ctx->c.kappa_max == 0) ctx->c.kappa_max = 5.0;
    if (ctx->c.alpha_frac == 0) ctx->c.alpha_frac = 0.05;
    ctx->st = (hipStream_t)hip_stream;
    for (int d = 0; d < 3; ++d) {
        ctx->n[d] = cfg->n[d];
        ctx->lo[d] = cfg->cpml[2 * d];
        ctx->hi[d] = cfg->cpml[2 * d + 1];
    }
    ctx->nmax = std::max(ctx->n[0], std::max(ctx->n[1], ctx->n[2]));
    ctx->P = (long)((ctx->n[0] + kR + 63) / 64) * 64;
    ctx->S = (long)(ctx->n[1] + 2 * kR) * ctx->P;
    // trailing pad: a z-march tile may overhang the last row by up to kTY - 1 rows (plus its halo)
    ctx->elems = (size_t)kLead + (size_t)(ctx->n[2] + 2 * kR) * ctx->S + (size_t)(kTY + 2 * kR) * ctx->P + 128;
    ctx->field_bytes = a256(ctx->elems * 4);
    ctx->prof_bytes = a256((size_t)3 * 3 * ctx->nmax * 4);
    ctx->total = (size_t)kNF * ctx->field_bytes + ctx->prof_bytes;
    ctx->prof.assign((size_t)3 * 3 * ctx->nmax, 0.0f);
    for (int d = 0; d < 3; ++d) {
        float *base = ctx->prof.data() + (size_t)d * 3 * ctx->nmax;
        pv_profile(ctx->n[d], ctx->lo[d], ctx->hi[d], ctx->c.lambda, ctx->c.R, ctx->c.kappa_max, ctx->c.alpha_frac,
                   base, base + ctx->nmax, base + 2 * ctx->nmax);
    }
    *out = ctx;
    return FDTD_OK;
}

int fdtd_pv_workspace_size(const fdtd_pv_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return FDTD_EINVAL;
    *bytes = ctx->total;
    return FDTD_OK;
}

int fdtd_pv_bind_workspace(fdtd_pv_ctx *ctx, void *dev_ptr, size_t bytes) {
    if (!ctx || !dev_ptr) return FDTD_EINVAL;
    if (((uintptr_t)dev_ptr) & 255) PVFAIL(ctx, FDTD_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < ctx->total) PVFAIL(ctx, FDTD_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, ctx->total);
    ctx->ws = (char *)dev_ptr;
    const size_t n16 = ((size_t)kNF * ctx->field_bytes) / 16;
    hipLaunchKernelGGL(k_pv_zero, dim3((unsigned)std::min<size_t>((n16 + 255) / 256, 65536)), dim3(256), 0, ctx->st,
                       (uint4 *)ctx->ws, n16);
    PVHIP(ctx, hipGetLastError());
    PVHIP(ctx, hipMemcpyAsync(ctx->ws + (size_t)kNF * ctx->field_bytes, ctx->prof.data(), ctx->prof.size() * 4,
                              hipMemcpyHostToDevice, ctx->st));
    PVHIP(ctx, hipStreamSynchronize(ctx->st));
    ctx->step = 0;
    ctx->rec0 = 0;
    return FDTD_OK;
}

static int pv_copy(fdtd_pv_ctx *ctx, float *dst, const float *src, int to_padded) {
    if (!ctx->ws) PVFAIL(ctx, FDTD_ESTATE, "no workspace bound");
    hipLaunchKernelGGL(k_pv_copy, dim3((ctx->n[0] + 255) / 256, ctx->n[1], ctx->n[2]), dim3(256), 0, ctx->st, dst,
                       src, ctx->n[0], ctx->n[1], ctx->P, ctx->S, to_padded);
    PVHIP(ctx, hipGetLastError());
    return FDTD_OK;
}

int fdtd_pv_set_pressure(fdtd_pv_ctx *ctx, const float *p_dev) {
    if (!ctx || !p_dev) return FDTD_EINVAL;
    return pv_copy(ctx, ctx->ws ? ctx->field(0) : nullptr, p_dev, 1);
}

int fdtd_pv_get_pressure(fdtd_pv_ctx *ctx, float *p_dev) {
    if (!ctx || !p_dev) return FDTD_EINVAL;
    return pv_copy(ctx, p_dev, ctx->ws ? ctx->field(0) : nullptr, 0);
}

int fdtd_pv_set_source(fdtd_pv_ctx *ctx, int32_t i, int32_t j, int32_t k, const float *w_dev, int32_t nt) {
    if (!ctx || !w_dev || nt <= 0) return FDTD_EINVAL;
    if (i < 0 || i >= ctx->n[0] || j < 0 || j >= ctx->n[1] || k < 0 || k >= ctx->n[2])
        PVFAIL(ctx, FDTD_EINVAL, "source (%d,%d,%d) outside the grid", i, j, k);
    ctx->src[0] = i;
    ctx->src[1] = j;
    ctx->src[2] = k;
    ctx->wav = w_dev;
    ctx->wav_n = nt;
    return FDTD_OK;
}

int fdtd_pv_set_receivers(fdtd_pv_ctx *ctx, const int32_t *rec_dev, int32_t nrec, float *traces_dev, int32_t cap) {
    if (!ctx || nrec < 0 || cap < 0 || (nrec > 0 && (!rec_dev || !traces_dev))) return FDTD_EINVAL;
    if (nrec > 0) {
        std::vector<int32_t> h((size_t)nrec * 3);
        PVHIP(ctx, hipMemcpyAsync(h.data(), rec_dev, h.size() * 4, hipMemcpyDeviceToHost, ctx->st));
        PVHIP(ctx, hipStreamSynchronize(ctx->st));
        for (int r = 0; r < nrec; ++r)
            for (int d = 0; d < 3; ++d)
                if (h[3 * r + d] < 0 || h[3 * r + d] >= ctx->n[d])
                    PVFAIL(ctx, FDTD_EINVAL, "receiver %d outside the grid", r);
    }
    ctx->rec = rec_dev;
    ctx->nrec = nrec;
    ctx->traces = traces_dev;
    ctx->cap = cap;
    ctx->rec0 = ctx->step;
    return FDTD_OK;
}

int fdtd_pv_step(fdtd_pv_ctx *ctx, int32_t nsteps) {
    if (!ctx || nsteps < 0) return FDTD_EINVAL;
    if (!ctx->ws) PVFAIL(ctx, FDTD_ESTATE, "no workspace bound");
    const dim3 grid((ctx->n[0] + 63) / 64, (ctx->n[1] + 3) / 4, ctx->n[2]), block(64, 4);
    const dim3 zgrid((ctx->n[0] + 63) / 64, (ctx->n[1] + kTY - 1) / kTY, (ctx->n[2] + kZC - 1) / kZC),
        zblock(64, kNW);
    // automatic choice: the z-march from 2^24 points up (measured crossover between
    // 224^3 and 256^3: below it its workgroups fill the chip in too few rounds)
    const double npts = (double)ctx->n[0] * ctx->n[1] * ctx->n[2];
    const bool naive = ctx->c.variant == 1 || (ctx->c.variant == 0 && npts < (double)(1L << 24));
    for (int s = 0; s < nsteps; ++s) {
        PvArgs g = pv_args(ctx);
        if (naive) {
            hipLaunchKernelGGL(k_pv_vel, grid, block, 0, ctx->st, g);
            hipLaunchKernelGGL(k_pv_pres, grid, block, 0, ctx->st, g);
        } else {
            hipLaunchKernelGGL(k_pv_vel_zm, zgrid, zblock, 0, ctx->st, g);
            hipLaunchKernelGGL(k_pv_pres_zm, zgrid, zblock, 0, ctx->st, g);
        }
        const long row = ctx->step - ctx->rec0;
        if (ctx->nrec > 0 && row < ctx->cap)
            hipLaunchKernelGGL(k_pv_rec, dim3((ctx->nrec + 255) / 256), dim3(256), 0, ctx->st, (const float *)g.p,
                               ctx->rec, ctx->nrec, ctx->P, ctx->S, ctx->traces + (size_t)row * ctx->nrec);
        ++ctx->step;
    }
    PVHIP(ctx, hipGetLastError());
    return FDTD_OK;
}

const char *fdtd_pv_last_error(const fdtd_pv_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void fdtd_pv_destroy(fdtd_pv_ctx *ctx) { delete ctx; }

}  // extern "C"
