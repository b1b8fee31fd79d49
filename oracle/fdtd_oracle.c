/*
 * fdtd_oracle.c -- FP64 reference for the second-order acoustic FDTD + CPML step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes (paper: "Model", first-order system and its implied scalar
 * wave equation p_tt = c^2 Lap p; "FDTD Verification", standing-wave MMS):
 *
 *   u^{n+1} = 2 u^n - u^{n-1} + m * sum_d Lt_d(u^n) + m * f^n,   m = v^2 dt^2
 *
 * with the radius-r central stencils of the paper's delta^(2r) operator
 * (section "First-Order Acoustic Model and Discrete Update") and, inside the
 * absorbing layer, the CFS/Roden-Gedney stretched derivative of section
 * "CPML Boundary Layers" applied twice (second-order form, kappa-inclusive):
 *
 *   psi_d  <- b_d psi_d  + a_d D1_d u^n                     (update, then use)
 *   eta_d   = kinv_d D2_d u^n + dkinv_d D1_d u^n + D1_d psi_d
 *   zeta_d <- b_d zeta_d + a_d eta_d
 *   Lt_d    = kinv_d eta_d + zeta_d
 *
 * psi_d, zeta_d live only where the layer coordinate rho_d > 0; elsewhere
 * kinv=1, dkinv=0, a=0 and Lt_d reduces to D2_d u exactly.  Profiles follow
 * the CPML section's sigma/kappa/alpha grading and its a,b recursion
 * coefficients, evaluated in FP64.
 *
 * Conventions taken where the paper is silent (the same list is kept with
 * the design notes):
 *   - finite-difference weights: standard central (Fornberg) weights of
 *     order 2r for the first and second derivative;
 *   - rho is node based: rho = 1 at the outermost node, step 1/L;
 *   - sigma_max = -(q+1) v_ref ln(R) / (2 L h), q = 3, natural log;
 *   - a = 0 wherever sigma = 0;
 *   - faces outside [0,n) are zero Dirichlet, or periodic per axis;
 *   - source: f^n = A w_n / (hx hy hz) at one node, added after the update.
 *
 * Arrays are x-fastest: idx = i + nx*(j + ny*k).  All arithmetic is double.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the loops below use. */
int og_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

typedef struct {
    int n[3];          /* nx, ny, nz                                      */
    double h[3];       /* spacing per axis (m)                            */
    double dt;         /* time step (s)                                   */
    int r;             /* stencil radius, 1..4 (the method uses 4)        */
    int periodic[3];   /* 1 = periodic axis, 0 = zero Dirichlet           */
    int cpml[6];       /* layer width per face: -x,+x,-y,+y,-z,+z          */
    double R;          /* target reflection (1e-8)                        */
    double kappa_max;  /* 5                                               */
    double alpha_frac; /* alpha_max / sigma_max (0.05)                    */
    double vref;       /* velocity scaling sigma_max (max of the model)   */
} og_t;

/* ---- finite-difference weights ---------------------------------------- */
/* Central weights for the first derivative (d1[1..r]) and the second
 * derivative (d2[0..r]) of spatial order 2r.  These are the classical
 * rational coefficients; the tests pin them by polynomial exactness and by
 * the paper's printed spatial-convergence table.                           */
int og_weights(int r, double *d1, double *d2)
{
    static const double D1[5][5] = {
        {0, 0, 0, 0, 0},
        {0, 1.0 / 2.0, 0, 0, 0},
        {0, 2.0 / 3.0, -1.0 / 12.0, 0, 0},
        {0, 3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0, 0},
        {0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0},
    };
    static const double D2[5][5] = {
        {0, 0, 0, 0, 0},
        {-2.0, 1.0, 0, 0, 0},
        {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0, 0, 0},
        {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0, 0},
        {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0},
    };
    if (r < 1 || r > 4) return -1;
    for (int l = 0; l <= r; ++l) {
        d1[l] = D1[r][l];
        d2[l] = D2[r][l];
    }
    return 0;
}

static long og_npts(const og_t *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

/* Value of f at integer coordinates, with the face rule applied. */
static double og_at(const og_t *g, const double *f, long c[3])
{
    long q[3];
    for (int d = 0; d < 3; ++d) {
        long n = g->n[d], x = c[d];
        if (x < 0 || x >= n) {
            if (!g->periodic[d]) return 0.0;
            x = ((x % n) + n) % n;
        }
        q[d] = x;
    }
    return f[q[0] + g->n[0] * (q[1] + (long)g->n[1] * q[2])];
}

/* D1 along axis d at point c:  sum_l d1_l (f(c+l e_d) - f(c-l e_d)) / h_d */
static double og_d1_at(const og_t *g, const double *w1, int d, const double *f, const long c[3])
{
    double s = 0.0;
    for (int l = 1; l <= g->r; ++l) {
        long p[3] = {c[0], c[1], c[2]}, m[3] = {c[0], c[1], c[2]};
        p[d] += l;
        m[d] -= l;
        s += w1[l] * (og_at(g, f, p) - og_at(g, f, m));
    }
    return s / g->h[d];
}

/* D2 along axis d at point c:  (d2_0 f(c) + sum_l d2_l (f(c+l) + f(c-l))) / h_d^2 */
static double og_d2_at(const og_t *g, const double *w2, int d, const double *f, const long c[3])
{
    long cc[3] = {c[0], c[1], c[2]};
    double s = w2[0] * og_at(g, f, cc);
    for (int l = 1; l <= g->r; ++l) {
        long p[3] = {c[0], c[1], c[2]}, m[3] = {c[0], c[1], c[2]};
        p[d] += l;
        m[d] -= l;
        s += w2[l] * (og_at(g, f, p) + og_at(g, f, m));
    }
    return s / (g->h[d] * g->h[d]);
}

static void og_coords(const og_t *g, long idx, long c[3])
{
    c[0] = idx % g->n[0];
    c[1] = (idx / g->n[0]) % g->n[1];
    c[2] = idx / ((long)g->n[0] * g->n[1]);
}

/* Whole-grid first / second derivative along one axis, and the Laplacian. */
int og_deriv1(const og_t *g, int d, const double *f, double *out)
{
    double w1[5], w2[5];
    if (og_weights(g->r, w1, w2)) return -1;
    long N = og_npts(g);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        long c[3];
        og_coords(g, i, c);
        out[i] = og_d1_at(g, w1, d, f, c);
    }
    return 0;
}

int og_deriv2(const og_t *g, int d, const double *f, double *out)
{
    double w1[5], w2[5];
    if (og_weights(g->r, w1, w2)) return -1;
    long N = og_npts(g);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        long c[3];
        og_coords(g, i, c);
        out[i] = og_d2_at(g, w2, d, f, c);
    }
    return 0;
}

int og_laplacian(const og_t *g, const double *f, double *out)
{
    double w1[5], w2[5];
    if (og_weights(g->r, w1, w2)) return -1;
    long N = og_npts(g);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        long c[3];
        og_coords(g, i, c);
        out[i] = og_d2_at(g, w2, 0, f, c) + og_d2_at(g, w2, 1, f, c) + og_d2_at(g, w2, 2, f, c);
    }
    return 0;
}

/* ---- CPML profiles (CPML section: sigma, kappa, alpha; a, b) ---------- */
/* For axis d, fills per-index arrays of length n[d]:
 *   rho (layer coordinate), b, a, kinv = 1/kappa, dkinv = d(1/kappa)/dx.
 * Returns -1 on an invalid layer (periodic axis with a layer, or layers
 * that overlap). */
int og_profile(const og_t *g, int d, double *rho, double *b, double *a, double *kinv, double *dkinv)
{
    const double q = 3.0;
    int n = g->n[d], Llo = g->cpml[2 * d], Lhi = g->cpml[2 * d + 1];
    if (Llo < 0 || Lhi < 0) return -1;
    if (g->periodic[d] && (Llo || Lhi)) return -1;
    if (Llo + Lhi > n) return -1;
    for (int i = 0; i < n; ++i) {
        double rh = 0.0, drho = 0.0;
        int L = 0;
        if (Llo > 0 && i < Llo) {
            L = Llo;
            rh = (double)(Llo - i) / Llo;
            drho = -1.0 / (Llo * g->h[d]);
        } else if (Lhi > 0 && i > n - 1 - Lhi) {
            L = Lhi;
            rh = (double)(i - (n - 1 - Lhi)) / Lhi;
            drho = 1.0 / (Lhi * g->h[d]);
        }
        rho[i] = rh;
        if (rh > 0.0) {
            double smax = -(q + 1.0) * g->vref * log(g->R) / (2.0 * L * g->h[d]);
            double sigma = smax * pow(rh, q);
            double kappa = 1.0 + (g->kappa_max - 1.0) * pow(rh, q);
            double alpha = g->alpha_frac * smax * (1.0 - rh);
            double bb = exp(-(sigma / kappa + alpha) * g->dt);
            b[i] = bb;
            a[i] = sigma > 0.0 ? sigma * (bb - 1.0) / (kappa * (sigma + kappa * alpha)) : 0.0;
            kinv[i] = 1.0 / kappa;
            /* d(1/kappa)/dx = -kappa'(rho) rho'(x) / kappa^2 */
            dkinv[i] = -(g->kappa_max - 1.0) * q * pow(rh, q - 1.0) * drho / (kappa * kappa);
        } else {
            b[i] = 0.0; /* unused: psi and zeta vanish outside the layer */
            a[i] = 0.0;
            kinv[i] = 1.0;
            dkinv[i] = 0.0;
        }
    }
    return 0;
}

/* prof layout: prof[((d*5 + field) * nmax) + i], field 0..4 = rho,b,a,kinv,dkinv */
static const double *og_pf(const double *prof, int nmax, int d, int field)
{
    return prof + ((long)(d * 5 + field)) * nmax;
}

int og_profiles_all(const og_t *g, int nmax, double *prof)
{
    for (int d = 0; d < 3; ++d) {
        double *base = prof + (long)d * 5 * nmax;
        if (og_profile(g, d, base, base + nmax, base + 2L * nmax, base + 3L * nmax, base + 4L * nmax))
            return -1;
    }
    return 0;
}

/* ---- one forward step ------------------------------------------------- */
/* On entry u = u^n, um1 = u^{n-1}, psi[d*N..], zeta[d*N..] = layer memory at
 * level n (full-size arrays, zero outside each layer).  On exit u = u^{n+1},
 * um1 = u^n, psi and zeta at level n+1.
 * src_index < 0 means no source; otherwise f^n = src_amp / (hx hy hz) at that
 * node.  If lapf is not NULL it receives Lt(u^n) + f^n (the factor that
 * multiplies m in the update; used for the model gradient).
 * work must hold N doubles. */
int og_step(const og_t *g, const double *m, const double *prof, int nmax,
            double *u, double *um1, double *psi, double *zeta,
            long src_index, double src_amp, double *lapf, double *work)
{
    double w1[5], w2[5];
    if (og_weights(g->r, w1, w2)) return -1;
    long N = og_npts(g);
    double f_src = src_amp / (g->h[0] * g->h[1] * g->h[2]);

    /* 1. psi_d <- b psi_d + a D1_d u^n, inside each layer */
    for (int d = 0; d < 3; ++d) {
        const double *rho = og_pf(prof, nmax, d, 0), *b = og_pf(prof, nmax, d, 1),
                     *a = og_pf(prof, nmax, d, 2);
        double *ps = psi + (long)d * N;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            long c[3];
            og_coords(g, i, c);
            if (rho[c[d]] > 0.0) ps[i] = b[c[d]] * ps[i] + a[c[d]] * og_d1_at(g, w1, d, u, c);
        }
    }

    /* 2-3. eta, zeta, stretched Laplacian and the leapfrog */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
        long c[3];
        og_coords(g, i, c);
        double lt = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double *rho = og_pf(prof, nmax, d, 0), *b = og_pf(prof, nmax, d, 1),
                         *a = og_pf(prof, nmax, d, 2), *ki = og_pf(prof, nmax, d, 3),
                         *dki = og_pf(prof, nmax, d, 4);
            long x = c[d];
            double eta = ki[x] * og_d2_at(g, w2, d, u, c) + dki[x] * og_d1_at(g, w1, d, u, c) +
                         og_d1_at(g, w1, d, psi + (long)d * N, c);
            double z = 0.0;
            if (rho[x] > 0.0) {
                z = b[x] * zeta[(long)d * N + i] + a[x] * eta;
                zeta[(long)d * N + i] = z;
            }
            lt += ki[x] * eta + z;
        }
        double f = (i == src_index) ? f_src : 0.0;
        work[i] = 2.0 * u[i] - um1[i] + m[i] * lt + m[i] * f;
        if (lapf) lapf[i] = lt + f;
    }

    /* 4. rotate levels */
    memcpy(um1, u, sizeof(double) * N);
    memcpy(u, work, sizeof(double) * N);
    return 0;
}

/* ---- one adjoint (transposed) step ------------------------------------ */
/* Exact transpose of og_step's linear map (source excluded), written in the
 * same leapfrog shape:  on entry lam = lambda^{n+1} (adjoint of u^{n+1},
 * including any receiver residual of step n), lamp = lambda^{n+2},
 * psib/zetab = adjoints of psi^{n+1}/zeta^{n+1}.  On exit lam = lambda^n,
 * lamp = lambda^{n+1}, psib/zetab = adjoints of psi^n/zeta^n.
 * Transposes used: D2 is symmetric, D1 antisymmetric (both face rules).
 * work must hold 7*N doubles. */
int og_adjoint_step(const og_t *g, const double *m, const double *prof, int nmax,
                    double *lam, double *lamp, double *psib, double *zetab, double *work)
{
    double w1[5], w2[5];
    if (og_weights(g->r, w1, w2)) return -1;
    long N = og_npts(g);
    double *lbar = work;           /* m * lambda^{n+1}                 */
    double *etab = work + N;       /* [3][N] adjoint of eta_d          */
    double *fd = work + 4 * N;     /* [3][N] a_d * (total psi adjoint) */

    for (long i = 0; i < N; ++i) lbar[i] = m[i] * lam[i];

    for (int d = 0; d < 3; ++d) {
        const double *rho = og_pf(prof, nmax, d, 0), *b = og_pf(prof, nmax, d, 1),
                     *a = og_pf(prof, nmax, d, 2), *ki = og_pf(prof, nmax, d, 3);
        double *eb = etab + (long)d * N, *zb = zetab + (long)d * N;
        /* Lt_d = kinv eta_d + zeta_d^{n+1};  zeta^{n+1} = b zeta^n + a eta */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            long c[3];
            og_coords(g, i, c);
            long x = c[d];
            if (rho[x] > 0.0) {
                double zt = zb[i] + lbar[i];
                eb[i] = ki[x] * lbar[i] + a[x] * zt;
                zb[i] = b[x] * zt;
            } else {
                eb[i] = ki[x] * lbar[i];
            }
        }
    }
    for (int d = 0; d < 3; ++d) {
        const double *rho = og_pf(prof, nmax, d, 0), *b = og_pf(prof, nmax, d, 1),
                     *a = og_pf(prof, nmax, d, 2);
        double *eb = etab + (long)d * N, *pb = psib + (long)d * N, *F = fd + (long)d * N;
        /* eta_d contains D1_d psi^{n+1}:  psib += D1^T eta_b = -D1 eta_b;
         * psi^{n+1} = b psi^n + a D1 u^n. */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            long c[3];
            og_coords(g, i, c);
            long x = c[d];
            if (rho[x] > 0.0) {
                double pt = pb[i] - og_d1_at(g, w1, d, eb, c);
                F[i] = a[x] * pt;
                pb[i] = b[x] * pt;
            } else {
                F[i] = 0.0;
            }
        }
    }
    double *out = lbar; /* lbar is no longer needed once the products below are formed */
    double *ke = (double *)malloc(sizeof(double) * 2 * N);
    if (!ke) return -2;
    double *de = ke + N;
    for (long i = 0; i < N; ++i) out[i] = 2.0 * lam[i] - lamp[i];
    for (int d = 0; d < 3; ++d) {
        const double *ki = og_pf(prof, nmax, d, 3), *dki = og_pf(prof, nmax, d, 4);
        double *eb = etab + (long)d * N, *F = fd + (long)d * N;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            long c[3];
            og_coords(g, i, c);
            ke[i] = ki[c[d]] * eb[i];
            de[i] = dki[c[d]] * eb[i];
        }
        /* u^n enters eta_d through kinv D2 u + dkinv D1 u, and psi^{n+1} through a D1 u */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) {
            long c[3];
            og_coords(g, i, c);
            out[i] += og_d2_at(g, w2, d, ke, c) - og_d1_at(g, w1, d, de, c) - og_d1_at(g, w1, d, F, c);
        }
    }
    free(ke);
    memcpy(lamp, lam, sizeof(double) * N);
    memcpy(lam, out, sizeof(double) * N);
    return 0;
}
