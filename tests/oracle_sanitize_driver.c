/* Host sanitizer run of the FP64 oracle (test infrastructure): the oracle's
 * translation unit is included whole and driven through every entry point on
 * small grids with uneven layers, a periodic axis and the smallest axis the
 * stencil allows, so that AddressSanitizer and UndefinedBehaviorSanitizer see
 * every loop's index range.  Prints "ok" when everything returned 0. */
#include "../oracle/fdtd_oracle.c"

#include <stdio.h>

static double frand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return ((*s >> 8) & 0xffffff) / (double)0x1000000 - 0.5;
}

static int run_case(int nx, int ny, int nz, const int cpml[6], const int periodic[3], int steps) {
    og_t g;
    memset(&g, 0, sizeof g);
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.h[0] = 10.0;
    g.h[1] = 12.0;
    g.h[2] = 9.0;
    g.dt = 1e-3;
    g.r = 4;
    for (int d = 0; d < 3; ++d) g.periodic[d] = periodic[d];
    for (int f = 0; f < 6; ++f) g.cpml[f] = cpml[f];
    g.R = 1e-8;
    g.kappa_max = 5.0;
    g.alpha_frac = 0.05;
    g.vref = 2500.0;
    const long N = (long)nx * ny * nz;
    int nmax = nx > ny ? nx : ny;
    nmax = nmax > nz ? nmax : nz;
    double *m = malloc(sizeof(double) * N), *u = calloc(N, sizeof(double)), *um1 = calloc(N, sizeof(double));
    double *psi = calloc(3 * N, sizeof(double)), *zeta = calloc(3 * N, sizeof(double));
    double *lapf = calloc(N, sizeof(double)), *work = calloc(7 * N, sizeof(double));
    double *prof = calloc(15 * (size_t)nmax, sizeof(double)), *out = calloc(N, sizeof(double));
    double *lam = calloc(N, sizeof(double)), *lamp = calloc(N, sizeof(double));
    double *psib = calloc(3 * N, sizeof(double)), *zetab = calloc(3 * N, sizeof(double));
    double *pr[5];
    for (int k = 0; k < 5; ++k) pr[k] = calloc(nmax, sizeof(double));
    unsigned s = 12345u;
    int rc = 0;
    for (long i = 0; i < N; ++i) {
        m[i] = 0.02 * (1.0 + 0.1 * frand(&s));
        u[i] = frand(&s);
        um1[i] = frand(&s);
        lam[i] = frand(&s);
        lamp[i] = frand(&s);
    }
    rc |= og_profiles_all(&g, nmax, prof);
    for (int d = 0; d < 3; ++d) {
        rc |= og_profile(&g, d, pr[0], pr[1], pr[2], pr[3], pr[4]);
        rc |= og_deriv1(&g, d, u, out);
        rc |= og_deriv2(&g, d, u, out);
    }
    rc |= og_laplacian(&g, u, out);
    for (int n = 0; n < steps; ++n) rc |= og_step(&g, m, prof, nmax, u, um1, psi, zeta, (int)(N / 2), 1.0, lapf, work);
    for (int n = 0; n < steps; ++n) rc |= og_adjoint_step(&g, m, prof, nmax, lam, lamp, psib, zetab, work);
    double acc = 0;
    for (long i = 0; i < N; ++i) acc += u[i] + lam[i];
    if (!(acc == acc)) rc |= 1;
    free(m); free(u); free(um1); free(psi); free(zeta); free(lapf); free(work); free(prof); free(out);
    free(lam); free(lamp); free(psib); free(zetab);
    for (int k = 0; k < 5; ++k) free(pr[k]);
    return rc;
}

int main(void) {
    const int c1[6] = {5, 7, 3, 6, 8, 4}, p1[3] = {0, 0, 0};
    const int c2[6] = {4, 4, 4, 4, 4, 4};
    const int c3[6] = {6, 5, 0, 0, 0, 0}, p3[3] = {0, 1, 1};
    const int c4[6] = {0, 0, 0, 0, 0, 0};
    int rc = run_case(24, 21, 19, c1, p1, 6);
    rc |= run_case(9, 9, 9, c2, p1, 4);       /* smallest axis with the widest layer */
    rc |= run_case(20, 14, 12, c3, p3, 5);    /* periodic y and z */
    rc |= run_case(11, 10, 13, c4, p1, 3);    /* no layer */
    if (rc) {
        printf("fail %d\n", rc);
        return 1;
    }
    printf("ok\n");
    return 0;
}
