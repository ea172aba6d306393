/*
 * AddressSanitizer / UndefinedBehaviorSanitizer run of the oracle's C
 * stepper (test infrastructure).  The stepper source is included so that
 * this file is the whole program: random coefficients on tiny and ragged 2D
 * and 3D grids, both memory schemes, global and per-point stencil weights,
 * sources and receivers, every array allocated to its exact size.  Exit
 * status 0 when every case ran and stayed finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/fw2_oracle.c"

static unsigned g_seed = 12345u;

static double urand(double lo, double hi)
{
    g_seed = g_seed * 1103515245u + 12345u;
    return lo + (hi - lo) * (double)((g_seed >> 8) & 0xffffff) / (double)0xffffff;
}

static double *arr(size_t n, double lo, double hi)
{
    double *a = (double *)malloc((n ? n : 1) * sizeof(double));
    for (size_t i = 0; i < n; ++i) a[i] = urand(lo, hi);
    return a;
}

static int run_case(int ndim, int nx, int ny, int nz, int L, int scheme, int per_point, int steps)
{
    oracle_problem P;
    memset(&P, 0, sizeof(P));
    const int64_t npts = (int64_t)nx * ny * nz;
    P.ndim = ndim;
    P.L = L;
    P.scheme = scheme;
    P.n[0] = nx;
    P.n[1] = ny;
    P.n[2] = nz;
    P.dt = 1e-8;
    const double h = 1e-4;
    const double g[4] = {1.15, -0.066, 0.0079, -0.00057};
    for (int k = 0; k < 4; ++k) P.g[k] = g[k] / h;
    P.g11 = 0.0067 / h;
    P.nl_A = 1.0;
    double *kap0 = arr(npts, 4.0e-10, 4.5e-10), *nlq = arr(npts, -3.0e-9, -2.0e-9);
    double *rho_v = arr(ndim * npts, 950.0, 1100.0), *kap_v = arr(ndim * npts, 4.0e-10, 4.5e-10);
    double *ik1 = arr(ndim * npts, 0.8, 1.2), *ik2 = arr(ndim * npts, 0.8, 1.2);
    const size_t nm = (size_t)ndim * L * npts;
    double *a1 = arr(nm, -1e-3, 0.0), *b1 = arr(nm, 0.5, 1.0), *a2 = arr(nm, -1e-3, 0.0), *b2 = arr(nm, 0.5, 1.0);
    double *e01 = arr(nm, -1e-4, 0.0), *e02 = arr(nm, -1e-4, 0.0);
    double *gwp = per_point ? arr(5 * npts, 0.0, 1e4) : NULL;
    double *gwv = per_point ? arr((size_t)ndim * 5 * npts, 0.0, 1e4) : NULL;
    P.kap0 = kap0;
    P.nlq = nlq;
    P.rho_v = rho_v;
    P.kap_v = kap_v;
    P.ik1 = ik1;
    P.ik2 = ik2;
    P.a1 = a1;
    P.b1 = b1;
    P.a2 = a2;
    P.b2 = b2;
    P.e0_1 = e01;
    P.e0_2 = e02;
    P.gw_p = gwp;
    P.gw_v = gwv;
    /* sources at the first and last points, receivers at the last and first */
    int64_t src[2] = {0, npts - 1}, rcv[2] = {npts - 1, 0};
    int32_t sig[2] = {0, 1};
    double w[2] = {1.0, -0.5};
    const int n_src = npts > 1 ? 2 : 1;
    double *signals = arr(2 * 5, -1e3, 1e3);
    P.n_src = n_src;
    P.src_idx = src;
    P.src_sig = sig;
    P.src_w = w;
    P.n_t = 5;
    P.signals = signals;
    P.n_rcv = n_src;
    P.rcv_idx = rcv;
    double *p = (double *)calloc(npts, sizeof(double));
    double *v = (double *)calloc(ndim * npts, sizeof(double));
    double *psi1 = (double *)calloc(nm ? nm : 1, sizeof(double));
    double *psi2 = (double *)calloc(nm ? nm : 1, sizeof(double));
    double *trace = (double *)malloc((size_t)steps * n_src * sizeof(double));
    int rc = oracle_run(&P, p, v, psi1, psi2, 0, steps, trace);
    int ok = rc == 0;
    for (int64_t i = 0; i < npts && ok; ++i) ok = isfinite(p[i]);
    for (int i = 0; i < steps * n_src && ok; ++i) ok = isfinite(trace[i]);
    free(kap0); free(nlq); free(rho_v); free(kap_v); free(ik1); free(ik2);
    free(a1); free(b1); free(a2); free(b2); free(e01); free(e02); free(gwp); free(gwv);
    free(signals); free(p); free(v); free(psi1); free(psi2); free(trace);
    if (!ok) printf("case %dD %dx%dx%d L=%d scheme=%d per_point=%d failed\n", ndim, nx, ny, nz, L, scheme, per_point);
    return ok;
}

int main(void)
{
    const int shapes[][4] = {{2, 1, 1, 1}, {2, 1, 7, 1}, {2, 7, 1, 1}, {2, 9, 6, 1}, {2, 13, 11, 1},
                             {3, 1, 1, 1}, {3, 3, 4, 5}, {3, 6, 5, 4}, {3, 9, 2, 7}};
    int n = 0, good = 0;
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (int L = 1; L <= 3; ++L)
            for (int scheme = 0; scheme <= 1; ++scheme)
                for (int pp = 0; pp <= 1; ++pp) {
                    ++n;
                    good += run_case(shapes[s][0], shapes[s][1], shapes[s][2], shapes[s][3], L, scheme, pp, 6);
                }
    printf("oracle sanitizer cases: %d of %d clean\n", good, n);
    return good == n ? 0 : 1;
}
