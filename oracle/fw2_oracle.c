/*
 * FP64 reference time stepper for the Fullwave 2 system (Sode & Pinton,
 * arXiv 2106.11476).  TEST INFRASTRUCTURE ONLY: used by the test suite, the
 * smoke check and the benchmark's CPU baseline; never by the product path.
 *
 * Plain nested loops over the grid, values outside the array read as zero.
 * Every per-point coefficient (stencil weights / h, memory-variable a and b,
 * 1/kappa, staggered medium values) is prepared by oracle/solver.py from the
 * paper's formulas and handed in as arrays; this file only advances the state.
 *
 * The stencil weights are either one global set or, in stencil mode 1, the
 * set of the local Courant number at each p and v point (gw_p, gw_v).
 *
 * One time step (Sec. 3.1 staggered scheme, Eqs. general5 and general6):
 *   1. pressure phase, every p point (integer position along each axis):
 *        D_a    = (D^- v_a)                       stencil of Sec. 3.1
 *        memory term M of each mechanism, either
 *          scheme 0 (Eq. relaxation_psi as printed, update then use):
 *            psi2 <- b2 psi2 + a2 D_a ;  M = psi2
 *          scheme 1 (time-centred convolution, D linear between samples):
 *            M = e0 D_a + psi2 ;  psi2 <- b2 psi2 + (a2 - e0 + b2 e0) D_a
 *        S      = sum_a ( ik2 D_a + sum_nu M )    Eq. relaxation4 (nabla_2)
 *        p     <- p - dt S / (kappa0 (1 + kappa0 B p))   Eq. general6,
 *                 B = 1 - 2 beta as printed (Eq. state2)
 *   2. sources:   p[idx] += w * signal[step]
 *   3. receivers: trace[step][r] = p[idx_r]
 *   4. velocity phase, every v_a point (half-integer position along a)
 *      strictly between two pressure samples (the sample past the last
 *      pressure sample along a lies outside the grid and stays zero):
 *        D      = (D^+ p)_a
 *        memory terms as in step 1 with (a1, b1, e0_1)
 *        S      = ik1 D + sum_nu M                     (nabla_1)
 *        v_a   <- v_a - dt S / (rho_a (1 + A kappa0_a pbar)),  pbar = mean of
 *                 the two pressures around the v point, A = 1 as printed
 *                 (Eq. state1)                          Eq. general5
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t ndim;
    int32_t L;
    int32_t scheme;          /* 0: printed recursion, 1: time-centred */
    int32_t pad_;
    int64_t n[3];            /* nx, ny, nz (nz = 1 in 2D); x fastest */
    double dt;
    double g[4];             /* g_m0 / h, m = 1..4 */
    double g11;              /* g_11 / h */
    const double *kap0;      /* [npts] equilibrium compressibility at p points */
    const double *nlq;       /* [npts] kappa0 B at p points (B = 1 - 2 beta as printed) */
    const double *rho_v;     /* [ndim][npts] density at v_a points */
    const double *kap_v;     /* [ndim][npts] compressibility at v_a points */
    const double *ik1;       /* [ndim][npts] 1/kappa_1 at v_a points */
    const double *ik2;       /* [ndim][npts] 1/kappa_2 at p points */
    const double *a1, *b1;   /* [ndim][L][npts] nabla_1 coefficients at v_a points */
    const double *a2, *b2;   /* [ndim][L][npts] nabla_2 coefficients at p points */
    const double *e0_1, *e0_2; /* [ndim][L][npts] newest-sample weights (scheme 1) */
    int32_t n_src;
    const int64_t *src_idx;
    const int32_t *src_sig;
    const double *src_w;
    int32_t n_t;
    const double *signals;   /* [n_sig][n_t] */
    int32_t n_rcv;
    const int64_t *rcv_idx;
    /* Per-point stencil weights (stencil mode 1), or NULL for the global g:
     * gw_p [5][npts] at p points, gw_v [ndim][5][npts] at v_a points; rows
     * g_10 .. g_40, g_11, all over h. */
    const double *gw_p;
    const double *gw_v;
    /* Coefficient A of the momentum multiplier rho_a (1 + A kappa0_a pbar)
     * (Eq. state1: A = 1); the mass multiplier's B is folded into nlq. */
    double nl_A;
} oracle_problem;

/* Field value at integer coordinate x (x[0] fastest); zero outside the grid. */
static double at(const double *f, const int64_t *n, const int64_t *x)
{
    for (int a = 0; a < 3; ++a)
        if (x[a] < 0 || x[a] >= n[a]) return 0.0;
    return f[(x[2] * n[1] + x[1]) * n[0] + x[0]];
}

/* Value of f at x + s1*e_a1 + s2*e_a2 (a2 < 0: no second shift). */
static double at_shift(const double *f, const int64_t *n, const int64_t *x,
                       int a1, int64_t s1, int a2, int64_t s2)
{
    int64_t y[3] = {x[0], x[1], x[2]};
    y[a1] += s1;
    if (a2 >= 0) y[a2] += s2;
    return at(f, n, y);
}

/* Stencil weights (g_10..g_40, g_11, over h) that apply at flat index idx:
 * the global set, or row k of the per-point table tab ([5][npts]). */
static void weights_at(const oracle_problem *P, const double *tab, int64_t npts, int64_t idx, double w[5])
{
    for (int k = 0; k < 5; ++k)
        w[k] = tab ? tab[k * npts + idx] : (k < 4 ? P->g[k] : P->g11);
}

/* (D^- v_a) at the p point x: v_a[k] sits at k + 1/2 along a. */
static double d_minus(const oracle_problem *P, const double *w, const double *va, int a, const int64_t *x)
{
    double s = 0.0;
    for (int m = 1; m <= 4; ++m)
        s += w[m - 1] * (at_shift(va, P->n, x, a, m - 1, -1, 0) -
                         at_shift(va, P->n, x, a, -m, -1, 0));
    for (int b = 0; b < P->ndim; ++b) {
        if (b == a) continue;
        for (int sg = -1; sg <= 1; sg += 2)
            s += w[4] * (at_shift(va, P->n, x, b, sg, -1, 0) -
                         at_shift(va, P->n, x, a, -1, b, sg));
    }
    return s;
}

/* (D^+ p)_a at the v_a point x (position x + 1/2 e_a). */
static double d_plus(const oracle_problem *P, const double *w, const double *p, int a, const int64_t *x)
{
    double s = 0.0;
    for (int m = 1; m <= 4; ++m)
        s += w[m - 1] * (at_shift(p, P->n, x, a, m, -1, 0) -
                         at_shift(p, P->n, x, a, -(m - 1), -1, 0));
    for (int b = 0; b < P->ndim; ++b) {
        if (b == a) continue;
        for (int sg = -1; sg <= 1; sg += 2)
            s += w[4] * (at_shift(p, P->n, x, a, 1, b, sg) -
                         at_shift(p, P->n, x, b, sg, -1, 0));
    }
    return s;
}

static void pressure_phase(const oracle_problem *P, double *p, const double *v, double *psi2)
{
    const int64_t nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const int64_t npts = nx * ny * nz;
    const int L = P->L;
#pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < ny * nz; ++row) {
        int64_t x[3];
        x[1] = row % ny;
        x[2] = row / ny;
        for (int64_t i = 0; i < nx; ++i) {
            x[0] = i;
            const int64_t idx = row * nx + i;
            double S = 0.0;
            double w[5];
            weights_at(P, P->gw_p, npts, idx, w);
            for (int a = 0; a < P->ndim; ++a) {
                const double D = d_minus(P, w, v + a * npts, a, x);
                double acc = 0.0;
                for (int nu = 0; nu < L; ++nu) {
                    const int64_t c = ((int64_t)a * L + nu) * npts + idx;
                    if (P->scheme == 0) {
                        psi2[c] = P->b2[c] * psi2[c] + P->a2[c] * D;
                        acc += psi2[c];
                    } else {
                        const double e0 = P->e0_2[c];
                        acc += e0 * D + psi2[c];
                        psi2[c] = P->b2[c] * psi2[c] + ((P->a2[c] - e0) + P->b2[c] * e0) * D;
                    }
                }
                S += P->ik2[a * npts + idx] * D + acc;
            }
            const double pold = p[idx];
            const double kappa = P->kap0[idx] * (1.0 + P->nlq[idx] * pold);
            p[idx] = pold - P->dt * S / kappa;
        }
    }
}

static void velocity_phase(const oracle_problem *P, const double *p, double *v, double *psi1)
{
    const int64_t nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const int64_t npts = nx * ny * nz;
    const int L = P->L;
#pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < ny * nz; ++row) {
        int64_t x[3];
        x[1] = row % ny;
        x[2] = row / ny;
        for (int64_t i = 0; i < nx; ++i) {
            x[0] = i;
            const int64_t idx = row * nx + i;
            for (int a = 0; a < P->ndim; ++a) {
                if (x[a] == P->n[a] - 1) continue;   /* outside the grid */
                double w[5];
                weights_at(P, P->gw_v ? P->gw_v + (int64_t)a * 5 * npts : NULL, npts, idx, w);
                const double D = d_plus(P, w, p, a, x);
                double acc = 0.0;
                for (int nu = 0; nu < L; ++nu) {
                    const int64_t c = ((int64_t)a * L + nu) * npts + idx;
                    if (P->scheme == 0) {
                        psi1[c] = P->b1[c] * psi1[c] + P->a1[c] * D;
                        acc += psi1[c];
                    } else {
                        const double e0 = P->e0_1[c];
                        acc += e0 * D + psi1[c];
                        psi1[c] = P->b1[c] * psi1[c] + ((P->a1[c] - e0) + P->b1[c] * e0) * D;
                    }
                }
                const double S = P->ik1[a * npts + idx] * D + acc;
                const double pbar = 0.5 * (at(p, P->n, x) + at_shift(p, P->n, x, a, 1, -1, 0));
                const double rho = P->rho_v[a * npts + idx] * (1.0 + P->nl_A * P->kap_v[a * npts + idx] * pbar);
                v[a * npts + idx] -= P->dt * S / rho;
            }
        }
    }
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Advance n_steps steps.  step0 is the global index of the first step (it
 * selects the source sample).  trace: [n_steps][n_rcv] or NULL. */
int oracle_run(const oracle_problem *P, double *p, double *v, double *psi1, double *psi2,
               int64_t step0, int64_t n_steps, double *trace)
{
    if (P->ndim < 2 || P->ndim > 3 || P->L < 0 || P->scheme < 0 || P->scheme > 1) return 1;
    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t step = step0 + s;
        pressure_phase(P, p, v, psi2);
        if (step < P->n_t)
            for (int32_t q = 0; q < P->n_src; ++q)
                p[P->src_idx[q]] += P->src_w[q] * P->signals[(int64_t)P->src_sig[q] * P->n_t + step];
        if (trace)
            for (int32_t r = 0; r < P->n_rcv; ++r)
                trace[s * P->n_rcv + r] = p[P->rcv_idx[r]];
        velocity_phase(P, p, v, psi1);
    }
    return 0;
}
