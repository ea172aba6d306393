// Host-side setup math of libfw2 (FP64).  See setup.hpp.
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace fw2 {

namespace {

// Solve the axial Taylor conditions sum_j (2j-1)^(2k-1) c_j = rhs[k] (k = 1..4).
void solve_axial(const double rhs[4], double c[4])
{
    double A[4][5];
    for (int k = 0; k < 4; ++k) {
        for (int j = 0; j < 4; ++j) A[k][j] = std::pow(2.0 * j + 1.0, 2.0 * k + 1.0);
        A[k][4] = rhs[k];
    }
    for (int col = 0; col < 4; ++col) {          // Gaussian elimination, partial pivoting
        int piv = col;
        for (int row = col + 1; row < 4; ++row)
            if (std::fabs(A[row][col]) > std::fabs(A[piv][col])) piv = row;
        if (piv != col)
            for (int j = 0; j < 5; ++j) std::swap(A[col][j], A[piv][j]);
        for (int row = col + 1; row < 4; ++row) {
            const double f = A[row][col] / A[col][col];
            for (int j = col; j < 5; ++j) A[row][j] -= f * A[col][j];
        }
    }
    for (int row = 3; row >= 0; --row) {
        double s = A[row][4];
        for (int j = row + 1; j < 4; ++j) s -= A[row][j] * c[j];
        c[row] = s / A[row][row];
    }
}

}  // namespace

void stencil_weights(double r, int ndim, double g[4], double *g11)
{
    // right-hand side r^(2k-2)
    double rhs[4], c[4];
    for (int k = 0; k < 4; ++k) rhs[k] = std::pow(r, 2.0 * k);
    solve_axial(rhs, c);
    *g11 = r * r / 24.0;
    for (int j = 0; j < 4; ++j) g[j] = c[j];
    g[0] = c[0] - 2.0 * (ndim - 1) * (*g11);
}

void stencil_polynomials(int ndim, double pw[4][4], double *g11_per_s)
{
    // The weights are linear in the right-hand side (1, s, s^2, s^3), s = r^2:
    // column k of the solution for the unit right-hand side e_k is the s^k
    // coefficient.  g_10 carries the cross-term correction -2(d-1) s / 24.
    for (int k = 0; k < 4; ++k) {
        double e[4] = {0.0, 0.0, 0.0, 0.0}, c[4];
        e[k] = 1.0;
        solve_axial(e, c);
        for (int j = 0; j < 4; ++j) pw[j][k] = c[j];
    }
    pw[0][1] -= 2.0 * (ndim - 1) / 24.0;
    *g11_per_s = 1.0 / 24.0;
}

double stability_factor(double r, int ndim, const double g[4], double g11)
{
    // The symbol of one axis depends only on that axis' wavenumber, so the
    // sines and cosines are tabulated once per sample (M of them) and the
    // sweep over the M^ndim wavenumber grid is arithmetic only.
    const int M = ndim == 2 ? 181 : 61;
    const double pi = 3.14159265358979323846;
    std::vector<double> ax(M), sh(M), co(M);
    for (int i = 0; i < M; ++i) {
        const double th = pi * i / (M - 1);
        double A = 0.0;
        for (int m = 1; m <= 4; ++m) A += g[m - 1] * std::sin((2 * m - 1) * th / 2.0);
        ax[i] = A;
        sh[i] = std::sin(th / 2.0);
        co[i] = std::cos(th);
    }
    double worst = 0.0;
    int cnt[3] = {M, M, ndim == 3 ? M : 1};
    for (int iz = 0; iz < cnt[2]; ++iz)
        for (int iy = 0; iy < cnt[1]; ++iy)
            for (int ix = 0; ix < cnt[0]; ++ix) {
                const int id[3] = {ix, iy, iz};
                double s2 = 0.0;
                for (int a = 0; a < ndim; ++a) {
                    double cs = 0.0;
                    for (int b = 0; b < ndim; ++b)
                        if (b != a) cs += co[id[b]];
                    const double A = ax[id[a]] + 2.0 * g11 * sh[id[a]] * cs;
                    s2 += A * A;
                }
                worst = std::max(worst, r * std::sqrt(s2));
            }
    return worst;
}

double boundary_distance(int64_t twice_x, int64_t n, int nb)
{
    const double x = 0.5 * (double)twice_x;
    double s = std::max(0.0, std::max((double)nb - x, x - (double)(n - 1 - nb)));
    return std::min(s, (double)nb);
}

void layer_profile(double s, double h, int nb, int ntr, double d0, double a0, int nu,
                   double d_target, int npoly, double *d, double *alpha)
{
    if (nb == 0 || s <= 0.0) {
        *d = d0;
        *alpha = a0;
        return;
    }
    if (nu == 1) {
        const double u = s / nb;                              // x / L_C-PML
        const double gp = std::pow(u, (double)npoly);         // polynomial transition
        *d = (d_target - d0) * gp + d0;
        *alpha = (0.0 - a0) * u + a0;                         // linear transition
        return;
    }
    double gc = 0.0;                                          // no transition layer: keep
    if (ntr > 0) {
        const double u = std::min(s, (double)ntr) / ntr;
        gc = 0.5 * (1.0 - std::cos(3.14159265358979323846 * u));   // cosine transition
    }
    *d = (0.0 - d0) * gc + d0;
    *alpha = (0.0 - a0) * gc + a0;
}

MechCoef mech_coef(double kappa, double d, double alpha, double dt)
{
    MechCoef m{0.0, 1.0, 0.0, 0.0};
    const double lam = d / kappa + alpha;
    m.b = std::exp(-lam * dt);
    if (d == 0.0) return m;                 // kernel vanishes: a = e0 = e1 = 0
    m.a = d / (kappa * (d + kappa * alpha)) * (m.b - 1.0);
    // e1 = -(d/kappa^2) int_0^dt tau exp(-lam tau) dtau / dt ; e0 = a - e1
    const double x = lam * dt;
    const double amp = -d / (kappa * kappa);
    const double i1 = (-std::expm1(-x) - x * std::exp(-x)) / (lam * x);
    m.e1 = amp * i1;
    m.e0 = m.a - m.e1;
    return m;
}

AxisTables build_axis_tables(const TableInput &in, int nabla, int nb, int ntr)
{
    AxisTables t;
    const int L = in.L;
    t.n_slots = nabla == 2 ? nb + 1 : nb + 2;
    t.w.assign((size_t)t.n_slots * in.n_labels, 0.0f);
    t.bc.assign((size_t)t.n_slots * in.n_labels * L * 2, 0.0f);
    const int row_len = 2 + 4 * L;
    for (int s = 0; s < t.n_slots; ++s) {
        double dist;
        if (nabla == 2) dist = (double)s;
        else dist = s == 0 ? 0.0 : std::min((double)s - 0.5, (double)nb);
        for (int lab = 0; lab < in.n_labels; ++lab) {
            const double *row = in.table + (size_t)lab * row_len;
            const double kappa = nabla == 1 ? row[0] : row[1];
            const double *dv = row + 2 + (nabla == 1 ? 0 : L);
            const double *av = row + 2 + 2 * L + (nabla == 1 ? 0 : L);
            double w = 1.0 / kappa;
            for (int nu = 0; nu < L; ++nu) {
                double d, al;
                layer_profile(dist, in.h, nb, ntr, dv[nu], av[nu], nu + 1, in.d_target, in.npoly, &d, &al);
                const MechCoef m = mech_coef(kappa, d, al, in.dt);
                double c;
                if (in.scheme == 0) {
                    c = m.a;
                } else {
                    w += m.e0;
                    c = m.e1 + m.b * m.e0;
                }
                const size_t o = (((size_t)s * in.n_labels + lab) * L + nu) * 2;
                t.bc[o] = (float)m.b;
                t.bc[o + 1] = (float)c;
            }
            t.w[(size_t)s * in.n_labels + lab] = (float)w;
        }
    }
    return t;
}

}  // namespace fw2
