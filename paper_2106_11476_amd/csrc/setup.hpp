// Host-side setup math of libfw2 (FP64): stencil weights, stability bound,
// boundary-layer profiles and memory-variable coefficient tables.
#pragma once

#include <cstdint>
#include <vector>

namespace fw2 {

// Staggered (8,4) weights for Courant number r (Sec. 3.1): g[m-1] = g_m0,
// g11 = g_11, before division by h.  The axial weights solve
// sum_j c_j (2j-1)^(2k-1) = r^(2k-2), k = 1..4; g11 = r^2/24 and the first
// on-axis weight gives up 2 (ndim-1) g11 to the cross terms.
void stencil_weights(double r, int ndim, double g[4], double *g11);

// The same weights as polynomials in s = r^2: g_m0(s) = sum_k pw[m-1][k] s^k,
// g_11(s) = g11_per_s * s.
void stencil_polynomials(int ndim, double pw[4][4], double *g11_per_s);

// Largest |sin(w dt / 2)| of the leapfrog with these weights over the
// Brillouin zone; the scheme is stable when it is below 1.
double stability_factor(double r, int ndim, const double g[4], double g11);

// Distance (cells) of a sample at coordinate twice_x / 2 from the inner edge
// of the boundary region of an axis with n samples and nb cells per side,
// clamped to [0, nb].
double boundary_distance(int64_t twice_x, int64_t n, int nb);

// Memory-variable coefficients of one mechanism at one position.
struct MechCoef {
    double a, b;     // Eqs. relaxation_a and relaxation_b
    double e0, e1;   // time-centred weights (newest sample, previous sample)
};

// (d, alpha) of mechanism nu (1-based) at distance s cells into the layer
// (Table 1): nu = 1 polynomial d to d~ and linear alpha to 0 over the whole
// layer; nu >= 2 cosine ramp to 0 over the transition layer (kept when
// there is none).
void layer_profile(double s, double h, int nb, int ntr, double d0, double a0, int nu,
                   double d_target, int npoly, double *d, double *alpha);

MechCoef mech_coef(double kappa, double d, double alpha, double dt);

// Per-axis tables.  Slot 0 is the interior; pressure-point slots k = 1..nb
// are distance k; velocity-point slots k = 1..nb+1 are distance k - 1/2
// (clamped to nb).  For each (slot, label): w = 1/kappa (+ sum_nu e0 when
// centred) and per mechanism (b, c) with c = a (printed) or e1 + b e0
// (centred).
struct AxisTables {
    int n_slots;
    std::vector<float> w;      // [slot][label]
    std::vector<float> bc;     // [slot][label][nu][2]
};

struct TableInput {
    int n_labels, L, scheme;
    const double *table;       // [n_labels][2 + 4L]
    double h, dt, d_target;
    int npoly;
};

// nabla = 1 builds the velocity-point (half-integer) table, nabla = 2 the
// pressure-point (integer) table, for an axis with nb / ntr layer cells.
AxisTables build_axis_tables(const TableInput &in, int nabla, int nb, int ntr);

}  // namespace fw2
