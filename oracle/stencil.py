"""Staggered-grid (2M,4) finite-difference weights, M = 4 (Sec. 3.1).

The paper writes the x-derivative of the (2M,4) operator as

    D_x p = (1/h) [ g_11 (p(1/2,1) - p(-1/2,1) + p(1/2,-1) - p(-1/2,-1))
                    + sum_{i=1..M} g_i0 (p(i-1/2,0) - p(-i+1/2,0)) ]

and defers the weights to Tan & Huang (2014), which is not reproduced in the
paper.  Reading used here (listed among the readings of the design notes):
the weights are the ones that make the leapfrog dispersion relation of the
scheme,  sin(w dt/2)/r = |A(theta)|,  exact to the stated orders, with one
global Courant number r = c_ref dt / h:

* axial (theta_y = theta_z = 0): with c_1 = g_10 + 2(d-1) g_11 and c_j = g_j0
  (j >= 2), sum_j c_j (2j-1)^(2k-1) = r^(2k-2) for k = 1..M;
* mixed fourth-order term theta_x^2 theta_y^2: g_11 = r^2 / 24.

At r = 0 this is the textbook eighth-order staggered set.

The paper's scheme comes from a time-space domain design whose weights depend
on the Courant number, i.e. on the velocity.  With stencil_mode 1 every point
takes the weights of its own Courant number r = c dt / h (the same Taylor
conditions solved at that r; local_weights below), instead of one r for the
whole grid.
"""
import numpy as np

M = 4


def stencil_weights(r: float, ndim: int):
    """Return (g, g11): g[m-1] = g_m0 for m = 1..4, and g11 (Sec. 3.1).

    r    -- Courant number c_ref * dt / h used for the time correction.
    ndim -- 2 or 3; the cross term appears over the ndim-1 other axes, so the
            on-axis first weight absorbs 2(ndim-1) g11.
    """
    k = np.arange(1, M + 1)
    j = np.arange(1, M + 1)
    # Row k: sum_j c_j (2j-1)^(2k-1) = r^(2k-2)
    A = np.array([[(2.0 * jj - 1.0) ** (2 * kk - 1) for jj in j] for kk in k])
    rhs = np.array([float(r) ** (2 * kk - 2) for kk in k])
    c = np.linalg.solve(A, rhs)
    g11 = float(r) ** 2 / 24.0
    g = c.copy()
    g[0] = c[0] - 2.0 * (ndim - 1) * g11
    return g, g11


def local_weights(r2, ndim: int):
    """Weights of stencil_weights for every entry of an array of r^2 values.

    Returns (g, g11) with g of shape (4,) + r2.shape: the Taylor conditions
    of stencil_weights solved at each r (one solve of the same 4 x 4 system
    with one right-hand side per point)."""
    r2 = np.asarray(r2, dtype=np.float64)
    k = np.arange(1, M + 1)
    j = np.arange(1, M + 1)
    A = np.array([[(2.0 * jj - 1.0) ** (2 * kk - 1) for jj in j] for kk in k])
    rhs = np.stack([r2.ravel() ** (kk - 1) for kk in k])        # r^(2k-2)
    c = np.linalg.solve(A, rhs).reshape((M,) + r2.shape)
    g11 = r2 / 24.0
    g = c.copy()
    g[0] = c[0] - 2.0 * (ndim - 1) * g11
    return g, g11


def scheme_phase_velocity_ratio(g, g11, r, ppw, angle, ndim=2):
    """Numerical / true phase velocity of the staggered leapfrog scheme.

    Derived from the update equations themselves (Sec. 3.1 scheme), not from
    the Taylor conditions above: a plane wave exp(i(k.x - w t)) through
    p^n = p^{n-1} - K dt (Dx u + Dy v), u^{n+1/2} = u^{n-1/2} - dt/rho Dx p
    gives  sin(w dt / 2) = r * sqrt(sum_a A_a^2)  with
    A_x = sum_m g_m0 sin((2m-1) th_x / 2) + 2 g11 sin(th_x/2) sum_{b!=x} cos(th_b),
    th = k h.  Returns c_num / c for wavelength ppw * h at the given angle
    (2D, radians from the x axis).
    """
    th = 2.0 * np.pi / ppw
    ths = [th * np.cos(angle), th * np.sin(angle)]
    if ndim == 3:
        ths.append(0.0)
    s2 = 0.0
    for a, ta in enumerate(ths):
        Aa = sum(g[m - 1] * np.sin((2 * m - 1) * ta / 2.0) for m in range(1, M + 1))
        Aa += 2.0 * g11 * np.sin(ta / 2.0) * sum(np.cos(tb) for b, tb in enumerate(ths) if b != a)
        s2 += Aa * Aa
    w_dt = 2.0 * np.arcsin(r * np.sqrt(s2))
    # true: w dt = c k dt = r * th
    return w_dt / (r * th)
