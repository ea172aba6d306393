"""Two-stage C-PML with a transition layer (Sec. 3.3, Table 1).

Reading used (see the design notes, "boundary geometry"):

* The boundary region of one side has thickness L_CPML = L_Tr + L_Bound
  (the paper's L_C-PML = L_Transition + L_Bound), measured from its inner
  edge; s is the distance of a sample from that inner edge (s = 0 inside the
  domain, s = L_CPML at the outer edge, clamped there for samples past it).
* nu = 1:  d  goes polynomially (Eq. polynomial_transition) from the local
  tissue value d_0 to d~ = -(N+1) c_p ln(R_c) / (2 L_CPML) over the whole
  L_CPML; alpha goes linearly (Eq. linear_transition) from alpha_0 to 0.
* nu >= 2: d and alpha go to 0 with the cosine ramp (Eq.
  cosine_transition) over the inner L_Tr and stay 0 beyond.  With no
  transition layer (L_Tr = 0) they keep their tissue values.
* kappa is unchanged (Table 1, target = initial value).
All through the general formula X(s) = (X~ - X0) g(s) + X0.
Profiles are directional: the x-derivative uses the x distance only.

Two other readings are available for the reflection study only (the library
and the workloads use reading A):
* reading "B": the nu = 1 ramps run over the outer L_Bound only (the
  polynomial and linear functions of Sec. 3.3 take L_B = L_Bound), the
  target d~ still with L_CPML as Table 1 prints it;
* reading "A_kappa": reading A with the target of each derivative scaled by
  its own kappa (d~_i = kappa_i d~), which keeps the ratio of the two
  stretch factors, and so the impedance, at the interior's value deep in the
  layer when kappa_1 != kappa_2;
* reading "A_alpha_tr": reading A with alpha^{nu=1} taken linearly to 0 over
  the inner L_Tr instead of the whole L_CPML (a tissue alpha far above the
  angular frequency otherwise turns the nu = 1 damping into a real stretch
  over most of the layer).
"""
import numpy as np


def g_polynomial(x, L, N):
    """Eq. polynomial_transition: (x/L)^N on [0, L]."""
    return (np.asarray(x, dtype=np.float64) / L) ** N


def g_linear(x, L):
    """Eq. linear_transition: x/L on [0, L]."""
    return np.asarray(x, dtype=np.float64) / L


def g_cosine(x, L):
    """Eq. cosine_transition: (1 - cos(pi x / L)) / 2 on [0, L]."""
    return 0.5 * (1.0 - np.cos(np.pi * np.asarray(x, dtype=np.float64) / L))


def blend(X0, Xt, g):
    """General formula of Sec. 3.3: X = (X~ - X0) g + X0."""
    return (Xt - X0) * g + X0


def d_target(c_p, R_c, N, L_cpml):
    """Table 1 target for d^{nu=1}: -(N+1) c_p log(R_c) / (2 L_CPML)."""
    return -(N + 1) * c_p * np.log(R_c) / (2.0 * L_cpml)


def boundary_distance(coord, n, nb):
    """Distance (in cells) of grid coordinate(s) from the inner edge of the
    boundary region of an axis with n samples and nb boundary cells per side.

    Samples sit at coordinates 0..n-1 (pressure) or k + 1/2 (staggered
    velocity).  The interior spans [nb, n-1-nb]; the result is clamped to nb.
    """
    coord = np.asarray(coord, dtype=np.float64)
    left = nb - coord
    right = coord - (n - 1 - nb)
    s = np.maximum(0.0, np.maximum(left, right))
    return np.minimum(s, float(nb))


def profile(s_cells, h, nb, ntr, d0, a0, nu, c_p, R_c, N, reading="A", kappa=1.0):
    """(d, alpha) of mechanism nu (1-based) at distance s_cells into the layer.

    d0, a0 are the local tissue values (Table 1 initial values); s_cells can be
    an array broadcastable against d0/a0.  reading and kappa: see the module
    notes (kappa is the derivative's own kappa, used by reading "A_kappa").
    """
    s = np.asarray(s_cells, dtype=np.float64)
    if nb == 0:
        return np.broadcast_to(d0, np.broadcast(s, d0).shape).astype(np.float64), \
            np.broadcast_to(a0, np.broadcast(s, a0).shape).astype(np.float64)
    if nu == 1:
        L = nb * h
        dt_ = d_target(c_p, R_c, N, L)
        if reading == "A_kappa":
            dt_ = dt_ * np.asarray(kappa, dtype=np.float64)
        if reading == "B" and nb > ntr:
            Lb = (nb - ntr) * h
            x = np.maximum(s - ntr, 0.0) * h
            return blend(d0, dt_, g_polynomial(x, Lb, N)), blend(a0, 0.0, g_linear(x, Lb))
        if reading not in ("A", "A_kappa", "B", "A_alpha_tr"):
            raise ValueError("unknown boundary reading %r" % (reading,))
        x = s * h
        d = blend(d0, dt_, g_polynomial(x, L, N))
        if reading == "A_alpha_tr" and ntr > 0:
            Ltr = ntr * h
            a = blend(a0, 0.0, g_linear(np.minimum(x, Ltr), Ltr))
        else:
            a = blend(a0, 0.0, g_linear(x, L))
        return d, a
    # nu >= 2: cosine ramp over the transition layer, zero past it.
    if ntr == 0:
        # No transition layer: nu >= 2 keeps its tissue values (the setting
        # the paper reports as unstable inside the C-PML).
        g = np.zeros_like(s)
    else:
        Ltr = ntr * h
        x = np.minimum(s * h, Ltr)
        g = g_cosine(x, Ltr)
    d = blend(d0, 0.0, g)
    a = blend(a0, 0.0, g)
    return d, a
