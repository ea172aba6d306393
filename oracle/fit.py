"""Relaxation-parameter fit to a power law (Sec. 4.1).

The cost of Eq. relaxation_parameter_optimization,
    J = w_a NMSE(alpha_model, alpha_target) + (1 - w_a) NMSE(c_model, c_target),
    NMSE(x, y) = mean((x - y)^2) / Var(y),  w_a = 0.1,
is minimised over the 2 + 4L isotropic parameters inside the bounds of Table 2
(kappa in [0.8, 1.2], d in [1e2, 1e10], alpha in [1e5, 1e12]; all but kappa on
a log scale).  The paper uses a coarse-to-fine grid search; this reading uses a
bounded least-squares solve (the same cost written as a sum of squares) from a
few seeded starting points, which is a different optimiser for the same
objective (the grid search itself is not part of the time stepper).
"""
import numpy as np
from scipy.optimize import least_squares

from . import physics, relaxation

W_ALPHA = 0.1
KAPPA_BOUNDS = (0.8, 1.2)
D_BOUNDS = (1e2, 1e10)
ALPHA_BOUNDS = (1e5, 1e12)

# Table 2 (two mechanisms, alpha0 = 0.5 dB/cm/MHz, y = 1):
#   k1, k2, d1(nu=1,2), d2(nu=1,2), alpha1(nu=1,2), alpha2(nu=1,2)
TABLE2 = np.array([0.835, 1.19,
                   9.82e5, 3.26e6,
                   4.40e4, 1.68e5,
                   2.83e8, 3.54e9,
                   8.35e6, 5.10e7])


def _unpack(theta, L):
    row = np.empty(2 + 4 * L)
    row[0:2] = theta[0:2]
    row[2:] = 10.0 ** theta[2:]
    return row


def _pack(row, L):
    th = np.empty(2 + 4 * L)
    th[0:2] = row[0:2]
    th[2:] = np.log10(row[2:])
    return th


def _bounds(L):
    lo = [KAPPA_BOUNDS[0]] * 2 + [np.log10(D_BOUNDS[0])] * (2 * L) + [np.log10(ALPHA_BOUNDS[0])] * (2 * L)
    hi = [KAPPA_BOUNDS[1]] * 2 + [np.log10(D_BOUNDS[1])] * (2 * L) + [np.log10(ALPHA_BOUNDS[1])] * (2 * L)
    return np.array(lo), np.array(hi)


def nmse(x, y):
    """NMSE of Sec. 4.1: mean squared error over the variance of the target."""
    return np.mean((x - y) ** 2) / np.var(y)


def cost(row, L, f, alpha0, y, c0, f_ref):
    """J of Eq. relaxation_parameter_optimization for one parameter tuple."""
    att, vel = relaxation.model_attenuation_velocity(f, c0, row, L)
    at = physics.power_law_db_cm(f, alpha0, y)
    ct = physics.kk_phase_velocity(f, alpha0, y, c0, f_ref)
    return W_ALPHA * nmse(att, at) + (1.0 - W_ALPHA) * nmse(vel, ct)


def fit_errors(row, L, f, alpha0, y, c0, f_ref):
    """Max relative attenuation and phase-velocity errors over f."""
    att, vel = relaxation.model_attenuation_velocity(f, c0, row, L)
    at = physics.power_law_db_cm(f, alpha0, y)
    ct = physics.kk_phase_velocity(f, alpha0, y, c0, f_ref)
    return float(np.max(np.abs(att / at - 1.0))), float(np.max(np.abs(vel / ct - 1.0)))


def _starts(L, alpha0, rng, n_random):
    """Seeded starting points: Table 2 stretched to L mechanisms, plus random."""
    out = []
    base = TABLE2
    k1, k2 = base[0], base[1]
    # Table 2 mechanisms, interpolated in log space across L mechanisms.
    def spread(v1, v2):
        if L == 1:
            return np.array([np.sqrt(v1 * v2)])
        return np.exp(np.linspace(np.log(v1), np.log(v2), L))
    s = alpha0 / 0.5
    row = np.concatenate([[k1, k2], spread(base[2], base[3]) * s, spread(base[4], base[5]) * s,
                          spread(base[6], base[7]), spread(base[8], base[9])])
    out.append(row)
    lo, hi = _bounds(L)
    for _ in range(n_random):
        th = lo + (hi - lo) * rng.random(lo.size)
        # keep random starts in the region where mechanisms matter
        th[2:2 + 2 * L] = rng.uniform(3.0, 7.5, 2 * L)
        th[2 + 2 * L:] = np.sort(rng.uniform(5.5, 10.0, 2 * L))
        out.append(_unpack(th, L))
    return out


def fit_power_law(alpha0, y, L, c0=1540.0, f_ref=3e6, f_band=(1e6, 20e6), n_freq=40,
                  seed=0, n_random=6, x0=None):
    """Fit the 2+4L relaxation tuple to alpha0 f^y with its KK velocity.

    Returns (row, info) with row = [k1, k2, d1[L], d2[L], alpha1[L], alpha2[L]].
    """
    f = np.linspace(f_band[0], f_band[1], n_freq)
    at = physics.power_law_db_cm(f, alpha0, y)
    ct = physics.kk_phase_velocity(f, alpha0, y, c0, f_ref)
    wa = np.sqrt(W_ALPHA / (f.size * np.var(at)))
    wc = np.sqrt((1.0 - W_ALPHA) / (f.size * np.var(ct)))

    def resid(theta):
        row = _unpack(theta, L)
        att, vel = relaxation.model_attenuation_velocity(f, c0, row, L)
        return np.concatenate([wa * (att - at), wc * (vel - ct)])

    lo, hi = _bounds(L)
    rng = np.random.default_rng(seed)
    starts = ([np.asarray(x0, dtype=np.float64)] if x0 is not None else []) + _starts(L, alpha0, rng, n_random)
    best = None
    for row0 in starts:
        th0 = np.clip(_pack(row0, L), lo + 1e-9, hi - 1e-9)
        try:
            res = least_squares(resid, th0, bounds=(lo, hi), method="trf", x_scale="jac",
                                max_nfev=4000, xtol=1e-12, ftol=1e-12)
        except (ValueError, FloatingPointError):
            continue
        J = float(2.0 * res.cost)
        if best is None or J < best[0]:
            best = (J, res.x)
    row = _unpack(best[1], L)
    ea, ec = fit_errors(row, L, f, alpha0, y, c0, f_ref)
    return row, {"J": best[0], "max_att_err": ea, "max_vel_err": ec, "f_ref": f_ref,
                 "band": list(f_band), "c0": c0}
