"""Closed-form physics used as targets and pins (test infrastructure only).

* Power-law attenuation alpha(f) = alpha0 f^y (Sec. 4.1) and the phase
  velocity the Kramers-Kronig relations attach to it (Sec. 4.1 names the
  relation but prints no formula; the standard nearly-local forms are used:
  y = 1:   1/c(w) = 1/c(w0) - (2/pi) a' ln(w/w0)
  y != 1:  1/c(w) = 1/c(w0) + a' tan(pi y / 2) (w^(y-1) - w0^(y-1))
  with alpha(w) = a' w^y in Np/m and c(w0) = c0 at the anchor frequency).
* Free-space Green's functions of the lossless wave equation (2D, 3D), used
  for the lossless-propagation pin.
* The exact pre-shock simple-wave solution of the 1D lossless form of Eqs.
  general5 / general6 (used for the nonlinearity pin, Sec. 4.5).
"""
import numpy as np
from scipy import special

DB_PER_NEPER = 20.0 / np.log(10.0)


def power_law_db_cm(f_hz, alpha0_db_cm_mhz, y):
    """Target attenuation alpha0 * f^y in dB/cm (f in MHz inside the law)."""
    return alpha0_db_cm_mhz * (np.asarray(f_hz, dtype=np.float64) / 1e6) ** y


def kk_phase_velocity(f_hz, alpha0_db_cm_mhz, y, c0, f_ref_hz):
    """Kramers-Kronig phase velocity of the power law, c(f_ref) = c0."""
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    w0 = 2.0 * np.pi * float(f_ref_hz)
    # a' in Np/m/(rad/s)^y:  alpha_Np/m(w) = a' w^y
    ap = alpha0_db_cm_mhz * 100.0 / DB_PER_NEPER / (2.0 * np.pi * 1e6) ** y
    if abs(y - 1.0) < 1e-12:
        inv = 1.0 / c0 - (2.0 / np.pi) * ap * np.log(w / w0)
    else:
        inv = 1.0 / c0 + ap * np.tan(np.pi * y / 2.0) * (w ** (y - 1.0) - w0 ** (y - 1.0))
    return 1.0 / inv


def greens_2d_freq(omega, r, c):
    """2D Green's function of (d_tt - c^2 lap) G = delta(x) delta(t), for the
    time convention exp(+i w t):  G(w, r) = -(i / (4 c^2)) H0^(2)(w r / c)."""
    return -1j / (4.0 * c * c) * special.hankel2(0, np.asarray(omega) * r / c)


def greens_3d_freq(omega, r, c):
    """3D counterpart: G(w, r) = exp(-i w r / c) / (4 pi c^2 r)."""
    return np.exp(-1j * np.asarray(omega) * r / c) / (4.0 * np.pi * c * c * r)


def simple_wave_speed(p, rho0, kappa0, beta, nl=(1.0, 1.0, -2.0)):
    """Local propagation speed 1/sqrt(rho(p) kappa(p)) of the 1D lossless
    system with rho = rho0 (1 + A kappa0 p), kappa = kappa0 (1 + kappa0 B p),
    B = B0 + B1 beta; nl = (A, B0, B1), as printed in Eqs. state1 / state2
    (1, 1, -2) by default."""
    A, B0, B1 = nl
    B = B0 + B1 * beta
    return 1.0 / np.sqrt(rho0 * (1.0 + A * kappa0 * p) * kappa0 * (1.0 + kappa0 * B * p))


def simple_wave_propagate(t, f_samples, dist, rho0, kappa0, beta, nl=(1.0, 1.0, -2.0)):
    """Pre-shock solution p(x0 + dist, t) of a right-going simple wave whose
    waveform at x0 is f (sampled on the uniform grid t).

    Each value f(tau) travels unchanged at speed c(f(tau)); so the waveform at
    distance dist is p(tau + dist / c(f(tau))) = f(tau).  The result is
    interpolated back onto t (valid while arrival times stay monotone, i.e.
    before a shock forms).
    """
    f = np.asarray(f_samples, dtype=np.float64)
    arrival = np.asarray(t, dtype=np.float64) + dist / simple_wave_speed(f, rho0, kappa0, beta, nl)
    if np.any(np.diff(arrival) <= 0):
        raise ValueError("characteristics cross: shock formed")
    return np.interp(t, arrival, f, left=0.0, right=0.0)
