"""Relaxation mechanisms: memory-variable coefficients and dispersion relation.

Sec. 2.1 (Eqs. relaxation1-3, convolution_kernel_x): each stretched derivative
is (1/kappa) d/dx + sum_nu zeta^nu * d/dx with the causal kernel
    zeta^nu(t) = -(d^nu / kappa^2) exp(-(d^nu/kappa + alpha^nu) t) H(t).
Sec. 3.2 (Eqs. relaxation_a, relaxation_b, relaxation_psi): the convolution is
advanced by psi^n = b psi^{n-1} + a (d/dx)^{n-1/2} with
    b = exp(-(d/kappa + alpha) dt),   a = d / (kappa (d + kappa alpha)) (b - 1).
Eqs. dispersion_relations and gamma1 give the plane-wave wavenumber.
"""
import numpy as np


def kernel_zeta(t, kappa, d, alpha):
    """zeta(t) of Eq. convolution_kernel_x (t >= 0 branch, H(t) = 1)."""
    return -(d / kappa**2) * np.exp(-(d / kappa + alpha) * t)


def memory_coefficients(kappa, d, alpha, dt):
    """(a, b) of Eqs. relaxation_a and relaxation_b, elementwise.

    a is defined as 0 where d == 0 (the kernel vanishes identically there);
    this also covers the 0/0 of d = alpha = 0.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    b = np.exp(-(d / kappa + alpha) * dt)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = d / (kappa * (d + kappa * alpha)) * (b - 1.0)
    a = np.where(d == 0.0, 0.0, a)
    return a, b


def centred_weights(kappa, d, alpha, dt):
    """(e0, e1) of the time-centred evaluation of the convolution (reading).

    The leapfrog applies a stretched derivative at the time t_k of its newest
    derivative sample D_k.  Evaluating the convolution of Sec. 3.2 at t_k with
    D taken linear between consecutive samples gives
        psi(t_k) = e0 D_k + sum_{j>=1} b^(j-1) (e1 + b e0) D_{k-j},
        e0 = int_0^dt zeta(tau) (1 - tau/dt) dtau,
        e1 = int_0^dt zeta(tau) (tau/dt) dtau,
    so e0 + e1 = a (the paper's Z(0)) and the history still decays by b.
    Returns arrays; both are 0 where d == 0.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    lam = d / kappa + alpha
    x = lam * dt
    amp = -d / kappa**2
    with np.errstate(divide="ignore", invalid="ignore"):
        # int_0^dt exp(-lam tau) dtau and int_0^dt tau exp(-lam tau) dtau / dt
        i0 = -np.expm1(-x) / lam
        i1 = (-np.expm1(-x) - x * np.exp(-x)) / (lam * x)
    e1 = amp * i1
    e0 = amp * i0 - e1
    e0 = np.where(d == 0.0, 0.0, e0)
    e1 = np.where(d == 0.0, 0.0, e1)
    return e0, e1


def gamma(omega, kappa, d_list, alpha_list):
    """gamma of Eq. gamma1: sum_nu (d/kappa^2) / (d/kappa + alpha + i w)."""
    omega = np.asarray(omega, dtype=np.float64)
    g = np.zeros_like(omega, dtype=np.complex128)
    for d, al in zip(d_list, alpha_list):
        g = g + (d / kappa**2) / (d / kappa + al + 1j * omega)
    return g


def wavenumber(omega, c, k1, k2, d1, d2, a1, a2):
    """Complex k of Eq. dispersion_relations for p ~ exp(i(w t - k x)).

    k = (w/c) (1/(k1 k2) - g1/k2 - g2/k1 + g1 g2)^(-1/2), principal root,
    which here has Re k > 0 and Im k < 0 (decay along +x).
    """
    g1 = gamma(omega, k1, d1, a1)
    g2 = gamma(omega, k2, d2, a2)
    inner = 1.0 / (k1 * k2) - g1 / k2 - g2 / k1 + g1 * g2
    return (np.asarray(omega) / c) * inner ** (-0.5)


NP_PER_M_TO_DB_PER_CM = 20.0 / np.log(10.0) / 100.0


def model_attenuation_velocity(f_hz, c, row, L):
    """Attenuation (dB/cm) and phase velocity (m/s) of one relaxation tuple.

    row = [k1, k2, d1[L], d2[L], alpha1[L], alpha2[L]] (the 2 + 4L isotropic
    parameters listed in Sec. 3.2).  alpha = -Im k (Np/m), c_ph = w / Re k.
    """
    k1, k2 = row[0], row[1]
    d1 = row[2:2 + L]
    d2 = row[2 + L:2 + 2 * L]
    al1 = row[2 + 2 * L:2 + 3 * L]
    al2 = row[2 + 3 * L:2 + 4 * L]
    w = 2.0 * np.pi * np.asarray(f_hz, dtype=np.float64)
    k = wavenumber(w, c, k1, k2, d1, d2, al1, al2)
    att = -k.imag * NP_PER_M_TO_DB_PER_CM
    vel = w / k.real
    return att, vel
