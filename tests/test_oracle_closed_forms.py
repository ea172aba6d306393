"""Pins of the oracle's host math against closed forms and definitions.

Each test checks an oracle function against something other than its own
formula: a textbook result, a definition evaluated by quadrature, a brute-force
sum, or a reduction to a known special case.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import fit, physics, pml, relaxation, stencil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------- stencil ---

def test_stencil_r0_is_textbook_eighth_order():
    """Sec. 3.1: at r -> 0 the (8,4) operator must reduce to the classical
    eighth-order staggered first derivative 1225/1024, -245/3072, 49/5120,
    -5/7168 (Fornberg's staggered weights), with no cross term."""
    for ndim in (2, 3):
        g, g11 = stencil.stencil_weights(0.0, ndim)
        assert g11 == 0.0
        np.testing.assert_allclose(g, [1225 / 1024, -245 / 3072, 49 / 5120, -5 / 7168], rtol=0, atol=1e-15)


def test_stencil_textbook_set_differentiates_polynomials_exactly():
    """Independent pin: the r = 0 weights differentiate x^k exactly for
    k <= 8 on the staggered points (eighth-order accuracy)."""
    g, _ = stencil.stencil_weights(0.0, 2)
    for k in range(0, 9):
        val = sum(g[m - 1] * ((m - 0.5) ** k - (-(m - 0.5)) ** k) for m in range(1, 5))
        exact = 1.0 if k == 1 else 0.0
        assert abs(val - exact) < 1e-12, k


@pytest.mark.parametrize("ndim", [2, 3])
def test_stencil_time_space_phase_velocity(ndim):
    """The (8,4) set at r = 0.4 keeps the numerical phase velocity of the
    leapfrog scheme within 2e-5 of c at 12 points per wavelength in every
    direction, while the same scheme with the r = 0 (space-only) weights is an
    order of magnitude worse: the time correction is really there."""
    r = 0.4
    g, g11 = stencil.stencil_weights(r, ndim)
    g0, g110 = stencil.stencil_weights(0.0, ndim)
    worst, worst0 = 0.0, 0.0
    for ang in np.linspace(0, np.pi / 2, 19):
        worst = max(worst, abs(stencil.scheme_phase_velocity_ratio(g, g11, r, 12, ang, ndim) - 1))
        worst0 = max(worst0, abs(stencil.scheme_phase_velocity_ratio(g0, g110, r, 12, ang, ndim) - 1))
    assert worst < 2e-5
    assert worst0 > 10 * worst


def test_stencil_phase_velocity_converges_with_ppw():
    """Phase error along the axis falls at least like ppw^-8 between 8 and 16
    points per wavelength (space order 8)."""
    r = 0.3
    g, g11 = stencil.stencil_weights(r, 2)
    e8 = abs(stencil.scheme_phase_velocity_ratio(g, g11, r, 6, 0.0) - 1)
    e16 = abs(stencil.scheme_phase_velocity_ratio(g, g11, r, 12, 0.0) - 1)
    assert e8 / e16 > 2 ** 7


# ------------------------------------------------------------- relaxation ---

PARAMS = [  # kappa, d, alpha: Table 2 mechanisms and a boundary-like one
    (0.835, 9.82e5, 2.83e8), (0.835, 3.26e6, 3.54e9), (1.19, 4.40e4, 8.35e6),
    (1.19, 1.68e5, 5.10e7), (1.0, 5.0e6, 0.0), (1.0, 1.0e7, 1.2e7)]


@pytest.mark.parametrize("kappa,d,alpha", PARAMS)
def test_memory_coefficients_match_kernel_integral(kappa, d, alpha):
    """Sec. 3.2: Z(m) = integral of zeta over [m dt, (m+1) dt] must equal
    a b^m, with zeta of Eq. convolution_kernel_x integrated by quadrature."""
    dt = 1.6667e-8
    a, b = relaxation.memory_coefficients(kappa, d, alpha, dt)
    for m in (0, 1, 2, 5):
        Z, _ = integrate.quad(lambda t: relaxation.kernel_zeta(t, kappa, d, alpha),
                              m * dt, (m + 1) * dt, epsabs=0, epsrel=1e-12)
        assert abs(a * b ** m - Z) <= 1e-9 * abs(a) + 1e-300


def test_memory_coefficients_d_zero_is_inert():
    a, b = relaxation.memory_coefficients(1.0, 0.0, 0.0, 1e-8)
    assert a == 0.0 and b == 1.0
    a, b = relaxation.memory_coefficients(0.9, 0.0, 3e6, 1e-8)
    assert a == 0.0 and abs(b - np.exp(-3e6 * 1e-8)) < 1e-15


def test_recursion_equals_brute_force_convolution():
    """Eq. relaxation_psi must reproduce the discrete convolution
    psi^n = sum_{m=0}^{n-1} Z(m) D^{n-m-1/2} (update-then-use: the newest
    derivative enters with weight Z(0) = a)."""
    rng = np.random.default_rng(3)
    dt = 2e-8
    kappa, d, alpha = 0.9, 2e6, 4e7
    a, b = relaxation.memory_coefficients(kappa, d, alpha, dt)
    D = rng.standard_normal(60)          # D[n-1] is the derivative at n - 1/2
    psi = 0.0
    for n in range(1, 61):
        psi = b * psi + a * D[n - 1]
        brute = sum(integrate.quad(lambda t: relaxation.kernel_zeta(t, kappa, d, alpha),
                                   m * dt, (m + 1) * dt, epsrel=1e-12)[0] * D[n - m - 1]
                    for m in range(n)) if n in (1, 2, 7, 60) else None
        if brute is not None:
            assert abs(psi - brute) < 1e-9 * max(1.0, abs(brute))


def test_gamma_is_fourier_transform_of_kernel():
    """Eq. gamma1: -sum gamma equals the Fourier transform of the kernels,
    evaluated here by quadrature of zeta(t) exp(-i w t)."""
    kappa, d, alpha = 1.19, 1.68e5, 5.10e7
    for f in (1e6, 7e6):
        w = 2 * np.pi * f
        rate = d / kappa + alpha
        T = 40.0 / rate
        re = integrate.quad(lambda t: relaxation.kernel_zeta(t, kappa, d, alpha) * np.cos(w * t), 0, T,
                            limit=2000)[0]
        im = integrate.quad(lambda t: -relaxation.kernel_zeta(t, kappa, d, alpha) * np.sin(w * t), 0, T,
                            limit=2000)[0]
        g = relaxation.gamma(w, kappa, [d], [alpha])
        assert abs((re + 1j * im) + g) < 1e-7 * abs(g)


def test_dispersion_single_mechanism_is_cpml_stretch():
    """Sec. 2.1 special case: with N = 1 and nabla_1 = nabla_2 the stretched
    derivative is the C-PML one, k = (w/c) s with the textbook stretch
    s = kappa + d / (alpha + i w) (Kuzuoglu-Mittra / Komatitsch-Martin)."""
    c = 1500.0
    for kappa, d, alpha in [(1.0, 3e6, 0.0), (1.3, 5e6, 2e6), (0.9, 1e5, 1e7)]:
        for f in (0.5e6, 2e6, 11e6):
            w = 2 * np.pi * f
            k = relaxation.wavenumber(w, c, kappa, kappa, [d], [d], [alpha], [alpha])
            s = kappa + d / (alpha + 1j * w)
            assert abs(k - (w / c) * s) < 1e-12 * abs(k)


def test_dispersion_lossless_limit():
    for f in (1e6, 9e6):
        w = 2 * np.pi * f
        k = relaxation.wavenumber(w, 1540.0, 1.0, 1.0, [0.0], [0.0], [1e6], [1e6])
        assert abs(k - w / 1540.0) < 1e-12 * abs(k)


def test_table2_reproduces_power_law_over_2_to_20_mhz():
    """Table 2 through Eq. dispersion_relations: attenuation within 5% of
    0.5 f dB/cm from 2 to 20 MHz and decaying waves (Im k < 0).  At 1 MHz the
    printed (3-digit) values give about -9%, recorded here as found."""
    row = np.array(fit.TABLE2)
    f = np.array([2, 3, 5, 8, 10, 15, 20]) * 1e6
    att, vel = relaxation.model_attenuation_velocity(f, 1540.0, row, 2)
    assert np.all(np.abs(att / (0.5 * f / 1e6) - 1) < 0.05)
    att1, _ = relaxation.model_attenuation_velocity(np.array([1e6]), 1540.0, row, 2)
    assert -0.11 < att1[0] / 0.5 - 1 < -0.07
    k = relaxation.wavenumber(2 * np.pi * f, 1540.0, row[0], row[1], row[2:4], row[4:6], row[6:8], row[8:10])
    assert np.all(k.imag < 0)
    # phase velocity follows the y = 1 Kramers-Kronig curve (anchored at 10 MHz) within 0.1 %
    ct = physics.kk_phase_velocity(f, 0.5, 1.0, vel[f == 10e6][0], 10e6)
    assert np.all(np.abs(vel / ct - 1) < 1e-3)


def test_kk_velocity_matches_numerical_kramers_kronig():
    """Pin of the nearly-local KK forms: the y = 1 and y = 1.5 laws' velocity
    differences must agree with the difference of their defining expressions
    obtained by numerically integrating d(1/c)/dw = -(2/pi) a'/w (y = 1) and
    a' tan(pi y/2) (y - 1) w^(y-2) (y != 1)."""
    c0, fr = 1540.0, 3e6
    f = np.array([1e6, 5e6, 20e6])
    for y in (1.0, 1.5):
        ap = 0.5 * 100 / physics.DB_PER_NEPER / (2 * np.pi * 1e6) ** y
        for fi, ci in zip(f, physics.kk_phase_velocity(f, 0.5, y, c0, fr)):
            if y == 1.0:
                dinv = integrate.quad(lambda w: -(2 / np.pi) * ap / w, 2 * np.pi * fr, 2 * np.pi * fi)[0]
            else:
                dinv = integrate.quad(lambda w: ap * np.tan(np.pi * y / 2) * (y - 1) * w ** (y - 2),
                                      2 * np.pi * fr, 2 * np.pi * fi)[0]
            assert abs(1 / ci - (1 / c0 + dinv)) < 1e-12 / c0


def test_stored_tissue_fits_meet_paper_accuracy():
    """Every stored relaxation tuple, re-evaluated through the dispersion
    relation, stays within the paper's fitting accuracy (Sec. 4.1 / Sec. 5.2:
    attenuation error < 5 %, phase velocity error < 0.5 % over 1-20 MHz)."""
    with open(os.path.join(ROOT, "workloads", "tissue_fits.json")) as fh:
        fits = json.load(fh)["fits"]
    assert len(fits) >= 70
    f = np.linspace(1e6, 20e6, 77)
    for key, v in fits.items():
        row = np.array(v["row"])
        ea, ec = fit.fit_errors(row, v["L"], f, v["alpha0"], v["y"], v["c0"], v["f_ref"])
        assert ea < 0.05, key
        assert ec < 0.005, key
        lo, hi = fit._bounds(v["L"])
        th = fit._pack(row, v["L"])
        assert np.all(th >= lo - 1e-9) and np.all(th <= hi + 1e-9), key


def test_fitter_objective_is_papers_cost():
    """The least-squares residual of fit.fit_power_law sums to J of Eq.
    relaxation_parameter_optimization (NMSE = MSE / Var(target), w_a = 0.1)."""
    row, info = fit.fit_power_law(0.5, 1.0, 2, n_random=0)
    f = np.linspace(1e6, 20e6, 40)
    att, vel = relaxation.model_attenuation_velocity(f, 1540.0, row, 2)
    at = 0.5 * f / 1e6
    ct = physics.kk_phase_velocity(f, 0.5, 1.0, 1540.0, 3e6)
    J = 0.1 * np.mean((att - at) ** 2) / np.var(at) + 0.9 * np.mean((vel - ct) ** 2) / np.var(ct)
    assert abs(J - info["J"]) < 1e-9 + 1e-6 * J
    assert info["max_att_err"] < 0.05 and info["max_vel_err"] < 0.005


# -------------------------------------------------------------------- PML ---

def test_profile_endpoints_follow_table1():
    """Table 1: initial values at the inner edge, targets at the outer edge
    (nu = 1: d -> d~, alpha -> 0; nu >= 2: both -> 0 at the end of the
    transition layer and beyond); kappa is not touched by the profile."""
    h, nb, ntr, cp, Rc, N = 1e-4, 48, 36, 1540.0, 1e-3, 2
    d0, a0 = 7e5, 3e8
    dtil = -(N + 1) * cp * np.log(Rc) / (2 * nb * h)
    d, a = pml.profile(0.0, h, nb, ntr, d0, a0, 1, cp, Rc, N)
    assert d == d0 and a == a0
    d, a = pml.profile(float(nb), h, nb, ntr, d0, a0, 1, cp, Rc, N)
    assert abs(d - dtil) < 1e-9 * dtil and abs(a) < 1e-9
    d, a = pml.profile(float(ntr), h, nb, ntr, d0, a0, 2, cp, Rc, N)
    assert abs(d) < 1e-9 and abs(a) < 1e-6
    d, a = pml.profile(float(nb), h, nb, ntr, d0, a0, 2, cp, Rc, N)
    assert d == 0 and a == 0
    d, a = pml.profile(ntr / 2.0, h, nb, ntr, d0, a0, 2, cp, Rc, N)
    assert abs(d - d0 / 2) < 1e-9 * d0          # cosine ramp midpoint


def test_profile_theoretical_reflection_is_Rc():
    """With kappa = 1 and alpha = 0 the continuous C-PML's normal-incidence
    round-trip reflection is exp(-(2/c) * integral of d over the layer); the
    target d~ of Table 1 must make it exactly R_c (quadrature of the profile)."""
    h, nb, cp, Rc, N = 5e-5, 48, 1540.0, 1e-3, 2
    val = integrate.quad(lambda s: pml.profile(s, h, nb, 36, 0.0, 0.0, 1, cp, Rc, N)[0], 0, nb)[0] * h
    assert abs(np.exp(-2 * val / cp) - Rc) < 1e-9


def test_boundary_distance_is_mirror_symmetric():
    n, nb = 40, 6
    s_int = pml.boundary_distance(np.arange(n), n, nb)
    assert np.array_equal(s_int, s_int[::-1])
    s_half = pml.boundary_distance(np.arange(n) + 0.5, n, nb)
    # v sample k (at k + 1/2) mirrors v sample n - 2 - k
    assert np.array_equal(s_half[:n - 1], s_half[:n - 1][::-1])
    assert s_int[nb] == 0 and s_int[0] == nb and s_half[nb - 1] == 0.5 and s_half[n - 1] == nb
