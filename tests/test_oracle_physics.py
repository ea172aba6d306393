"""Physics pins of the FP64 oracle against what the paper and the mathematics
fix: free-space Green's function, plane-wave attenuation / dispersion
(Sec. 4.1, Fig. 2), two-stage C-PML reflection (Secs. 4.2-4.3, Fig. 3) and
nonlinear steepening against the exact pre-shock simple wave (Sec. 4.5)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import physics, relaxation, solver

C0 = 1540.0


# --------------------------------------------------------- Green's function ---

def _green_run(ppw, cfl, f0=2e6, dists=(5, 8)):
    lam = ppw
    n = int(2 * (max(dists) * lam + 20) + 2 * 4 * lam)
    prob = W.homogeneous((n, n), L=1, row=W.lossless_row(1), nb=(4 * lam,) * 2, ntr=(3 * lam,) * 2,
                         f0=f0, ppw=ppw, cfl=cfl)
    prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    h, dt = prob.h, prob.dt
    nt = int((max(dists) * lam * h / C0 + 12 * 3 / (4 * f0)) / dt) + 50
    sig = W.gaussian_pulse(nt, dt, f0, 3, amp=1.0)
    ctr = n // 2
    prob.signals = sig[None]
    prob.src_idx = prob.flat(np.array([ctr]), np.array([ctr]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    rs = [(d * lam, 0) for d in dists] + [(int(round(d * lam / np.sqrt(2))),) * 2 for d in dists]
    prob.rcv_idx = prob.flat(np.array([ctr + a for a, b in rs]), np.array([ctr + b for a, b in rs]))
    _, tr = solver.run(prob, nt)
    # Additive injection of s_n after the pressure update is a source term
    # dp/dt += (h^2/dt) s(t) delta(x) with s_n at t = (n+1/2) dt; p of trace row n
    # is at (n+1) dt.  p = G * d/dt(source).
    N = 8 * nt
    s = np.zeros(N)
    s[:nt] = sig
    S = np.fft.rfft(s)
    w = 2 * np.pi * np.fft.rfftfreq(N, dt)
    errs = []
    for k, (a, b) in enumerate(rs):
        r = np.hypot(a, b) * h
        P = np.zeros_like(S)
        P[1:] = physics.greens_2d_freq(w[1:], r, C0) * 1j * w[1:] * (h * h / dt) * S[1:] * np.exp(1j * w[1:] * dt / 2)
        pa = np.fft.irfft(P, N)[:nt]
        errs.append(np.linalg.norm(tr[:, k] - pa) / np.linalg.norm(pa))
    return np.array(errs)


def test_lossless_point_source_matches_2d_greens_function(oracle_lib):
    """Lossless homogeneous medium, 12 ppw, CFL 0.4: traces at 5 and 8
    wavelengths (on axis and diagonal) match the analytic 2D Green's function
    convolution within 1 % (rel L2); halving the time step cuts the error
    about four-fold (the source term is second order in time)."""
    e = _green_run(12, 0.4)
    assert np.all(e < 1e-2), e
    e2 = _green_run(12, 0.2)
    assert np.all(e2 < e / 3.0), (e, e2)


# ------------------------------------------- attenuation and dispersion (E1) ---

def _plane_wave_measure(row, L, f0, scheme=1, ppw=12, cfl=0.4, width=64, dist_lam=10):
    """Plane pulse from a full-width line source; attenuation (dB/cm) and
    phase velocity between two receivers dist_lam wavelengths apart, at the
    spectral line nearest f0 (Sec. 4.1 measurement)."""
    lam = ppw
    nb, ntr = 4 * lam, 3 * lam
    nx = width + 2 * nb
    ys = nb + 4
    y1 = ys + 2 * lam
    y2 = y1 + dist_lam * lam
    ny = y2 + 2 * lam + nb
    prob = W.homogeneous((nx, ny), L=L, row=row, nb=(nb, nb), ntr=(ntr, ntr), f0=f0, ppw=ppw, cfl=cfl)
    prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    prob.relax_scheme = scheme
    h, dt = prob.h, prob.dt
    npulse = W.pulse_length(dt, f0, 3)
    nt = int((y2 - ys) * h / C0 / dt) + npulse + 200
    xs = np.arange(nx)
    prob.src_idx = prob.flat(xs, np.full_like(xs, ys))
    prob.src_sig = np.zeros(nx, np.int32)
    prob.src_w = np.ones(nx, np.float32)
    prob.signals = W.gaussian_pulse(npulse, dt, f0, 3, 1.0)[None]
    cx = nx // 2
    prob.rcv_idx = prob.flat(np.array([cx, cx]), np.array([y1, y2]))
    _, tr = solver.run(prob, nt)
    N = 4 * nt
    P1, P2 = np.fft.rfft(tr[:, 0], N), np.fft.rfft(tr[:, 1], N)
    f = np.fft.rfftfreq(N, dt)
    k = np.argmin(np.abs(f - f0))
    dx = (y2 - y1) * h
    att = np.log(np.abs(P1[k]) / np.abs(P2[k])) / dx * relaxation.NP_PER_M_TO_DB_PER_CM
    w = 2 * np.pi * f[k]
    tau0 = dx / C0
    tau = tau0 - np.angle(P2[k] / P1[k] * np.exp(1j * w * tau0)) / w
    return f[k], att, dx / tau


FREQS = [1e6, 2e6, 5e6, 10e6, 20e6]


def test_attenuation_and_dispersion_follow_power_law(oracle_lib):
    """Sec. 4.1 / Fig. 2: a pulse propagated 10 wavelengths at 12 ppw,
    CFL 0.4, in the fitted alpha0 = 0.5 dB/cm/MHz, y = 1 medium (two
    mechanisms): measured attenuation within 1 % and phase velocity within
    5e-5 of the dispersion relation (Eq. dispersion_relations), hence within
    the paper's 5 % / 0.5 % of alpha0 f^y and its Kramers-Kronig velocity."""
    row = W.tissue_row(0.5, 1.0, 2, 2e6)
    for f0 in FREQS:
        fk, att, vel = _plane_wave_measure(row, 2, f0)
        a_an, c_an = relaxation.model_attenuation_velocity(np.array([fk]), C0, np.array(row), 2)
        assert abs(att / a_an[0] - 1) < 0.01, (f0, att, a_an)
        assert abs(vel / c_an[0] - 1) < 5e-5, (f0, vel, c_an)
        assert abs(att / physics.power_law_db_cm(fk, 0.5, 1.0) - 1) < 0.05
        assert abs(vel / physics.kk_phase_velocity(fk, 0.5, 1.0, C0, 2e6) - 1) < 0.005


@pytest.mark.parametrize("L", [4, 6, 8])
def test_attenuation_y_not_one_and_many_mechanisms(oracle_lib, L):
    """Same measurement for a y = 1.3 law with four mechanisms (the kind of
    tuple the heterogeneous 2D workload uses) and with six and eight, at 3
    and 12 MHz.  Phase velocity: within 2e-4 of the dispersion relation with
    four mechanisms, 3e-4 with six and eight (measured 2.0e-4 and 2.2e-4 at
    12 MHz), in all cases more than an order of magnitude inside the
    paper's 0.5 %."""
    row = W.tissue_row(1.5, 1.3, L, 3e6)
    for f0 in (3e6, 12e6):
        fk, att, vel = _plane_wave_measure(row, L, f0)
        a_an, c_an = relaxation.model_attenuation_velocity(np.array([fk]), C0, np.array(row), L)
        assert abs(att / a_an[0] - 1) < 0.01
        assert abs(vel / c_an[0] - 1) < (2e-4 if L <= 4 else 3e-4)
        assert abs(att / physics.power_law_db_cm(fk, 1.5, 1.3) - 1) < 0.05


def test_printed_recursion_loses_attenuation(oracle_lib):
    """The literal update-then-use recursion (Eq. relaxation_psi entering
    the step that produced it) applies psi half a step late: at 12 ppw /
    CFL 0.4 the measured attenuation falls 10-30 % below the dispersion
    relation (this is why the time-centred evaluation is the default)."""
    row = W.tissue_row(0.5, 1.0, 2, 2e6)
    fk, att, vel = _plane_wave_measure(row, 2, 2e6, scheme=0)
    a_an, _ = relaxation.model_attenuation_velocity(np.array([fk]), C0, np.array(row), 2)
    assert -0.30 < att / a_an[0] - 1 < -0.10


# ----------------------------------------------------- C-PML reflection (E2/E3) ---
# The reflection sweeps take minutes, so tests/golden/make_reflection_figures.py
# (oracle only) stores the measured figures; the pins below read them, and
# test_stored_reflection_figures_match_the_oracle recomputes one case.

_FIG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _figures():
    with open(os.path.join(_FIG, "reflection_figures.json")) as fh:
        return {k: np.array(v["dB"]) for k, v in json.load(fh).items()}


def test_stored_reflection_figures_match_the_oracle(oracle_lib):
    """The stored figures are the current oracle's: one case (Table 2 verbatim,
    3 + 1 lambda, normal incidence) recomputed gives the stored value."""
    sys.path.insert(0, _FIG)
    import make_reflection_figures as mk
    key, row, L, angles, kw = [c for c in mk.cases() if c[0] == "table2 3+1"][0]
    assert np.allclose(mk.measure(row, L, angles, kw), _figures()[key], atol=1e-6, rtol=0)


def test_cpml_reflection_over_the_stated_angles(golden):
    """Secs. 4.2-4.3 at 16 ppw, CFL 0.2, 3 lambda transition + 1 lambda bound:
    the stated bound of about -49 dB from 0 to 80 degrees and the -50 dB of
    the 3 + 1 lambda layer, read from the fixture.  R_c is not stated: with
    R_c = 1e-4 the C-PML special case (lossless interior) meets the bound at
    every angle; with the library's R_c = 1e-3 the fitted two-mechanism
    tissue meets it up to 60 degrees, and above that reflects more (recorded
    finding: -46.6 dB at 70, -34.6 dB at 80 degrees).  In this measurement
    (point source one wavelength above the layer) the reflection grows with
    the angle: the minimum near 45 degrees of the paper's figure is not
    reproduced (recorded finding)."""
    st = golden.stated()
    fig = _figures()
    bound, b31 = st["reflection_db_all_angles_max"], st["reflection_db_tr3_bd1"]
    assert (st["ppw_reflection"], st["cfl_reflection"]) == (16, 0.2)
    r = fig["lossless 3+1 R_c 1e-4"]
    assert np.all(r <= bound), r
    assert r[0] <= b31, r
    rf = fig["fitted 3+1"]
    assert rf[0] <= b31, rf
    assert np.all(rf[:4] <= bound), rf                       # 0 .. 60 degrees
    assert -49.0 < rf[4] < -44.0 and -38.0 < rf[5] < -31.0, rf   # 70, 80 degrees: above the bound
    for curve in (r, rf):                                     # grows with the angle: no minimum at 45
        assert np.all(np.diff(curve) > 0), curve


def test_cpml_reflection_thickness_and_table2(golden):
    """Sec. 4.2: about -50 dB with a 3 + 1 lambda layer and -60 dB with
    5 + 1 lambda, read from the fixture, at normal incidence.  The lossless
    special case meets the 5 + 1 figure with the library's R_c = 1e-3 (and
    the 3 + 1 figure, checked over the angles above).  Table 2 verbatim
    does not (recorded finding: about -38.7 dB at 3 + 1): its nu = 1 nabla_1
    mechanism has alpha = 2.83e8 1/s, twenty times the angular frequency of
    the 2 MHz pulse, and with alpha ramped linearly to 0 over the whole layer
    (Table 1) the damping d / (alpha + i omega) of that derivative is nearly
    real over most of the layer, so the layer absorbs only part of what R_c
    promises.  Two checks of that reading of the finding: the reflection
    follows R_c at about 10 dB per decade (with R_c = 1e-5 Table 2 meets both
    stated figures), and taking alpha to 0 over the transition layer instead
    (oracle reading "A_alpha_tr", a study reading, not the library's) brings
    Table 2 below -50 dB at R_c = 1e-3."""
    st = golden.stated()
    fig = _figures()
    b31, b51 = st["reflection_db_tr3_bd1"], st["reflection_db_tr5_bd1"]
    assert fig["lossless 5+1"][0] <= b51
    t3 = fig["table2 3+1"][0]
    assert -42.0 < t3 < -35.0, t3
    t3e = fig["table2 3+1 R_c 1e-5"][0]
    assert t3e <= b31 and -24.0 < t3e - t3 < -17.0, (t3, t3e)
    assert fig["table2 5+1 R_c 1e-5"][0] <= b51
    ta = fig["table2 3+1 alpha over the transition"][0]
    assert ta <= b31 and ta < t3 - 10.0, (t3, ta)


# ------------------------------------------------ nonlinear steepening (E5) ---

@pytest.mark.parametrize("form", ["printed", "westervelt"])
def test_nonlinear_plane_wave_matches_exact_simple_wave(oracle_lib, form):
    """Sec. 4.5: lossless plane pulse (1 MHz, 4 cycles), 20 ppw, CFL 0.4.
    The waveform recorded at receiver 1 is propagated to receiver 2 with the
    exact pre-shock simple-wave solution of the same equations (each value
    travels at 1/sqrt(rho(p) kappa(p))); at sigma ~ 0.35 the first four
    harmonic levels agree within 1 dB.  As printed (Eqs. state1 / state2:
    rho0 (1 + kappa0 p), kappa0 (1 + kappa0 (1 - 2 beta) p)) the effective
    coefficient is beta - 1; the custom form A = 0, B = -2 beta (the
    multipliers rho0 and kappa0 (1 - 2 beta kappa0 p)) gives beta itself, the
    Westervelt value of Sec. 2.2.  With the nonlinear terms switched off
    (beta = 1/2 in Eq. general6 and amplitude far smaller) the second
    harmonic is absent, so the match is not a linear-propagation artefact."""
    f0, ppw, cfl, beta = 1e6, 20, 0.4, 3.5
    nl = (1.0, 1.0, -2.0) if form == "printed" else (0.0, 0.0, -2.0)
    beta_eff = -(nl[0] + nl[1] + nl[2] * beta) / 2.0      # beta - 1, or beta
    assert beta_eff == (beta - 1 if form == "printed" else beta)
    p0 = 2e6 * 2.5 / beta_eff                               # the same sigma for both forms
    lam = ppw
    nb, ntr = 4 * lam, 3 * lam
    nx = 48 + 2 * nb
    ys = nb + 4
    y1 = ys + 3 * lam
    dist_lam = 26
    y2 = y1 + dist_lam * lam
    ny = y2 + 2 * lam + nb
    prob = W.homogeneous((nx, ny), L=1, row=W.lossless_row(1), nb=(nb, nb), ntr=(ntr, ntr), f0=f0,
                         ppw=ppw, cfl=cfl, beta=beta)
    if form != "printed":
        prob.nonlinear_form, (prob.nl_A, prob.nl_B0, prob.nl_B1) = 1, nl
    h, dt = prob.h, prob.dt
    npulse = W.pulse_length(dt, f0, 4)
    nt = int((y2 - ys) * h / C0 / dt) + npulse + 100
    xs = np.arange(nx)
    prob.src_idx = prob.flat(xs, np.full_like(xs, ys))
    prob.src_sig = np.zeros(nx, np.int32)
    prob.src_w = np.ones(nx, np.float32)
    sig = W.gaussian_pulse(npulse, dt, f0, 4, 1.0)
    cx = nx // 2
    prob.rcv_idx = prob.flat(np.array([cx, cx]), np.array([y1, y2]))
    # amplitude calibration with a quasi-linear run: peak p0 at receiver 1
    prob.signals = sig[None]
    _, tr = solver.run(prob, y1 * 0 + int((y1 - ys) * h / C0 / dt) + npulse)
    prob.signals = (sig * p0 / np.abs(tr[:, 0]).max())[None].astype(np.float32)
    _, tr = solver.run(prob, nt)
    t = (np.arange(nt) + 1) * dt
    kap0 = 1.0 / (1000.0 * C0 ** 2)
    dist = (y2 - y1) * h
    pex = physics.simple_wave_propagate(t, tr[:, 0], dist, 1000.0, kap0, beta, nl)
    sigma = beta_eff * p0 * kap0 * (2 * np.pi * f0 / C0) * dist
    assert 0.3 < sigma < 0.45
    N = 8 * nt
    f = np.fft.rfftfreq(N, dt)
    F2, FE = np.abs(np.fft.rfft(tr[:, 1], N)), np.abs(np.fft.rfft(pex, N))
    for n in range(1, 5):
        k = np.argmin(np.abs(f - n * f0))
        assert abs(20 * np.log10(F2[k] / FE[k])) < 1.0, n
    if form != "printed":
        # the wrong coefficient (beta - 1, the printed form's) misses the
        # harmonics of this run: the pin tells the two forms apart
        pwr = physics.simple_wave_propagate(t, tr[:, 0], dist, 1000.0, kap0, beta)
        FW = np.abs(np.fft.rfft(pwr, N))
        k2 = np.argmin(np.abs(f - 2 * f0))
        assert abs(20 * np.log10(F2[k2] / FW[k2])) > 2.0
        return
    # the generated second harmonic is a real nonlinear effect
    prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    prob.signals = (sig * 1e-3)[None].astype(np.float32)
    _, trl = solver.run(prob, nt)
    FL = np.abs(np.fft.rfft(trl[:, 1], N))
    k1, k2 = np.argmin(np.abs(f - f0)), np.argmin(np.abs(f - 2 * f0))
    assert F2[k2] / F2[k1] > 30 * FL[k2] / FL[k1]


def test_nonlinear_harmonics_one_to_seven(oracle_lib):
    """Sec. 4.5 reports agreement up to the seventh harmonic.  With the
    Taylor-matched weights (the stencil reading) that needs about 4.5 points
    per wavelength at the seventh harmonic, i.e. 32 at the fundamental: a
    lossless plane pulse (1 MHz, 4 cycles, CFL 0.4) propagated 10
    wavelengths to sigma = 0.65 matches the exact pre-shock simple wave of
    the same equations in harmonics 1-7 within 1 dB (the seventh lies 33 dB
    below the fundamental)."""
    f0, ppw, cfl, beta, sigma, dist_lam = 1e6, 32, 0.4, 3.5, 0.65, 10
    lam = ppw
    nb, ntr = 4 * lam, 3 * lam                   # along the propagation axis
    nbx, ntrx = 2 * lam, 3 * lam // 2            # lateral layers only absorb edge waves
    nx = int(2.4 * lam) + 2 * nbx
    ys = nb + 4
    y1 = ys + 3 * lam
    y2 = y1 + dist_lam * lam
    ny = y2 + 2 * lam + nb
    prob = W.homogeneous((nx, ny), L=1, row=W.lossless_row(1), nb=(nbx, nb), ntr=(ntrx, ntr), f0=f0,
                         ppw=ppw, cfl=cfl, beta=beta)
    h, dt = prob.h, prob.dt
    kap0 = 1.0 / (1000.0 * C0 ** 2)
    dist = (y2 - y1) * h
    p0 = sigma / ((beta - 1) * kap0 * (2 * np.pi * f0 / C0) * dist)
    npulse = W.pulse_length(dt, f0, 4)
    nt = int((y2 - ys) * h / C0 / dt) + npulse + 100
    xs = np.arange(nx)
    prob.src_idx = prob.flat(xs, np.full_like(xs, ys))
    prob.src_sig = np.zeros(nx, np.int32)
    prob.src_w = np.ones(nx, np.float32)
    sig = W.gaussian_pulse(npulse, dt, f0, 4, 1.0)
    cx = nx // 2
    prob.rcv_idx = prob.flat(np.array([cx, cx]), np.array([y1, y2]))
    prob.signals = sig[None]
    _, tr = solver.run(prob, int((y1 - ys) * h / C0 / dt) + npulse)
    prob.signals = (sig * p0 / np.abs(tr[:, 0]).max())[None].astype(np.float32)
    _, tr = solver.run(prob, nt)
    t = (np.arange(nt) + 1) * dt
    pex = physics.simple_wave_propagate(t, tr[:, 0], dist, 1000.0, kap0, beta)
    N = 8 * nt
    f = np.fft.rfftfreq(N, dt)
    F2, FE = np.abs(np.fft.rfft(tr[:, 1], N)), np.abs(np.fft.rfft(pex, N))
    k1 = np.argmin(np.abs(f - f0))
    for n in range(1, 8):
        k = np.argmin(np.abs(f - n * f0))
        assert abs(20 * np.log10(F2[k] / FE[k])) < 1.0, n
    k7 = np.argmin(np.abs(f - 7 * f0))
    assert 20 * np.log10(FE[k7] / FE[k1]) > -40.0          # the seventh harmonic is really there


def test_reduced_order_eight_ppw_half_cfl(oracle_lib):
    """Sec. 5: 8 points per wavelength with CFL 0.2 is offered as the
    reduced-order setting, with a slight increase of the attenuation error.
    The plane-wave measurement there stays within 1 % of the dispersion
    relation in attenuation and 5e-5 in phase velocity, within the paper's
    5 % of the power law, and its attenuation error at 2-20 MHz is larger
    than at 12 ppw / CFL 0.4."""
    row = W.tissue_row(0.5, 1.0, 2, 2e6)
    for f0 in (1e6, 2e6, 5e6, 20e6):
        fk, att, vel = _plane_wave_measure(row, 2, f0, ppw=8, cfl=0.2)
        a_an, c_an = relaxation.model_attenuation_velocity(np.array([fk]), C0, np.array(row), 2)
        assert abs(att / a_an[0] - 1) < 0.01, (f0, att, a_an)
        assert abs(vel / c_an[0] - 1) < 5e-5, (f0, vel, c_an)
        assert abs(att / physics.power_law_db_cm(fk, 0.5, 1.0) - 1) < 0.05
        if f0 >= 2e6:
            fk12, att12, _ = _plane_wave_measure(row, 2, f0)
            a12, _ = relaxation.model_attenuation_velocity(np.array([fk12]), C0, np.array(row), 2)
            assert abs(att / a_an[0] - 1) > abs(att12 / a12[0] - 1), f0
