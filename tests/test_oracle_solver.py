"""Pins of the oracle's time stepper: twin cross-check, invariants and
special cases that any correct implementation of the scheme must satisfy."""
import numpy as np
import pytest

import workloads as W
from oracle import solver


def _random_problem(shape, L, seed, nb=5, ntr=3, n_labels=2):
    rng = np.random.default_rng(seed)
    prob = W.homogeneous(shape, L=L, nb=(nb,) * len(shape), ntr=(ntr,) * len(shape))
    grid = prob.c.shape
    prob.c = rng.uniform(1450, 1620, grid).astype(np.float32)
    prob.rho = rng.uniform(950, 1120, grid).astype(np.float32)
    prob.beta = rng.uniform(3.5, 5.5, grid).astype(np.float32)
    rows = []
    for k in range(n_labels):
        r = [rng.uniform(0.85, 1.15), rng.uniform(0.85, 1.15)]
        r += list(10 ** rng.uniform(4, 6.5, 2 * L)) + list(10 ** rng.uniform(6, 9.5, 2 * L))
        rows.append(r)
    prob.relax_table = np.array(rows)
    prob.label = rng.integers(0, n_labels, grid).astype(np.uint8)
    prob.dt = 0.4 * prob.h / float(prob.c.max())
    return prob


def _random_state(prob, seed):
    p, v, psi1, psi2 = W.random_state(prob.ndim, prob.n_relax, prob.shape, seed)
    st = solver.State(prob.ndim, prob.n_relax, prob.c.shape)
    st.p, st.v = p.astype(np.float64), v.astype(np.float64)
    st.psi1, st.psi2 = psi1.astype(np.float64), psi2.astype(np.float64)
    return st


@pytest.mark.parametrize("shape,L", [((37, 29), 2), ((23, 19), 4), ((13, 11, 9), 2), ((12, 10, 9), 1), ((21, 17), 7)])
def test_c_stepper_matches_numpy_twin(oracle_lib, shape, L):
    """Two independent codings of the same steps (plain loops with explicit
    bounds checks vs. whole-array shifts of a zero-padded field) agree."""
    prob = _random_problem(shape, L, seed=11)
    g = prob.c.shape
    rng = np.random.default_rng(5)
    prob.src_idx = np.array([3, prob.npts // 2, prob.npts - 4], np.int64)
    prob.src_sig = np.array([0, 1, 0], np.int32)
    prob.src_w = np.array([1.0, -0.5, 2.0], np.float32)
    prob.signals = (1e4 * rng.standard_normal((2, 25))).astype(np.float32)
    prob.rcv_idx = np.array([0, 7, prob.npts // 3, prob.npts - 1], np.int64)
    st0 = _random_state(prob, 9)
    m = solver.coefficient_maps(prob)
    a, ta = solver.run(prob, 30, st0.copy(), m)
    b, tb = solver.numpy_run(prob, 30, st0.copy(), m)
    for name in ("p", "v", "psi1", "psi2"):
        x, y = getattr(a, name), getattr(b, name)
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y)), name
    assert np.max(np.abs(ta - tb)) <= 1e-12 * np.max(np.abs(tb))
    assert a.step == 30


def test_zero_input_stays_zero(oracle_lib):
    prob = _random_problem((30, 24), 2, seed=1)
    st, tr = solver.run(prob, 40)
    assert not st.p.any() and not st.v.any() and not st.psi1.any() and not st.psi2.any()


def test_split_run_equals_single_run(oracle_lib):
    prob = W.plain_2d(interior=96, n_steps=0, n_rcv=8)
    s1, t1 = solver.run(prob, 150)
    s2, ta = solver.run(prob, 70)
    s2, tb = solver.run(prob, 80, s2)
    assert np.array_equal(s1.p, s2.p) and np.array_equal(s1.psi1, s2.psi1)
    assert np.array_equal(t1, np.concatenate([ta, tb]))


def test_mirror_symmetry(oracle_lib):
    """A medium and source symmetric under x -> nx-1-x give a symmetric p
    (the staggered v_x mirrors onto -v_x at nx-2-x)."""
    prob = W.homogeneous((41, 36), L=2, nb=(6, 6), ntr=(4, 4))
    rng = np.random.default_rng(2)
    half = rng.uniform(1450, 1620, (36, 21)).astype(np.float32)
    prob.c = np.concatenate([half, half[:, :20][:, ::-1]], axis=1)
    prob.dt = 0.4 * prob.h / float(prob.c.max())
    prob.src_idx = prob.flat(np.array([20]), np.array([12]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.signals = W.gaussian_pulse(200, prob.dt, 2e6, 3, 1e5)[None]
    st, _ = solver.run(prob, 200)
    assert np.max(np.abs(st.p - st.p[:, ::-1])) <= 1e-11 * np.max(np.abs(st.p))
    vx = st.v[0]
    assert np.max(np.abs(vx[:, :40] + vx[:, :40][:, ::-1])) <= 1e-11 * np.max(np.abs(vx))


def test_superposition_without_nonlinearity(oracle_lib):
    """beta = 1/2 removes the mass-equation nonlinearity; with tiny
    amplitudes the remaining momentum term is below 1e-9 relative, so the
    response to two sources is the sum of the responses (the relaxation and
    boundary parts are linear)."""
    prob = _random_problem((40, 34), 2, seed=4)
    prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    prob.signals = W.gaussian_pulse(300, prob.dt, 3e6, 3, 1e-3)[None]
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.src_idx = prob.flat(np.array([12]), np.array([10]))
    a, _ = solver.run(prob, 250)
    prob.src_idx = prob.flat(np.array([27]), np.array([22]))
    b, _ = solver.run(prob, 250)
    prob.src_idx = prob.flat(np.array([12, 27]), np.array([10, 22]))
    prob.src_sig = np.zeros(2, np.int32)
    prob.src_w = np.ones(2, np.float32)
    ab, _ = solver.run(prob, 250)
    assert np.max(np.abs(ab.p - (a.p + b.p))) <= 1e-8 * np.max(np.abs(ab.p))


def _energy(prob, st):
    kap0 = 1.0 / (prob.rho.astype(np.float64) * prob.c.astype(np.float64) ** 2)
    return 0.5 * np.sum(kap0 * st.p ** 2) + 0.5 * np.sum(prob.rho.astype(np.float64) * np.sum(st.v ** 2, axis=0))


def test_lossless_closed_box_keeps_discrete_energy(oracle_lib):
    """No relaxation, no boundary layer, linear regime: the staggered leapfrog
    conserves E = 1/2 sum kappa0 (p^n)^2 + 1/2 sum rho_a v^{n-1/2} v^{n+1/2}
    exactly when D^- = -(D^+)^T (the two stencils are adjoint, cross terms and
    grid edges included).  A wrong index or sign in either stencil breaks it."""
    prob = W.homogeneous((48, 40), L=1, row=W.lossless_row(1), nb=(0, 0), ntr=(0, 0))
    rng = np.random.default_rng(8)
    prob.c = rng.uniform(1450, 1620, prob.c.shape).astype(np.float32)
    prob.rho = rng.uniform(950, 1120, prob.c.shape).astype(np.float32)
    prob.dt = 0.4 * prob.h / float(prob.c.max())
    prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    m = solver.coefficient_maps(prob)
    st = solver.State(2, 1, prob.c.shape)
    st.p = 1e-3 * rng.standard_normal(prob.c.shape)

    def energy(s_prev_v, s):
        e = 0.5 * np.sum(m.kap0 * s.p ** 2)
        for a in range(2):
            e += 0.5 * np.sum(m.rho_v[a] * s_prev_v[a] * s.v[a])
        return e

    st, _ = solver.run(prob, 1, st, m, record=False)
    es = []
    for _ in range(20):
        st, _ = solver.run(prob, 199, st, m, record=False)
        vprev = st.v.copy()
        st, _ = solver.run(prob, 1, st, m, record=False)
        es.append(energy(vprev, st))
    es = np.array(es)
    assert np.max(np.abs(es / es[0] - 1)) < 1e-9


def test_relaxation_dissipates_energy(oracle_lib):
    """Interior relaxation (Table 2 tissue, no boundary layer) removes energy:
    block averages of the energy decrease."""
    prob = W.homogeneous((48, 40), L=2, nb=(0, 0), ntr=(0, 0), f0=6e6)
    prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    st = solver.State(2, 2, prob.c.shape)
    yy, xx = np.mgrid[0:40, 0:48]
    st.p = 1e-3 * np.exp(-((xx - 24.0) ** 2 + (yy - 20.0) ** 2) / 3.0)
    blocks = []
    for _ in range(8):
        acc = 0.0
        for _ in range(10):
            st, _ = solver.run(prob, 25, st, record=False)
            acc += _energy(prob, st)
        blocks.append(acc)
    assert np.all(np.diff(blocks) < 0)


def test_boundary_layer_absorbs(oracle_lib):
    """With the two-stage layer the field leaves the domain: after the pulse
    has crossed the grid several times the energy left is tiny."""
    prob = W.homogeneous((80, 80), L=2, nb=(24, 24), ntr=(18, 18), f0=2e6)
    st = solver.State(2, 2, prob.c.shape)
    yy, xx = np.mgrid[0:80, 0:80]
    st.p = 1e3 * np.exp(-((xx - 40.0) ** 2 + (yy - 40.0) ** 2) / 8.0)
    e0 = _energy(prob, st)
    st, _ = solver.run(prob, 1500, st, record=False)
    assert _energy(prob, st) < 1e-4 * e0
