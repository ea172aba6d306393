"""Pins of the oracle's per-point (velocity-dependent) stencil weights
(stencil_mode 1): every point takes the (8,4) weights of its own Courant
number r = c dt / h, a v point the mean of its two cells' r^2.

What fixes them: the scheme's own plane-wave dispersion relation (closed
form), equality with the global-weight scheme wherever the local r is one
value, locality of the stencil, and mirror symmetry."""
import numpy as np
import pytest

import workloads as W
from oracle import solver, stencil


def _copy(prob, **kw):
    q = W.Problem(**{k: getattr(prob, k) for k in prob.__dataclass_fields__})
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def _random_problem(shape, L, seed, c=None, nb=5, ntr=3, n_labels=2):
    rng = np.random.default_rng(seed)
    prob = W.homogeneous(shape, L=L, nb=(nb,) * len(shape), ntr=(ntr,) * len(shape))
    grid = prob.c.shape
    prob.c = (rng.uniform(1450, 1620, grid) if c is None else np.full(grid, c)).astype(np.float32)
    prob.rho = rng.uniform(950, 1120, grid).astype(np.float32)
    prob.beta = rng.uniform(3.5, 5.5, grid).astype(np.float32)
    rows = []
    for k in range(n_labels):
        r = [rng.uniform(0.85, 1.15), rng.uniform(0.85, 1.15)]
        r += list(10 ** rng.uniform(4, 6.5, 2 * L)) + list(10 ** rng.uniform(6, 9.5, 2 * L))
        rows.append(r)
    prob.relax_table = np.array(rows)
    prob.label = rng.integers(0, n_labels, grid).astype(np.uint8)
    prob.dt = 0.4 * prob.h / 1620.0
    prob.pml_cp = 1620.0
    return prob


def _state(prob, seed):
    p, v, psi1, psi2 = W.random_state(prob.ndim, prob.n_relax, prob.shape, seed)
    st = solver.State(prob.ndim, prob.n_relax, prob.c.shape)
    st.p, st.v = p.astype(np.float64), v.astype(np.float64)
    st.psi1, st.psi2 = psi1.astype(np.float64), psi2.astype(np.float64)
    return st


def test_local_weights_are_the_taylor_weights_of_each_r():
    """The batched solve gives, at every r, the weights whose leapfrog phase
    velocity (closed form from the update equations) is within 2e-5 of c at
    12 points per wavelength in every direction, and equals the single-r
    solve."""
    r = np.array([[0.05, 0.2], [0.33, 0.45]])
    g, g11 = stencil.local_weights(r ** 2, 2)
    assert g.shape == (4, 2, 2) and g11.shape == (2, 2)
    for idx in np.ndindex(r.shape):
        gs, g11s = stencil.stencil_weights(r[idx], 2)
        np.testing.assert_allclose(g[(slice(None),) + idx], gs, rtol=1e-13, atol=1e-15)
        assert abs(g11[idx] - g11s) <= 1e-15
        worst = max(abs(stencil.scheme_phase_velocity_ratio(g[(slice(None),) + idx], g11[idx], r[idx], 12, a) - 1)
                    for a in np.linspace(0, np.pi / 2, 10))
        assert worst < 2e-5


def test_local_r_reduces_dispersion_in_slow_tissue():
    """Why the mode exists: with one r set by the fastest tissue, a slower
    tissue propagates with the weights of the wrong r; its own weights cut the
    phase error (closed form, 12 and 8 points per wavelength)."""
    r_max = 0.4
    for c_ratio in (0.9, 0.8):
        r = r_max * c_ratio
        gg, gg11 = stencil.stencil_weights(r_max, 2)
        gl, gl11 = stencil.stencil_weights(r, 2)
        for ppw in (12, 8):
            e_glob = abs(stencil.scheme_phase_velocity_ratio(gg, gg11, r, ppw, 0.3) - 1)
            e_loc = abs(stencil.scheme_phase_velocity_ratio(gl, gl11, r, ppw, 0.3) - 1)
            assert e_loc < 0.5 * e_glob, (c_ratio, ppw, e_loc, e_glob)


@pytest.mark.parametrize("shape", [(31, 27), (13, 11, 9)])
def test_constant_c_equals_global_weights(oracle_lib, shape):
    """Where c is one value (density, nonlinearity and relaxation still
    vary), every local r is c dt / h, so the per-point run equals the
    global-weight run with that r."""
    prob = _random_problem(shape, 2, seed=3, c=1530.0)
    loc = _copy(prob, stencil_mode=1)
    glob = _copy(prob, stencil_mode=0, fd_r=1530.0 * prob.dt / prob.h)
    st0 = _state(prob, 4)
    a, _ = solver.run(loc, 25, st0.copy())
    b, _ = solver.run(glob, 25, st0.copy())
    for name in ("p", "v", "psi1", "psi2"):
        x, y = getattr(a, name), getattr(b, name)
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y)), name


def test_far_from_an_interface_each_side_uses_its_own_r(oracle_lib):
    """Two tissues meeting at x = 24: after one step, p at least 5 cells and
    v at least 10 cells from the interface equal the global-weight runs with
    that side's r (the stencil reaches 4 cells per phase)."""
    prob = _random_problem((48, 30), 2, seed=7)
    grid = prob.c.shape
    xx = np.arange(grid[1])[None, :] + np.zeros(grid)
    c1, c2 = 1455.0, 1615.0
    prob.c = np.where(xx < 24, c1, c2).astype(np.float32)
    st0 = _state(prob, 8)
    a, _ = solver.run(_copy(prob, stencil_mode=1), 1, st0.copy())
    b1, _ = solver.run(_copy(prob, fd_r=c1 * prob.dt / prob.h), 1, st0.copy())
    b2, _ = solver.run(_copy(prob, fd_r=c2 * prob.dt / prob.h), 1, st0.copy())
    x = np.arange(grid[1])
    # v_x samples sit at x + 1/2: distance to the interface plane at 23.5
    for lo, ref in (((x <= 23 - 5), b1), ((x >= 24 + 5), b2)):
        np.testing.assert_allclose(a.p[:, lo], ref.p[:, lo], rtol=0, atol=1e-12 * np.abs(ref.p).max())
    for lo, ref in (((x <= 23 - 10), b1), ((x >= 24 + 10), b2)):
        np.testing.assert_allclose(a.v[:, :, lo], ref.v[:, :, lo], rtol=0, atol=1e-12 * np.abs(ref.v).max())
    # and the two global runs do differ there (the test can see the weights)
    assert np.abs(b1.p[:, x <= 18] - b2.p[:, x <= 18]).max() > 1e-6 * np.abs(b1.p).max()


def test_mirror_symmetry_with_local_weights(oracle_lib):
    """A heterogeneous medium and source symmetric under x -> nx-1-x give a
    symmetric p and an antisymmetric v_x: the v-point r^2 is symmetric in
    its two cells."""
    prob = W.homogeneous((41, 36), L=2, nb=(6, 6), ntr=(4, 4))
    rng = np.random.default_rng(2)
    half = rng.uniform(1450, 1620, (36, 21)).astype(np.float32)
    prob.c = np.concatenate([half, half[:, :20][:, ::-1]], axis=1)
    prob.dt = 0.4 * prob.h / float(prob.c.max())
    prob.stencil_mode = 1
    prob.src_idx = prob.flat(np.array([20]), np.array([12]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.signals = W.gaussian_pulse(200, prob.dt, 2e6, 3, 1e5)[None]
    st, _ = solver.run(prob, 200)
    assert np.max(np.abs(st.p - st.p[:, ::-1])) <= 1e-11 * np.max(np.abs(st.p))
    vx = st.v[0]
    assert np.max(np.abs(vx[:, :40] + vx[:, :40][:, ::-1])) <= 1e-11 * np.max(np.abs(vx))
    # the global-weight run of the same medium differs (the mode is active)
    g, _ = solver.run(_copy(prob, stencil_mode=0), 200)
    assert np.max(np.abs(g.p - st.p)) > 1e-6 * np.max(np.abs(st.p))


@pytest.mark.parametrize("shape,L", [((29, 23), 2), ((12, 10, 9), 3)])
def test_c_stepper_matches_numpy_twin_with_local_weights(oracle_lib, shape, L):
    prob = _random_problem(shape, L, seed=12)
    prob.stencil_mode = 1
    st0 = _state(prob, 3)
    m = solver.coefficient_maps(prob)
    a, _ = solver.run(prob, 20, st0.copy(), m)
    b, _ = solver.numpy_run(prob, 20, st0.copy(), m)
    for name in ("p", "v", "psi1", "psi2"):
        x, y = getattr(a, name), getattr(b, name)
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y)), name
