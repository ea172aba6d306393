"""Pins of the oracle's FP64 discrete adjoint: its forward recomputation is
the oracle's stepper, and its sound-speed gradient equals central finite
differences of the misfit (computed with the C stepper)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, solver


def _problem(shape=(34, 30), L=2, seed=3, n_steps=110):
    rng = np.random.default_rng(seed)
    prob = W.random_medium(shape, L, 2, seed=seed, nb=6, ntr=4, f0=3e6)
    prob.n_steps = n_steps
    prob.beta = prob.beta.astype(np.float32)
    # fixed stencil Courant number and layer speed: c enters only via kappa0
    prob.fd_r = float(prob.c.max()) * prob.dt / prob.h
    prob.pml_cp = float(prob.c.max())
    nx, ny = shape
    prob.src_idx = prob.flat(np.array([nx // 2, nx // 2 + 1]), np.array([ny // 3, ny // 3]))
    prob.src_sig = np.zeros(2, np.int32)
    prob.src_w = np.array([1.0, 0.5], np.float32)
    prob.signals = W.gaussian_pulse(n_steps, prob.dt, 3e6, 3, 2e5)[None]
    prob.rcv_idx = prob.flat(np.array([4, 12, 20, 29]), np.array([ny - 8, ny - 9, ny - 7, 10]))
    return prob


def _obs(prob, n_steps, seed=7):
    pert = W.Problem(**{k: getattr(prob, k) for k in prob.__dataclass_fields__})
    rng = np.random.default_rng(seed)
    pert.c = (prob.c * (1.0 + 0.01 * rng.standard_normal(prob.c.shape))).astype(np.float32)
    pert.c = np.minimum(pert.c, prob.c.max())
    _, tr = solver.run(pert, n_steps)
    return tr


def test_adjoint_forward_is_the_oracle_stepper(oracle_lib):
    prob = _problem()
    obs = np.zeros((prob.n_steps, len(prob.rcv_idx)))
    J, g, tr = adjoint.misfit_and_gradient(prob, obs, prob.n_steps)
    _, tr2 = solver.run(prob, prob.n_steps)
    assert np.max(np.abs(tr - tr2)) <= 1e-12 * np.max(np.abs(tr2))


@pytest.mark.parametrize("L,nonlinear", [(2, True), (3, False), (1, True)])
def test_adjoint_gradient_matches_central_differences(oracle_lib, L, nonlinear):
    """dJ/dc from the reversed steps against (J(c + e) - J(c - e)) / 2e at
    points in the interior, in the boundary layers and next to the source and
    a receiver; the nonlinear multipliers, the memory variables and the
    staggered means are all exercised."""
    prob = _problem(L=L, seed=L + 5)
    if not nonlinear:
        prob.beta = np.full(prob.c.shape, 0.5, np.float32)
    obs = _obs(prob, prob.n_steps)
    J, g, _ = adjoint.misfit_and_gradient(prob, obs, prob.n_steps)
    assert J > 0
    nx, ny = prob.shape
    pts = [(nx // 2, ny // 2), (2, 3), (nx // 2, ny // 3 + 1), (12, ny - 9), (nx - 3, ny // 2), (9, 17)]
    for (x, y) in pts:
        c0 = float(prob.c[y, x])
        eps = 1e-3
        cp = prob.c.copy(); cp[y, x] = c0 + eps
        cm = prob.c.copy(); cm[y, x] = c0 - eps
        prob.c = cp
        Jp = adjoint.misfit(prob, obs, prob.n_steps)
        prob.c = cm
        Jm = adjoint.misfit(prob, obs, prob.n_steps)
        prob.c = prob.c.copy(); prob.c[y, x] = c0
        fd = (Jp - Jm) / (float(cp[y, x]) - float(cm[y, x]))
        scale = np.max(np.abs(g))
        assert abs(fd - g[y, x]) <= 1e-5 * scale + 1e-4 * abs(fd), ((x, y), fd, g[y, x], scale)


def test_adjoint_3d_matches_central_differences(oracle_lib):
    prob = W.random_medium((14, 12, 11), 2, 2, seed=2, nb=3, ntr=2, f0=3e6)
    n = 40
    prob.fd_r = float(prob.c.max()) * prob.dt / prob.h
    prob.pml_cp = float(prob.c.max())
    prob.src_idx = prob.flat(np.array([7]), np.array([6]), np.array([5]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.signals = W.gaussian_pulse(n, prob.dt, 3e6, 3, 2e5)[None]
    prob.rcv_idx = prob.flat(np.array([3, 10]), np.array([4, 8]), np.array([8, 2]))
    obs = _obs(prob, n)
    J, g, _ = adjoint.misfit_and_gradient(prob, obs, n)
    for (x, y, z) in [(7, 6, 6), (2, 2, 2), (9, 5, 4)]:
        c0 = float(prob.c[z, y, x])
        cp = prob.c.copy(); cp[z, y, x] = c0 + 1e-3
        cm = prob.c.copy(); cm[z, y, x] = c0 - 1e-3
        prob.c = cp; Jp = adjoint.misfit(prob, obs, n)
        prob.c = cm; Jm = adjoint.misfit(prob, obs, n)
        prob.c = prob.c.copy(); prob.c[z, y, x] = c0
        fd = (Jp - Jm) / (float(cp[z, y, x]) - float(cm[z, y, x]))
        assert abs(fd - g[z, y, x]) <= 1e-5 * np.max(np.abs(g)) + 1e-4 * abs(fd)
