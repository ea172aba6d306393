"""FP64 discrete adjoint of the oracle's time stepper (test infrastructure).

Sec. 5 (extension to full waveform inversion): the memory-variable
recursion dissipates, so a gradient cannot come from stepping the forward
scheme backwards in time.  This module transposes the linearised discrete
scheme of oracle.solver (memory scheme 1, time-centred), in reverse-mode
form, for the misfit J = 1/2 sum_n sum_r (trace[n][r] - obs[n][r])^2.

Forward step n (input state p, v, m1 = psi1, m2 = psi2; x = kappa0):
  pressure:  D_a = (D^- v_a);  S = sum_a (w2_a D_a + sum_nu m2_a,nu)
             m2' = b2 m2 + c2 D;  K = x (1 + nlq p), nlq = x B (B = 1 - 2 beta
             as printed);  p' = p - dt S / K
  sources:   p'' = p' + s_n
  receivers: trace_n = p''[R]
  velocity:  D' = (D^+ p'')_a;  S' = w1 D' + sum_nu m1;  m1' = b1 m1 + c1 D'
             Q = rho_a (1 + A x_a pbar), x_a and pbar the means of the two cells
             (A = 1 as printed)
             v' = v - dt S' / Q     (only for v samples inside the grid)
with w = 1/kappa + sum_nu e0, c = e1 + b e0 (oracle.relaxation.centred_weights).
The adjoint uses (D^-)^T = -(D^+) and (D^+)^T = -(D^-) (zero outside the grid,
v samples past the grid excluded), which the discrete-energy pin checks.

The gradient with respect to the sound speed comes through kappa0 = 1/(rho c^2)
only (the stencil Courant number and the layer's c_p are fixed inputs):
  dJ/dc = dJ/dkappa0 * (-2 kappa0 / c).
"""
import numpy as np

from . import solver

PAD = solver.PAD


def _sh(f, ndim, grid, off):
    return solver._shift(np.pad(f, PAD), ndim, grid, off)


def _e(a, s=1):
    o = [0, 0, 0]
    o[a] = s
    return o


def _add(o1, o2):
    return [o1[k] + o2[k] for k in range(3)]


def d_minus(f, a, maps):
    """(D^- f)_a at pressure points for a field f at v_a points."""
    nd, grid = maps.ndim, maps.grid
    D = np.zeros(grid)
    for mm in range(1, 5):
        D += maps.g[mm - 1] * (_sh(f, nd, grid, _e(a, mm - 1)) - _sh(f, nd, grid, _e(a, -mm)))
    for b in range(nd):
        if b == a:
            continue
        for sg in (-1, 1):
            D += maps.g11 * (_sh(f, nd, grid, _e(b, sg)) - _sh(f, nd, grid, _add(_e(a, -1), _e(b, sg))))
    return D


def d_plus(f, a, maps):
    """(D^+ f)_a at v_a points for a field f at pressure points."""
    nd, grid = maps.ndim, maps.grid
    D = np.zeros(grid)
    for mm in range(1, 5):
        D += maps.g[mm - 1] * (_sh(f, nd, grid, _e(a, mm)) - _sh(f, nd, grid, _e(a, -(mm - 1))))
    for b in range(nd):
        if b == a:
            continue
        for sg in (-1, 1):
            D += maps.g11 * (_sh(f, nd, grid, _add(_e(a, 1), _e(b, sg))) - _sh(f, nd, grid, _e(b, sg)))
    return D


def inside_v(maps, a):
    """Mask of the v_a samples inside the grid (the last along a is outside)."""
    nd, grid = maps.ndim, maps.grid
    ax = nd - 1 - a
    m = np.arange(grid[ax]) < grid[ax] - 1
    shape = [1] * nd
    shape[ax] = grid[ax]
    return np.broadcast_to(m.reshape(shape), grid)


def _weights(maps, which):
    """(w[a], b[a][nu], c[a][nu]) of the centred scheme for nabla_1 or nabla_2."""
    if which == 1:
        ik, A, B, E0 = maps.ik1, maps.a1, maps.b1, maps.e0_1
    else:
        ik, A, B, E0 = maps.ik2, maps.a2, maps.b2, maps.e0_2
    w = ik + E0.sum(axis=1)
    c = (A - E0) + B * E0
    return w, B, c


def _sources(prob, step, grid):
    s = np.zeros(int(np.prod(grid)))
    sig = np.asarray(prob.signals, np.float64)
    if sig.ndim == 1:
        sig = sig[None]
    if step < sig.shape[1]:
        idx = np.asarray(prob.src_idx, np.int64)
        np.add.at(s, idx, np.asarray(prob.src_w, np.float64) * sig[np.asarray(prob.src_sig), step])
    return s.reshape(grid)


def forward_step(prob, maps, st, step):
    """One forward step of the centred scheme; returns the new state, the
    trace row and the intermediates the adjoint needs."""
    nd, L, grid = maps.ndim, maps.L, maps.grid
    w2, b2, c2 = _weights(maps, 2)
    w1, b1, c1 = _weights(maps, 1)
    S = np.zeros(grid)
    m2n = np.empty_like(st.psi2)
    for a in range(nd):
        D = d_minus(st.v[a], a, maps)
        S += w2[a] * D + st.psi2[a].sum(axis=0)
        for nu in range(L):
            m2n[a, nu] = b2[a, nu] * st.psi2[a, nu] + c2[a, nu] * D
    K = maps.kap0 * (1.0 + maps.nlq * st.p)
    pp = st.p - maps.dt * S / K + _sources(prob, step, grid)
    tr = pp.reshape(-1)[np.asarray(prob.rcv_idx, np.int64)]
    vn = st.v.copy()
    m1n = st.psi1.copy()
    for a in range(nd):
        ins = inside_v(maps, a)
        D = d_plus(pp, a, maps)
        Sv = w1[a] * D + st.psi1[a].sum(axis=0)
        pbar = 0.5 * (pp + _sh(pp, nd, grid, _e(a, 1)))
        Q = maps.rho_v[a] * (1.0 + maps.nl_A * maps.kap_v[a] * pbar)
        vn[a] = np.where(ins, st.v[a] - maps.dt * Sv / Q, st.v[a])
        for nu in range(L):
            m1n[a, nu] = np.where(ins, b1[a, nu] * st.psi1[a, nu] + c1[a, nu] * D, st.psi1[a, nu])
    new = solver.State(nd, L, grid)
    new.p, new.v, new.psi1, new.psi2, new.step = pp, vn, m1n, m2n, st.step + 1
    return new, tr


def reverse_step(prob, maps, st, lam, residual, gk):
    """Adjoint of one forward step from input state st.  lam (State) holds the
    adjoint of the step's outputs on entry and of its inputs on exit; residual
    is trace_n - obs_n; gk accumulates dJ/dkappa0."""
    nd, L, grid = maps.ndim, maps.L, maps.grid
    w2, b2, c2 = _weights(maps, 2)
    w1, b1, c1 = _weights(maps, 1)
    dt = maps.dt
    # forward recompute of the pressure phase
    S = np.zeros(grid)
    for a in range(nd):
        S += w2[a] * d_minus(st.v[a], a, maps) + st.psi2[a].sum(axis=0)
    K = maps.kap0 * (1.0 + maps.nlq * st.p)
    pp = st.p - dt * S / K + _sources(prob, st.step, grid)
    # velocity phase, reversed (v' = v - dt S'/Q: dv/dv = 1)
    lam_pp = lam.p.copy()
    for a in range(nd):
        ins = inside_v(maps, a)
        D = d_plus(pp, a, maps)
        Sv = w1[a] * D + st.psi1[a].sum(axis=0)
        pnext = _sh(pp, nd, grid, _e(a, 1))
        pbar = 0.5 * (pp + pnext)
        Q = maps.rho_v[a] * (1.0 + maps.nl_A * maps.kap_v[a] * pbar)
        lv = np.where(ins, lam.v[a], 0.0)
        lS = -dt * lv / Q
        lQ = dt * Sv * lv / (Q * Q)
        lpbar = lQ * maps.rho_v[a] * maps.nl_A * maps.kap_v[a]
        lk = lQ * maps.rho_v[a] * maps.nl_A * pbar
        lD = w1[a] * lS
        for nu in range(L):
            lm1n = np.where(ins, lam.psi1[a, nu], 0.0)
            lD = lD + c1[a, nu] * lm1n
            lam.psi1[a, nu] = np.where(ins, lS + b1[a, nu] * lm1n, lam.psi1[a, nu])
        lD = np.where(ins, lD, 0.0)
        lpbar = np.where(ins, lpbar, 0.0)
        lk = np.where(ins, lk, 0.0)
        # D' = D^+ pp  ->  lam_pp += (D^+)^T lD = -(D^- lD)
        lam_pp += -d_minus(lD, a, maps)
        # pbar = (pp_i + pp_{i+e})/2, x_a = (x_i + x_{i+e})/2
        lam_pp += 0.5 * (lpbar + _sh(lpbar, nd, grid, _e(a, -1)))
        gk += 0.5 * (lk + _sh(lk, nd, grid, _e(a, -1)))
    # receivers: trace = pp[R]
    flat = lam_pp.reshape(-1)
    np.add.at(flat, np.asarray(prob.rcv_idx, np.int64), residual)
    # sources are additive constants: lam_p' = lam_pp.  Pressure phase, reversed.
    lS = -dt * lam_pp / K
    lK = dt * S * lam_pp / (K * K)
    lam.p = lam_pp + lK * maps.kap0 * maps.nlq
    gk += lK * (1.0 + 2.0 * maps.nlq * st.p)
    for a in range(nd):
        lD = w2[a] * lS
        for nu in range(L):
            lm2n = lam.psi2[a, nu]
            lD = lD + c2[a, nu] * lm2n
            lam.psi2[a, nu] = lS + b2[a, nu] * lm2n
        # D = D^- v_a  ->  lam_v += (D^-)^T lD = -(D^+ lD), only inside the grid
        lam.v[a] = lam.v[a] + np.where(inside_v(maps, a), -d_plus(lD, a, maps), 0.0)
    return lam


def misfit_and_gradient(prob, obs, n_steps, maps=None):
    """J and dJ/dc (FP64) by storing every forward state (small grids)."""
    if maps is None:
        maps = solver.coefficient_maps(prob)
    if maps.scheme != 1:
        raise ValueError("the adjoint is derived for the time-centred memory scheme")
    if maps.stencil_mode != 0:
        raise ValueError("the adjoint is derived for one global stencil")
    st = solver.State(maps.ndim, maps.L, maps.grid)
    states, traces = [], []
    for n in range(n_steps):
        states.append(st)
        st, tr = forward_step(prob, maps, st, n)
        traces.append(tr)
    traces = np.array(traces)
    res = traces - obs[:n_steps]
    J = 0.5 * float(np.sum(res * res))
    lam = solver.State(maps.ndim, maps.L, maps.grid)
    gk = np.zeros(maps.grid)
    for n in reversed(range(n_steps)):
        lam = reverse_step(prob, maps, states[n], lam, res[n], gk)
    c = np.asarray(prob.c, np.float64).reshape(maps.grid)
    grad_c = gk * (-2.0 * maps.kap0 / c)
    return J, grad_c, traces


def misfit(prob, obs, n_steps):
    """J with the C stepper (FP64), for finite differences."""
    _, tr = solver.run(prob, n_steps)
    r = tr - obs[:n_steps]
    return 0.5 * float(np.sum(r * r))
