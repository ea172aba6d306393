"""FP64 oracle solver: per-point coefficient maps and the time loop.

Test infrastructure only.  Follows the paper's method as written:

* Sec. 2.1 / 3.2: two stretched derivatives, nabla_1 (acting on p, evaluated
  at the velocity points) and nabla_2 (acting on v, at the pressure points),
  each with 1/kappa and L memory variables (Eqs. relaxation_a, relaxation_b,
  relaxation_psi, relaxation4); the isotropic tuple
  (kappa1, kappa2, d1[L], d2[L], alpha1[L], alpha2[L]) is assigned per point.
* Sec. 3.3 / Table 1: the boundary layer modifies d and alpha of each axis'
  derivative with the directional two-stage profile.
* Eqs. general5 / general6 with the equation of state of Eqs. state1 /
  state2: rho = rho0 (1 + kappa0 p), kappa = kappa0 (1 + kappa0 (1-2 beta) p).
  prob.nonlinear_form 1 replaces them by rho0 (1 + A kappa0 p) and
  kappa0 (1 + kappa0 (B0 + B1 beta) p) (A = 1, B0 = 1, B1 = -2 as printed;
  A = 0, B0 = 0, B1 = -2 gives a plane-wave nonlinearity coefficient beta).
* Sec. 3.1: staggered leapfrog with the (8,4) stencil.
* Memory variables, two schemes (prob.relax_scheme):
  0 -- Eq. relaxation_psi as printed: psi^n = b psi^{n-1} + a D^{n-1/2}, the
       updated psi entering the same step (update-then-use);
  1 -- time-centred (default): the same exponential convolution evaluated at
       the time of the newest derivative sample, with the derivative linear
       between samples (weights of relaxation.centred_weights).  Scheme 0
       places psi half a step after the derivative it modifies and loses
       about a fifth of the attenuation at 12 ppw / CFL 0.4; scheme 1
       reproduces the dispersion relation (see the attenuation pins).

Readings taken where the paper is silent (all listed in the design notes):
staggered rho and kappa0 are the mean of the two neighbouring cells, the cell
past the last one repeating the last value; a velocity sample takes the
relaxation tuple of the cell it is attached to (index k for position k+1/2);
velocity samples lie strictly between two pressure samples (along axis a the
sample past the last pressure sample is outside the grid and stays zero), so
the staggered grid is mirror symmetric; the momentum multiplier uses the mean
of the two neighbouring pressures at the current level, the mass multiplier the pressure of the previous level; fields
are zero outside the grid; sources add to p after the pressure phase and
receivers read p after the sources; with stencil_mode 1 the stencil weights
are those of the local Courant number (pressure point: its cell; v point: the
mean of the two cells' r^2).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import pml, relaxation, stencil

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libfw2_oracle.so")
_SRC = os.path.join(_HERE, "fw2_oracle.c")


def build(force=False):
    """Compile the C stepper with gcc (plain -O2, OpenMP, IEEE double)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("L", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("pad_", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
        ("dt", ctypes.c_double), ("g", ctypes.c_double * 4), ("g11", ctypes.c_double),
        ("kap0", ctypes.c_void_p), ("nlq", ctypes.c_void_p),
        ("rho_v", ctypes.c_void_p), ("kap_v", ctypes.c_void_p),
        ("ik1", ctypes.c_void_p), ("ik2", ctypes.c_void_p),
        ("a1", ctypes.c_void_p), ("b1", ctypes.c_void_p),
        ("a2", ctypes.c_void_p), ("b2", ctypes.c_void_p),
        ("e0_1", ctypes.c_void_p), ("e0_2", ctypes.c_void_p),
        ("n_src", ctypes.c_int32), ("src_idx", ctypes.c_void_p), ("src_sig", ctypes.c_void_p),
        ("src_w", ctypes.c_void_p), ("n_t", ctypes.c_int32), ("signals", ctypes.c_void_p),
        ("n_rcv", ctypes.c_int32), ("rcv_idx", ctypes.c_void_p),
        ("gw_p", ctypes.c_void_p), ("gw_v", ctypes.c_void_p),
        ("nl_A", ctypes.c_double),
    ]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build()
        lib = ctypes.CDLL(_SO)
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_run.argtypes = [ctypes.POINTER(_Problem)] + [ctypes.c_void_p] * 4 + \
            [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_threads.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def threads():
    """OpenMP threads the C stepper uses (OMP_NUM_THREADS or all cores)."""
    return int(_lib().oracle_threads())


# ---------------------------------------------------------------------------
# Per-point coefficient maps
# ---------------------------------------------------------------------------

def _np_axis(ndim, a):
    """numpy axis of physical axis a (0 = x, fastest)."""
    return ndim - 1 - a


def _next_along(f, ndim, a):
    """f at the next cell along axis a; past the last cell, the last value."""
    ax = _np_axis(ndim, a)
    n = f.shape[ax]
    idx = np.minimum(np.arange(1, n + 1), n - 1)
    return np.take(f, idx, axis=ax)


def _along(vec, ndim, a):
    """Reshape a 1-D array over axis a so it broadcasts against the grid."""
    shape = [1] * ndim
    shape[_np_axis(ndim, a)] = vec.size
    return vec.reshape(shape)


class Maps:
    """All per-point FP64 coefficient arrays of one problem."""


def nonlinear_coefficients(prob):
    """(A, B0, B1) of the multipliers rho0 (1 + A kappa0 p) and
    kappa0 (1 + kappa0 (B0 + B1 beta) p): Eqs. state1 / state2 as printed
    give (1, 1, -2); prob.nonlinear_form = 1 takes prob.nl_A, nl_B0, nl_B1."""
    if int(getattr(prob, "nonlinear_form", 0)) == 1:
        return float(prob.nl_A), float(prob.nl_B0), float(prob.nl_B1)
    return 1.0, 1.0, -2.0


def coefficient_maps(prob):
    """Compute every derived coefficient from the problem's inputs (FP64).

    prob is a workloads.Problem (inputs only).  Returns a Maps object whose
    arrays are C-contiguous float64 with the grid shape (x fastest).
    """
    ndim = len(prob.shape)
    L = int(prob.n_relax)
    grid = tuple(prob.shape[::-1])
    c = np.asarray(prob.c, dtype=np.float64).reshape(grid)
    rho = np.asarray(prob.rho, dtype=np.float64).reshape(grid)
    beta = np.asarray(prob.beta, dtype=np.float64).reshape(grid)
    m = Maps()
    m.ndim, m.L, m.grid = ndim, L, grid
    m.dt, m.h = float(prob.dt), float(prob.h)

    # Medium: kappa0 = 1/(rho0 c^2) (compressibility, Sec. 2.2), kappa0 B with
    # B = 1 - 2 beta as printed (Eq. state2), and the momentum multiplier's A.
    kap0 = 1.0 / (rho * c * c)
    m.kap0 = kap0
    A, B0, B1 = nonlinear_coefficients(prob)
    m.nl_A = A
    m.nlq = kap0 * (B0 + B1 * beta)
    m.rho_v = np.stack([0.5 * (rho + _next_along(rho, ndim, a)) for a in range(ndim)])
    m.kap_v = np.stack([0.5 * (kap0 + _next_along(kap0, ndim, a)) for a in range(ndim)])

    # Stencil (Sec. 3.1), one global Courant number.
    cmax = float(np.max(c))
    r = float(prob.fd_r) if prob.fd_r and prob.fd_r > 0 else cmax * m.dt / m.h
    g, g11 = stencil.stencil_weights(r, ndim)
    m.r, m.g, m.g11 = r, g / m.h, g11 / m.h
    # stencil_mode 1: the weights of the local Courant number at every point.
    # A pressure point takes r^2 = (c dt / h)^2 of its cell; a v_a point the
    # mean of the r^2 of the two cells it lies between (the cell past the
    # last one repeating the last value).  Rows: g_10..g_40, g_11, over h.
    m.stencil_mode = int(getattr(prob, "stencil_mode", 0))
    m.gw_p = m.gw_v = None
    if m.stencil_mode == 1:
        r2 = (c * m.dt / m.h) ** 2
        gp, g11p = stencil.local_weights(r2, ndim)
        m.gw_p = np.concatenate([gp, g11p[None]]) / m.h
        gv = []
        for a in range(ndim):
            ga, g11a = stencil.local_weights(0.5 * (r2 + _next_along(r2, ndim, a)), ndim)
            gv.append(np.concatenate([ga, g11a[None]]) / m.h)
        m.gw_v = np.stack(gv)
    elif m.stencil_mode != 0:
        raise ValueError("stencil_mode must be 0 or 1")

    # Relaxation tuple per point.
    table = np.asarray(prob.relax_table, dtype=np.float64)
    lab = np.zeros(grid, dtype=np.intp) if prob.label is None else \
        np.asarray(prob.label).reshape(grid).astype(np.intp)
    k1 = table[lab, 0]
    k2 = table[lab, 1]
    d1 = [table[lab, 2 + nu] for nu in range(L)]
    d2 = [table[lab, 2 + L + nu] for nu in range(L)]
    al1 = [table[lab, 2 + 2 * L + nu] for nu in range(L)]
    al2 = [table[lab, 2 + 3 * L + nu] for nu in range(L)]

    c_p = float(prob.pml_cp) if prob.pml_cp and prob.pml_cp > 0 else cmax
    Rc, N = float(prob.pml_Rc), int(prob.pml_npoly)
    # boundary-layer reading: "A" (the library's); "B" and "A_kappa" serve the
    # reflection study only (oracle.pml)
    reading = getattr(prob, "pml_reading", "A")

    npts = int(np.prod(grid))
    m.ik1 = np.stack([1.0 / k1 for _ in range(ndim)])
    m.ik2 = np.stack([1.0 / k2 for _ in range(ndim)])
    m.a1 = np.zeros((ndim, L) + grid)
    m.b1 = np.zeros((ndim, L) + grid)
    m.a2 = np.zeros((ndim, L) + grid)
    m.b2 = np.zeros((ndim, L) + grid)
    m.scheme = int(getattr(prob, "relax_scheme", 1))
    m.e0_1 = np.zeros((ndim, L) + grid)
    m.e0_2 = np.zeros((ndim, L) + grid)
    for a in range(ndim):
        n_a = prob.shape[a]
        nb, ntr = int(prob.bound_cells[a]), int(prob.trans_cells[a])
        s_int = _along(pml.boundary_distance(np.arange(n_a), n_a, nb), ndim, a)
        s_half = _along(pml.boundary_distance(np.arange(n_a) + 0.5, n_a, nb), ndim, a)
        for nu in range(L):
            # nabla_2 at pressure points (integer positions along a)
            dd, aa = pml.profile(s_int, m.h, nb, ntr, d2[nu], al2[nu], nu + 1, c_p, Rc, N, reading, k2)
            A, B = relaxation.memory_coefficients(k2, dd, aa, m.dt)
            m.a2[a, nu], m.b2[a, nu] = A, B
            m.e0_2[a, nu] = relaxation.centred_weights(k2, dd, aa, m.dt)[0]
            # nabla_1 at velocity points (half-integer positions along a)
            dd, aa = pml.profile(s_half, m.h, nb, ntr, d1[nu], al1[nu], nu + 1, c_p, Rc, N, reading, k1)
            A, B = relaxation.memory_coefficients(k1, dd, aa, m.dt)
            m.a1[a, nu], m.b1[a, nu] = A, B
            m.e0_1[a, nu] = relaxation.centred_weights(k1, dd, aa, m.dt)[0]
    m.npts = npts
    return m


class State:
    """FP64 solver state: p, v[ndim], psi1[ndim][L], psi2[ndim][L], step."""

    def __init__(self, ndim, L, grid):
        self.p = np.zeros(grid)
        self.v = np.zeros((ndim,) + grid)
        self.psi1 = np.zeros((ndim, L) + grid)
        self.psi2 = np.zeros((ndim, L) + grid)
        self.step = 0

    def copy(self):
        s = State.__new__(State)
        s.p, s.v, s.psi1, s.psi2 = self.p.copy(), self.v.copy(), self.psi1.copy(), self.psi2.copy()
        s.step = self.step
        return s


def _sources(prob):
    idx = np.ascontiguousarray(np.asarray(prob.src_idx, dtype=np.int64))
    sig = np.ascontiguousarray(np.asarray(prob.src_sig, dtype=np.int32))
    w = np.ascontiguousarray(np.asarray(prob.src_w, dtype=np.float64))
    signals = np.ascontiguousarray(np.asarray(prob.signals, dtype=np.float64))
    if signals.ndim == 1:
        signals = signals[None, :]
    return idx, sig, w, signals


def run(prob, n_steps, state=None, maps=None, record=True):
    """Advance the problem n_steps with the C stepper.

    Returns (state, trace) with trace [n_steps][n_rcv] (FP64) or None.
    """
    if maps is None:
        maps = coefficient_maps(prob)
    if state is None:
        state = State(maps.ndim, maps.L, maps.grid)
    idx, sig, w, signals = _sources(prob)
    ridx = np.ascontiguousarray(np.asarray(prob.rcv_idx, dtype=np.int64))
    P = _Problem()
    P.ndim, P.L, P.scheme = maps.ndim, maps.L, maps.scheme
    n3 = list(prob.shape) + [1] * (3 - maps.ndim)
    for k in range(3):
        P.n[k] = int(n3[k])
    P.dt = maps.dt
    for k in range(4):
        P.g[k] = float(maps.g[k])
    P.g11 = float(maps.g11)
    keep = []

    def ptr(arr, dtype=np.float64):
        arr = np.ascontiguousarray(arr, dtype=dtype)
        keep.append(arr)
        return arr.ctypes.data

    P.kap0, P.nlq = ptr(maps.kap0), ptr(maps.nlq)
    P.rho_v, P.kap_v = ptr(maps.rho_v), ptr(maps.kap_v)
    P.ik1, P.ik2 = ptr(maps.ik1), ptr(maps.ik2)
    P.a1, P.b1, P.a2, P.b2 = ptr(maps.a1), ptr(maps.b1), ptr(maps.a2), ptr(maps.b2)
    P.e0_1, P.e0_2 = ptr(maps.e0_1), ptr(maps.e0_2)
    P.n_src = int(idx.size)
    P.src_idx, P.src_sig, P.src_w = ptr(idx, np.int64), ptr(sig, np.int32), ptr(w)
    P.n_t = int(signals.shape[1])
    P.signals = ptr(signals)
    P.n_rcv = int(ridx.size)
    P.rcv_idx = ptr(ridx, np.int64)
    P.gw_p = ptr(maps.gw_p) if maps.gw_p is not None else None
    P.gw_v = ptr(maps.gw_v) if maps.gw_v is not None else None
    P.nl_A = float(maps.nl_A)
    for name in ("p", "v", "psi1", "psi2"):
        arr = getattr(state, name)
        if not (arr.flags.c_contiguous and arr.dtype == np.float64):
            setattr(state, name, np.ascontiguousarray(arr, dtype=np.float64))
    trace = np.zeros((int(n_steps), int(ridx.size))) if (record and ridx.size) else None
    rc = _lib().oracle_run(ctypes.byref(P), state.p.ctypes.data, state.v.ctypes.data,
                           state.psi1.ctypes.data, state.psi2.ctypes.data,
                           int(state.step), int(n_steps),
                           trace.ctypes.data if trace is not None else None)
    if rc != 0:
        raise RuntimeError("oracle_run failed (%d)" % rc)
    state.step += int(n_steps)
    return state, trace


# ---------------------------------------------------------------------------
# Vectorised NumPy twin of the C stepper (tiny grids; cross-checks indexing)
# ---------------------------------------------------------------------------

PAD = 5


def _shift(fp, ndim, grid, off):
    """View of the zero-padded field fp at x + off (off in x, y, z order)."""
    sl = []
    for npax in range(ndim):
        a = ndim - 1 - npax
        start = PAD + off[a]
        sl.append(slice(start, start + grid[npax]))
    return fp[tuple(sl)]


def _pad(f):
    return np.pad(f, PAD)


def _memory(scheme, psi, a, nu, A, B, E0, D):
    """Advance one memory variable in place; return its term in the sum."""
    if scheme == 0:
        psi[a, nu] = B[a, nu] * psi[a, nu] + A[a, nu] * D
        return psi[a, nu].copy()
    term = E0[a, nu] * D + psi[a, nu]
    psi[a, nu] = B[a, nu] * psi[a, nu] + ((A[a, nu] - E0[a, nu]) + B[a, nu] * E0[a, nu]) * D
    return term


def numpy_run(prob, n_steps, state=None, maps=None):
    """Same algorithm as fw2_oracle.c, written with array shifts."""
    if maps is None:
        maps = coefficient_maps(prob)
    ndim, L, grid = maps.ndim, maps.L, maps.grid
    if state is None:
        state = State(ndim, L, grid)
    idx, sig, w, signals = _sources(prob)
    ridx = np.asarray(prob.rcv_idx, dtype=np.int64)
    trace = np.zeros((int(n_steps), ridx.size))

    def e(a, s=1):
        o = [0, 0, 0]
        o[a] = s
        return o

    def add(o1, o2):
        return [o1[k] + o2[k] for k in range(3)]

    if maps.stencil_mode == 1:
        wp = [maps.gw_p[k] for k in range(5)]
        wv = [[maps.gw_v[a, k] for k in range(5)] for a in range(ndim)]
    else:
        wp = list(maps.g) + [maps.g11]
        wv = [wp] * ndim

    for s in range(int(n_steps)):
        step = state.step
        # pressure phase
        S = np.zeros(grid)
        for a in range(ndim):
            vp = _pad(state.v[a])
            D = np.zeros(grid)
            for mm in range(1, 5):
                D += wp[mm - 1] * (_shift(vp, ndim, grid, e(a, mm - 1)) -
                                   _shift(vp, ndim, grid, e(a, -mm)))
            for b in range(ndim):
                if b == a:
                    continue
                for sg in (-1, 1):
                    D += wp[4] * (_shift(vp, ndim, grid, e(b, sg)) -
                                  _shift(vp, ndim, grid, add(e(a, -1), e(b, sg))))
            acc = np.zeros(grid)
            for nu in range(L):
                acc += _memory(maps.scheme, state.psi2, a, nu, maps.a2, maps.b2, maps.e0_2, D)
            S += maps.ik2[a] * D + acc
        kappa = maps.kap0 * (1.0 + maps.nlq * state.p)
        state.p = state.p - maps.dt * S / kappa
        flat = state.p.reshape(-1)
        if step < signals.shape[1]:
            for q in range(idx.size):
                flat[idx[q]] += w[q] * signals[sig[q], step]
        trace[s] = flat[ridx] if ridx.size else trace[s]
        # velocity phase
        pp = _pad(state.p)
        psi1_old = [None] * ndim
        for a in range(ndim):
            D = np.zeros(grid)
            for mm in range(1, 5):
                D += wv[a][mm - 1] * (_shift(pp, ndim, grid, e(a, mm)) -
                                      _shift(pp, ndim, grid, e(a, -(mm - 1))))
            for b in range(ndim):
                if b == a:
                    continue
                for sg in (-1, 1):
                    D += wv[a][4] * (_shift(pp, ndim, grid, add(e(a, 1), e(b, sg))) -
                                     _shift(pp, ndim, grid, e(b, sg)))
            acc = np.zeros(grid)
            psi1_old[a] = [state.psi1[a, nu].copy() for nu in range(L)]
            for nu in range(L):
                acc += _memory(maps.scheme, state.psi1, a, nu, maps.a1, maps.b1, maps.e0_1, D)
            Sv = maps.ik1[a] * D + acc
            pbar = 0.5 * (state.p + _shift(pp, ndim, grid, e(a, 1)))
            vnew = state.v[a] - maps.dt * Sv / (maps.rho_v[a] * (1.0 + maps.nl_A * maps.kap_v[a] * pbar))
            # the sample past the last pressure sample along a is outside
            inside = _along(np.arange(grid[_np_axis(ndim, a)]) < grid[_np_axis(ndim, a)] - 1, ndim, a)
            state.v[a] = np.where(inside, vnew, state.v[a])
            for nu in range(L):
                state.psi1[a, nu] = np.where(inside, state.psi1[a, nu], psi1_old[a][nu])
        state.step += 1
    return state, trace


def stencil_maps(prob):
    """The part of coefficient_maps that divergence() needs (grid, stencil
    weights), without the per-point relaxation maps (large grids)."""
    ndim = len(prob.shape)
    m = Maps()
    m.ndim, m.grid = ndim, tuple(prob.shape[::-1])
    m.h, m.dt = float(prob.h), float(prob.dt)
    m.stencil_mode = int(getattr(prob, "stencil_mode", 0))
    if m.stencil_mode != 0:
        return coefficient_maps(prob)
    cmax = float(np.max(np.asarray(prob.c, dtype=np.float64)))
    r = float(prob.fd_r) if prob.fd_r and prob.fd_r > 0 else cmax * m.dt / m.h
    g, g11 = stencil.stencil_weights(r, ndim)
    m.r, m.g, m.g11 = r, g / m.h, g11 / m.h
    return m


def divergence(v, maps):
    """Sum over the axes of (D^- v_a) at every pressure point (Sec. 3.1
    stencil, the operator of the pressure phase), FP64.

    v is [ndim] + grid (any float dtype); the weights are the problem's own
    (global, or per point with stencil_mode 1).  With no memory variables and
    p = 0 before the step, the pressure phase sets p = -dt S / kappa0 with S
    this divergence, which is how the function is pinned against the C
    stepper.  Used to compare the part of a velocity field that drives the
    pressure."""
    ndim, grid = maps.ndim, maps.grid
    v = np.asarray(v, dtype=np.float64)
    if maps.stencil_mode == 1:
        wp = [maps.gw_p[k] for k in range(5)]
    else:
        wp = list(maps.g) + [maps.g11]

    def e(a, s=1):
        o = [0, 0, 0]
        o[a] = s
        return o

    out = np.zeros(grid)
    for a in range(ndim):
        vp = _pad(v[a])
        for mm in range(1, 5):
            out += wp[mm - 1] * (_shift(vp, ndim, grid, e(a, mm - 1)) -
                                 _shift(vp, ndim, grid, e(a, -mm)))
        for b in range(ndim):
            if b == a:
                continue
            for sg in (-1, 1):
                o2 = e(a, -1)
                o2[b] += sg
                out += wp[4] * (_shift(vp, ndim, grid, e(b, sg)) - _shift(vp, ndim, grid, o2))
    return out
