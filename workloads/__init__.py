"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds input data and random draws only: grids, medium maps
(c, rho, beta), tissue labels with their relaxation tuples, source signals and
positions, receiver positions.  It contains none of the method's arithmetic;
derived coefficients (stencil weights, memory-variable coefficients, boundary
profiles) are computed separately by the oracle and by the HIP library.

Relaxation tuples are the paper's Table 2 (alpha0 = 0.5 dB/cm/MHz, y = 1,
two mechanisms) or entries of tissue_fits.json, written by
oracle/make_tissue_fits.py with the paper's fitting objective (Sec. 4.1).

The paper's 2D and 3D application datasets (a segmented Visible Human abdomen
and a micro-CT rat skull) are not available; configs 2 and 3 are synthetic
stand-ins with the shapes, property ranges and structure stated for them.
"""
import json
import os
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

# Table 2 of the paper: two mechanisms fitted to alpha0 = 0.5 dB/cm/MHz, y = 1.
# Column order: k1, k2, d1[nu=1,2], d2[nu=1,2], alpha1[nu=1,2], alpha2[nu=1,2].
TABLE2_ROW = [0.835, 1.19, 9.82e5, 3.26e6, 4.40e4, 1.68e5, 2.83e8, 3.54e9, 8.35e6, 5.10e7]

# Medium without attenuation or dispersion: unit stretch, no mechanisms.
def lossless_row(L):
    return [1.0, 1.0] + [0.0] * (4 * L)


_FITS = None


def tissue_fits():
    global _FITS
    if _FITS is None:
        with open(os.path.join(_HERE, "tissue_fits.json")) as fh:
            _FITS = json.load(fh)["fits"]
    return _FITS


def tissue_row(alpha0, y, L, f_ref):
    """Relaxation tuple for alpha0 f^y with L mechanisms (stored fit)."""
    k = "a%.2f_y%.2f_L%d_f%.1f" % (alpha0, y, L, f_ref / 1e6)
    return list(tissue_fits()[k]["row"])


ALPHA0_GRID = [0.4, 0.6, 0.8, 1.0, 1.2, 1.5]
Y_GRID = [1.0, 1.1, 1.2, 1.3]


@dataclass
class Problem:
    """Inputs of one simulation (what create_domain / add_source / add_receivers take).

    Arrays are numpy with shape shape[::-1] (x fastest); flat indices are
    x + nx * (y + ny * z).
    """
    shape: Tuple[int, ...]
    h: float
    dt: float
    n_relax: int
    c: np.ndarray
    rho: np.ndarray
    beta: np.ndarray
    relax_table: np.ndarray                  # [n_labels, 2 + 4L] float64
    label: Optional[np.ndarray] = None       # uint8, or None = all label 0
    bound_cells: Tuple[int, ...] = (0, 0, 0)
    trans_cells: Tuple[int, ...] = (0, 0, 0)
    pml_Rc: float = 1e-3
    pml_npoly: int = 2
    pml_cp: float = 0.0                      # 0: largest c of the map
    fd_r: float = 0.0                        # 0: largest c * dt / h
    relax_scheme: int = 1                    # 0: printed recursion, 1: time-centred
    stencil_mode: int = 0                    # 0: one global r, 1: r of the local sound speed
    nonlinear_form: int = 0                  # 0: multipliers as printed; 1: the coefficients below
    nl_A: float = 1.0                        # rho0 (1 + A kappa0 p)
    nl_B0: float = 1.0                       # kappa0 (1 + kappa0 (B0 + B1 beta) p)
    nl_B1: float = -2.0
    src_idx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    src_sig: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    src_w: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    signals: np.ndarray = field(default_factory=lambda: np.zeros((1, 1), np.float32))
    rcv_idx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    n_steps: int = 0
    name: str = ""

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def flat(self, *coords):
        """Flat index of (x, y[, z]) (arrays allowed)."""
        idx = np.zeros_like(np.asarray(coords[0]), dtype=np.int64)
        stride = 1
        for a, x in enumerate(coords):
            idx = idx + np.asarray(x, dtype=np.int64) * stride
            stride *= self.shape[a]
        return idx


def gaussian_pulse(n_t, dt, f0, n_cycles, amp=1.0):
    """Gaussian-modulated sinusoid (the pulse shape the paper's experiments
    use).  Sample n belongs to step n, i.e. to t_n = (n + 1/2) dt; envelope
    standard deviation n_cycles / (4 f0), centred at six deviations."""
    sig = n_cycles / (4.0 * f0)
    t0 = 6.0 * sig
    t = (np.arange(n_t) + 0.5) * dt
    return (amp * np.sin(2 * np.pi * f0 * (t - t0)) * np.exp(-0.5 * ((t - t0) / sig) ** 2)).astype(np.float32)


def pulse_length(dt, f0, n_cycles):
    """Samples covering the pulse (twelve envelope deviations)."""
    return int(np.ceil(12.0 * n_cycles / (4.0 * f0) / dt)) + 1


def grid_spacing(c_ref, f0, ppw):
    return c_ref / (ppw * f0)


# ---------------------------------------------------------------------------
# Generic homogeneous problem (tests)
# ---------------------------------------------------------------------------

def homogeneous(shape, L=2, c=1540.0, rho=1000.0, beta=3.5, row=None, ppw=12, f0=2e6,
                cfl=0.4, nb=None, ntr=None, n_steps=100, name="homogeneous"):
    ndim = len(shape)
    h = grid_spacing(1540.0, f0, ppw)
    dt = cfl * h / c
    grid = tuple(shape[::-1])
    if row is None:
        row = TABLE2_ROW if L == 2 else lossless_row(L)
    if nb is None:
        nb = (0,) * ndim
    if ntr is None:
        ntr = tuple(int(round(0.75 * b)) for b in nb)
    return Problem(shape=tuple(shape), h=h, dt=dt, n_relax=L,
                   c=np.full(grid, c, np.float32), rho=np.full(grid, rho, np.float32),
                   beta=np.full(grid, beta, np.float32),
                   relax_table=np.asarray([row], np.float64), label=None,
                   bound_cells=tuple(nb), trans_cells=tuple(ntr), n_steps=n_steps, name=name)


def random_medium(shape, L, n_labels, seed, nb=8, ntr=6, ppw=12, f0=3e6, cfl=0.4, n_steps=50,
                  name="random"):
    """Piecewise-random medium: labels, c, rho, beta drawn per cell (tests)."""
    rng = np.random.default_rng(seed)
    ndim = len(shape)
    grid = tuple(shape[::-1])
    h = grid_spacing(1540.0, f0, ppw)
    c = rng.uniform(1450.0, 1620.0, grid).astype(np.float32)
    rho = rng.uniform(950.0, 1120.0, grid).astype(np.float32)
    beta = rng.uniform(3.5, 5.5, grid).astype(np.float32)
    dt = cfl * h / float(c.max())
    rows = []
    for k in range(n_labels):
        a0 = ALPHA0_GRID[rng.integers(len(ALPHA0_GRID))]
        y = Y_GRID[rng.integers(len(Y_GRID))]
        if L in (2, 3, 4):
            rows.append(tissue_row(a0, y, L, 3e6))
        elif 5 <= L <= 8:                    # fits stored for two tissues only
            rows.append(tissue_row(*((1.5, 1.3) if k % 2 == 0 else (0.5, 1.0)), L, 3e6))
        else:
            rows.append(lossless_row(L))
    label = rng.integers(0, n_labels, grid).astype(np.uint8)
    return Problem(shape=tuple(shape), h=h, dt=dt, n_relax=L, c=c, rho=rho, beta=beta,
                   relax_table=np.asarray(rows, np.float64), label=label,
                   bound_cells=(nb,) * ndim, trans_cells=(ntr,) * ndim, n_steps=n_steps, name=name)


def random_state(ndim, L, shape, seed, scale=1.0):
    """Seeded random initial state (p, v, psi1, psi2) in float32, scaled to
    acoustic magnitudes: p ~ scale * 1e5 Pa, v ~ p / (rho c), psi ~ v / h."""
    rng = np.random.default_rng(seed)
    grid = tuple(shape[::-1])
    p = (scale * 1e5 * rng.standard_normal(grid)).astype(np.float32)
    v = (scale * 1e5 / 1.5e6 * rng.standard_normal((ndim,) + grid)).astype(np.float32)
    psi1 = (scale * 1e5 * 1e-2 * rng.standard_normal((ndim, L) + grid)).astype(np.float32)
    psi2 = (scale * 1e5 / 1.5e6 * 1e2 * rng.standard_normal((ndim, L) + grid)).astype(np.float32)
    return p, v, psi1, psi2


# ---------------------------------------------------------------------------
# Workload 1: plain 2D, 384^2 interior + 4 wavelength boundary, water, L = 2
# ---------------------------------------------------------------------------

def plain_2d(interior=384, ppw=12, f0=2e6, cfl=0.4, n_steps=1000, n_rcv=64, seed=1):
    """384x384 interior + 48-cell (3 lambda transition + 1 lambda bound)
    boundary each side; water c 1540, rho 1000, beta 3.5; L = 2 fitted to
    0.5 dB/MHz^1.1/cm; 12 ppw at 2 MHz, CFL 0.4; 3-cycle line source; 1000
    steps; 64 receivers.  seed is unused (the workload is deterministic)."""
    lam = ppw
    nb, ntr = 4 * lam, 3 * lam
    n = interior + 2 * nb
    h = grid_spacing(1540.0, f0, ppw)
    c = 1540.0
    dt = cfl * h / c
    grid = (n, n)
    row = tissue_row(0.5, 1.1, 2, 2e6)
    prob = Problem(shape=(n, n), h=h, dt=dt, n_relax=2,
                   c=np.full(grid, c, np.float32), rho=np.full(grid, 1000.0, np.float32),
                   beta=np.full(grid, 3.5, np.float32), relax_table=np.asarray([row]),
                   bound_cells=(nb, nb), trans_cells=(ntr, ntr), n_steps=n_steps,
                   name="plain_2d_%d" % n)
    xs = np.arange(nb, nb + interior)
    prob.src_idx = prob.flat(xs, np.full_like(xs, nb + 8))
    prob.src_sig = np.zeros(xs.size, np.int32)
    prob.src_w = np.ones(xs.size, np.float32)
    nt = pulse_length(dt, f0, 3)
    prob.signals = gaussian_pulse(nt, dt, f0, 3, amp=1e5)[None, :]
    rx = np.round(np.linspace(nb, nb + interior - 1, n_rcv)).astype(np.int64)
    ry = min(nb + 300, n - nb - 1)
    prob.rcv_idx = prob.flat(rx, np.full_like(rx, ry))
    return prob


# ---------------------------------------------------------------------------
# Workload 2: heterogeneous abdominal-wall-like 2D medium, L = 4
# ---------------------------------------------------------------------------

def abdominal_2d(nx=4096, ny=2048, seed=2, n_steps=12000, ppw=12, f0=3e6, cfl=0.4,
                 n_interfaces=8, n_scatter=100000, n_elem=128, L=4):
    """Layered fat/muscle/connective medium with undulating interfaces and
    single-cell sound-speed scatterers; a linear array transmits a plane wave
    (zero delays) and receives on its element centres.  nx is the lateral
    (fastest) axis, ny the depth.  Smaller nx, ny give the same recipe on a
    smaller grid (parity tests)."""
    rng = np.random.default_rng(seed)
    lam = ppw
    nb, ntr = 4 * lam, 3 * lam
    h = grid_spacing(1540.0, f0, ppw)
    grid = (ny, nx)
    W = nx * h
    depth = (ny - 2 * nb) * h
    # interfaces: y_k(x) = y_k0 + sum_m A_m sin(2 pi m x / W + phi_m), A <= 1 mm
    x = np.arange(nx) * h
    y0 = np.sort(rng.uniform(0.05, 0.95, n_interfaces)) * depth + nb * h
    ifc = np.empty((n_interfaces, nx))
    for k in range(n_interfaces):
        amp = rng.uniform(0.0, 1e-3, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        ifc[k] = y0[k] + sum(amp[m] * np.sin(2 * np.pi * (m + 1) * x / W + ph[m]) for m in range(3))
    yy = (np.arange(ny) * h)[:, None]
    layer = np.zeros(grid, np.int32)
    for k in range(n_interfaces):
        layer += (yy >= ifc[k][None, :]).astype(np.int32)
    n_layers = n_interfaces + 1
    # per-layer tissue class and properties
    classes = rng.integers(0, 3, n_layers)     # 0 fat, 1 muscle, 2 connective
    c_l = rng.uniform(1450.0, 1620.0, n_layers)
    rho_l = rng.uniform(950.0, 1120.0, n_layers)
    beta_l = rng.uniform(3.5, 5.5, n_layers)
    a0_l = [ALPHA0_GRID[i] for i in rng.integers(0, len(ALPHA0_GRID), n_layers)]
    y_l = [Y_GRID[i] for i in rng.integers(0, len(Y_GRID), n_layers)]
    if L <= 4:
        rows = [tissue_row(a0_l[k], y_l[k], L, 3e6) for k in range(n_layers)]
    else:
        # 5..8 mechanisms are fitted for two laws only: fat layers take
        # 0.5 dB/MHz/cm, muscle and connective layers 1.5 dB/MHz^1.3/cm
        rows = [tissue_row(0.5, 1.0, L, 3e6) if classes[k] == 0 else tissue_row(1.5, 1.3, L, 3e6)
                for k in range(n_layers)]
    c = c_l[layer].astype(np.float32)
    rho = rho_l[layer].astype(np.float32)
    beta = beta_l[layer].astype(np.float32)
    label = layer.astype(np.uint8)
    # sub-resolution scatterers: single cells (< lambda/10 in size), c * (1 + 0.02 N(0,1))
    n_sc = int(min(n_scatter, nx * ny // 16))
    sx = rng.integers(0, nx, n_sc)
    sy = rng.integers(0, ny, n_sc)
    c[sy, sx] = (c[sy, sx] * (1.0 + 0.02 * rng.standard_normal(n_sc))).astype(np.float32)
    dt = cfl * h / float(c.max())
    prob = Problem(shape=(nx, ny), h=h, dt=dt, n_relax=L, c=c, rho=rho, beta=beta,
                   relax_table=np.asarray(rows, np.float64), label=label,
                   bound_cells=(nb, nb), trans_cells=(ntr, ntr), n_steps=n_steps,
                   name="abdominal_2d_%dx%d" % (nx, ny) + ("" if L == 4 else "_L%d" % L))
    prob.meta = {"classes": classes.tolist(), "alpha0": a0_l, "y": y_l}
    # linear array: pitch 12 cells (~ lambda), element width 10 cells, 8 cells
    # below the top boundary layer; fewer elements if the grid is narrow
    pitch, width = 12, 10
    n_el = int(min(n_elem, (nx - 2 * nb) // pitch))
    x0 = nx // 2 - (n_el * pitch) // 2
    ey = nb + 8
    ex = np.concatenate([x0 + e * pitch + np.arange(width) for e in range(n_el)])
    prob.src_idx = prob.flat(ex, np.full_like(ex, ey))
    prob.src_sig = np.repeat(np.arange(n_el, dtype=np.int32), width)
    prob.src_w = np.ones(ex.size, np.float32)
    nt = pulse_length(dt, f0, 3)
    pulse = gaussian_pulse(nt, dt, f0, 3, amp=1e5)
    prob.signals = np.repeat(pulse[None, :], n_el, axis=0)   # plane wave: zero delays
    centres = x0 + np.arange(n_el) * pitch + width // 2
    prob.rcv_idx = prob.flat(centres, np.full_like(centres, ey))
    return prob


# ---------------------------------------------------------------------------
# Workload 3: 3D transcranial-like medium, L = 2
# ---------------------------------------------------------------------------

def skull_3d(n=1024, nb=48, ntr=36, seed=3, n_steps=4000, ppw=12, f0=1e6, cfl=0.4, n_rcv=1024, L=2):
    """Cube of n^3 points including nb-cell layers: brain-like background
    (c 1540, rho 1040, beta 4; Table 2 tuple), a curved bone-like shell
    (thickness 4-8 cells = 0.5-1 mm at 12 ppw / 1 MHz; c 2800, rho 1900,
    alpha0 8 dB/MHz/cm fitted with two mechanisms; +-10% porosity noise on c
    and rho) between a focused spherical-cap source (aperture 0.49 of the
    domain, radius of curvature equal to it, apex 8 cells below the top
    layer) and its focus; receivers on the focal axis.  The geometry scales
    with n (same recipe on smaller cubes for parity tests).  z is the depth
    (slowest) axis.  With L = 5..8 the two tissues take the fitted 5..8
    mechanism tuples of 0.5 dB/MHz/cm (background) and 1.5 dB/MHz^1.3/cm
    (shell), the only laws fitted with that many mechanisms."""
    if L != 2 and not 5 <= L <= 8:
        raise ValueError("skull_3d takes L = 2 or 5..8")
    rng = np.random.default_rng(seed)
    h = grid_spacing(1540.0, f0, ppw)
    Ldom = n * h
    grid = (n, n, n)
    c = np.full(grid, 1540.0, np.float32)
    rho = np.full(grid, 1040.0, np.float32)
    beta = np.full(grid, 4.0, np.float32)
    label = np.zeros(grid, np.uint8)
    ctr = (n - 1) / 2.0
    apex = nb + 8
    Rcurv = 0.49 * n                        # cells
    aper = 0.245 * n                        # aperture radius, cells
    zf = apex + Rcurv                       # geometric focus on the axis
    # shell: sphere about a point below the focus, upper part only
    R_sk = 0.30 * n
    zc = zf + 0.05 * n
    ph = rng.uniform(0, 2 * np.pi, 4)
    km = rng.normal(0, 1, (6, 3))
    km = km / np.linalg.norm(km, axis=1, keepdims=True) * rng.uniform(0.15, 0.6, (6, 1))   # rad / cell
    pm = rng.uniform(0, 2 * np.pi, 6)
    am = rng.uniform(0.5, 1.0, 6)
    am = am / am.sum()
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float32)
    for z in range(n):
        dz = z - zc
        if dz > 0:
            continue
        r = np.sqrt((xx - ctr) ** 2 + (yy - ctr) ** 2 + dz * dz)
        th = np.arctan2(yy - ctr, xx - ctr)
        el = np.arccos(np.clip(-dz / np.maximum(r, 1e-6), -1, 1))
        thick = 6.0 + 2.0 * np.sin(3 * th + ph[0]) * np.cos(4 * el + ph[1])
        m = (r >= R_sk) & (r <= R_sk + thick)
        if not m.any():
            continue
        noise = np.zeros(int(m.sum()), np.float32)
        px, py = xx[m], yy[m]
        for q in range(6):
            noise += am[q] * np.sin(km[q, 0] * px + km[q, 1] * py + km[q, 2] * z + pm[q])
        c[z][m] = (2800.0 * (1.0 + 0.1 * noise)).astype(np.float32)
        rho[z][m] = (1900.0 * (1.0 + 0.1 * noise)).astype(np.float32)
        label[z][m] = 1
    dt = cfl * h / float(c.max())
    if L == 2:
        rows = [TABLE2_ROW, tissue_row(8.0, 1.0, 2, 1e6)]
    else:
        rows = [tissue_row(0.5, 1.0, L, 3e6), tissue_row(1.5, 1.3, L, 3e6)]
    prob = Problem(shape=(n, n, n), h=h, dt=dt, n_relax=L, c=c, rho=rho, beta=beta,
                   relax_table=np.asarray(rows, np.float64), label=label,
                   bound_cells=(nb,) * 3, trans_cells=(ntr,) * 3, n_steps=n_steps,
                   name="skull_3d_%d" % n + ("" if L == 2 else "_L%d" % L))
    # focused spherical cap: voxels within half a cell of the sphere of radius
    # Rcurv about the focus, inside the aperture, above the focus
    zs = np.arange(apex, int(np.ceil(zf)))
    pts = []
    for z in zs:
        dz = z - zf
        rho_xy2 = Rcurv * Rcurv - dz * dz
        if rho_xy2 <= 0:
            continue
        r = np.sqrt((xx - ctr) ** 2 + (yy - ctr) ** 2 + dz * dz)
        m = (np.abs(r - Rcurv) <= 0.5) & ((xx - ctr) ** 2 + (yy - ctr) ** 2 <= aper * aper)
        if m.any():
            pts.append(prob.flat(xx[m].astype(np.int64), yy[m].astype(np.int64), np.full(int(m.sum()), z)))
    prob.src_idx = np.unique(np.concatenate(pts)).astype(np.int64)
    prob.src_sig = np.zeros(prob.src_idx.size, np.int32)
    prob.src_w = np.ones(prob.src_idx.size, np.float32)
    nt = pulse_length(dt, f0, 3)
    prob.signals = gaussian_pulse(nt, dt, f0, 3, amp=1e5)[None, :]
    zr = np.unique(np.round(np.linspace(apex + 2, n - nb - 1, n_rcv)).astype(np.int64))
    ci = int(round(ctr))
    prob.rcv_idx = prob.flat(np.full(zr.size, ci), np.full(zr.size, ci), zr)
    return prob


# ---------------------------------------------------------------------------
# Workload 4: stream of 2D requests for batched serving
# ---------------------------------------------------------------------------

def serving_requests(n=256, seed=4, sides=(1024, 3072), side_step=256, f0_range=(1e6, 5e6),
                     L_choices=(2, 3, 4), steps_per_depth=2.5, rate=None, max_steps=None):
    """Seeded stream of n square 2D requests.  Request i uses seed 4000 + i:
    side drawn from {sides[0], sides[0] + side_step, ..., sides[1]}, f0 from
    U[f0_range], L from L_choices, the layered abdominal recipe with
    scatterers scaled by area, and n_steps = steps_per_depth * side (one depth
    crossing at CFL 0.4), capped at max_steps.  With a rate, arrivals are a
    Poisson process of that rate (requests per second); otherwise all arrive
    at t = 0.  Returns a list of (problem, n_steps, arrival)."""
    rng = np.random.default_rng(seed)
    side_set = np.arange(sides[0], sides[1] + 1, side_step)
    t = 0.0
    out = []
    for i in range(n):
        r = np.random.default_rng(4000 + i)
        side = int(side_set[r.integers(len(side_set))])
        f0 = float(r.uniform(*f0_range))
        L = int(L_choices[r.integers(len(L_choices))])
        steps = int(round(steps_per_depth * side))
        if max_steps:
            steps = min(steps, int(max_steps))
        n_sc = int(1e5 * side * side / (4096 * 2048))
        prob = abdominal_2d(nx=side, ny=side, seed=4000 + i, n_steps=steps, f0=f0, L=L,
                            n_scatter=max(n_sc, 1), n_elem=min(128, max(4, (side - 96) // 12)))
        prob.name = "request_%d_%dx%d_L%d" % (i, side, side, L)
        if rate:
            t += rng.exponential(1.0 / rate)
        out.append((prob, steps, t if rate else 0.0))
    return out


# ---------------------------------------------------------------------------
# Workload 5: 2D sound-speed inversion (gradient of a trace misfit), L = 2
# ---------------------------------------------------------------------------

def inversion_2d(n=1536, seed=5, shot=0, n_steps=6000, ppw=12, f0=2e6, cfl=0.4, L=2,
                 n_src=64, n_rcv=256, n_blobs=8, blob_amp=0.03):
    """One shot of a seeded inversion problem on an n x n grid (including the
    4-wavelength boundary layers).  The background is the layered abdominal
    recipe at f0 without scatterers; the true medium multiplies its sound
    speed by (1 + sum_k s_k blob_amp G_k) with n_blobs Gaussian blobs G_k
    (peak 1, radius 0.02-0.06 of the interior, signs s_k = +-1) inside the
    interior.  n_src point sources sit on one row 8 cells below the top
    boundary layer, evenly spaced across the interior; this problem fires
    source `shot` with a 3-cycle pulse (1e5 Pa).  n_rcv receivers sit on the
    same row.  The stencil's Courant number and the boundary layer's speed
    are fixed from the background (they do not vary with c), and the time
    step keeps the true medium at the stated CFL.  Returns (problem with the
    background c, true c)."""
    prob = abdominal_2d(nx=n, ny=n, seed=seed, n_steps=n_steps, ppw=ppw, f0=f0, cfl=cfl,
                        n_scatter=0, n_elem=1, L=L)
    rng = np.random.default_rng(seed + 1000)
    nb = prob.bound_cells[0]
    inner = n - 2 * nb
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pert = np.zeros((n, n))
    for _ in range(n_blobs):
        r = rng.uniform(0.02, 0.06) * inner
        cx, cy = rng.uniform(nb + 2 * r, n - nb - 2 * r, 2)
        s = 1.0 if rng.random() < 0.5 else -1.0
        pert += s * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * r * r))
    c_bg = np.asarray(prob.c, np.float64)
    c_true = (c_bg * (1.0 + blob_amp * pert)).astype(np.float32)
    prob.dt = cfl * prob.h / float(c_true.max())
    prob.fd_r = float(c_true.max()) * prob.dt / prob.h
    prob.pml_cp = float(c_bg.max())
    ey = nb + 8
    sx = nb + (np.arange(n_src) * inner) // n_src + inner // (2 * n_src)
    rx = nb + (np.arange(n_rcv) * inner) // n_rcv + inner // (2 * n_rcv)
    prob.src_idx = prob.flat(np.array([sx[shot]]), np.array([ey]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    nt = pulse_length(prob.dt, f0, 3)
    prob.signals = gaussian_pulse(nt, prob.dt, f0, 3, amp=1e5)[None, :]
    prob.rcv_idx = prob.flat(rx, np.full_like(rx, ey))
    prob.name = "inversion_2d_%d_shot%d" % (n, shot)
    return prob, c_true
