"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bar: relative L2 <= 1e-4 and max-abs <= 1e-3 of the peak pressure.
  - p and the receiver traces: both, always (the relative L2 of the final p
    is waived only when the pulse has left the grid and the final field is
    below 1e-5 of the peak: it then measures FP32 rounding of a residue).
  - v, psi1, psi2: max-abs after conversion to pressure units (rho c |dv|,
    h |dpsi1|, h rho c |dpsi2|), always.  While the pulse is in the grid
    (final max|p| at least a tenth of the peak) each is also held to the
    relative L2 bar.  After it has left, FP32 rounding leaves a small
    residual in v and psi2 that the pressure phase does not feel (their
    relative L2 can exceed 1e-4 while p stays within 1e-5); there the
    combination of v and psi2 that drives p, the pressure phase's S (one
    oracle step's pressure increment from the GPU state against that from
    the oracle state), is held to the relative L2 bar, waived below 1e-5 of
    the peak like p.  The divergence of v is printed beside them.
Every test prints its case before touching the GPU."""
import numpy as np
import pytest

import workloads as W
from oracle import solver

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
MAX_ABS = 1e-3
DECAYED = 1e-5          # final field below this fraction of the peak: the pulse has left the grid
LIVE = 0.1              # final max|p| at least this fraction of the peak: the pulse is in the grid


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def gpu_run(prob, n_steps, state=None, chunks=None, graph_chunk=None, cap=None):
    torch = _torch()
    from paper_2106_11476_amd import fw2
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=cap if cap else max(n_steps, 1))
    if graph_chunk is not None:
        dom.set_graph_chunk(graph_chunk)
    if state is not None:
        dom.write_fields(state)
    for n in (chunks or [n_steps]):
        dom.step(n)
    torch.cuda.synchronize()
    f = dom.read_fields(fw2.FIELD_ALL)
    tr = dom.trace.cpu().numpy() if dom.trace is not None else None
    step = dom.current_step()
    dom.destroy_domain()
    return f, tr, step


def oracle_run(prob, n_steps, state=None):
    st = None
    if state is not None:
        st = solver.State(prob.ndim, prob.n_relax, prob.c.shape)
        st.p = state["p"].astype(np.float64)
        st.v = state["v"].astype(np.float64)
        st.psi1 = state["psi1"].astype(np.float64)
        st.psi2 = state["psi2"].astype(np.float64)
    st, tr = solver.run(prob, n_steps, st)
    return st, tr


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def pressure_drive(prob, fields, step, maps):
    """One oracle step's pressure increment from the given state: -dt S / K
    plus the sources of that step, where S is what the pressure phase forms
    from v and psi2 (the part of the state that drives p)."""
    st = solver.State(prob.ndim, prob.n_relax, tuple(prob.shape[::-1]))
    st.p, st.v = fields["p"].astype(np.float64), fields["v"].astype(np.float64)
    st.psi1, st.psi2 = fields["psi1"].astype(np.float64), fields["psi2"].astype(np.float64)
    st.step = int(step)
    p0 = st.p.copy()
    s1, _ = solver.run(prob, 1, st, maps=maps, record=False)
    return s1.p - p0


def compare(f, tr, ref, rtr, label, check_all=True, prob=None):
    """Prints every figure, then asserts the bars (module docstring)."""
    peak = np.abs(ref.p).max()
    if rtr is not None and rtr.size:
        peak = max(peak, np.abs(rtr).max())
    e_p = rel_l2(f["p"], ref.p)
    m_p = np.abs(f["p"] - ref.p).max() / peak
    a_p = np.abs(ref.p).max() / peak
    _say(label, "p rel %.2e max/peak %.2e (final max|p| %.1e of peak)" % (e_p, m_p, a_p))
    if rtr is not None and rtr.size:
        e_t = rel_l2(tr[:rtr.shape[0]], rtr)
        m_t = np.abs(tr[:rtr.shape[0]] - rtr).max() / peak
        _say(label, "trace rel %.2e max/peak %.2e" % (e_t, m_t))
    fields = []
    if check_all:
        z = float(np.max(np.asarray(prob.rho, np.float64) * np.asarray(prob.c, np.float64)))
        h = prob.h
        scale = {"v": z, "psi1": h, "psi2": h * z}
        for name in ("v", "psi1", "psi2"):
            r = getattr(ref, name)
            d = np.abs(f[name] - r).max() * scale[name] / peak
            a = np.abs(r).max() * scale[name] / peak
            e = rel_l2(f[name], r)
            fields.append((name, d, a, e))
            _say(label, "%s max-abs (pressure units)/peak %.2e, rel L2 %.2e (max %.1e of peak)" % (name, d, e, a))
        maps = solver.stencil_maps(prob)
        e_d = rel_l2(solver.divergence(f["v"], maps), solver.divergence(ref.v, maps))
        _say(label, "div(v) rel L2 %.2e" % e_d)
        drive = None
        if a_p < LIVE or prob.ndim == 2 or np.prod(prob.shape) <= 2e6:
            cm = solver.coefficient_maps(prob)
            gd = pressure_drive(prob, f, ref.step, cm)
            rd = pressure_drive(prob, {"p": ref.p, "v": ref.v, "psi1": ref.psi1, "psi2": ref.psi2}, ref.step, cm)
            drive = (rel_l2(gd, rd), np.abs(rd).max() / peak)
            _say(label, "pressure drive rel L2 %.2e (max %.1e of peak)" % drive)
    assert m_p <= MAX_ABS, (label, m_p)
    assert e_p <= REL_L2 or a_p < DECAYED, (label, e_p)
    if rtr is not None and rtr.size:
        assert e_t <= REL_L2 and m_t <= MAX_ABS, (label, e_t, m_t)
    for name, d, a, e in fields:
        assert d <= MAX_ABS, (label, name, d)
        if a_p >= LIVE:
            assert e <= REL_L2, (label, name, e)
    if check_all and a_p < LIVE:
        assert drive[0] <= REL_L2 or drive[1] < DECAYED, (label, "pressure drive", drive)


def _state(prob, seed):
    p, v, psi1, psi2 = W.random_state(prob.ndim, prob.n_relax, prob.shape, seed)
    # samples past the grid along their axis are held at zero
    for a in range(prob.ndim):
        sl = [slice(None)] * prob.ndim
        sl[prob.ndim - 1 - a] = -1
        v[a][tuple(sl)] = 0
        for nu in range(prob.n_relax):
            psi1[a, nu][tuple(sl)] = 0
    return {"p": p, "v": v, "psi1": psi1, "psi2": psi2}


# --------------------------------------------------------------- workloads ---

def test_plain_2d_full_workload():
    """384^2 interior + 4 lambda layer, water, L = 2 fitted to 0.5 dB/MHz^1.1/cm,
    12 ppw at 2 MHz, CFL 0.4, line source, 1000 steps, 64 receivers."""
    prob = W.plain_2d()
    _say("plain_2d 480x480 L=2 1000 steps")
    f, tr, step = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    assert step == prob.n_steps
    compare(f, tr, ref, rtr, "plain_2d", prob=prob)


def test_heterogeneous_2d_small_grid():
    """The layered abdominal-wall recipe (L = 4, labels, scatterers, array
    source) on a 320 x 224 grid, 1500 steps."""
    prob = W.abdominal_2d(nx=320, ny=224, n_steps=1500, n_scatter=2000)
    _say("abdominal_2d 320x224 L=4 1500 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    compare(f, tr, ref, rtr, "abdominal_2d_small", prob=prob)


def test_heterogeneous_2d_mid_run_all_fields():
    """The heterogeneous recipe on 320 x 224 after 300 steps, while the pulse
    is inside the grid: every field, v and the memory variables included."""
    prob = W.abdominal_2d(nx=320, ny=224, n_steps=300, n_scatter=2000)
    _say("abdominal_2d 320x224 L=4 300 steps (pulse in the grid)")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    compare(f, tr, ref, rtr, "abdominal_2d_small_300", prob=prob)


def test_heterogeneous_2d_stated_step_count_small_grid():
    """The abdominal recipe for its stated 12000 steps on a 320 x 224 grid
    (FP32 drift over the whole run; the full-size grid is compared with
    stored oracle results in test_gpu_long_runs)."""
    prob = W.abdominal_2d(nx=320, ny=224, n_steps=12000, n_scatter=2000)
    _say("abdominal_2d 320x224 L=4 12000 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    _say("final max|p| / peak trace %.3e" % (np.abs(ref.p).max() / np.abs(rtr).max()))
    compare(f, tr, ref, rtr, "abdominal_2d_small_12000", prob=prob)


def test_skull_3d_stated_step_count_small_cube():
    """The transcranial recipe for its stated 4000 steps on a 64^3 cube."""
    prob = W.skull_3d(n=64, nb=10, ntr=6, n_steps=4000)
    _say("skull_3d 64^3 L=2 4000 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    _say("final max|p| / peak trace %.3e" % (np.abs(ref.p).max() / np.abs(rtr).max()))
    compare(f, tr, ref, rtr, "skull_3d_64_4000", prob=prob)


def test_heterogeneous_2d_full_size_random_state():
    """Full 4096 x 2048 grid of the heterogeneous workload in the benchmark's
    launch configuration (graph chunks): a seeded random state advanced a few
    steps matches the oracle everywhere."""
    prob = W.abdominal_2d()
    st = _state(prob, 21)
    _say("abdominal_2d 4096x2048 L=4 random state, 6 steps (graph chunk 2)")
    f, tr, _ = gpu_run(prob, 6, state=st, graph_chunk=2)
    ref, rtr = oracle_run(prob, 6, state=st)
    compare(f, tr, ref, rtr, "abdominal_2d_full", prob=prob)


def test_heterogeneous_2d_eight_mechanisms():
    """The same recipe with L = 8 (fitted 8-mechanism tuples per layer): on a
    320 x 224 grid for 1200 steps, and on the full 4096 x 2048 grid from a
    seeded random state in the benchmark's launch configuration."""
    prob = W.abdominal_2d(nx=320, ny=224, n_steps=1200, n_scatter=2000, L=8)
    _say("abdominal_2d 320x224 L=8 1200 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    compare(f, tr, ref, rtr, "abdominal_2d_small_L8", prob=prob)
    prob = W.abdominal_2d(L=8)
    st = _state(prob, 22)
    _say("abdominal_2d 4096x2048 L=8 random state, 4 steps (graph chunk 2)")
    f, tr, _ = gpu_run(prob, 4, state=st, graph_chunk=2)
    ref, rtr = oracle_run(prob, 4, state=st)
    compare(f, tr, ref, rtr, "abdominal_2d_full_L8", prob=prob)


def test_medium_upload_in_chunks_with_a_partial_last_chunk():
    """A long 3D grid (24 x 24 x 9000) whose medium is uploaded in two chunks
    of planes (8192 and 808 planes of 64 x 32 padded points), the last one
    partial; c, rho, beta and the label differ at every point, so a plane
    placed at the wrong depth changes the fields.  A seeded random state over
    the whole grid advanced 2 steps matches the oracle everywhere."""
    prob = W.random_medium((24, 24, 9000), 1, 3, seed=77, nb=6, ntr=2)
    st = _state(prob, 23)
    _say("random_medium 24x24x9000 L=1 random state, 2 steps")
    f, tr, _ = gpu_run(prob, 2, state=st)
    ref, rtr = oracle_run(prob, 2, state=st)
    compare(f, tr, ref, rtr, "chunked_upload_3d", prob=prob)


# -------------------------------------------------------- random states ---

@pytest.mark.parametrize("shape,L,scheme,labels", [
    ((67, 45), 1, 1, 1), ((67, 45), 2, 0, 3), ((131, 70), 3, 1, 4), ((64, 64), 4, 1, 2),
    ((19, 23, 17), 2, 1, 2), ((33, 20, 21), 4, 0, 3), ((9, 7, 6), 1, 1, 1),
])
def test_random_state_parity(shape, L, scheme, labels):
    prob = W.random_medium(shape, L, labels, seed=sum(shape) + L, nb=min(6, min(shape) // 2 - 1), ntr=2)
    prob.relax_scheme = scheme
    rng = np.random.default_rng(3)
    n = prob.npts
    prob.src_idx = np.unique(rng.integers(0, n, 7)).astype(np.int64)
    prob.src_sig = rng.integers(0, 2, prob.src_idx.size).astype(np.int32)
    prob.src_w = rng.uniform(-1, 1, prob.src_idx.size).astype(np.float32)
    prob.signals = (1e4 * rng.standard_normal((2, 30))).astype(np.float32)
    prob.rcv_idx = rng.integers(0, n, 9).astype(np.int64)
    st = _state(prob, 5)
    _say("random state", shape, "L", L, "scheme", scheme, "labels", labels)
    f, tr, _ = gpu_run(prob, 25, state=st)
    ref, rtr = oracle_run(prob, 25, state=st)
    compare(f, tr, ref, rtr, "random %s" % (shape,), prob=prob)


def test_3d_point_source():
    prob = W.homogeneous((40, 36, 34), L=2, nb=(8, 8, 8), ntr=(6, 6, 6))
    prob.src_idx = prob.flat(np.array([20]), np.array([18]), np.array([17]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.signals = W.gaussian_pulse(300, prob.dt, 2e6, 3, 1e5)[None]
    prob.rcv_idx = prob.flat(np.array([5, 20, 33]), np.array([18, 30, 4]), np.array([17, 10, 28]))
    _say("3d 40x36x34 point source 300 steps")
    f, tr, _ = gpu_run(prob, 300)
    ref, rtr = oracle_run(prob, 300)
    compare(f, tr, ref, rtr, "3d point", prob=prob)


def test_skull_3d_small_cube():
    """The 3D transcranial recipe (shell, porosity noise, two labels, focused
    cap source, axis receivers) on a 96^3 cube with 12-cell layers."""
    prob = W.skull_3d(n=96, nb=12, ntr=9, n_steps=260)
    _say("skull_3d 96^3 L=2 260 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    compare(f, tr, ref, rtr, "skull_3d_96", prob=prob)


def test_skull_3d_small_cube_eight_mechanisms():
    """The transcranial recipe with the fitted 8-mechanism tuples on a 64^3
    cube with 10-cell layers."""
    prob = W.skull_3d(n=64, nb=10, ntr=6, n_steps=160, L=8)
    _say("skull_3d 64^3 L=8 160 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    compare(f, tr, ref, rtr, "skull_3d_64_L8", prob=prob)


def test_skull_3d_full_size_window():
    """The 1024^3 grid of the transcranial workload in the benchmark's launch
    configuration (plane-prefetch sweeps over 64 x 8 columns, 64 planes per
    block, graph-captured steps), checked where the oracle can follow it: a
    96^3 window at the centre holds a heterogeneous two-tissue medium (c
    1540-3080, the workload's two relaxation tuples, layers 48 cells thick as
    in the workload), the rest is the brain-like background, and a seeded
    random state fills a 16^3 block in the middle of the window.  One step
    moves information at most 8 cells along an axis, so after 3 steps every
    nonzero sample lies within 28 cells of the block, inside the window's
    interior.  The same window as its own 96^3 grid (same h, dt, stencil r and
    layer constants; 6-cell layers outside that reach) run by the oracle must
    give the same fields over the whole window."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    N, n, blk, steps = 1024, 96, 16, 3
    h = W.grid_spacing(1540.0, 1e6, 12)
    c_max = 3080.0
    dt = 0.4 * h / c_max
    rows = np.asarray([W.TABLE2_ROW, W.tissue_row(8.0, 1.0, 2, 1e6)], np.float64)
    rng = np.random.default_rng(1024)
    wc = rng.uniform(1540.0, c_max, (n, n, n)).astype(np.float32)
    wr = (1040.0 + (wc - 1540.0) * (860.0 / 1540.0)).astype(np.float32)
    wb = rng.uniform(3.5, 5.5, (n, n, n)).astype(np.float32)
    wl = (wc > 2300.0).astype(np.uint8)

    def problem(size, nb, ntr):
        grid = (size,) * 3
        return W.Problem(shape=grid, h=h, dt=dt, n_relax=2, c=np.full(grid, 1540.0, np.float32),
                         rho=np.full(grid, 1040.0, np.float32), beta=np.full(grid, 4.0, np.float32),
                         relax_table=rows, label=np.zeros(grid, np.uint8), bound_cells=(nb,) * 3,
                         trans_cells=(ntr,) * 3, pml_cp=c_max, fd_r=c_max * dt / h, n_steps=steps)

    small = problem(n, 6, 4)
    small.c[...], small.rho[...], small.beta[...], small.label[...] = wc, wr, wb, wl
    st = {"p": np.zeros((n, n, n), np.float32), "v": np.zeros((3, n, n, n), np.float32),
          "psi1": np.zeros((3, 2, n, n, n), np.float32), "psi2": np.zeros((3, 2, n, n, n), np.float32)}
    b0 = (n - blk) // 2
    inner = (slice(b0, b0 + blk),) * 3
    for name, arr in zip(("p", "v", "psi1", "psi2"), W.random_state(3, 2, (blk,) * 3, 77)):
        st[name][(Ellipsis,) + inner] = arr

    big = problem(N, 48, 36)
    o = (N - n) // 2
    win = (slice(o, o + n),) * 3
    big.c[win], big.rho[win], big.beta[win], big.label[win] = wc, wr, wb, wl
    _say("skull_3d-like 1024^3, 96^3 window, random 16^3 block, %d steps (graph chunk 2)" % steps)
    dom = fw2.from_problem(big, device="cuda:0", cap_steps=steps)
    dom.set_graph_chunk(2)
    buf = torch.zeros(dom.field_numel(), dtype=torch.float32, device="cuda:0")
    views = dom.field_views(buf)
    for name, arr in st.items():
        views[name][(Ellipsis,) + win] = torch.from_numpy(arr).to("cuda:0")
    dom.write_fields_device(buf)
    del buf, views
    dom.step(steps)
    torch.cuda.synchronize()
    out = dom.read_fields_device()
    views = dom.field_views(out)
    f = {name: views[name][(Ellipsis,) + win].cpu().numpy() for name in st}
    for name in st:                      # every sample outside the window is still exactly zero
        views[name][(Ellipsis,) + win] = 0.0
    outside = float(out.abs().max().item())
    del out, views
    dom.destroy_domain()
    torch.cuda.empty_cache()
    assert outside == 0.0, outside
    ref, _ = oracle_run(small, steps, state=st)
    # in the oracle nothing reached the window's 6-cell layers (an 8-cell margin is zero)
    for name in st:
        a = np.abs(getattr(ref, name))
        for ax in range(3):
            lo = [slice(None)] * a.ndim
            hi = [slice(None)] * a.ndim
            lo[a.ndim - 3 + ax] = slice(0, 8)
            hi[a.ndim - 3 + ax] = slice(n - 8, n)
            assert a[tuple(lo)].max() == 0.0 and a[tuple(hi)].max() == 0.0, (name, ax)
    compare(f, None, ref, None, "skull_3d_1024_window", prob=small)


def test_largest_2d_grid_far_corner_window():
    """The largest 2D grid the library accepts, 32697 x 32759 ((nx + 72)(ny + 8)
    = 2^30 - 1; padded rows of 32768 floats, so the sweeps' 32-bit byte offsets
    reach 4.29e9 of the 2^32 they can hold), in the default launch
    configuration with graph-captured steps, checked where the oracle can
    follow it: a 128^2 window at the far corner (the highest offsets, and the
    far boundary layers) holds a heterogeneous two-tissue medium, and a seeded
    random state fills a 16^2 block 16 cells from both far edges, inside the
    far layers.  After 3 steps the pressure reaches the far edges, and every
    nonzero sample lies within 28 cells of the block.  The same
    window as its own 128^2 grid (same h, dt, stencil r, layer constants and
    48-cell layers, so its far layers are the big grid's) run by the oracle
    must give the same fields over the whole window."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    nx, ny, n, blk, steps = 32697, 32759, 128, 16, 3
    h = W.grid_spacing(1540.0, 1e6, 12)
    c_max = 3080.0
    dt = 0.4 * h / c_max
    rows = np.asarray([W.TABLE2_ROW, W.tissue_row(8.0, 1.0, 2, 1e6)], np.float64)
    rng = np.random.default_rng(32697)
    wc = rng.uniform(1540.0, c_max, (n, n)).astype(np.float32)
    wr = (1040.0 + (wc - 1540.0) * (860.0 / 1540.0)).astype(np.float32)
    wb = rng.uniform(3.5, 5.5, (n, n)).astype(np.float32)
    wl = (wc > 2300.0).astype(np.uint8)

    def problem(gx, gy):
        arr = (gy, gx)
        return W.Problem(shape=(gx, gy), h=h, dt=dt, n_relax=2, c=np.full(arr, 1540.0, np.float32),
                         rho=np.full(arr, 1040.0, np.float32), beta=np.full(arr, 4.0, np.float32),
                         relax_table=rows, label=np.zeros(arr, np.uint8), bound_cells=(48, 48),
                         trans_cells=(36, 36), pml_cp=c_max, fd_r=c_max * dt / h, n_steps=steps)

    small = problem(n, n)
    small.c[...], small.rho[...], small.beta[...], small.label[...] = wc, wr, wb, wl
    st = {"p": np.zeros((n, n), np.float32), "v": np.zeros((2, n, n), np.float32),
          "psi1": np.zeros((2, 2, n, n), np.float32), "psi2": np.zeros((2, 2, n, n), np.float32)}
    b0 = n - 16 - blk
    inner = (slice(b0, b0 + blk),) * 2
    for name, arr in zip(("p", "v", "psi1", "psi2"), W.random_state(2, 2, (blk,) * 2, 78)):
        st[name][(Ellipsis,) + inner] = arr

    big = problem(nx, ny)
    win = (slice(ny - n, ny), slice(nx - n, nx))
    big.c[win], big.rho[win], big.beta[win], big.label[win] = wc, wr, wb, wl
    _say("largest 2D grid %dx%d, far-corner %d^2 window, random %d^2 block, %d steps (graph chunk 2)"
         % (nx, ny, n, blk, steps))
    dom = fw2.from_problem(big, device="cuda:0", cap_steps=steps)
    del big
    dom.set_graph_chunk(2)
    buf = torch.zeros(dom.field_numel(), dtype=torch.float32, device="cuda:0")
    views = dom.field_views(buf)
    for name, arr in st.items():
        views[name][(Ellipsis,) + win] = torch.from_numpy(arr).to("cuda:0")
    dom.write_fields_device(buf)
    del buf, views
    dom.step(steps)
    torch.cuda.synchronize()
    out = dom.read_fields_device()
    views = dom.field_views(out)
    f = {name: views[name][(Ellipsis,) + win].cpu().numpy() for name in st}
    for name in st:                      # every sample outside the window is still exactly zero
        views[name][(Ellipsis,) + win] = 0.0
    outside = float(out.abs().max().item())
    del out, views
    dom.destroy_domain()
    torch.cuda.empty_cache()
    assert outside == 0.0, outside
    ref, _ = oracle_run(small, steps, state=st)
    # nothing reached the window's near layers (an 8-cell margin is zero); the
    # far edges, shared with the big grid, are reached
    for name in st:
        a = np.abs(getattr(ref, name))
        for ax in range(2):
            lo = [slice(None)] * a.ndim
            lo[a.ndim - 2 + ax] = slice(0, 8)
            assert a[tuple(lo)].max() == 0.0, (name, ax)
    assert np.abs(ref.p[:, -1]).max() > 0 and np.abs(ref.p[-1, :]).max() > 0
    compare(f, None, ref, None, "largest_2d_far_corner", prob=small)


def test_largest_3d_cube_far_corner_window():
    """A 1400^3 cube, about the largest that fits the GPU's memory (a 215 GB
    workspace; every array holds 2.74e9 > 2^31 elements), in the default
    launch configuration: a 128^3 window at its far corner (the highest
    addresses, and the far boundary layers) holds a heterogeneous two-tissue
    medium, a point source 52 cells from the far faces plays a seeded random
    signal, and 27 receivers sit around it and inside the far layers.  After
    40 steps the wave has moved a few cells; what the stencil carries further
    is below FP32 range long before the window's near faces.  The same window
    as its own 128^3 grid (same h, dt, stencil r, layer constants, 48-cell
    layers) run by the oracle must give the same traces and final pressure
    in the window."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    torch.cuda.empty_cache()
    N, n, steps = 1400, 128, 40
    h = W.grid_spacing(1540.0, 1e6, 12)
    c_max = 3080.0
    dt = 0.4 * h / c_max
    rows = np.asarray([W.TABLE2_ROW, W.tissue_row(8.0, 1.0, 2, 1e6)], np.float64)
    rng = np.random.default_rng(1400)
    wc = rng.uniform(1540.0, c_max, (n, n, n)).astype(np.float32)
    wr = (1040.0 + (wc - 1540.0) * (860.0 / 1540.0)).astype(np.float32)
    wb = rng.uniform(3.5, 5.5, (n, n, n)).astype(np.float32)
    wl = (wc > 2300.0).astype(np.uint8)
    signal = rng.standard_normal((1, steps)).astype(np.float32) * 1e5
    s0 = n - 52                                       # source, window coordinates
    r = np.array([s0 - 6, s0, s0 + 6, s0 + 30, s0 + 45])
    rx, ry, rz = [g.ravel() for g in np.meshgrid(r[:3], r[:3], r[:3], indexing="ij")]
    rx = np.concatenate([rx[:-2], r[3:]])
    ry = np.concatenate([ry[:-2], r[3:]])
    rz = np.concatenate([rz[:-2], r[3:][::-1]])

    def problem(size, off):
        grid = (size,) * 3
        prob = W.Problem(shape=grid, h=h, dt=dt, n_relax=2, c=np.full(grid, 1540.0, np.float32),
                         rho=np.full(grid, 1040.0, np.float32), beta=np.full(grid, 4.0, np.float32),
                         relax_table=rows, label=np.zeros(grid, np.uint8), bound_cells=(48,) * 3,
                         trans_cells=(36,) * 3, pml_cp=c_max, fd_r=c_max * dt / h, n_steps=steps)
        prob.src_idx = prob.flat(np.array([off + s0]), np.array([off + s0]), np.array([off + s0]))
        prob.src_sig = np.zeros(1, np.int32)
        prob.src_w = np.ones(1, np.float32)
        prob.signals = signal
        prob.rcv_idx = prob.flat(off + rx, off + ry, off + rz)
        return prob

    small = problem(n, 0)
    small.c[...], small.rho[...], small.beta[...], small.label[...] = wc, wr, wb, wl
    big = problem(N, N - n)
    win = (slice(N - n, N),) * 3
    big.c[win], big.rho[win], big.beta[win], big.label[win] = wc, wr, wb, wl
    _say("largest 3D cube %d^3, far-corner %d^3 window, point source and %d receivers, %d steps"
         % (N, n, len(rx), steps))
    dom = fw2.from_problem(big, device="cuda:0", cap_steps=steps)
    del big
    dom.step(steps)
    torch.cuda.synchronize()
    tr = dom.trace[:steps].cpu().numpy()
    out = dom.read_fields_device(fw2.FIELD_P)
    pv = dom.field_views(out, fw2.FIELD_P)["p"]
    f = {"p": pv[win].cpu().numpy()}
    pv[win] = 0.0
    outside = float(out.abs().max().item())
    del out, pv
    dom.destroy_domain()
    torch.cuda.empty_cache()
    ref, rtr = oracle_run(small, steps)
    _say("largest 3D cube: max |p| outside the window %.2e of the window's peak" % (outside / np.abs(ref.p).max()))
    assert outside <= 1e-20 * np.abs(ref.p).max()
    compare(f, tr, ref, rtr, "largest_3d_far_corner", check_all=False, prob=small)


# ---------------------------------------------------------- edge cases ---

def test_degenerate_grids():
    for shape in [(1, 1), (1, 7), (5, 1), (2, 3, 1), (1, 1, 1)]:
        prob = W.homogeneous(shape, L=1, nb=(0,) * len(shape), ntr=(0,) * len(shape))
        st = _state(prob, 1)
        _say("degenerate", shape)
        f, tr, _ = gpu_run(prob, 4, state=st)
        ref, _ = oracle_run(prob, 4, state=st)
        compare(f, None, ref, None, "degenerate %s" % (shape,), prob=prob)


def test_split_steps_graph_and_direct_are_bitwise_equal():
    prob = W.plain_2d(interior=120, n_steps=200, n_rcv=8)
    _say("bitwise split/graph 216x216")
    a, ta, sa = gpu_run(prob, 200, graph_chunk=0)
    b, tb, sb = gpu_run(prob, 200, chunks=[0, 37, 100, 63], graph_chunk=16)
    c, tc, _ = gpu_run(prob, 200, graph_chunk=200)
    assert sa == sb == 200
    for k in a:
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    assert np.array_equal(ta, tb) and np.array_equal(ta, tc)


def test_moving_a_domain_between_streams_is_bitwise():
    """fw2_set_stream: steps split over two streams (the domain moved between
    them, graph chunks included) end bitwise where one stream ends."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.plain_2d(interior=120, n_steps=200, n_rcv=8)
    _say("stream move 216x216")
    a, ta, _ = gpu_run(prob, 200)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dom = fw2.from_problem(prob, device="cuda:0", stream=s1, cap_steps=200)
    dom.step(70)
    dom.set_stream(s2)
    dom.step(90)
    dom.set_stream(s1)
    dom.step(40)
    s1.synchronize()
    assert dom.current_step() == 200
    f = dom.read_fields(fw2.FIELD_ALL)
    tr = dom.trace.cpu().numpy()
    dom.destroy_domain()
    for k in a:
        assert np.array_equal(a[k], f[k]), k
    assert np.array_equal(ta, tr)


def test_checkpoint_resume_is_bitwise():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.abdominal_2d(nx=256, ny=160, n_steps=300, n_scatter=500)
    _say("checkpoint/resume 256x160")
    full, tf, _ = gpu_run(prob, 300)
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=300)
    dom.step(140)
    ck = dom.read_fields(fw2.FIELD_ALL)
    step = dom.current_step()
    dom.destroy_domain()
    dom2 = fw2.from_problem(prob, device="cuda:0", cap_steps=300)
    dom2.write_fields(ck)
    dom2.set_current_step(step)
    dom2.step(160)
    torch.cuda.synchronize()
    res = dom2.read_fields(fw2.FIELD_ALL)
    t2 = dom2.trace.cpu().numpy()
    dom2.destroy_domain()
    for k in full:
        assert np.array_equal(full[k], res[k]), k
    assert np.array_equal(tf[140:], t2[140:])


def test_zero_steps_and_write_read_roundtrip():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.random_medium((37, 29, 11), 3, 2, seed=4, nb=3, ntr=2)
    st = _state(prob, 8)
    _say("roundtrip 37x29x11")
    dom = fw2.from_problem(prob, device="cuda:0")
    dom.write_fields(st)
    dom.step(0)
    back = dom.read_fields(fw2.FIELD_ALL)
    dev = dom.read_fields_device(fw2.FIELD_P | fw2.FIELD_PSI2).cpu().numpy()
    dom.destroy_domain()
    for k in st:
        assert np.array_equal(back[k], st[k]), k
    assert np.array_equal(dev, np.concatenate([st["p"].ravel(), st["psi2"].ravel()]))


def test_invalid_calls_and_watchdog():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.plain_2d(interior=64, n_steps=10, n_rcv=4)
    _say("invalid calls 160x160")
    dom = fw2.from_problem(prob, device="cuda:0")
    with pytest.raises(fw2.Fw2Error):
        dom.add_source([5, 5], [0, 0], [1, 1], np.ones((1, 3)))          # duplicate index
    with pytest.raises(fw2.Fw2Error):
        dom.add_source([prob.npts], [0], [1], np.ones((1, 3)))          # out of range
    with pytest.raises(fw2.Fw2Error):
        dom.add_receivers([-1], 5)
    with pytest.raises(fw2.Fw2Error):
        dom.step(-1)
    dom.step(10)
    dom.check_finite(1e12)
    f = dom.read_fields(fw2.FIELD_P)
    f["p"][3, 4] = np.nan
    dom.write_fields(f)
    with pytest.raises(fw2.Fw2Error) as e:
        dom.check_finite(1e12)
    assert e.value.status == 5
    dom.destroy_domain()
    # a time step above the stability bound is refused at creation
    bad = W.plain_2d(interior=64, n_steps=10)
    bad.dt *= 1.8
    with pytest.raises(fw2.Fw2Error):
        fw2.from_problem(bad, device="cuda:0")


def test_kernel_timing_counts_launches():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.plain_2d(interior=64, n_steps=50, n_rcv=4)
    _say("kernel timing 160x160")
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=600)
    dom.enable_kernel_timing(True)
    dom.step(300)
    ms, cnt = dom.get_kernel_timing()
    assert cnt == [300, 300] and ms[0] > 0 and ms[1] > 0
    dom.enable_kernel_timing(False)
    dom.destroy_domain()


# ------------------------------------------------- kernel variants / tiles ---

@pytest.mark.parametrize("config", ["0,32,16", "1,32,16", "1,64,5", "1,32,1", "1,16,7", "2,32,16", "2,64,5", "2,16,1"])
@pytest.mark.parametrize("shape,L,scheme", [((37, 21, 19), 2, 1), ((70, 33, 24), 3, 0), ((16, 16, 40), 1, 1)])
def test_3d_kernel_variants_match_oracle(monkeypatch, config, shape, L, scheme):
    """3D plane-sweep tiles (32x16 and 64x8 columns, ragged in every axis,
    one-plane tiles), with and without the plane prefetch (variant 2), and
    the generic kernel give oracle results."""
    monkeypatch.setenv("FW2_KERNEL_CONFIG", config)
    prob = W.random_medium(shape, L, 3, seed=9, nb=5, ntr=3)
    prob.relax_scheme = scheme
    st = _state(prob, 17)
    _say("3d variant", config, shape, "L", L, "scheme", scheme)
    f, tr, _ = gpu_run(prob, 8, state=st)
    ref, rtr = oracle_run(prob, 8, state=st)
    compare(f, tr, ref, rtr, "3d variant %s %s" % (config, shape), prob=prob)


@pytest.mark.parametrize("config", ["0,64,16", "1,64,16", "1,128,7", "1,256,33", "1,64,1", "2,64,8", "2,256,5"])
@pytest.mark.parametrize("shape,L,scheme", [((70, 45), 2, 1), ((257, 131), 4, 1), ((131, 90), 3, 0)])
def test_kernel_variants_match_oracle(monkeypatch, config, shape, L, scheme):
    """Every kernel variant and tile shape (including tiles that overhang
    the grid and one-row tiles) gives oracle results."""
    monkeypatch.setenv("FW2_KERNEL_CONFIG", config)
    prob = W.random_medium(shape, L, 3, seed=7, nb=8, ntr=5)
    prob.relax_scheme = scheme
    st = _state(prob, 13)
    _say("variant", config, shape, "L", L, "scheme", scheme)
    f, tr, _ = gpu_run(prob, 12, state=st)
    ref, rtr = oracle_run(prob, 12, state=st)
    compare(f, tr, ref, rtr, "variant %s %s" % (config, shape), prob=prob)


# ------------------------------------------------- more than four mechanisms ---

@pytest.mark.parametrize("config", [None, "0,64,16"])
@pytest.mark.parametrize("shape,L,scheme", [((70, 45), 5, 1), ((131, 40), 6, 0), ((64, 48), 8, 1),
                                            ((19, 17, 15), 6, 1), ((21, 18, 13), 8, 0)])
def test_many_mechanisms_match_oracle(monkeypatch, config, shape, L, scheme):
    """L = 5..8 (fitted tuples) in 2D and 3D, both memory schemes, default
    sweep kernels and the generic kernel."""
    if config:
        monkeypatch.setenv("FW2_KERNEL_CONFIG", config if len(shape) == 2 else "0,32,16")
    prob = W.random_medium(shape, L, 2, seed=L + len(shape), nb=5, ntr=3)
    prob.relax_scheme = scheme
    st = _state(prob, 29)
    _say("mechanisms", L, shape, "scheme", scheme, "config", config)
    f, tr, _ = gpu_run(prob, 10, state=st)
    ref, rtr = oracle_run(prob, 10, state=st)
    compare(f, tr, ref, rtr, "L=%d %s" % (L, shape), prob=prob)


def test_many_mechanisms_point_source_run():
    """A 2D pulse through a medium fitted with six mechanisms, 400 steps."""
    prob = W.random_medium((96, 80), 6, 2, seed=31, nb=10, ntr=6)
    prob.src_idx = prob.flat(np.array([48]), np.array([40]))
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.signals = W.gaussian_pulse(400, prob.dt, 3e6, 3, 1e5)[None]
    prob.rcv_idx = prob.flat(np.array([10, 80]), np.array([15, 60]))
    _say("six mechanisms, point source, 400 steps")
    f, tr, _ = gpu_run(prob, 400)
    ref, rtr = oracle_run(prob, 400)
    compare(f, tr, ref, rtr, "L=6 point source", prob=prob)
