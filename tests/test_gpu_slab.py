"""Slabs of a 3D grid split along z (one GPU's share of a decomposed grid).

The halo calls move exactly the planes the header states, and a grid split
into slabs and stepped with halo exchange after each phase gives bitwise the
fields and traces of the whole-grid run (the per-point arithmetic does not
depend on where a slab starts), which itself matches the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _say, _state, _torch, compare, oracle_run

pytestmark = pytest.mark.gpu


def _padded(buf, shape, k):
    """Array k of a state block, padded [nz+8][ny+8][pitch]: (x, y, z) at
    [z+4, y+4, x+4] (the library's layout: 4-cell halos, pitch a multiple of
    64)."""
    nx, ny, nz = shape
    pitch = ((nx + 8 + 63) // 64) * 64
    stride = pitch * (ny + 8) * (nz + 8)
    return buf[k * stride:(k + 1) * stride].reshape(nz + 8, ny + 8, pitch)


def test_halo_pack_and_unpack_move_the_stated_planes():
    torch = _torch()
    from paper_2106_11476_amd import fw2, slab
    prob = W.random_medium((40, 36, 24), 2, 3, seed=21, nb=4, ntr=3)
    lo_p, hi_p = slab.split_problem(prob, [0, 12, 24])[0]
    _say("halo pack/unpack 40x36x24 split at 12")
    A = fw2.Domain(lo_p, device="cuda:0")
    B = fw2.Domain(hi_p, device="cuda:0")
    sa, sb = _state(lo_p, 1), _state(hi_p, 2)
    A.write_fields(sa)
    B.write_fields(sb)
    nx, ny, nz = lo_p.shape
    assert A.halo_numel(fw2.HALO_P) == 4 * nx * ny
    assert A.halo_numel(fw2.HALO_V) == 6 * nx * ny
    assert A.halo_numel(fw2.HALO_MEDIUM) == 2 * nx * ny
    fa, fb = A.read_fields(), B.read_fields()
    for kind in (fw2.HALO_P, fw2.HALO_V):
        up = torch.empty(A.halo_numel(kind), dtype=torch.float32, device="cuda:0")
        down = torch.empty_like(up)
        A.halo_pack(kind, fw2.HIGH, up)
        B.halo_unpack(kind, fw2.LOW, up)
        B.halo_pack(kind, fw2.LOW, down)
        A.halo_unpack(kind, fw2.HIGH, down)
        torch.cuda.synchronize()
        u = up.cpu().numpy().reshape(-1, ny, nx)
        d = down.cpu().numpy().reshape(-1, ny, nx)
        if kind == fw2.HALO_P:
            assert np.array_equal(u, fa["p"][-4:]) and np.array_equal(d, fb["p"][:4])
        else:
            assert np.array_equal(u[:4], fa["v"][2][-4:]) and np.array_equal(d[:4], fb["v"][2][:4])
            assert np.array_equal(u[4], fa["v"][0][-1]) and np.array_equal(u[5], fa["v"][1][-1])
            assert np.array_equal(d[4], fb["v"][0][0]) and np.array_equal(d[5], fb["v"][1][0])
    sta, stb = A.new_state_buffer(), B.new_state_buffer()
    A.save_state(sta)
    B.save_state(stb)
    torch.cuda.synchronize()
    sta, stb = sta.cpu().numpy(), stb.cpu().numpy()
    inner = (slice(4, 4 + ny), slice(4, 4 + nx))
    # B's low p halo holds A's top four planes, its high halo stays zero
    pb = _padded(stb, hi_p.shape, 0)
    assert np.array_equal(pb[0:4][(slice(None),) + inner], fa["p"][-4:])
    assert not pb[nz + 4:].any()
    pa = _padded(sta, lo_p.shape, 0)
    assert np.array_equal(pa[nz + 4:][(slice(None),) + inner], fb["p"][:4])
    assert not pa[0:4].any()
    # v: four planes of v_z, one of v_x and v_y, nothing else in the halos
    vzb, vxb, vyb = _padded(stb, hi_p.shape, 3), _padded(stb, hi_p.shape, 1), _padded(stb, hi_p.shape, 2)
    assert np.array_equal(vzb[0:4][(slice(None),) + inner], fa["v"][2][-4:])
    assert np.array_equal(vxb[3][inner], fa["v"][0][-1]) and not vxb[0:3].any()
    assert np.array_equal(vyb[3][inner], fa["v"][1][-1]) and not vyb[0:3].any()
    for arr in (pb, vzb, vxb, vyb):                   # halo rows and columns of every plane stay zero
        assert not arr[:, :4].any() and not arr[:, 4 + ny:].any() and not arr[:, :, :4].any()
    # the memory variables are never exchanged
    for k in range(4, 4 + 2 * 3 * 2):
        assert not _padded(stb, hi_p.shape, k)[:4].any()
    A.destroy_domain()
    B.destroy_domain()


def test_halo_and_phase_errors():
    _torch()
    from paper_2106_11476_amd import fw2, slab
    prob = W.random_medium((24, 20, 16), 2, 2, seed=3, nb=4, ntr=3)
    whole = fw2.Domain(prob, device="cuda:0")
    with pytest.raises(fw2.Fw2Error) as e:
        whole.halo_numel(fw2.HALO_P)
    assert e.value.status == 6
    s = fw2.Domain(slab.split_problem(prob, [0, 8, 16])[0][0], device="cuda:0")
    with pytest.raises(fw2.Fw2Error) as e:
        s.step_phase(fw2.PHASE_VELOCITY)
    assert e.value.status == 4
    s.step_phase(fw2.PHASE_PRESSURE)
    with pytest.raises(fw2.Fw2Error) as e:
        s.step(1)
    assert e.value.status == 4
    with pytest.raises(fw2.Fw2Error) as e:
        s.step_phase(fw2.PHASE_PRESSURE)
    assert e.value.status == 4
    s.step_phase(fw2.PHASE_VELOCITY)
    assert s.current_step() == 1
    with pytest.raises(fw2.Fw2Error) as e:
        s.halo_numel(7)
    assert e.value.status == 1
    whole.destroy_domain()
    s.destroy_domain()


CASES = [
    # (label, problem factory, z bounds, steps, kernel config or None)
    ("skull 96^3, three uneven slabs", lambda: W.skull_3d(n=96, nb=12, ntr=9, n_steps=150),
     [0, 29, 60, 96], 150, None),
    ("skull 96^3, plane sweeps without prefetch", lambda: W.skull_3d(n=96, nb=12, ntr=9, n_steps=90),
     [0, 40, 96], 90, "1,32,16"),
    ("skull 96^3, one thread per point", lambda: W.skull_3d(n=96, nb=12, ntr=9, n_steps=90),
     [0, 50, 96], 90, "0,64,8"),
    ("skull 64^3, eight mechanisms", lambda: W.skull_3d(n=64, nb=10, ntr=6, n_steps=100, L=8),
     [0, 20, 44, 64], 100, None),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_slab_run_equals_the_whole_grid_run_and_the_oracle(case, monkeypatch):
    torch = _torch()
    from paper_2106_11476_amd import fw2, slab
    label, make, bounds, steps, config = case
    if config:
        monkeypatch.setenv("FW2_KERNEL_CONFIG", config)
    prob = make()
    _say(label, "bounds", bounds, "steps", steps, "config", config)
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=steps)
    dom.step(steps)
    torch.cuda.synchronize()
    f = dom.read_fields(fw2.FIELD_ALL)
    tr = dom.trace.cpu().numpy()
    dom.destroy_domain()
    ss = slab.SlabSet(prob, bounds, device="cuda:0", cap_steps=steps)
    ss.step(steps)
    torch.cuda.synchronize()
    g = ss.read_fields(fw2.FIELD_ALL)
    tg = ss.traces()
    assert all(d.current_step() == steps for d in ss.domains)
    ss.destroy()
    for name in ("p", "v", "psi1", "psi2"):
        assert np.array_equal(f[name], g[name]), (label, name, np.abs(f[name] - g[name]).max())
    assert np.array_equal(tr, tg), label
    assert np.abs(f["p"]).max() > 0
    if config is None:
        ref, rtr = oracle_run(prob, steps)
        compare(g, tg, ref, rtr, label, prob=prob)


@pytest.mark.parametrize("shape,L", [((70, 45), 3), ((26, 21, 19), 2)])
def test_zero_halos_stay_zero_after_stepping(shape, L):
    """Outside the grid every field is zero (the stencils read the halo cells
    instead of testing bounds): after steps from a random state with sources
    and receivers, every halo cell of p, v and the memory variables in the
    state block is still exactly zero, and so is the v sample past the last
    pressure sample along its axis."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.random_medium(shape, L, 3, seed=13, nb=5, ntr=3)
    nd = len(shape)
    mid = [s // 2 for s in shape]
    prob.src_idx = prob.flat(*[np.array([m]) for m in mid])
    prob.src_sig = np.zeros(1, np.int32)
    prob.src_w = np.ones(1, np.float32)
    prob.signals = W.gaussian_pulse(60, prob.dt, 3e6, 3, 1e5)[None]
    prob.rcv_idx = prob.flat(*[np.array([m + 1]) for m in mid])
    _say("zero halos after stepping", shape, "L", L)
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=40)
    dom.write_fields(_state(prob, 9))
    dom.step(40)
    buf = dom.new_state_buffer()
    dom.save_state(buf)
    torch.cuda.synchronize()
    f = dom.read_fields(fw2.FIELD_V)
    dom.destroy_domain()
    buf = buf.cpu().numpy()
    n3 = list(shape) + [1] * (3 - nd)
    nx, ny, nz = n3
    pitch = ((nx + 8 + 63) // 64) * 64
    planes = nz + 8 if nd == 3 else 1
    stride = pitch * (ny + 8) * planes
    n_arr = 1 + nd + 2 * nd * L
    assert buf.size == n_arr * stride
    for k in range(n_arr):
        a = buf[k * stride:(k + 1) * stride].reshape(planes, ny + 8, pitch)
        win = ((slice(4, 4 + nz) if nd == 3 else slice(0, 1)), slice(4, 4 + ny), slice(4, 4 + nx))
        assert a[win].any(), k
        halo = np.ones(a.shape, bool)
        halo[win] = False
        assert not a[halo].any(), ("halo cell written", k)
    for a in range(nd):                            # the v sample past the grid along its axis
        sl = [slice(None)] * nd
        sl[nd - 1 - a] = -1
        assert not f["v"][a][tuple(sl)].any(), a


def test_benchmark_cube_in_eight_real_slabs_is_bitwise_the_whole_grid_run():
    """The benchmark's 1024^3 transcranial cube split into eight 1024 x 1024 x
    128 slabs, one GPU's share each on eight GPUs, stepped with the halo
    exchange after each phase, gives bit for bit the whole grid's pressure
    and focal-axis traces after 200 steps, when the pulse is at a third of
    its peak."""
    torch = _torch()
    from paper_2106_11476_amd import fw2, slab
    steps = 200
    prob = W.skull_3d(n=1024, L=2)
    _say("skull_3d 1024^3: whole grid against eight 128-plane slabs, %d steps" % steps)
    torch.cuda.empty_cache()
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=steps)
    dom.step(steps)
    torch.cuda.synchronize()
    p_whole = dom.read_fields_device(fw2.FIELD_P)
    tr_whole = dom.trace.cpu().numpy()
    dom.destroy_domain()
    del dom
    torch.cuda.empty_cache()
    ss = slab.SlabSet(prob, list(range(0, 1025, 128)), device="cuda:0", cap_steps=steps)
    ss.step(steps)
    torch.cuda.synchronize()
    whole = p_whole.view(1024, 1024, 1024)
    for k, d in enumerate(ss.domains):
        part = d.read_fields_device(fw2.FIELD_P).view(128, 1024, 1024)
        assert torch.equal(part, whole[128 * k:128 * (k + 1)]), k
        del part
    tr_slab = ss.traces()
    ss.destroy()
    del p_whole, whole
    torch.cuda.empty_cache()
    assert np.array_equal(tr_slab, tr_whole)
    assert np.abs(tr_whole).max() > 0
