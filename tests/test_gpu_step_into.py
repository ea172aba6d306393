"""Out-of-place stepping (fw2_step_into), which the adjoint's checkpointed
recomputation uses: n steps through caller-owned state blocks give, block by
block, bitwise the states that stepping in place passes through, with the
same traces, for every kernel family, through a HIP graph and without one;
the domain's own fields are left as they were.  Every test prints its case
before touching the GPU."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _say, _state, _torch

pytestmark = pytest.mark.gpu

CASES = [
    ((257, 131), 4, 1, None),             # 2D row sweeps with prefetch (default)
    ((70, 45), 2, 0, "0,64,16"),           # generic one-thread-per-point kernels
    ((131, 90), 3, 1, "1,128,7"),          # row sweeps without prefetch
    ((70, 45), 6, 1, None),                # more than four mechanisms
    ((37, 21, 19), 2, 1, None),            # 3D plane sweeps (default variant)
    ((37, 21, 19), 3, 0, "0,32,16"),       # 3D generic kernels
    ((40, 33, 30), 2, 1, "1,32,16"),       # 3D plane sweeps without prefetch
    ((131, 90), 3, 1, "local"),            # per-point stencil weights, 2D
    ((37, 21, 19), 2, 0, "local"),         # per-point stencil weights, 3D
]


def _problem(shape, L, scheme, n_steps):
    prob = W.random_medium(shape, L, 3, seed=5 + L, nb=5, ntr=3)
    prob.relax_scheme = scheme
    prob.n_steps = n_steps
    mid = [s // 2 for s in shape]
    prob.src_idx = prob.flat(*[np.array([m, m]) if a == 0 else np.array([m, m + 1])
                               for a, m in enumerate(mid)])
    prob.src_sig = np.zeros(2, np.int32)
    prob.src_w = np.array([1.0, -0.5], np.float32)
    prob.signals = W.gaussian_pulse(n_steps, prob.dt, 3e6, 3, 2e5)[None]
    prob.rcv_idx = prob.flat(*[np.array([2, s // 3, s - 2]) for s in shape])
    return prob


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "direct"])
@pytest.mark.parametrize("shape,L,scheme,config", CASES)
def test_steps_into_blocks_are_the_in_place_states(monkeypatch, shape, L, scheme, config, graph):
    torch = _torch()
    from paper_2106_11476_amd import fw2
    if config and config != "local":
        monkeypatch.setenv("FW2_KERNEL_CONFIG", config)
    n0, n = 5, 9
    prob = _problem(shape, L, scheme, n0 + n)
    if config == "local":
        prob.stencil_mode = fw2.STENCIL_LOCAL
    st = _state(prob, 23)
    _say("step_into", shape, "L", L, "scheme", scheme, "config", config, "graph", graph)
    a = fw2.from_problem(prob, device="cuda:0", cap_steps=n0 + n)
    b = fw2.from_problem(prob, device="cuda:0", cap_steps=n0 + n)
    for d in (a, b):
        d.write_fields(st)
        d.step(n0)
    if not graph:
        a.set_graph_chunk(0)
    first = a.new_state_buffer()
    a.save_state(first)
    torch.cuda.synchronize()
    before = a.read_fields()
    blocks = a.new_state_buffer(n)
    a.step_into(n, first, blocks)
    ref = b.new_state_buffer(n)
    for i in range(n):
        b.step(1)
        b.save_state(ref[i])
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(blocks[i], ref[i]), ("block", i)
    assert a.current_step() == n0 + n
    assert torch.equal(a.trace, b.trace)
    after = a.read_fields()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    # the same blocks again: the captured graph is replayed
    a.set_current_step(n0)
    blocks.zero_()
    a.step_into(n, first, blocks)
    torch.cuda.synchronize()
    assert torch.equal(blocks, ref)
    a.destroy_domain()
    b.destroy_domain()


def test_step_into_checks_its_arguments():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = _problem((64, 48), 2, 1, 10)
    _say("step_into argument checks")
    d = fw2.from_problem(prob, device="cuda:0")
    blocks = d.new_state_buffer(4)
    with pytest.raises(fw2.Fw2Error):
        d.step_into(3, blocks[1], blocks)           # first inside the destination blocks
    with pytest.raises(fw2.Fw2Error):
        d.step_into(-1, blocks[0], blocks[1:])
    d.step_phase(fw2.PHASE_PRESSURE)
    with pytest.raises(fw2.Fw2Error):
        d.step_into(2, blocks[0], blocks[1:])       # half a step done
    d.step_phase(fw2.PHASE_VELOCITY)
    d.step_into(0, blocks[0], blocks[1:])
    torch.cuda.synchronize()
    assert d.current_step() == 1
    d.destroy_domain()
    from paper_2106_11476_amd import slab
    cube = W.skull_3d(n=32, nb=6, ntr=4, n_steps=4)
    part = slab.split_problem(cube, [0, 16, 32], only=[0])[0][0]
    s = fw2.Domain(part, device="cuda:0")
    sb = s.new_state_buffer(3)
    with pytest.raises(fw2.Fw2Error):
        s.step_into(2, sb[0], sb[1:])               # slabs exchange halos between phases
    s.destroy_domain()
