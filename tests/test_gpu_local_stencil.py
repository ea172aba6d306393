"""GPU parity of the per-point stencil weights (stencil mode 1) against the
FP64 oracle, through the C ABI, for every kernel family (2D sweeps with
their tiles, the generic kernels, the 3D plane sweeps), plus the heterogeneous
workload recipe and its full-size grid.  Same bar as the global-weight
parity tests.  Every test prints its case before touching the GPU."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _say, _state, _torch, compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


def _local(prob):
    prob.stencil_mode = 1
    return prob


@pytest.mark.parametrize("config", ["0,64,16", "1,256,4", "1,64,8", "1,128,7", "2,64,8"])
@pytest.mark.parametrize("shape,L,scheme", [((70, 45), 2, 1), ((257, 131), 4, 1), ((131, 90), 3, 0)])
def test_local_stencil_2d_matches_oracle(monkeypatch, config, shape, L, scheme):
    monkeypatch.setenv("FW2_KERNEL_CONFIG", config)
    prob = _local(W.random_medium(shape, L, 3, seed=7, nb=8, ntr=5))
    prob.relax_scheme = scheme
    st = _state(prob, 13)
    _say("local stencil 2D", config, shape, "L", L, "scheme", scheme)
    f, tr, _ = gpu_run(prob, 12, state=st)
    ref, rtr = oracle_run(prob, 12, state=st)
    compare(f, tr, ref, rtr, "local %s %s" % (config, shape), prob=prob)


@pytest.mark.parametrize("config", ["0,32,16", "1,32,16", "1,64,5", "1,16,7", "2,32,16"])
@pytest.mark.parametrize("shape,L,scheme", [((37, 21, 19), 2, 1), ((33, 20, 21), 4, 0)])
def test_local_stencil_3d_matches_oracle(monkeypatch, config, shape, L, scheme):
    monkeypatch.setenv("FW2_KERNEL_CONFIG", config)
    prob = _local(W.random_medium(shape, L, 3, seed=9, nb=5, ntr=3))
    prob.relax_scheme = scheme
    st = _state(prob, 17)
    _say("local stencil 3D", config, shape, "L", L, "scheme", scheme)
    f, tr, _ = gpu_run(prob, 8, state=st)
    ref, rtr = oracle_run(prob, 8, state=st)
    compare(f, tr, ref, rtr, "local 3d %s %s" % (config, shape), prob=prob)


def test_local_stencil_heterogeneous_recipe():
    """The layered abdominal-wall recipe on 320 x 224, 1500 steps, array
    source and receivers, per-point weights."""
    prob = _local(W.abdominal_2d(nx=320, ny=224, n_steps=1500, n_scatter=2000))
    _say("local stencil abdominal_2d 320x224 L=4 1500 steps")
    f, tr, _ = gpu_run(prob, prob.n_steps)
    ref, rtr = oracle_run(prob, prob.n_steps)
    compare(f, tr, ref, rtr, "local abdominal small", prob=prob)


def test_local_stencil_full_size_random_state():
    """Full 4096 x 2048 benchmark grid, per-point weights, in the graph-chunk
    launch configuration: a seeded random state advanced 4 steps."""
    prob = _local(W.abdominal_2d())
    st = _state(prob, 23)
    _say("local stencil abdominal_2d 4096x2048 random state, 4 steps")
    f, tr, _ = gpu_run(prob, 4, state=st, graph_chunk=2)
    ref, rtr = oracle_run(prob, 4, state=st)
    compare(f, tr, ref, rtr, "local abdominal full", prob=prob)


def test_local_stencil_is_refused_by_the_adjoint():
    """The discrete adjoint is derived for global weights (with per-point
    weights c would also enter through the stencil); the batched path takes
    per-point weights (tested with the batch)."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = _local(W.random_medium((40, 36), 2, 2, seed=3, nb=4, ntr=2))
    _say("local stencil refused by the adjoint")
    dom = fw2.Domain(prob, device="cuda:0")
    with pytest.raises(fw2.Fw2Error, match="UNSUPPORTED"):
        dom.adjoint_begin()
    torch.cuda.synchronize()
    dom.destroy_domain()
