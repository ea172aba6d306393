"""Descriptor options of the C ABI on the GPU: the nonlinear form as
coefficients (Sec. 2.2, Eqs. state1 / state2), medium maps handed over in
device memory, and relaxation maps turned into labels."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _say, _state, _torch, compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

WESTERVELT = dict(nonlinear_form=1, nl_A=0.0, nl_B0=0.0, nl_B1=-2.0)


@pytest.mark.parametrize("shape,L", [((61, 47), 3), ((21, 18, 17), 2)])
def test_custom_nonlinear_form_matches_the_oracle(shape, L):
    """A = 0, B = -2 beta (plane-wave nonlinearity coefficient beta) on a
    random medium from a random state, with pressures large enough that the
    multipliers matter."""
    _torch()
    prob = W.random_medium(shape, L, 3, seed=31, nb=6, ntr=4)
    for k, v in WESTERVELT.items():
        setattr(prob, k, v)
    st = _state(prob, 5)
    st["p"] = st["p"] * 50.0                       # ~5 MPa: kappa0 B p of order 1e-3
    _say("nonlinear form A=0 B=-2beta", shape, "L", L)
    f, _, _ = gpu_run(prob, 24, state=st)
    ref, _ = oracle_run(prob, 24, state=st)
    compare(f, None, ref, None, "westervelt %s" % (shape,), prob=prob)
    # the coefficients change the result (the test is not vacuous)
    prob.nonlinear_form = 0
    f0, _, _ = gpu_run(prob, 24, state=st)
    assert np.abs(f0["p"] - f["p"]).max() > 1e-6 * np.abs(f["p"]).max()


@pytest.mark.parametrize("shape,L,nl", [((77, 53), 4, False), ((77, 53), 2, True), ((23, 19, 21), 2, False)])
def test_device_maps_give_bitwise_the_host_domain(shape, L, nl):
    """c, rho, beta and labels passed as device arrays are converted on the
    GPU with the host conversion's FP64 arithmetic: after stepping from the
    same state the fields are bitwise those of the host-map domain."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.random_medium(shape, L, 4, seed=41, nb=6, ntr=4)
    if nl:
        for k, v in WESTERVELT.items():
            setattr(prob, k, v)
    st = _state(prob, 7)
    _say("device maps", shape, "L", L, "custom nonlinear form", nl)
    out = []
    for dev in (False, True):
        d = fw2.Domain(prob, device="cuda:0", device_maps=dev)
        d.write_fields(st)
        d.step(20)
        torch.cuda.synchronize()
        out.append(d.read_fields(fw2.FIELD_ALL))
        d.destroy_domain()
    for name in out[0]:
        assert np.array_equal(out[0][name], out[1][name]), name


def test_invalid_device_maps_are_rejected():
    _torch()
    from paper_2106_11476_amd import fw2
    prob = W.random_medium((40, 30), 2, 2, seed=3, nb=4, ntr=3)
    prob.c = prob.c.copy()
    prob.c[7, 9] = -1.0
    with pytest.raises(fw2.Fw2Error) as e:
        fw2.Domain(prob, device="cuda:0", device_maps=True)
    assert e.value.status == 1
    prob = W.random_medium((40, 30), 2, 2, seed=3, nb=4, ntr=3)
    prob.label = prob.label.copy()
    prob.label[3, 3] = 5
    with pytest.raises(fw2.Fw2Error) as e:
        fw2.Domain(prob, device="cuda:0", device_maps=True)
    assert e.value.status == 1


def test_dense_relaxation_maps_label_into_the_same_domain():
    """Per-point relaxation maps (Sec. 3.2's 2 + 4L parameters at every point)
    labelled by fw2_label_relaxation_map give the same simulation as the
    generator's labels and table."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.random_medium((64, 48), 3, 5, seed=11, nb=6, ntr=4)
    table = np.asarray(prob.relax_table)
    dense = np.moveaxis(table[prob.label.astype(np.intp)], -1, 0)
    lab, tab = fw2.label_relaxation_map(dense, prob.n_relax)
    st = _state(prob, 3)
    _say("dense relaxation maps 64x48 L=3")
    f1, _, _ = gpu_run(prob, 15, state=st)
    prob.label, prob.relax_table = lab, tab
    f2, _, _ = gpu_run(prob, 15, state=st)
    torch.cuda.synchronize()
    for name in f1:
        assert np.array_equal(f1[name], f2[name]), name
