"""fw2_batch_create_noalloc, the batch that allocates nothing (its table is
the library's own file-scope device array): through the C ABI, two calls in
a row, the second with a smaller input, each give bitwise the fields and
traces of the same batch built on a caller workspace (fw2_batch_create); a
second no-allocation batch on the same GPU is refused while the first
exists; more than 64 domains are refused."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _run_batch(mix, noalloc, tile=(256, 4)):
    torch = _torch()
    from paper_2106_11476_amd import fw2
    stream = torch.cuda.Stream()
    doms = [fw2.from_problem(p, device="cuda:0", stream=stream, cap_steps=n) for p, n in mix]
    b = fw2.Batch(max_domains=len(mix), stream=stream, noalloc=noalloc)
    b.set_tile(*tile)
    b.set_domains(doms, [n for _, n in mix])
    left = max(n for _, n in mix)
    while left > 0:
        k = min(left, 77)
        b.step(k)
        left -= k
    stream.synchronize()
    out = []
    for (p, n), d in zip(mix, doms):
        assert d.current_step() == n
        out.append((d.read_fields(fw2.FIELD_ALL), d.trace.cpu().numpy()))
    b.set_domains([], [])
    b.destroy()
    for d in doms:
        d.destroy_domain()
    return out


def test_noalloc_batch_matches_the_workspace_batch_twice():
    _torch()
    rs = W.serving_requests(n=4, seed=23, sides=(192, 416), side_step=32, max_steps=400)
    first = [(p, n) for p, n, _ in rs]
    small = W.serving_requests(n=2, seed=29, sides=(96, 160), side_step=32, max_steps=250)
    second = [(p, n) for p, n, _ in small]
    assert sum(p.npts for p, _ in second) < sum(p.npts for p, _ in first)
    for label, mix in (("first call", first), ("second call, smaller input", second)):
        _say("no-alloc batch", label, [(p.shape, p.n_relax, n) for p, n in mix])
        ref = _run_batch(mix, noalloc=False)
        got = _run_batch(mix, noalloc=True)
        for (p, _), (f, tr), (g, tg) in zip(mix, ref, got):
            for key in f:
                assert np.array_equal(f[key], g[key]), (label, p.name, key)
            assert np.array_equal(tr, tg), (label, p.name)
            assert np.abs(tr).max() > 0


def test_noalloc_batch_is_one_per_gpu_and_bounded():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    _say("no-alloc batch: second holder refused, size limit")
    b = fw2.Batch(max_domains=4, noalloc=True)
    with pytest.raises(fw2.Fw2Error) as e:
        fw2.Batch(max_domains=2, noalloc=True)
    assert e.value.status == 4
    b.destroy()
    c = fw2.Batch(max_domains=64, noalloc=True)          # free again after destroy
    c.destroy()
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream()
    assert fw2.lib().fw2_batch_create_noalloc(65, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)) == 1
    assert b"64" in fw2.lib().fw2_last_error()
