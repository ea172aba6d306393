"""GPU tests of batched stepping and continuous-batching serving: every
request's result is the same alone and in the mix (bitwise: the batched
launch runs the single-domain per-tile code), admission respects the memory
budget, and the batched fields match the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import solver

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _solo(prob, n_steps):
    torch = _torch()
    from paper_2106_11476_amd import fw2
    dom = fw2.from_problem(prob, device="cuda:0", cap_steps=n_steps)
    dom.step(n_steps)
    torch.cuda.synchronize()
    f = dom.read_fields(fw2.FIELD_ALL)
    tr = dom.trace.cpu().numpy()
    dom.destroy_domain()
    return f, tr


def _mix():
    rs = W.serving_requests(n=5, seed=11, sides=(224, 480), side_step=32, max_steps=700)
    return [(p, n) for p, n, _ in rs]


@pytest.mark.parametrize("tile", [(256, 4), (64, 8), (64, 1)])
def test_batched_steps_equal_solo_runs_bitwise(tile):
    torch = _torch()
    from paper_2106_11476_amd import fw2
    mix = _mix()
    _say("batch of", [(p.shape, p.n_relax, n) for p, n in mix])
    solo = [_solo(p, n) for p, n in mix]
    stream = torch.cuda.Stream()
    doms = [fw2.from_problem(p, device="cuda:0", stream=stream, cap_steps=n) for p, n in mix]
    b = fw2.Batch(max_domains=8, stream=stream)
    b.set_tile(*tile)
    b.set_domains(doms, [n for _, n in mix])
    left = max(n for _, n in mix)
    while left > 0:                       # uneven chunks, some past each domain's end
        k = min(left, 97)
        b.step(k)
        left -= k
    stream.synchronize()
    for (p, n), d, (f, tr) in zip(mix, doms, solo):
        assert d.current_step() == n
        g = d.read_fields(fw2.FIELD_ALL)
        for key in f:
            assert np.array_equal(f[key], g[key]), (p.name, key)
        assert np.array_equal(tr, d.trace.cpu().numpy()), p.name
    b.set_domains([], [])
    b.destroy()
    for d in doms:
        d.destroy_domain()


def test_batched_fields_match_oracle():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    p, n = _mix()[1]
    n = 300
    _say("batch vs oracle", p.shape, p.n_relax)
    stream = torch.cuda.Stream()
    d = fw2.from_problem(p, device="cuda:0", stream=stream, cap_steps=n)
    b = fw2.Batch(max_domains=2, stream=stream)
    b.set_domains([d], [n])
    b.step(n)
    stream.synchronize()
    f = d.read_fields(fw2.FIELD_P)
    ref, rtr = solver.run(p, n)
    peak = max(np.abs(ref.p).max(), np.abs(rtr).max())
    assert np.linalg.norm(f["p"] - ref.p) / np.linalg.norm(ref.p) < 1e-4
    assert np.abs(f["p"] - ref.p).max() / peak < 1e-3
    tr = d.trace.cpu().numpy()
    assert np.linalg.norm(tr - rtr) / np.linalg.norm(rtr) < 1e-4
    b.set_domains([], [])
    b.destroy()
    d.destroy_domain()


def test_continuous_batching_results_are_mix_independent():
    """Requests arriving while others run are admitted at chunk boundaries
    (staggered starts, different step counts); each trace equals its solo
    trace, and the resident bytes never exceed the budget."""
    torch = _torch()
    from paper_2106_11476_amd import serve
    mix = _mix()
    _say("continuous batching", len(mix))
    solo = [_solo(p, n)[1] for p, n in mix]
    reqs = [serve.Request(rid=i, problem=p, n_steps=n, arrival=0.02 * i) for i, (p, n) in enumerate(mix)]
    budget = int(2.2 * max(serve.footprint_bytes(p, n) for p, n in mix))
    srv = serve.Server(budget_bytes=budget, max_active=4, chunk=48)
    st = srv.run(reqs)
    srv.close()
    assert st.completed == len(mix)
    assert st.peak_bytes <= budget
    assert st.peak_active >= 2                    # work really overlapped
    for r, tr in zip(reqs, solo):
        assert np.array_equal(r.trace, tr), r.rid
    s = st.summary()
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_autotuner_picks_a_candidate():
    _torch()
    from paper_2106_11476_amd import serve
    probs = [p for p, _ in _mix()[:3]]
    cands = ((256, 4), (64, 8))
    best, t = serve.autotune_tile(probs, candidates=cands, steps=16)
    assert best in cands and all(v > 0 for v in t.values())


def test_batch_refuses_more_than_four_mechanisms():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    prob = W.random_medium((40, 36), 5, 2, seed=3, nb=4, ntr=2)
    _say("batch refuses L = 5")
    dom = fw2.Domain(prob, device="cuda:0")
    batch = fw2.Batch(max_domains=2, device="cuda:0")
    with pytest.raises(fw2.Fw2Error, match="UNSUPPORTED"):
        batch.set_domains([dom], [10])
    torch.cuda.synchronize()
    batch.destroy()
    dom.destroy_domain()
