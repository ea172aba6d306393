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
    # arrivals 3 ms apart: each request alone takes 15-20 ms, so later ones
    # arrive while earlier ones are on the device
    reqs = [serve.Request(rid=i, problem=p, n_steps=n, arrival=0.003 * i) for i, (p, n) in enumerate(mix)]
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


def test_serving_steps_large_requests_alone_in_arrival_order():
    """With a size threshold inside the mix, the larger requests are stepped
    alone (single-domain kernels, one at a time in arrival order) while the
    smaller ones share the batched launch; every trace is still bitwise the
    solo trace, and the large requests finish in arrival order."""
    torch = _torch()
    from paper_2106_11476_amd import serve
    mix = _mix()
    sizes = sorted(p.npts for p, _ in mix)
    cut = sizes[len(sizes) // 2]
    _say("hybrid serving, solo from", cut, "points", [(p.npts, n) for p, n in mix])
    solo = [_solo(p, n)[1] for p, n in mix]
    reqs = [serve.Request(rid=i, problem=p, n_steps=n, arrival=0.002 * i) for i, (p, n) in enumerate(mix)]
    budget = int(4 * max(serve.footprint_bytes(p, n) for p, n in mix))
    srv = serve.Server(budget_bytes=budget, max_active=4, chunk=48, solo_points=cut, solo_chunk=16)
    seen = []
    st = srv.run(reqs, on_done=lambda r: seen.append(r.rid))
    srv.close()
    assert st.completed == len(mix) and st.peak_bytes <= budget
    assert seen == [r.rid for r in sorted(reqs, key=lambda r: r.done)]          # one call per completion
    for r, tr in zip(reqs, solo):
        assert np.array_equal(r.trace, tr), r.rid
    big = [r for r in reqs if r.problem.npts >= cut]
    assert len(big) >= 2
    assert [r.rid for r in sorted(big, key=lambda r: r.done)] == [r.rid for r in big]


def test_autotuner_picks_a_candidate():
    _torch()
    from paper_2106_11476_amd import serve
    probs = [p for p, _ in _mix()[:3]]
    cands = ((256, 4), (64, 8))
    best, t = serve.autotune_tile(probs, candidates=cands, steps=16)
    assert best in cands and all(v > 0 for v in t.values())


def _variant_mix():
    """Domains of every launch class: global and per-point stencil weights,
    1..4 and 5..8 mechanisms, both memory schemes, uneven sizes and steps."""
    out = []
    for k, (shape, L, mode, scheme, n) in enumerate([((200, 136), 3, 1, 1, 260), ((264, 96), 2, 0, 1, 300),
                                                     ((150, 170), 6, 0, 1, 240), ((97, 131), 8, 1, 0, 200),
                                                     ((320, 64), 4, 1, 0, 280)]):
        p = W.random_medium(shape, L, 2, seed=40 + k, nb=8, ntr=6)
        p.stencil_mode, p.relax_scheme = mode, scheme
        rng = np.random.default_rng(k)
        p.src_idx = np.unique(rng.integers(0, p.npts, 5)).astype(np.int64)
        p.src_sig = np.zeros(p.src_idx.size, np.int32)
        p.src_w = np.ones(p.src_idx.size, np.float32)
        p.signals = W.gaussian_pulse(120, p.dt, 3e6, 3, 1e5)[None]
        p.rcv_idx = rng.integers(0, p.npts, 7).astype(np.int64)
        p.name = "variant_%d_L%d_mode%d" % (k, L, mode)
        out.append((p, n))
    return out


@pytest.mark.parametrize("tile", [(256, 4), (256, 8), (64, 4)])
def test_batch_of_every_launch_class_equals_solo_runs_bitwise(tile):
    """Per-point stencil weights and 5..8 mechanisms in the batch (launches of
    their own), mixed with the common class: every domain ends bitwise where
    it ends alone.  64-column tiles take the domains with at most four
    mechanisms and refuse the others."""
    torch = _torch()
    from paper_2106_11476_amd import fw2
    mix = _variant_mix()
    if tile[0] == 64:
        many = [(p, n) for p, n in mix if p.n_relax > 4]
        mix = [(p, n) for p, n in mix if p.n_relax <= 4]
    _say("batch of every class, tile", tile, [(p.shape, p.n_relax, p.stencil_mode, n) for p, n in mix])
    solo = [_solo(p, n) for p, n in mix]
    stream = torch.cuda.Stream()
    doms = [fw2.from_problem(p, device="cuda:0", stream=stream, cap_steps=n) for p, n in mix]
    b = fw2.Batch(max_domains=8, stream=stream)
    b.set_tile(*tile)
    if tile[0] == 64:
        big = fw2.from_problem(many[0][0], device="cuda:0", stream=stream, cap_steps=many[0][1])
        with pytest.raises(fw2.Fw2Error, match="UNSUPPORTED"):
            b.set_domains(doms + [big], [n for _, n in mix] + [many[0][1]])
        big.destroy_domain()
    b.set_domains(doms, [n for _, n in mix])
    left = max(n for _, n in mix)
    while left > 0:
        k = min(left, 71)
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


def test_batched_per_point_weights_match_oracle():
    torch = _torch()
    from paper_2106_11476_amd import fw2
    p, _ = _variant_mix()[0]
    n = 200
    _say("batch with per-point weights vs oracle", p.shape, p.n_relax)
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


def test_autotuner_keeps_256_columns_for_many_mechanisms():
    _torch()
    from paper_2106_11476_amd import serve
    probs = [p for p, _ in _variant_mix()[1:3]]
    best, t = serve.autotune_tile(probs, candidates=((256, 4), (64, 8)), steps=8)
    assert best == (256, 4) and set(t) == {(256, 4)}


def test_served_workload_request_matches_the_oracle():
    """Requests of the served workload's recipe at their own size and step
    count (1024^2, 2560 steps, L and f0 as the stream draws them), served
    together in the batched launch (no solo threshold): the first one's
    traces against the oracle at the parity bar (relative L2 <= 1e-4,
    max-abs <= 1e-3 of the peak)."""
    _torch()
    from paper_2106_11476_amd import serve
    from test_gpu_parity import oracle_run, rel_l2
    raw = W.serving_requests(n=3, seed=4, sides=(1024, 1024))
    _say("served workload, three 1024^2 requests batched", [(p.n_relax, n) for p, n, _ in raw])
    reqs = [serve.Request(rid=i, problem=p, n_steps=n, arrival=0.0) for i, (p, n, _) in enumerate(raw)]
    budget = int(4 * max(serve.footprint_bytes(p, n) for p, n, _ in raw))
    srv = serve.Server(budget_bytes=budget, max_active=4, chunk=64, solo_points=1 << 40)
    st = srv.run(reqs)
    srv.close()
    assert st.completed == 3 and st.peak_active == 3
    p0, n0, _ = raw[0]
    _, rtr = oracle_run(p0, n0)
    peak = np.abs(rtr).max()
    e = rel_l2(reqs[0].trace[:n0], rtr)
    m = np.abs(reqs[0].trace[:n0] - rtr).max() / peak
    _say("request 0 (L %d, %d steps): trace rel L2 %.2e, max/peak %.2e" % (p0.n_relax, n0, e, m))
    assert e <= 1e-4 and m <= 1e-3
