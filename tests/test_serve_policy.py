"""CPU tests of the serving host logic: admission order, memory budget and
slot limits (no GPU)."""
from paper_2106_11476_amd.serve import Request, Stats, admit


def _q(specs):
    return [Request(rid=i, problem=None, n_steps=10, arrival=a, footprint=f) for i, (a, f) in enumerate(specs)]


def test_admits_arrived_requests_in_order_within_budget():
    q = _q([(0.0, 40), (0.1, 30), (0.2, 50), (5.0, 1)])
    got = admit(q, active_bytes=0, budget=100, free_slots=8, now=1.0)
    assert [r.rid for r in got] == [0, 1]          # third does not fit, fourth has not arrived


def test_blocked_head_is_not_overtaken():
    q = _q([(0.0, 90), (0.0, 5)])
    assert admit(q, active_bytes=20, budget=100, free_slots=8, now=0.5) == []


def test_slot_limit():
    q = _q([(0.0, 1)] * 5)
    assert len(admit(q, 0, 100, free_slots=3, now=0.0)) == 3


def test_nothing_before_arrival():
    q = _q([(2.0, 1)])
    assert admit(q, 0, 100, 4, now=1.0) == []


def test_stats_summary_percentiles():
    s = Stats(completed=4, makespan=2.0, latencies=[1.0, 2.0, 3.0, 4.0])
    d = s.summary()
    assert d["sims_per_s"] == 2.0 and d["p50_latency_s"] == 2.5 and 3.9 < d["p99_latency_s"] <= 4.0
