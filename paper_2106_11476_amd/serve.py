"""Continuous-batching request loop over libfw2's batched stepping.

Requests (2D simulations of any size, mechanism count and step count) arrive
over time.  The server keeps every admitted simulation resident in HBM and
advances all of them together with fw2_batch_step, one launch per phase over
the tiles of every active domain.  At each chunk boundary finished requests
hand back their receiver traces and free their memory, and queued requests
are admitted in arrival order while the device-memory budget and the slot
count allow.  Work of different requests therefore overlaps on the device,
and a request's results do not depend on what it was batched with.

The plain baseline runs the same requests one at a time in arrival order
with the single-domain path of the same library.
"""
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import fw2


@dataclass
class Request:
    rid: int
    problem: object              # workloads.Problem-like inputs (2D)
    n_steps: int
    arrival: float = 0.0         # seconds after the stream starts
    admitted: Optional[float] = None
    done: Optional[float] = None
    trace: Optional[np.ndarray] = None
    footprint: int = 0


def footprint_bytes(prob, n_steps):
    """Device bytes a request holds while resident: workspace, trace buffer,
    source tables."""
    ws = fw2.workspace_bytes(prob)
    n_rcv = max(len(prob.rcv_idx), 1)
    src = len(prob.src_idx) * (8 + 4 + 4) + np.asarray(prob.signals).size * 4
    return int(ws + n_steps * n_rcv * 4 + src + 8 * n_rcv)


def admit(queue, active_bytes, budget, free_slots, now):
    """Arrival-order admission: take queued requests that have arrived while
    the memory budget and the free slots allow; a request that does not fit
    blocks the ones behind it (no overtaking, so no starvation)."""
    chosen = []
    used = active_bytes
    for r in queue:
        if r.arrival > now or len(chosen) >= free_slots:
            break
        if used + r.footprint > budget:
            break
        chosen.append(r)
        used += r.footprint
    return chosen


@dataclass
class Stats:
    completed: int = 0
    makespan: float = 0.0
    latencies: List[float] = field(default_factory=list)
    peak_bytes: int = 0
    peak_active: int = 0
    # host time by activity (s): building domains, batch table updates,
    # waiting for the device, handing back finished requests
    t_build: float = 0.0
    t_table: float = 0.0
    t_wait: float = 0.0
    t_finish: float = 0.0
    chunks: int = 0

    def summary(self):
        lat = np.asarray(self.latencies) if self.latencies else np.zeros(1)
        return {"completed": self.completed, "makespan_s": round(self.makespan, 4),
                "sims_per_s": round(self.completed / self.makespan, 4) if self.makespan > 0 else None,
                "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                "peak_resident_bytes": int(self.peak_bytes), "peak_active": int(self.peak_active),
                "host_s": {"build": round(self.t_build, 4), "table": round(self.t_table, 4),
                           "wait": round(self.t_wait, 4), "finish": round(self.t_finish, 4)},
                "chunks": int(self.chunks)}


class Server:
    """Continuous batching on one GPU.

    budget_bytes -- device memory the resident requests may hold together
    max_active   -- largest number of requests advanced by one launch (<= 64)
    chunk        -- steps between admission / completion points
    solo_points  -- requests of at least this many points are stepped alone
    solo_chunk   -- steps between those points while a solo request runs
                    (newcomers cannot run before it finishes, so its chunks
                    can be longer; the host turnaround at each boundary
                    leaves the device idle)

    Host work overlaps device work: arrived requests are admitted (arrival
    order, memory budget and slots counted over running, built and admitted
    requests); their domains are built on a separate setup stream while a
    chunk of steps runs on the serving stream, and join at the next chunk
    boundary, when finished requests also hand back their traces.  With
    requests waiting to be built, chunks are kept short so that they join
    early.

    Requests too small to fill the GPU share the batched launch.  A request
    that fills it alone gains nothing from sharing and loses the reuse of its
    fields in the device's last-level cache between the two phases of a step
    (a batched phase sweeps every domain before the next phase starts), so
    such requests are stepped alone with the single-domain kernels, one at a
    time in arrival order; the others wait resident, with their setup and
    read-back still overlapping the device work.  The device serves the
    oldest work first: in each chunk it runs either the batch (when its oldest
    request arrived before the next solo request) or that solo request, not
    both, so neither waits behind a chunk of the other that has just started
    and large requests complete in arrival order as they would one at a time.
    """

    def __init__(self, budget_bytes, max_active=32, chunk=64, device="cuda:0", tile=(256, 4),
                 solo_points=1_000_000, solo_chunk=512):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.stream = torch.cuda.Stream(device=self.device)
        self.setup_stream = torch.cuda.Stream(device=self.device)
        self.batch = fw2.Batch(max_domains=self.max_active, device=self.device, stream=self.stream)
        self.tile = tuple(tile)
        self.batch.set_tile(*tile)
        self.solo_points = int(solo_points)
        self.solo_chunk = int(solo_chunk) if solo_chunk else self.chunk

    def _start(self, r):
        dom = fw2.Domain(r.problem, device=self.device, stream=self.setup_stream)
        if len(r.problem.src_idx):
            dom.add_source(r.problem.src_idx, r.problem.src_sig, r.problem.src_w, r.problem.signals)
        dom.add_receivers(r.problem.rcv_idx, r.n_steps)
        return dom

    def run(self, requests, clock=time.perf_counter, on_done=None):
        """Serve the requests (sorted by arrival); returns Stats.  on_done(r),
        if given, is called as each request completes."""
        queue = sorted(requests, key=lambda r: (r.arrival, r.rid))
        if self.tile[0] != 256 and any(int(r.problem.n_relax) > 4 and r.problem.npts < self.solo_points
                                       for r in queue):
            raise ValueError("requests with more than four mechanisms need 256-column tiles")
        for r in queue:
            r.footprint = footprint_bytes(r.problem, r.n_steps)
            if r.footprint > self.budget:
                raise ValueError("request %d needs %d bytes, above the budget" % (r.rid, r.footprint))
        active = []               # (request, domain) in the batch
        solo = []                 # (request, domain) stepped alone, in arrival order
        staged = []               # (request, domain) built, joining at the next boundary
        pending = []              # admitted requests (memory reserved) not built yet
        in_flight = False         # a chunk is queued on the serving stream
        stats = Stats()
        t0 = clock()

        def build_one():
            r = pending.pop(0)
            tb = clock()
            staged.append((r, self._start(r)))
            stats.t_build += clock() - tb

        while queue or active or solo or staged or pending:
            # admit arrived requests (arrival order; memory and slots counted
            # over running, built and admitted-but-unbuilt requests)
            held = [r for r, _ in active] + [r for r, _ in solo] + [r for r, _ in staged] + pending
            new = admit(queue, sum(r.footprint for r in held), self.budget, self.max_active - len(held),
                        clock() - t0)
            for r in new:
                queue.remove(r)
                r.admitted = clock() - t0
                pending.append(r)
            # build while the device is busy with the chunk in flight; with an
            # idle device build one, so that stepping can start
            if pending and not (in_flight or active or solo or staged):
                build_one()
            while pending and in_flight and not self.stream.query():
                build_one()
            changed = False
            finished = []
            if in_flight:
                tw = clock()
                self.stream.synchronize()
                stats.t_wait += clock() - tw
                in_flight = False
                finished = [(r, d) for r, d in active + solo if d.current_step() >= r.n_steps]
                if finished:
                    tf = clock()
                    changed = any(d.current_step() >= r.n_steps for r, d in active)
                    active = [(r, d) for r, d in active if d.current_step() < r.n_steps]
                    solo = [(r, d) for r, d in solo if d.current_step() < r.n_steps]
                    for r, d in finished:
                        r.trace = d.trace.cpu().numpy()
                        r.done = clock() - t0
                        stats.latencies.append(r.done - r.arrival)
                        stats.completed += 1
                        if on_done:
                            on_done(r)
                    stats.t_finish += clock() - tf
            for r, d in staged:
                if r.problem.npts >= self.solo_points:
                    d.set_stream(self.stream)
                    solo.append((r, d))
                else:
                    active.append((r, d))
                    changed = True
            staged = []
            if changed or finished:
                tt = clock()
                if changed:
                    # the batch table stops referring to finished domains before they go
                    self.batch.set_domains([d for _, d in active], [r.n_steps for r, _ in active])
                for _, d in finished:
                    d.destroy_domain()
                stats.t_table += clock() - tt
            if not active and not solo:
                if queue and not pending:
                    wait = queue[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            stats.peak_bytes = max(stats.peak_bytes, sum(r.footprint for r, _ in active + solo))
            stats.peak_active = max(stats.peak_active, len(active) + len(solo))
            # oldest work first: the batch if its oldest request arrived before
            # the solo request in turn, else that solo request
            run_batch = bool(active) and (not solo or min((r.arrival, r.rid) for r, _ in active)
                                          <= (solo[0][0].arrival, solo[0][0].rid))
            # run until the next event: the first completion of the work in
            # turn, or (when requests wait to join) the next chunk boundary
            left = [r.n_steps - d.current_step() for r, d in (active if run_batch else solo[:1])]
            to_done = min(left)
            waiting = pending or (queue and len(active) + len(solo) < self.max_active)
            chunk = self.chunk if run_batch else self.solo_chunk
            k = max(int(min(to_done, chunk) if waiting else to_done), 1)
            if run_batch:
                self.batch.step(k)
            else:
                r, d = solo[0]
                d.step(min(k, r.n_steps - d.current_step()))
            stats.chunks += 1
            in_flight = True
        stats.makespan = clock() - t0
        return stats

    def close(self):
        self.batch.destroy()


def run_plain(requests, device="cuda:0", clock=time.perf_counter, on_done=None):
    """The same requests one at a time in arrival order (single-domain path);
    on_done(r), if given, is called as each request completes."""
    import torch
    dev = torch.device(device)
    stream = torch.cuda.Stream(device=dev)
    stats = Stats()
    t0 = clock()
    for r in sorted(requests, key=lambda q: (q.arrival, q.rid)):
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        r.admitted = clock() - t0
        tb = clock()
        dom = fw2.Domain(r.problem, device=dev, stream=stream)
        if len(r.problem.src_idx):
            dom.add_source(r.problem.src_idx, r.problem.src_sig, r.problem.src_w, r.problem.signals)
        dom.add_receivers(r.problem.rcv_idx, r.n_steps)
        stats.t_build += clock() - tb
        dom.step(r.n_steps)
        tw = clock()
        stream.synchronize()
        stats.t_wait += clock() - tw
        tf = clock()
        r.trace = dom.trace.cpu().numpy()
        dom.destroy_domain()
        stats.t_finish += clock() - tf
        r.done = clock() - t0
        stats.latencies.append(r.done - r.arrival)
        stats.completed += 1
        stats.peak_active = 1
        if on_done:
            on_done(r)
    stats.makespan = clock() - t0
    return stats


def autotune_tile(problems, candidates=((256, 2), (256, 4), (256, 8), (64, 4), (64, 8), (64, 16)),
                  steps=32, device="cuda:0"):
    """Pick the batched sweep's tile (columns, rows) by timing each candidate
    on a batch of zero-state copies of the given problems (sources are not
    attached, so the fields stay zero and nothing is consumed).  Domains with
    more than four mechanisms run in 256-column tiles only, so with such a
    problem in the mix the 64-column candidates are left out."""
    import torch
    if any(int(p.n_relax) > 4 for p in problems):
        candidates = tuple(c for c in candidates if c[0] == 256)
    if not candidates:
        raise ValueError("no candidate tile fits the problems")
    dev = torch.device(device)
    stream = torch.cuda.Stream(device=dev)
    doms = [fw2.Domain(p, device=dev, stream=stream) for p in problems]
    best, timings = None, {}
    batch = fw2.Batch(max_domains=max(len(doms), 1), device=dev, stream=stream)
    for rows in candidates:
        batch.set_domains([], [])
        batch.set_tile(*rows)
        batch.set_domains(doms, [10 ** 9] * len(doms))
        batch.step(steps)                          # warm-up (also builds the graph)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.step(steps)
        e1.record(stream)
        stream.synchronize()
        timings[rows] = e0.elapsed_time(e1) / steps
        if best is None or timings[rows] < timings[best]:
            best = rows
    batch.set_domains([], [])
    batch.destroy()
    for d in doms:
        d.destroy_domain()
    return best, timings
