#!/usr/bin/env python
"""Benchmark of the Fullwave 2 time stepper on one MI355X.

A step is one time step of the whole hot path: pressure kernel, sources,
receivers, velocity kernel.  The headline workload is the largest one that
fits one GPU: the 3D transcranial-like cube (1024^3 points including the
4-wavelength boundary, L = 2 relaxation mechanisms, 2 tissue labels, a
focused spherical-cap source, 1 MHz).

Prints one JSON line: Gpoint-updates/s over the timed steps, the roofline of
the dominant kernel (HIP-event durations on the domain's stream, algorithmic
bytes per launch), the same cube with per-point stencil weights, one GPU's
slab of that cube split along z with its halo exchange timed, the 2D
abdominal-wall workload (4096 x 2048, L = 4, 12000 steps) as a sub-object,
batched-serving sims/s and p50/p99 latency against the plain one-at-a-time
solver, the sound-speed gradient of one shot of the 1536^2 inversion workload
(checkpointed forward + reverse steps, with the reverse step's own
roofline), the FP64 CPU oracle timed on a bounded sample (all host threads,
and one thread), and the paper's own runtimes as context.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload skull_3d|abdominal_2d|plain_2d]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
XGMI_LINK_GBS = 153.0   # one xGMI link, one direction
CSRC = os.path.join(ROOT, "paper_2106_11476_amd", "csrc")
# the step kernels are templates in step_kernels.hpp over the layout of kernels.hpp
KERNEL_SOURCE = [os.path.join(CSRC, "step_kernels.hpp"), os.path.join(CSRC, "kernels.hpp")]
ADJOINT_SOURCE = os.path.join(CSRC, "adjoint.hip")
ADJOINT_WORKLOAD = "inversion_2d_1536"
PROFILES = os.path.join(ROOT, "profiles")

# The paper's own runtimes (Sec. 4.6, Fig. 6): context, not the target.
PAPER_CONTEXT = {
    "source": "Sec. 4.6 (computational performance), Fig. 6",
    "hardware": "1x NVIDIA RTX 4090 (24 GB), CUDA 12.6",
    "precision": "not stated",
    "settings": "12 ppw, CFL 0.4, N = 2 relaxation mechanisms",
    "saturated_gcells_per_s_2d": 1.5,
    "saturated_gcells_per_s_3d": 0.75,
    "grid_1024x1024_s_per_1000_steps": 0.667,
    "grid_2048x2048_s_per_1000_steps": 2.74,
    "grid_256x256x256_s_per_1000_steps": 22.6,
}


def kernel_source_sha(path=None):
    import hashlib
    paths = KERNEL_SOURCE if path is None else ([path] if isinstance(path, str) else list(path))
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_values(path):
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    return vals


def measured_adjoint_traffic():
    """HBM bytes per point of one reverse step (both kernels, sparse ones
    included) from the committed counter summary, or None when there is none
    or the adjoint kernels changed since the counters were taken."""
    path = os.path.join(PROFILES, "traffic_adjoint_step_%s.txt" % ADJOINT_WORKLOAD)
    if not os.path.exists(path):
        return None
    vals = _profile_values(path)
    if vals.get("adjoint_source_sha256_16") != kernel_source_sha(ADJOINT_SOURCE):
        return None
    try:
        return float(vals["hbm_bytes_per_point_reverse_step"])
    except (KeyError, ValueError):
        return None


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload, or None when there is none or the kernel source changed
    since the counters were taken."""
    path = os.path.join(PROFILES, "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    vals = _profile_values(path)
    if vals.get("kernel_source_sha256_16") != kernel_source_sha():
        return None
    try:
        return int(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_bytes(ndim, L, labels):
    """Algorithmic bytes per point of each kernel (every array it must touch,
    read once and written once; the label byte only when tissues vary).
    pressure: reads v (ndim), p, psi2 (ndim L), kappa0, kappa0(1-2 beta);
              writes p, psi2.
    velocity: reads p, v (ndim), psi1 (ndim L), rho, kappa0; writes v, psi1.
    step:     each state array read and written once, three medium arrays
              read once, the label once."""
    lab = 1 if labels else 0
    p_b = 4 * (ndim + 1 + ndim * L + 2) + lab + 4 * (1 + ndim * L)
    v_b = 4 * (1 + ndim + ndim * L + 2) + lab + 4 * (ndim + ndim * L)
    state = 1 + ndim + 2 * ndim * L
    step_b = 8 * state + 12 + lab
    return p_b, v_b, step_b


def make_workload(name, n3d=1024, relax=None):
    """relax: mechanism count, None for the workload's own (4 in 2D, 2 in 3D)."""
    import workloads as W
    if name == "abdominal_2d":
        return W.abdominal_2d(L=4 if relax is None else relax)
    if name == "plain_2d" and relax is None:
        return W.plain_2d()
    if name == "skull_3d":
        return W.skull_3d(n=n3d, L=2 if relax is None else relax)
    raise SystemExit("unknown workload %s, or one without a --relax option" % name)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, %r)
import workloads as W
from oracle import solver
prob = W.skull_3d(n=96, nb=12, ntr=9) if %r else W.abdominal_2d(nx=512, ny=512)
maps = solver.coefficient_maps(prob)
st = solver.State(maps.ndim, maps.L, maps.grid)
t0 = time.perf_counter(); solver.run(prob, 1, st, maps, record=False); per = time.perf_counter() - t0
k = int(max(1, min(200, %r / max(per, 1e-6))))
t0 = time.perf_counter(); solver.run(prob, k, st, maps, record=False); el = time.perf_counter() - t0
print(json.dumps({"value": prob.npts * k / el / 1e9, "threads": solver.threads(),
                  "sample": "%%d steps of the full %%s grid, %%.1f s" %% (k, prob.name, el)}))
"""


def single_thread_oracle(three_d, target_s=8.0):
    """The oracle on one host thread, in a child process (OMP_NUM_THREADS=1;
    the child touches no GPU): a bounded sample of the same recipe."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = _ORACLE_SAMPLE % (ROOT, bool(three_d), float(target_s))
    out = subprocess.check_output([sys.executable, "-c", code], env=env, timeout=600)
    r = json.loads(out.decode().strip().splitlines()[-1])
    return {"value": round(r["value"], 6), "unit": "Gpoint-updates/s", "cores": r["threads"], "sample": r["sample"]}


def cpu_baseline(prob, target_s=15.0):
    """The FP64 oracle, as is, on the same workload: a bounded number of
    steps on the full grid from the zero state (setup not timed), on all host
    threads; plus a one-thread sample.  For the 3D cube, whose FP64 state
    does not fit host memory, the same recipe on a 192^3 cube is the sample."""
    from oracle import solver
    three_d = prob.ndim == 3
    if three_d and prob.npts > 192 ** 3:
        import workloads as W
        prob = W.skull_3d(n=192, nb=24, ntr=18)
    maps = solver.coefficient_maps(prob)
    st = solver.State(maps.ndim, maps.L, maps.grid)
    t0 = time.perf_counter()
    solver.run(prob, 2, st, maps, record=False)
    per = (time.perf_counter() - t0) / 2
    k = int(max(2, min(400, target_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    solver.run(prob, k, st, maps, record=False)
    el = time.perf_counter() - t0
    out = {"value": prob.npts * k / el / 1e9, "unit": "Gpoint-updates/s", "cores": solver.threads(),
           "kind": "oracle", "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
           "sample": "%d steps of the full %s grid (FP64 C stepper, OpenMP, %d threads), %.1f s"
                     % (k, prob.name, solver.threads(), el)}
    del maps, st
    try:
        out["single_thread"] = single_thread_oracle(three_d)
    except Exception as e:                      # reported, not fatal to the benchmark line
        out["single_thread"] = {"error": str(e)[:200]}
    return out


def probe_copy(torch, dev, mib, reps=10):
    """Plain device-to-device copy of `mib` MiB (one torch copy kernel per rep)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * n * 4
    del src, dst
    return {"bytes_per_copy": moved, "ms": round(ms, 4), "GBps": round(moved / ms / 1e6, 1), "reps": reps}


def library_probe(torch, dev, kind, nbytes, reps=10):
    """HBM rate of one of the library's streaming probes (fw2_stream_probe)
    over a device buffer of nbytes holding random normal FP32 values (all-zero
    buffers stream about 5% faster on this GPU), timed with events on torch's
    current stream, which the probe is launched on."""
    from paper_2106_11476_amd import fw2
    buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    buf.view(torch.float32).normal_()
    n = fw2.stream_probe_elements(kind, nbytes)
    moved = 2 * 16 * n if kind == fw2.PROBE_COPY else 21 * 4 * n
    for _ in range(2):
        fw2.stream_probe(kind, buf)
    torch.cuda.synchronize(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fw2.stream_probe(kind, buf)
    e1.record()
    torch.cuda.synchronize(dev)
    ms = e0.elapsed_time(e1) / reps
    del buf
    return {"bytes": moved, "ms": round(ms, 4), "GBps": round(moved / ms / 1e6, 1), "reps": reps}


def stream_reference(torch, dev, roofline, mib=2048):
    """What plain streaming kernels reach on this GPU, beside the dominant
    kernel's algorithmic rate and its measured HBM traffic rate: torch's
    device copy, the library's one-thread-per-float4 copy, and the library's
    probe with the velocity phase's byte mix (12 arrays read, 9 written, 4 B
    per lane, no stencil)."""
    from paper_2106_11476_amd import fw2
    ref = probe_copy(torch, dev, mib)
    out = {"kind": "plain device-to-device copy (one torch copy kernel)", "bytes_per_copy": ref["bytes_per_copy"],
           "ms": ref["ms"], "GBps": ref["GBps"], "reps": ref["reps"],
           "kernel_algorithmic_over_copy": round(roofline["achieved"] / ref["GBps"], 3)}
    copy16 = library_probe(torch, dev, fw2.PROBE_COPY, 2 * mib << 20)
    mix = library_probe(torch, dev, fw2.PROBE_VELOCITY_MIX, 21 * (512 << 20))
    out["probe_copy16"] = dict(copy16, kind="fw2_stream_probe copy, one float4 per thread")
    out["probe_velocity_mix"] = dict(mix, kind="fw2_stream_probe, 12 FP32 arrays read and 9 written per point")
    out["kernel_algorithmic_over_copy16"] = round(roofline["achieved"] / copy16["GBps"], 3)
    if roofline.get("traffic"):
        traffic_gbs = roofline["traffic"] / (roofline["launch_ms"] * 1e-3) / 1e9
        out["kernel_traffic_GBps"] = round(traffic_gbs, 1)
        out["kernel_traffic_over_copy"] = round(traffic_gbs / ref["GBps"], 3)
        out["kernel_traffic_over_velocity_mix"] = round(traffic_gbs / mix["GBps"], 3)
    return out


STATED_SERVING_REQUESTS = 256     # the served workload's stream


def serving_leg(seed=4, workload_requests=16, only_workload=False, solo_points=1_000_000, solo_chunk=512,
                passes="all", rate=None):
    """Continuous batching vs the plain one-at-a-time solver on four seeded
    request streams of the heterogeneous 2D recipe: `workload_requests` of
    the served workload's requests (1024^2-3072^2 at their own step counts;
    the stated stream has 256, the default 16 is a subsample), 48 at
    512^2-1024^2, 96 small 128^2-384^2 grids, and 48 small grids mixing every
    launch class (3, 4 or 8 mechanisms; every third request with per-point
    stencil weights).  Capacity: all requests queued at t = 0.  Latency:
    Poisson arrivals at 1.2x the plain solver's capacity.  target_met: the
    batched capacity is at least twice the plain one.  passes: "all", or
    "capacity" or "poisson" alone (the latter at the given arrival rate), so
    that a long stream can be measured in two runs."""
    import workloads as W
    from paper_2106_11476_amd import fw2, serve
    out = {}
    streams = [("workload_1024_3072", (workload_requests, (1024, 3072), 256, (2, 3, 4), 0))]
    if not only_workload:
        streams += [("heterogeneous_512_1024", (48, (512, 1024), 128, (2, 3, 4), 0)),
                    ("small_128_384", (96, (128, 384), 64, (2, 3, 4), 0)),
                    ("mixed_classes_128_384", (48, (128, 384), 64, (3, 4, 8), 3))]
    for name, (n, sides, step, L_choices, local_every) in streams:
        raw = W.serving_requests(n=n, seed=seed, sides=sides, side_step=step, L_choices=L_choices)
        if local_every:
            for i, (p, _, _) in enumerate(raw):
                if i % local_every == local_every - 1:
                    p.stencil_mode = fw2.STENCIL_LOCAL
        upd = sum(p.npts * k for p, k, _ in raw)
        mk = lambda arr: [serve.Request(i, p, k, a) for i, ((p, k, _), a) in enumerate(zip(raw, arr))]
        # the tuning set holds a domain with more than four mechanisms when
        # the stream does, so that the tile chosen can run every request
        tune = [p for p, _, _ in raw[:4]]
        many = [p for p, _, _ in raw if p.n_relax > 4]
        if many and all(p.n_relax <= 4 for p in tune):
            tune.append(many[0])
        tile, _ = serve.autotune_tile(tune, steps=32)
        med = float(np.median([serve.footprint_bytes(p, k) for p, k, _ in raw]))
        budget = int(24 * med)
        srv = serve.Server(budget_bytes=budget, max_active=32, chunk=64, tile=tile, solo_points=solo_points,
                           solo_chunk=solo_chunk)

        def progress(label):
            # long streams: a line every 16 completed requests
            count = 0

            def done(r):
                nonlocal count
                count += 1
                if count % 16 == 0:
                    print("[serving] %s %s: %d of %d done" % (name, label, count, n), file=sys.stderr, flush=True)
            return done
        res = {"requests": n, "sides": list(sides), "relax_mechanisms": list(L_choices),
               "per_point_weights_every": local_every, "tile": list(tile), "budget_bytes": budget}
        lam = rate
        if passes in ("all", "capacity"):
            p0 = serve.run_plain(mk([0.0] * n), on_done=progress("capacity plain"))
            b0 = srv.run(mk([0.0] * n), on_done=progress("capacity served"))
            lam = 1.2 * p0.completed / p0.makespan
            res.update({
                "capacity_sims_per_s": {"plain": round(p0.completed / p0.makespan, 3),
                                        "batched": round(b0.completed / b0.makespan, 3)},
                "capacity_gpoint_updates_per_s": {"plain": round(upd / p0.makespan / 1e9, 3),
                                                  "batched": round(upd / b0.makespan / 1e9, 3)},
                "capacity_speedup": round(p0.makespan / b0.makespan, 3),
                "target_met": bool(p0.makespan / b0.makespan >= 2.0),
                "capacity_host_s": {"plain": p0.summary()["host_s"], "batched": b0.summary()["host_s"]}})
        if passes in ("all", "poisson"):
            if not lam:
                raise SystemExit("the Poisson pass alone needs --serving-rate")
            arr = np.cumsum(np.random.default_rng(seed + 40).exponential(1.0 / lam, n))
            pl = serve.run_plain(mk(arr), on_done=progress("poisson plain"))
            bt = srv.run(mk(arr), on_done=progress("poisson served"))
            res.update({"poisson_rate_per_s": round(lam, 3),
                        "poisson": {"plain": pl.summary(), "batched": bt.summary()}})
        srv.close()
        out[name] = res
        if name == "workload_1024_3072":
            out[name]["stated_stream_requests"] = STATED_SERVING_REQUESTS
            out[name]["subsample"] = n < STATED_SERVING_REQUESTS
    return out


def local_stencil_leg(prob, steps, warmup=20):
    """The benchmark workload with per-point stencil weights (every point the
    weights of its own Courant number): Gpoint-updates/s and both kernels'
    HIP-event durations.  The pressure kernel then also reads rho (+4 B per
    point); the step's algorithmic bytes are unchanged (rho is read once per
    step already)."""
    import torch
    from paper_2106_11476_amd import fw2
    dev = torch.device("cuda:0")
    loc = type(prob)(**{k: getattr(prob, k) for k in prob.__dataclass_fields__})
    loc.stencil_mode = fw2.STENCIL_LOCAL
    stream = torch.cuda.Stream(device=dev)
    dom = fw2.from_problem(loc, device=dev, stream=stream, cap_steps=steps + warmup)
    dom.step(warmup)
    torch.cuda.synchronize(dev)
    dom.enable_kernel_timing(True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    dom.step(steps)
    torch.cuda.synchronize(dev)
    el = time.perf_counter() - t0
    ms, cnt = dom.get_kernel_timing()
    dom.check_finite(1e9)
    dom.destroy_domain()
    labels = prob.label is not None and np.asarray(prob.relax_table).shape[0] > 1
    p_b, v_b, step_b = kernel_bytes(prob.ndim, prob.n_relax, labels)
    p_b += 4
    avg = [ms[0] / max(cnt[0], 1), ms[1] / max(cnt[1], 1)]
    gpts = prob.npts * steps / el / 1e9
    return {"steps": steps, "value": round(gpts, 3), "unit": "Gpoint-updates/s",
            "ms_per_step": round(el / steps * 1e3, 5),
            "pressure_kernel": {"launch_ms": round(avg[0], 5), "alg_bytes_per_point": p_b,
                                "frac": round(p_b * prob.npts / (avg[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "velocity_kernel": {"launch_ms": round(avg[1], 5), "alg_bytes_per_point": v_b,
                                "frac": round(v_b * prob.npts / (avg[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "step_frac": round(gpts * step_b / HBM_PEAK_GBS, 4)}


def adjoint_bytes(ndim, L, labels):
    """Algorithmic HBM bytes per point of one reverse step: the forward state
    at the step's input read once, the adjoint state (same arrays) read and
    written once, the medium (kappa0, its nonlinear factor, rho) read once,
    the gradient accumulator read and written once, plus the 1-byte label."""
    n_state = 1 + ndim + 2 * ndim * L
    return 4 * n_state + 8 * n_state + 12 + 8 + (1 if labels else 0)


def adjoint_leg(steps=6000, K=64, shot=31, timed_reverse=200):
    """Gradient of the receiver-trace misfit for one shot of the 1536^2
    inversion workload: observed traces from the true medium, then the
    checkpointed forward (one state block every K steps) and the backward
    (segment recompute + reverse steps).  The reverse step alone is timed
    with HIP events on the domain's stream for the roofline."""
    import torch
    import workloads as W
    from paper_2106_11476_amd import adjoint, fw2
    dev = torch.device("cuda:0")
    prob, c_true = W.inversion_2d(shot=shot, n_steps=steps)
    truth = W.Problem(**{k: getattr(prob, k) for k in prob.__dataclass_fields__})
    truth.c = c_true
    dom = fw2.from_problem(truth, device=dev, cap_steps=steps)
    dom.step(steps)
    torch.cuda.synchronize(dev)
    obs = dom.trace[:steps].clone()
    dom.destroy_domain()
    c = torch.tensor(np.asarray(prob.c, np.float64), requires_grad=True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    J = adjoint.misfit(c, obs, prob, steps, checkpoint_every=K)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize(dev)
    t2 = time.perf_counter()
    g = c.grad.numpy()
    # reverse step alone
    stream = torch.cuda.Stream(device=dev)
    dom = fw2.from_problem(prob, device=dev, stream=stream, cap_steps=steps)
    dom.step(400)
    st = dom.new_state_buffer()
    dom.save_state(st)
    res = torch.zeros((1, len(prob.rcv_idx)), device=dev)
    dom.adjoint_begin()
    # steady state of the backward sweep: consecutive steps, each call handed
    # the state of the step before (the same block stands in for every state)
    s0 = max(steps - 1, 20 + timed_reverse)
    for k in range(20):
        dom.adjoint_step(st, s0 - k, res[0], prev=st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(20, 20 + timed_reverse):
        dom.adjoint_step(st, s0 - k, res[0], prev=st)
    e1.record(stream)
    stream.synchronize()
    ms = e0.elapsed_time(e1) / timed_reverse
    dom.destroy_domain()
    labels = prob.label is not None and np.asarray(prob.relax_table).shape[0] > 1
    b = adjoint_bytes(prob.ndim, prob.n_relax, labels)
    gbs = b * prob.npts / (ms * 1e-3) / 1e9
    return {"workload": prob.name, "grid": list(prob.shape), "steps": steps, "checkpoint_every": K,
            "sources_per_shot": 1, "receivers": int(len(prob.rcv_idx)),
            "misfit": float(J.item()), "gradient_finite": bool(np.isfinite(g).all()),
            "forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
            "gradient_s_per_shot": round(t2 - t0, 3),
            "reverse_step_ms": round(ms, 5),
            "reverse_gpts": round(prob.npts / (ms * 1e-3) / 1e9, 3),
            "reverse_roofline": {"bound": "hbm", "alg_bytes_per_point": b, "achieved": round(gbs, 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                 "traffic_bytes_per_point": measured_adjoint_traffic()}}


def full_gradient_leg(n_shots=64, steps=6000, K=64):
    """The inversion workload's whole gradient: the misfit summed over
    n_shots shots (each source fired alone, every shot recorded on the 256
    receivers), dJ/dc accumulated over the shots.  Per shot: the observed
    traces from the true medium, the checkpointed forward and the backward.
    Times the whole job on the host clock around each shot."""
    import torch
    import workloads as W
    from paper_2106_11476_amd import adjoint, fw2
    dev = torch.device("cuda:0")
    total = None
    J_sum = 0.0
    t_obs = t_grad = 0.0
    for shot in range(n_shots):
        prob, c_true = W.inversion_2d(shot=shot, n_steps=steps)
        truth = W.Problem(**{k: getattr(prob, k) for k in prob.__dataclass_fields__})
        truth.c = c_true
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        dom = fw2.from_problem(truth, device=dev, cap_steps=steps)
        dom.step(steps)
        torch.cuda.synchronize(dev)
        obs = dom.trace[:steps].clone()
        dom.destroy_domain()
        t1 = time.perf_counter()
        c = torch.tensor(np.asarray(prob.c, np.float64), requires_grad=True)
        J = adjoint.misfit(c, obs, prob, steps, checkpoint_every=K)
        J.backward()
        torch.cuda.synchronize(dev)
        t2 = time.perf_counter()
        t_obs += t1 - t0
        t_grad += t2 - t1
        J_sum += float(J.item())
        g = c.grad.numpy()
        total = g.copy() if total is None else total + g
    return {"workload": "inversion_2d_1536", "shots": n_shots, "receivers": 256, "steps": steps,
            "checkpoint_every": K, "misfit_sum": J_sum, "gradient_finite": bool(np.isfinite(total).all()),
            "gradient_rms": float(np.sqrt(np.mean(total ** 2))),
            "observed_traces_s": round(t_obs, 3), "gradient_s": round(t_grad, 3),
            "gradient_s_per_shot": round(t_grad / n_shots, 4)}


def _db_rows(db, sql):
    import sqlite3
    con = sqlite3.connect(db)
    try:
        return list(con.execute(sql))
    finally:
        con.close()


def summarize_stats_only(stats_db, name, title, commands):
    """Write profiles/kernel_stats_<name>.txt from a kernel-trace database."""
    stats = _db_rows(stats_db, "select name, total_calls, total_duration, average from top_kernels")
    lines = ["rocprofv3 kernel statistics: %s" % title, "commands:"] + ["  " + c for c in commands]
    lines.append("kernel_source_sha256_16: %s" % kernel_source_sha())
    lines.append("%-70s %8s %12s %10s" % ("kernel", "calls", "total_us", "avg_us"))
    for kname, calls, tot, avg in stats:
        lines.append("%-70s %8d %12.1f %10.3f" % (kname[:70], calls, tot, avg))
    with open(os.path.join(PROFILES, "kernel_stats_%s.txt" % name), "w") as fh:
        fh.write("\n".join(lines) + "\n")


CALIBRATION_BYTES = {"copy16": 512 << 20, "mix": 21 * (64 << 20)}   # buffer of each calibration probe


def calibration_probe(reps=5):
    """The library's streaming probes on fixed buffers (random data), reps
    dispatches each, for the HBM counter passes that check the counters'
    scale on known-size kernels; prints the bytes each dispatch must move."""
    import torch
    from paper_2106_11476_amd import fw2
    dev = torch.device("cuda:0")
    out = {}
    for name, kind in (("copy16", fw2.PROBE_COPY), ("mix", fw2.PROBE_VELOCITY_MIX)):
        nbytes = CALIBRATION_BYTES[name]
        buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        buf.view(torch.float32).normal_()
        n = fw2.stream_probe_elements(kind, nbytes)
        for _ in range(reps):
            fw2.stream_probe(kind, buf)
        torch.cuda.synchronize(dev)
        del buf
        rd, wr = (16 * n, 16 * n) if kind == fw2.PROBE_COPY else (48 * n, 36 * n)
        out[name] = {"read_bytes": rd, "write_bytes": wr, "dispatches": reps}
    print(json.dumps({"calibration_probe": out}))
    return out


def summarize_calibration(fetch_db, write_db, commands):
    """Write profiles/traffic_calibration_stream_probes.txt: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) of the library's probes against the bytes
    they must read and write, i.e. the scale factors of the counters measured
    on two known-size kernels other than the copy the traffic summaries use."""
    from paper_2106_11476_amd import fw2
    fetch = {r[0]: r for r in _db_rows(fetch_db, "select name, avg(counter_value), count(*) from pmc_events group by name")}
    write = {r[0]: r for r in _db_rows(write_db, "select name, avg(counter_value), count(*) from pmc_events group by name")}
    lines = ["HBM counter scale on known-size kernels: the library's streaming probes (fw2_stream_probe)", "commands:"]
    lines += ["  " + c for c in commands]
    for name, kind in (("copy16", fw2.PROBE_COPY), ("mix", fw2.PROBE_VELOCITY_MIX)):
        n = fw2.stream_probe_elements(kind, CALIBRATION_BYTES[name])
        rd, wr = (16 * n, 16 * n) if kind == fw2.PROBE_COPY else (48 * n, 36 * n)
        fk = [k for k in fetch if ("probe_copy16" if name == "copy16" else "probe_mix") in k][0]
        wk = [k for k in write if ("probe_copy16" if name == "copy16" else "probe_mix") in k][0]
        f_raw, w_raw = fetch[fk][1], write[wk][1]
        lines += ["%s_kernel: %s" % (name, fk),
                  "%s_read_kib_per_dispatch: %.1f" % (name, rd / 1024.0),
                  "%s_fetch_kib_per_dispatch_raw: %.1f" % (name, f_raw),
                  "%s_fetch_scale: %.4f" % (name, rd / 1024.0 / f_raw),
                  "%s_write_kib_per_dispatch: %.1f" % (name, wr / 1024.0),
                  "%s_write_kib_per_dispatch_raw: %.1f" % (name, w_raw),
                  "%s_write_scale: %.4f" % (name, wr / 1024.0 / w_raw)]
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, "traffic_calibration_stream_probes.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_profiles(stats_db, fetch_db, write_db, workload, copy_bytes, commands, n3d=1024, relax=None):
    """Write profiles/*.txt from rocprofv3 results (kernel-trace stats and the
    FETCH_SIZE / WRITE_SIZE passes).  Counter values are KiB per dispatch;
    each is scaled by what it reads for the plain copy that reads and writes
    copy_bytes."""
    import glob
    stats = _db_rows(stats_db, "select name, total_calls, total_duration, average from top_kernels")
    fetch = _db_rows(fetch_db, "select name, avg(counter_value), max(counter_value), count(*) from pmc_events group by name")
    write = _db_rows(write_db, "select name, avg(counter_value), max(counter_value), count(*) from pmc_events group by name")
    fmax = {r[0]: r for r in fetch}
    wmax = {r[0]: r for r in write}
    copy_name = "__amd_rocclr_copyBuffer"
    f_scale = copy_bytes / 1024.0 / fmax[copy_name][2]
    w_scale = copy_bytes / 1024.0 / wmax[copy_name][2]
    sha = kernel_source_sha()
    os.makedirs(PROFILES, exist_ok=True)
    prob = make_workload(workload, n3d, relax)
    lines = ["rocprofv3 kernel statistics of the first command (benchmark workload %s; "
             "kernels of the other legs that command runs are listed too)" % prob.name, "commands:"]
    lines += ["  " + c for c in commands]
    lines.append("kernel_source_sha256_16: %s" % sha)
    lines.append("%-70s %8s %12s %10s" % ("kernel", "calls", "total_us", "avg_us"))
    for name, calls, tot, avg in stats:
        lines.append("%-70s %8d %12.1f %10.3f" % (name[:70], calls, tot, avg))
    if workload == "skull_3d":
        name = prob.name
    else:
        name = workload + ("" if prob.n_relax == 4 else "_L%d" % prob.n_relax)
    with open(os.path.join(PROFILES, "kernel_stats_%s.txt" % name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    labels = prob.label is not None and np.asarray(prob.relax_table).shape[0] > 1
    p_b, v_b, _ = kernel_bytes(prob.ndim, prob.n_relax, labels)
    # the benchmark's sweep kernels carry the mechanism count as their first
    # template argument (other legs of a run may launch other instances)
    tag = "<%d, " % prob.n_relax
    for short, key, alg in (("pressure_kernel", "pressure_", p_b), ("velocity_kernel", "velocity_", v_b)):
        names = [n for n in fmax if key in n and tag in n]
        if not names:
            continue
        n = names[0]
        fk, wk = fmax[n][1], wmax[n][1]
        hbm = int(round((fk * f_scale + wk * w_scale) * 1024))
        algb = alg * prob.npts
        avg_us = [r[3] for r in stats if r[0] == n]
        txt = ["HBM traffic of %s on workload %s" % (n, prob.name), "commands:"]
        txt += ["  " + c for c in commands]
        txt += ["kernel_source_sha256_16: %s" % sha,
                "dispatches_counted: %d" % fmax[n][3],
                "fetch_kib_per_dispatch_raw: %.1f" % fk,
                "write_kib_per_dispatch_raw: %.1f" % wk,
                "copy_probe_bytes: %d" % copy_bytes,
                "copy_fetch_kib_raw: %.1f" % fmax[copy_name][2],
                "copy_write_kib_raw: %.1f" % wmax[copy_name][2],
                "fetch_scale: %.4f" % f_scale,
                "write_scale: %.4f" % w_scale,
                "hbm_bytes_per_launch: %d" % hbm,
                "algorithmic_bytes_per_launch: %d" % algb,
                "traffic_over_algorithmic: %.4f" % (hbm / algb),
                "avg_duration_us_kernel_trace: %s" % (("%.3f" % avg_us[0]) if avg_us else "n/a")]
        with open(os.path.join(PROFILES, "traffic_%s_%s.txt" % (short, prob.name)), "w") as fh:
            fh.write("\n".join(txt) + "\n")
    print("profiles written to", PROFILES)


def summarize_adjoint(stats_db, fetch_db, write_db, copy_bytes, commands):
    """Write the kernel statistics and the per-kernel traffic of the adjoint
    leg (FETCH_SIZE / WRITE_SIZE passes, KiB per dispatch, scaled by what the
    counters read for the plain copy of copy_bytes)."""
    stats = _db_rows(stats_db, "select name, total_calls, total_duration, average from top_kernels")
    fetch = _db_rows(fetch_db, "select name, avg(counter_value), max(counter_value), count(*) from pmc_events group by name")
    write = _db_rows(write_db, "select name, avg(counter_value), max(counter_value), count(*) from pmc_events group by name")
    fmax = {r[0]: r for r in fetch}
    wmax = {r[0]: r for r in write}
    copy_name = "__amd_rocclr_copyBuffer"
    f_scale = copy_bytes / 1024.0 / fmax[copy_name][2]
    w_scale = copy_bytes / 1024.0 / wmax[copy_name][2]
    sha = kernel_source_sha(ADJOINT_SOURCE)
    npts = 1536 * 1536
    os.makedirs(PROFILES, exist_ok=True)
    lines = ["rocprofv3 kernel statistics: adjoint leg of the benchmark: one shot of the 1536^2 inversion "
             "workload (forward with checkpoints, segment recompute and reverse-step kernels)", "commands:"]
    lines += ["  " + c for c in commands]
    lines.append("adjoint_source_sha256_16: %s" % sha)
    lines.append("%-70s %8s %12s %10s" % ("kernel", "calls", "total_us", "avg_us"))
    for name, calls, tot, avg in stats:
        lines.append("%-70s %8d %12.1f %10.3f" % (name[:70], calls, tot, avg))
    with open(os.path.join(PROFILES, "kernel_stats_%s_adjoint.txt" % ADJOINT_WORKLOAD), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # the steady reverse step: velocity kernel (deferred A3), receivers,
    # pressure kernel with the fused A0 of the step before, sources
    parts = [("velocity", "adj_velocity<2, 2, true>"), ("pressure", "adj_pressure<2, 2, true>"),
             ("receivers", "adj_receivers("), ("sources", "adj_sources(")]
    txt = ["HBM traffic of one reverse step of the adjoint (2D, L = 2) on the 1536^2 inversion workload",
           "commands:"] + ["  " + c for c in commands]
    txt += ["adjoint_source_sha256_16: %s" % sha, "points: %d" % npts, "copy_probe_bytes: %d" % copy_bytes,
            "fetch_scale: %.4f" % f_scale, "write_scale: %.4f" % w_scale]
    total = 0.0
    for short, key in parts:
        names = [n for n in fmax if key in n]
        if not names:
            continue
        n = names[0]
        fk, wk = fmax[n][1], wmax[n][1]
        b = (fk * f_scale + wk * w_scale) * 1024.0
        total += b
        avg_us = [r[3] for r in stats if r[0] == n]
        txt += ["%s_kernel: %s" % (short, n),
                "%s_fetch_kib_per_dispatch_raw: %.1f" % (short, fk),
                "%s_write_kib_per_dispatch_raw: %.1f" % (short, wk),
                "%s_hbm_bytes_per_point: %.2f" % (short, b / npts),
                "%s_avg_duration_us_kernel_trace: %s" % (short, ("%.3f" % avg_us[0]) if avg_us else "n/a")]
    alg = adjoint_bytes(2, 2, True)
    txt += ["hbm_bytes_per_point_reverse_step: %.2f" % (total / npts),
            "algorithmic_bytes_per_point_reverse_step: %d" % alg,
            "traffic_over_algorithmic: %.4f" % (total / npts / alg)]
    with open(os.path.join(PROFILES, "traffic_adjoint_step_%s.txt" % ADJOINT_WORKLOAD), "w") as fh:
        fh.write("\n".join(txt) + "\n")
    print("profiles written to", PROFILES)


def slab_leg(prob, steps=20, warmup=3, planes=128):
    """One GPU's share of the cube split along z into slabs of `planes`
    planes (the 1024^3 cube over 8 GPUs: 1024 x 1024 x 128 each): three
    consecutive slabs around the middle of the cube, stepped with the halo
    exchange after each phase (pack into a face buffer, unpack into the
    neighbour's halo; on several GPUs the face would cross xGMI between the
    two).  HIP events on the slabs' stream time the decomposed step, the step
    kernels alone and the exchange alone."""
    import torch
    from paper_2106_11476_amd import fw2, slab
    dev = torch.device("cuda:0")
    nx, ny, nz = prob.shape
    mid = nz // 2 - planes // 2
    bounds = [0, mid - planes, mid, mid + planes, mid + 2 * planes, nz]
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        ss = slab.SlabSet(prob, bounds, device=dev, stream=stream, cap_steps=2 * steps + warmup + 4, only=[1, 2, 3])
    ss.step(warmup)
    stream.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1) / steps            # ms per step of the three slabs

    def kernels_only():
        for d in ss.domains:
            d.step_phase(fw2.PHASE_PRESSURE)
        for d in ss.domains:
            d.step_phase(fw2.PHASE_VELOCITY)

    def exchange_only():
        ss.exchange(fw2.HALO_P)
        ss.exchange(fw2.HALO_V)

    t_full = timed(lambda: ss.step(1))
    t_kern = timed(kernels_only)
    t_xch = timed(exchange_only)
    face_p = ss.domains[1].halo_numel(fw2.HALO_P) * 4
    face_v = ss.domains[1].halo_numel(fw2.HALO_V) * 4
    for d in ss.domains:
        d.check_finite(1e9)
    ss.destroy()
    npts = nx * ny * planes
    n_if = 2                                            # interfaces between the three slabs
    xch_per_slab = t_xch / n_if                         # a middle slab takes part in two
    moved = n_if * 2 * (face_p + face_v) * 4            # each face packed and unpacked: read + write twice
    return {"slab_shape": [nx, ny, planes], "grid": list(prob.shape), "slabs_timed": 3,
            "z_planes": [bounds[1], bounds[4]], "steps": steps,
            "step_ms_per_slab": round(t_full / 3, 4),
            "gpts_per_slab": round(npts / (t_full / 3 * 1e-3) / 1e9, 3),
            "kernels_ms_per_slab": round(t_kern / 3, 4),
            "exchange_ms_per_slab": round(xch_per_slab, 4),
            "exchange_over_kernels": round(xch_per_slab / (t_kern / 3), 4),
            "face_bytes_per_step": {"p": face_p, "v": face_v, "total": face_p + face_v},
            "pack_unpack_GBps": round(moved / (t_xch * 1e-3) / 1e9, 1),
            "xgmi_ms_per_face_per_step_at_153GBps": round((face_p + face_v) / (XGMI_LINK_GBS * 1e9) * 1e3, 4)}


def measure(prob, K, Wm):
    """The benchmark proper: Wm untimed steps, then K steps timed on the
    host clock around fw2_step with HIP-event timing of both kernels on the
    domain's stream."""
    import torch
    from paper_2106_11476_amd import fw2
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    t_setup = time.perf_counter()
    dom = fw2.from_problem(prob, device=dev, stream=stream, cap_steps=K + Wm)
    torch.cuda.synchronize(dev)
    setup_s = time.perf_counter() - t_setup
    dom.step(Wm)
    torch.cuda.synchronize(dev)
    dom.enable_kernel_timing(True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    dom.step(K)
    torch.cuda.synchronize(dev)
    el = time.perf_counter() - t0
    ms, cnt = dom.get_kernel_timing()
    dom.enable_kernel_timing(False)
    dom.check_finite(1e9)
    dom.destroy_domain()
    npts = prob.npts
    gpts = npts * K / el / 1e9
    labels = prob.label is not None and np.asarray(prob.relax_table).shape[0] > 1
    p_b, v_b, step_b = kernel_bytes(prob.ndim, prob.n_relax, labels)
    avg = [ms[0] / max(cnt[0], 1), ms[1] / max(cnt[1], 1)]     # ms per launch
    dom_k = 0 if avg[0] >= avg[1] else 1
    kb = (p_b, v_b)[dom_k] * npts
    achieved = kb / (avg[dom_k] * 1e-3) / 1e9
    kname = ("pressure_kernel", "velocity_kernel")[dom_k]
    roof = {"bound": "hbm", "kernel": kname,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, prob.name),
            "alg_bytes_per_point": (p_b, v_b)[dom_k], "points_per_launch": npts,
            "launch_ms": round(avg[dom_k], 5),
            "other_kernel_ms": round(avg[1 - dom_k], 5),
            "step_alg_bytes_per_point": step_b,
            "step_frac": round(gpts * step_b / HBM_PEAK_GBS, 4)}
    return {"value": round(gpts, 3), "steps": K, "warmup": Wm, "ms_per_step": round(el / K * 1e3, 5),
            "config": {"workload": prob.name, "grid": list(prob.shape), "points": npts,
                       "relax_mechanisms": prob.n_relax,
                       "labels": int(np.asarray(prob.relax_table).shape[0]),
                       "relax_scheme": "centred" if prob.relax_scheme == 1 else "printed",
                       "parallelism": "single GPU"},
            "roofline": roof,
            # host-side setup (FP64 coefficients, uploads, sources, receivers); not in the timed region
            "setup_s": round(setup_s, 3)}


def launch_leg(steps=1000):
    """The launch-bound workload (plain_2d: 480^2 points, about 23 MB moved
    per step): time per step with the steps captured in HIP graphs of 32 and
    with direct launches, beside the time the step's algorithmic bytes take
    at the HBM peak."""
    import torch
    from paper_2106_11476_amd import fw2
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    prob = make_workload("plain_2d")
    dom = fw2.from_problem(prob, device=dev, stream=stream, cap_steps=steps)
    dom.step(steps)
    torch.cuda.synchronize(dev)
    out = {"workload": prob.name, "points": prob.npts, "steps": steps}
    for mode, chunk in (("graph", 32), ("direct", 0)):
        dom.set_graph_chunk(chunk)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        dom.step(steps)
        torch.cuda.synchronize(dev)
        el = time.perf_counter() - t0
        out[mode] = {"ms_per_step": round(el / steps * 1e3, 5), "gpts": round(prob.npts * steps / el / 1e9, 3)}
    dom.destroy_domain()
    labels = prob.label is not None and np.asarray(prob.relax_table).shape[0] > 1
    step_b = kernel_bytes(prob.ndim, prob.n_relax, labels)[2]
    out["alg_bytes_per_step"] = step_b * prob.npts
    out["hbm_peak_ms_per_step"] = round(step_b * prob.npts / (HBM_PEAK_GBS * 1e9) * 1e3, 5)
    return out


def main():
    global PROFILES
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 30 for skull_3d, 12000 in 2D)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 5 for skull_3d, 200 in 2D)")
    ap.add_argument("--workload", default="skull_3d")
    ap.add_argument("--n3d", type=int, default=1024, help="cube side of the skull_3d workload")
    ap.add_argument("--relax", type=int, default=None,
                    help="relaxation mechanisms (abdominal_2d: 3..8, default 4; skull_3d: 2 or 5..8, default 2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched-serving leg")
    ap.add_argument("--serving-requests", type=int, default=16,
                    help="requests of the served workload's stream (the stated stream has 256)")
    ap.add_argument("--serving-solo-points", type=int, default=1_000_000,
                    help="serving: requests of at least this many points are stepped alone")
    ap.add_argument("--serving-solo-chunk", type=int, default=512,
                    help="serving: steps between admission points while a solo request runs")
    ap.add_argument("--serving-passes", choices=("all", "capacity", "poisson"), default="all",
                    help="serving: both passes, or the capacity or the Poisson pass alone")
    ap.add_argument("--serving-rate", type=float, default=None,
                    help="serving: arrival rate per second of the Poisson pass run alone")
    ap.add_argument("--serving-only-workload", action="store_true",
                    help="serving leg: only the served workload's stream")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) leg")
    ap.add_argument("--adjoint-steps", type=int, default=6000, help="steps of the adjoint leg's shot")
    ap.add_argument("--adjoint-shots", type=int, default=0,
                    help="also compute the whole gradient over this many shots (the workload has 64)")
    ap.add_argument("--no-local-stencil", action="store_true",
                    help="skip the leg with per-point stencil weights")
    ap.add_argument("--no-slab", action="store_true", help="skip the slab (one GPU's share) leg")
    ap.add_argument("--no-abdominal", action="store_true",
                    help="with the 3D headline, skip the 2D abdominal-wall sub-object")
    ap.add_argument("--no-launch-bound", action="store_true",
                    help="skip the launch-bound workload (plain_2d, graphs against direct launches)")
    ap.add_argument("--no-stream-reference", action="store_true",
                    help="skip the plain-copy streaming reference beside the headline roofline")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first time a plain device copy of this size (bandwidth reference, "
                         "and the known-size kernel for scaling HBM counters)")
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_DB", "FETCH_DB", "WRITE_DB"),
                    help="write profiles/*.txt from rocprofv3 result databases and exit")
    ap.add_argument("--copy-read-bytes", type=int, default=256 * (1 << 20),
                    help="bytes the probe copy reads (and writes) per dispatch")
    ap.add_argument("--commands", nargs="*", default=[])
    ap.add_argument("--summarize-stats", nargs=3, metavar=("STATS_DB", "NAME", "TITLE"),
                    help="write profiles/kernel_stats_NAME.txt from one kernel-trace database and exit")
    ap.add_argument("--calibration-probe", action="store_true",
                    help="only run the library's streaming probes on fixed buffers (for the counter-scale check) and exit")
    ap.add_argument("--summarize-calibration", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write profiles/traffic_calibration_stream_probes.txt from the two counter passes and exit")
    ap.add_argument("--summarize-adjoint", nargs=3, metavar=("STATS_DB", "FETCH_DB", "WRITE_DB"),
                    help="write the adjoint leg's kernel statistics and traffic summaries and exit")
    ap.add_argument("--profiles-dir", default=PROFILES, help="where the summaries go")
    args = ap.parse_args()
    PROFILES = args.profiles_dir
    if args.summarize_calibration:
        summarize_calibration(*args.summarize_calibration, commands=args.commands)
        return
    if args.calibration_probe:
        calibration_probe()
        return
    if args.summarize_adjoint:
        summarize_adjoint(*args.summarize_adjoint, copy_bytes=args.copy_read_bytes, commands=args.commands)
        return
    if args.summarize_stats:
        summarize_stats_only(*args.summarize_stats, commands=args.commands)
        return
    if args.summarize:
        summarize_profiles(*args.summarize, workload=args.workload, n3d=args.n3d, relax=args.relax, copy_bytes=args.copy_read_bytes,
                           commands=args.commands)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    copy_probe = None
    if args.copy_probe_mib > 0:
        copy_probe = probe_copy(torch, dev, args.copy_probe_mib)
    three_d = args.workload == "skull_3d"
    K = args.steps if args.steps is not None else (30 if three_d else 12000)
    Wm = args.warmup if args.warmup is not None else (5 if three_d else 200)
    prob = make_workload(args.workload, args.n3d, args.relax)
    head = measure(prob, K, Wm)
    out = {"metric": "Gpoint-updates/s", "value": head["value"], "unit": "Gpoint-updates/s",
           "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": head["config"], "roofline": head["roofline"],
           "setup_s": head["setup_s"]}
    print("[bench] headline %s: %.3f Gpoint-updates/s" % (prob.name, head["value"]), file=sys.stderr, flush=True)
    if copy_probe is not None:
        out["copy_probe"] = copy_probe
    if not args.no_stream_reference:
        out["stream_reference"] = stream_reference(torch, dev, out["roofline"])
    if not args.no_launch_bound:
        out["launch_bound"] = launch_leg()
    if not args.no_local_stencil:
        out["local_stencil"] = local_stencil_leg(prob, max(1, min(K, 2000)))
    if three_d and not args.no_slab and prob.shape[2] >= 512:
        out["slab"] = slab_leg(prob)
        print("[bench] slab leg done", file=sys.stderr, flush=True)
    if three_d and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    if three_d:
        del prob
    if three_d and not args.no_abdominal:
        p2 = make_workload("abdominal_2d")
        sub = measure(p2, 12000, 200)
        if not args.no_local_stencil:
            sub["local_stencil"] = local_stencil_leg(p2, 2000)
        out["workloads"] = {p2.name: sub}
        print("[bench] 2D workload done", file=sys.stderr, flush=True)
    if not args.no_serving:
        out["serving"] = serving_leg(workload_requests=args.serving_requests,
                                     only_workload=args.serving_only_workload,
                                     solo_points=args.serving_solo_points, solo_chunk=args.serving_solo_chunk,
                                     passes=args.serving_passes, rate=args.serving_rate)
        print("[bench] serving leg done", file=sys.stderr, flush=True)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(steps=args.adjoint_steps)
        print("[bench] adjoint leg done", file=sys.stderr, flush=True)
    if args.adjoint_shots > 0:
        out["adjoint_full_gradient"] = full_gradient_leg(n_shots=args.adjoint_shots, steps=args.adjoint_steps)
        print("[bench] full gradient done", file=sys.stderr, flush=True)
    if not three_d and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
