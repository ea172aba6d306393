"""Write the FP64 oracle's results for the long-run parity tests.

Calls only the oracle (and the seeded input generator).  Each run takes a
workload at its stated step count and stores, in float32:

  trace     receiver traces, [n_steps][n_rcv / rcv_stride]: every
            rcv_stride-th receiver (1 for both runs: every receiver)
  p_dec     the final pressure on a decimated subgrid (every `stride`-th
            point along each axis, starting at 0)
  div_dec   the divergence sum_a D^-_a v_a of the final velocity at the same
            points
  drive_dec the pressure increment of one more oracle step from the final
            state at the same points: -dt S / K plus that step's sources,
            S being what the pressure phase forms from v and psi2
  peak      max |p| over the final full-resolution field and the traces

Workloads:
  abdominal   the 2D heterogeneous abdominal-wall recipe, 4096 x 2048, L = 4,
              12000 steps (stride 8)
  skull256    the 3D transcranial recipe on a 256^3 cube, L = 2, 4000 steps
              (stride 4)

The oracle needs hours on a few cores for each; --checkpoint-dir keeps the
state every --every steps so that an interrupted run resumes (a finished
run's checkpoint rewrites the output without stepping).

    python tests/golden/make_long_runs.py abdominal [--checkpoint-dir DIR]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import solver  # noqa: E402

RUNS = {
    "abdominal": dict(make=lambda: W.abdominal_2d(), stride=8, rcv_stride=1,
                      out="long_abdominal_2d_4096x2048.npz"),
    "skull256": dict(make=lambda: W.skull_3d(n=256), stride=4, rcv_stride=1,
                     out="long_skull_3d_256.npz"),
}


def decimate(f, ndim, stride):
    return f[(slice(None, None, stride),) * ndim]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("run", choices=sorted(RUNS))
    ap.add_argument("--checkpoint-dir", default=None)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--out-dir", default=HERE)
    args = ap.parse_args()
    spec = RUNS[args.run]
    prob = spec["make"]()
    n_total = int(prob.n_steps)
    t0 = time.time()
    maps = solver.coefficient_maps(prob)
    print("%s: %s, %d steps, coefficient maps %.1f s, %d threads"
          % (args.run, prob.name, n_total, time.time() - t0, solver.threads()), flush=True)
    state = solver.State(maps.ndim, maps.L, maps.grid)
    traces = []
    ck = None
    if args.checkpoint_dir:
        os.makedirs(args.checkpoint_dir, exist_ok=True)
        ck = os.path.join(args.checkpoint_dir, args.run + "_state.npz")
        if os.path.exists(ck):
            z = np.load(ck)
            state.p, state.v, state.psi1, state.psi2 = z["p"], z["v"], z["psi1"], z["psi2"]
            state.step = int(z["step"])
            traces = [z["trace"]]
            print("resumed at step %d" % state.step, flush=True)
    t0 = time.time()
    while state.step < n_total:
        n = min(args.every, n_total - state.step)
        s0 = state.step
        state, tr = solver.run(prob, n, state=state, maps=maps)
        traces.append(tr)
        el = time.time() - t0
        print("step %d / %d  %.0f s  %.2f Mpoint-updates/s"
              % (state.step, n_total, el, prob.npts * (state.step - s0) / max(el, 1e-9) / 1e6), flush=True)
        t0 = time.time()
        if ck:
            tmp = ck + ".tmp.npz"
            np.savez(tmp, p=state.p, v=state.v, psi1=state.psi1, psi2=state.psi2, step=state.step,
                     trace=np.concatenate(traces))
            os.replace(tmp, ck)
    trace = np.concatenate(traces)
    nd, s = maps.ndim, spec["stride"]
    div = solver.divergence(state.v, maps)
    p_last = state.p.copy()
    nxt, _ = solver.run(prob, 1, state=state.copy(), maps=maps, record=False)
    drive = nxt.p - p_last
    peak = max(float(np.abs(state.p).max()), float(np.abs(trace).max()))
    out = os.path.join(args.out_dir, spec["out"])
    rs = spec["rcv_stride"]
    np.savez_compressed(out, trace=trace[:, ::rs].astype(np.float32), rcv_stride=np.int64(rs),
                        p_dec=decimate(state.p, nd, s).astype(np.float32),
                        div_dec=decimate(div, nd, s).astype(np.float32),
                        drive_dec=decimate(drive, nd, s).astype(np.float32),
                        peak=np.float64(peak), stride=np.int64(s), n_steps=np.int64(n_total),
                        name=np.array(prob.name))
    print("wrote %s (peak %.6g, |p_final|max %.6g)" % (out, peak, float(np.abs(state.p).max())), flush=True)


if __name__ == "__main__":
    main()
