"""Write workloads/tissue_fits.json: relaxation tuples fitted with oracle.fit.

The synthetic workloads draw tissue attenuation (alpha0 in dB/cm/MHz^y and the
exponent y) from a small grid; each grid point needs a relaxation tuple that
reproduces alpha0 f^y over 1-20 MHz (Sec. 4.1).  This script computes them
once with the oracle's fitter and stores them as plain input data.

    python -m oracle.make_tissue_fits [--jobs N] [--missing]
"""
import argparse
import json
import os
from concurrent.futures import ProcessPoolExecutor

from oracle import fit

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "workloads", "tissue_fits.json")

ALPHA0_GRID = [0.4, 0.6, 0.8, 1.0, 1.2, 1.5]
Y_GRID = [1.0, 1.1, 1.2, 1.3]


def key(alpha0, y, L, f_ref):
    return "a%.2f_y%.2f_L%d_f%.1f" % (alpha0, y, L, f_ref / 1e6)


def wanted():
    jobs = [(0.5, 1.1, 2, 2e6),        # plain 2D water-like medium
            (8.0, 1.0, 2, 1e6),        # 3D bone-like shell
            (0.5, 1.0, 2, 2e6)]        # adjoint workload background
    for L in (2, 3, 4):
        for a0 in ALPHA0_GRID:
            for y in Y_GRID:
                jobs.append((a0, y, L, 3e6))
    for L in (5, 6, 7, 8):                # more mechanisms than the workloads use
        jobs.append((1.5, 1.3, L, 3e6))
        jobs.append((0.5, 1.0, L, 3e6))
    return jobs


def _one(job):
    a0, y, L, f_ref = job
    row, info = fit.fit_power_law(a0, y, L, f_ref=f_ref, n_random=3, seed=1)
    return key(a0, y, L, f_ref), {"alpha0": a0, "y": y, "L": L, "row": [float(v) for v in row], **info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--missing", action="store_true", help="keep the stored fits, compute only absent ones")
    args = ap.parse_args()
    out = {}
    jobs = wanted()
    if args.missing and os.path.exists(OUT):
        with open(OUT) as fh:
            out = json.load(fh)["fits"]
        jobs = [j for j in jobs if key(*j) not in out]
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for k, v in ex.map(_one, jobs):
            out[k] = v
            print(k, "att_err %.4f vel_err %.2e" % (v["max_att_err"], v["max_vel_err"]), flush=True)
    out = dict(sorted(out.items()))
    with open(OUT, "w") as fh:
        json.dump({"generator": "oracle/make_tissue_fits.py",
                   "columns": "k1, k2, d1[L], d2[L], alpha1[L], alpha2[L]",
                   "fits": out}, fh, indent=1)
    print("wrote", OUT, len(out))


if __name__ == "__main__":
    main()
