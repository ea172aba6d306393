"""Write the two-stage C-PML reflection figures the reflection pins read.

Calls only the oracle (oracle.reflection, Secs. 4.2-4.3: a point source one
wavelength above the bottom layer, 16 ppw, CFL 0.2) and the seeded input
rows of `workloads`, and stores the measured reflection in dB of each case
in tests/golden/reflection_figures.json.  The sweep takes a few minutes; the
tests compare the stored figures with the paper's and recompute one case to
show that the file matches the current oracle.

    python tests/golden/make_reflection_figures.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import reflection  # noqa: E402

ANGLES = (0, 20, 45, 60, 70, 80)


def cases():
    """(key, relaxation row, L, angles, layer and boundary settings)."""
    fit = W.tissue_row(0.5, 1.0, 2, 2e6)
    return [
        ("lossless 3+1 R_c 1e-4", W.lossless_row(1), 1, ANGLES, {"pml_Rc": 1e-4}),
        ("fitted 3+1", fit, 2, ANGLES, {}),
        ("lossless 5+1", W.lossless_row(1), 1, (0,), {"ntr_l": 5}),
        ("table2 3+1", W.TABLE2_ROW, 2, (0,), {}),
        ("table2 3+1 R_c 1e-5", W.TABLE2_ROW, 2, (0,), {"pml_Rc": 1e-5}),
        ("table2 5+1 R_c 1e-5", W.TABLE2_ROW, 2, (0,), {"ntr_l": 5, "pml_Rc": 1e-5}),
        ("table2 3+1 alpha over the transition", W.TABLE2_ROW, 2, (0,), {"pml_reading": "A_alpha_tr"}),
    ]


def measure(row, L, angles, kw):
    pml = {k: v for k, v in kw.items() if k != "ntr_l"}
    r = reflection.reflection_db(row, L, angles, ntr_l=kw.get("ntr_l", 3), **pml)
    return [float(x) for x in r]


def main():
    out = {}
    for key, row, L, angles, kw in cases():
        out[key] = {"L": L, "angles_deg": list(angles), "settings": kw, "dB": measure(row, L, angles, kw)}
        print(key, [round(x, 2) for x in out[key]["dB"]], flush=True)
    with open(os.path.join(HERE, "reflection_figures.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
