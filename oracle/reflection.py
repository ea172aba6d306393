"""Reflection of the two-stage C-PML measured with the oracle (Secs.
4.2-4.3): the measurement used by the reflection pins and by the study
below.  Test infrastructure only.

A point source sits one wavelength (D_l) above the bottom boundary layer;
run A has the layer there, run B is the same but deeper, by just enough that
its own layer sends nothing back within the window.  The reflection at
incidence angle theta is max|p_A - p_B| at a receiver at the source depth,
offset 2 D tan(theta), over the direct-wave peak at the image distance
2 D / cos(theta).  The window covers the direct wave to the image distance
and the round trip to the layer's outer wall.

    python -m oracle.reflection        prints the study behind the design notes
"""
import json
import sys

import numpy as np

import workloads as W

from . import solver

C0 = 1540.0


def reflection_db(row, L, angles, ppw=16, cfl=0.2, ntr_l=3, nbd_l=1, D_l=1.0, f0=2e6,
                   margin_l=2, **pml):
    """Reflection of the bottom two-stage layer at the given incidence
    angles: run A has the layer D_l wavelengths below a point source; run B
    is identical but deeper, by just enough that its own layer sends nothing
    back within the window.
    R = max|p_A - p_B| at a receiver at the source depth, offset 2 D tan(theta),
    over the direct-wave peak at the image distance 2 D / cos(theta).  The
    window covers the direct wave to the image distance and the round trip
    to the layer's outer wall (everything the layer sends back).  pml:
    pml_Rc, pml_cp or pml_reading overrides of the problem."""
    lam = ppw
    nb, ntr = (ntr_l + nbd_l) * lam, ntr_l * lam
    D = int(round(D_l * lam))
    offs = [int(round(2 * D * np.tan(np.radians(a)))) for a in angles]
    rimg = [2 * D / np.cos(np.radians(a)) for a in angles]
    half = max(max(offs), int(max(rimg))) + margin_l * lam
    nx = 2 * half + 2 * nb + 1
    top = margin_l * lam
    ny_a = nb + top + D + nb
    wall = 2.0 * np.sqrt((D + nb) ** 2 + (0.5 * max(offs)) ** 2)
    # window in cells of travel: the farther arrival plus 4 wavelengths, then
    # the pulse length (12 envelope deviations = 9 cycles at 3 cycles); run
    # B's layer starts so far down that a round trip to it is longer
    reach = max(max(rimg), wall) + 4 * lam + 9 * lam
    ext = int(np.ceil(max(0.0, reach / 2.0 - D))) + lam
    res = {}
    for name, ny in (("A", ny_a), ("B", ny_a + ext)):
        prob = W.homogeneous((nx, ny), L=L, row=row, nb=(nb, nb), ntr=(ntr, ntr), f0=f0, ppw=ppw, cfl=cfl)
        for k, v in pml.items():
            setattr(prob, k, v)
        h, dt = prob.h, prob.dt
        sx, sy = nx // 2, nb + top
        npulse = W.pulse_length(dt, f0, 3)
        nt = int((max(max(rimg), wall) + 4 * lam) * h / C0 / dt) + npulse
        prob.src_idx = prob.flat(np.array([sx]), np.array([sy]))
        prob.src_sig = np.zeros(1, np.int32)
        prob.src_w = np.ones(1, np.float32)
        prob.signals = W.gaussian_pulse(npulse, dt, f0, 3, 1.0)[None]
        rx = np.array([sx + o for o in offs] + [sx - int(round(r)) for r in rimg])
        prob.rcv_idx = prob.flat(rx, np.full(rx.size, sy))
        _, res[name] = solver.run(prob, nt)
    A, B = res["A"], res["B"]
    n = len(angles)
    return np.array([20 * np.log10(np.abs(A[:, k] - B[:, k]).max() / np.abs(B[:, n + k]).max())
                     for k in range(n)])


STUDY_ANGLES = (0, 10, 20, 30, 40, 45, 50, 60, 70, 80)


def study():
    """Yield (label, angles, dB) over media, layer thickness, R_c, c_p, N and
    the boundary readings (lossless special case, the fitted 0.5 dB/MHz/cm
    tissue, Table 2)."""
    fit = W.tissue_row(0.5, 1.0, 2, 2e6)
    cases = [
        ("lossless 3+1", W.lossless_row(1), 1, STUDY_ANGLES, {}),
        ("lossless 3+1 R_c 1e-4", W.lossless_row(1), 1, STUDY_ANGLES, {"pml_Rc": 1e-4}),
        ("fitted 3+1", fit, 2, STUDY_ANGLES, {}),
        ("fitted 3+1 R_c 1e-4", fit, 2, STUDY_ANGLES, {"pml_Rc": 1e-4}),
        ("table2 3+1", W.TABLE2_ROW, 2, STUDY_ANGLES, {}),
        ("table2 3+1 R_c 1e-5", W.TABLE2_ROW, 2, STUDY_ANGLES, {"pml_Rc": 1e-5}),
        ("table2 3+1 alpha over the transition", W.TABLE2_ROW, 2, STUDY_ANGLES, {"pml_reading": "A_alpha_tr"}),
        ("table2 3+1 kappa-scaled target", W.TABLE2_ROW, 2, (0,), {"pml_reading": "A_kappa"}),
        ("table2 3+1 reading B", W.TABLE2_ROW, 2, (0,), {"pml_reading": "B"}),
        ("lossless 3+1 reading B", W.lossless_row(1), 1, (0,), {"pml_reading": "B"}),
    ]
    for N in (1, 3, 4):
        cases.append(("table2 3+1 N %d" % N, W.TABLE2_ROW, 2, (0,), {"pml_npoly": N}))
    for rc in (1e-2, 1e-4):
        cases.append(("table2 3+1 R_c %g" % rc, W.TABLE2_ROW, 2, (0,), {"pml_Rc": rc}))
    for f in (0.7, 1.5):
        cases.append(("table2 3+1 c_p %.1f c" % f, W.TABLE2_ROW, 2, (0,), {"pml_cp": f * C0}))
    for label, row, L, rc in (("lossless", W.lossless_row(1), 1, 1e-3), ("fitted", fit, 2, 1e-3),
                              ("fitted", fit, 2, 1e-4), ("table2", W.TABLE2_ROW, 2, 1e-3),
                              ("table2", W.TABLE2_ROW, 2, 1e-5)):
        cases.append(("%s 5+1 R_c %g" % (label, rc), row, L, (0,), {"ntr_l": 5, "pml_Rc": rc}))
    for label, row, L, angles, kw in cases:
        pml = {k: v for k, v in kw.items() if k != "ntr_l"}
        r = reflection_db(row, L, angles, ntr_l=kw.get("ntr_l", 3), **pml)
        yield label, angles, [round(float(x), 2) for x in r]


if __name__ == "__main__":
    for label, angles, r in study():
        print(json.dumps({"case": label, "angles_deg": list(angles), "dB": r}), flush=True)
    sys.exit(0)
