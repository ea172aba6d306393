"""The stored oracle results of the long-run parity tests
(tests/golden/make_long_runs.py) describe the workloads the GPU tests run:
name, step count, receiver count, decimation and array shapes."""
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FILES = [("long_abdominal_2d_4096x2048.npz", lambda: W.abdominal_2d(), 8),
         ("long_skull_3d_256.npz", lambda: W.skull_3d(n=256), 4)]


@pytest.mark.parametrize("fname,make,stride", FILES, ids=[f[0] for f in FILES])
def test_stored_long_run_matches_its_workload(fname, make, stride):
    z = np.load(os.path.join(GOLDEN, fname))
    prob = make()
    assert str(z["name"]) == prob.name
    assert int(z["n_steps"]) == prob.n_steps and int(z["stride"]) == stride
    rs = int(z["rcv_stride"])
    assert z["trace"].shape == (prob.n_steps, len(range(0, len(prob.rcv_idx), rs)))
    dec = tuple(len(range(0, n, stride)) for n in prob.shape[::-1])
    for key in ("p_dec", "div_dec", "drive_dec"):
        assert z[key].shape == dec, key
        assert np.all(np.isfinite(z[key])), key
    peak = float(z["peak"])
    assert peak > 0 and np.abs(z["trace"]).max() <= peak
