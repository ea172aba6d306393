"""Host logic of the benchmark script: the one-GPU refusal, the algorithmic
byte accounting of the roofline, the gate that withholds measured traffic
once the kernel source has changed, and the workload names that key the
committed counter summaries.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _arrays(ndim, L, labels):
    """Arrays each kernel touches once per point, listed one by one (Sec. 3.1
    leapfrog with the memory variables of Sec. 3.2): (name, bytes)."""
    lab = [("label", 1)] if labels else []
    f = 4
    pres_read = [("v%d" % a, f) for a in range(ndim)] + [("p", f)] + \
        [("psi2_%d_%d" % (a, l), f) for a in range(ndim) for l in range(L)] + \
        [("kappa0", f), ("kappa0_nl", f)] + lab
    pres_write = [("p", f)] + [("psi2_%d_%d" % (a, l), f) for a in range(ndim) for l in range(L)]
    vel_read = [("p", f)] + [("v%d" % a, f) for a in range(ndim)] + \
        [("psi1_%d_%d" % (a, l), f) for a in range(ndim) for l in range(L)] + \
        [("rho", f), ("kappa0", f)] + lab
    vel_write = [("v%d" % a, f) for a in range(ndim)] + \
        [("psi1_%d_%d" % (a, l), f) for a in range(ndim) for l in range(L)]
    state = {n for n, _ in pres_write + vel_write}
    medium = {"kappa0", "kappa0_nl", "rho"}
    step = 2 * f * len(state) + f * len(medium) + (1 if labels else 0)
    return (sum(b for _, b in pres_read + pres_write), sum(b for _, b in vel_read + vel_write), step)


@pytest.mark.parametrize("ndim,L,labels", [(2, 4, True), (2, 8, True), (3, 2, True), (3, 8, True),
                                           (2, 1, False), (3, 5, False)])
def test_algorithmic_bytes_match_the_arrays_each_kernel_touches(ndim, L, labels):
    assert bench.kernel_bytes(ndim, L, labels) == _arrays(ndim, L, labels)


def test_benchmark_configuration_bytes():
    """The figures quoted for the benchmark lines: 2D L = 4 velocity 93 B and
    step 165 B; 3D L = 2 pressure 77 B, velocity 85 B, step 141 B."""
    assert bench.kernel_bytes(2, 4, True) == (89, 93, 165)
    assert bench.kernel_bytes(3, 2, True) == (77, 85, 141)


def test_traffic_is_withheld_when_the_kernel_source_changed(tmp_path, monkeypatch):
    path = tmp_path / "traffic_velocity_kernel_w.txt"
    path.write_text("kernel_source_sha256_16: abc\nhbm_bytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda *a: "abc")
    assert bench.measured_traffic("velocity_kernel", "w") == 1234
    monkeypatch.setattr(bench, "kernel_source_sha", lambda *a: "def")
    assert bench.measured_traffic("velocity_kernel", "w") is None
    assert bench.measured_traffic("velocity_kernel", "missing") is None


def test_workload_names_carry_the_mechanism_count():
    assert bench.make_workload("skull_3d", 32).name == "skull_3d_32"
    assert bench.make_workload("skull_3d", 32, 8).name == "skull_3d_32_L8"
    with pytest.raises(SystemExit):
        bench.make_workload("plain_2d", relax=3)
    with pytest.raises(ValueError):
        bench.make_workload("skull_3d", 32, 4)


def test_stream_reference_relates_the_kernel_to_a_plain_copy(monkeypatch):
    """The stream reference relates the dominant kernel's algorithmic and
    measured-traffic rates to torch's copy and to the library's probes."""
    import bench
    from paper_2106_11476_amd import fw2
    monkeypatch.setattr(bench, "probe_copy", lambda torch, dev, mib, reps=10: {
        "bytes_per_copy": 2 * mib * (1 << 20), "ms": 1.0, "GBps": 5000.0, "reps": reps})
    rates = {fw2.PROBE_COPY: 6250.0, fw2.PROBE_VELOCITY_MIX: 5200.0}
    monkeypatch.setattr(bench, "library_probe", lambda torch, dev, kind, nbytes, reps=10: {
        "bytes": nbytes, "ms": 1.0, "GBps": rates[kind], "reps": reps})
    roof = {"achieved": 4000.0, "traffic": 10 * 10 ** 9, "launch_ms": 2.0}
    r = bench.stream_reference(None, None, roof)
    assert r["kernel_algorithmic_over_copy"] == 0.8
    assert r["kernel_traffic_GBps"] == 5000.0 and r["kernel_traffic_over_copy"] == 1.0
    assert r["kernel_algorithmic_over_copy16"] == 0.64
    assert r["kernel_traffic_over_velocity_mix"] == round(5000.0 / 5200.0, 3)
    assert r["probe_copy16"]["GBps"] == 6250.0 and r["probe_velocity_mix"]["GBps"] == 5200.0
    r = bench.stream_reference(None, None, {"achieved": 4000.0, "traffic": None, "launch_ms": 2.0})
    assert "kernel_traffic_GBps" not in r


def test_calibration_summary_reads_the_counter_scale_of_each_probe(tmp_path, monkeypatch):
    """summarize_calibration divides the bytes each probe must move by the
    counters' KiB per dispatch (fake databases with the pmc_events table)."""
    import sqlite3
    from paper_2106_11476_amd import fw2

    def db(path, values):
        con = sqlite3.connect(path)
        con.execute("create table pmc_events (name text, counter_value real)")
        for name, v in values:
            con.executemany("insert into pmc_events values (?, ?)", [(name, v)] * 3)
        con.commit()
        con.close()
        return str(path)

    n_copy = fw2.stream_probe_elements(fw2.PROBE_COPY, bench.CALIBRATION_BYTES["copy16"])
    n_mix = fw2.stream_probe_elements(fw2.PROBE_VELOCITY_MIX, bench.CALIBRATION_BYTES["mix"])
    kib = lambda b: b / 1024.0
    f = db(tmp_path / "f.db", [("ns::probe_copy16(args)", kib(16 * n_copy) / 2), ("ns::probe_mix(args)", kib(48 * n_mix) / 2)])
    w = db(tmp_path / "w.db", [("ns::probe_copy16(args)", kib(16 * n_copy)), ("ns::probe_mix(args)", kib(36 * n_mix))])
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    bench.summarize_calibration(f, w, ["cmd"])
    vals = bench._profile_values(str(tmp_path / "traffic_calibration_stream_probes.txt"))
    assert vals["copy16_fetch_scale"] == "2.0000" and vals["mix_fetch_scale"] == "2.0000"
    assert vals["copy16_write_scale"] == "1.0000" and vals["mix_write_scale"] == "1.0000"
