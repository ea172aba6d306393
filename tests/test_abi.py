"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/fw2.h declares, and its host-only validation (fw2_workspace_bytes)
rejects bad descriptors.  No compute call is made here (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2106_11476_amd import fw2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fw2.h")).read()
    return sorted(set(re.findall(r"\b(fw2_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = fw2.lib()
    declared = _declared()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(fw2.EXPORTS) == declared


def test_desc_struct_matches_header_layout():
    # offsets of a few fields must match the C layout (natural alignment)
    assert fw2.DomainDesc.n.offset == 8
    assert fw2.DomainDesc.h.offset == 32
    assert ctypes.sizeof(fw2.DomainDesc) % 8 == 0


def test_workspace_bytes_counts_every_array():
    prob = W.plain_2d()
    nb = fw2.workspace_bytes(prob)
    pitch = ((480 + 8 + 63) // 64) * 64
    stride = pitch * (480 + 8)
    n_arrays = 1 + 2 + 2 * 2 * 2 + 3
    assert nb >= n_arrays * stride * 4
    assert nb < n_arrays * stride * 4 + 1 << 20
    prob3 = W.homogeneous((20, 18, 16), L=3, nb=(4, 4, 4))
    assert fw2.workspace_bytes(prob3) >= (1 + 3 + 18 + 3) * 16 * 24 * 26 * 4


@pytest.mark.parametrize("mutate,msg", [
    (lambda p: setattr(p, "bound_cells", (300, 48)), "wider"),
    (lambda p: setattr(p, "trans_cells", (60, 30)), "trans_cells"),
    (lambda p: setattr(p, "n_relax", 9), "n_relax"),
    (lambda p: setattr(p, "dt", -1.0), "positive"),
    (lambda p: setattr(p, "pml_Rc", 1.5), "pml_Rc"),
    (lambda p: setattr(p, "relax_scheme", 3), "relax_scheme"),
    (lambda p: setattr(p, "relax_table", np.array([[0.0, 1.0, 1, 1, 1, 1, 1, 1, 1, 1]])), "kappa"),
    (lambda p: setattr(p, "relax_table", np.array([[1.0, 1.0, -1, 1, 1, 1, 1, 1, 1, 1]])), ">= 0"),
    (lambda p: setattr(p, "nonlinear_form", 3), "nonlinear_form"),
    (lambda p: (setattr(p, "nonlinear_form", 1), setattr(p, "nl_A", float("inf"))), "finite"),
    (lambda p: setattr(p, "slab_nz", 480), "slab domains are 3D"),
    # 2D sweeps address the padded grid with 32-bit byte offsets
    (lambda p: setattr(p, "shape", (32768, 32768)), "2^30"),
    (lambda p: setattr(p, "shape", (1 << 20, 1100)), "2^30"),
])
def test_workspace_bytes_rejects_bad_descriptors(mutate, msg):
    prob = W.plain_2d()
    mutate(prob)
    with pytest.raises(fw2.Fw2Error) as e:
        fw2.workspace_bytes(prob)
    assert e.value.status == 1 and msg in str(e.value)


def test_null_arguments_are_rejected_without_a_gpu():
    lib = fw2.lib()
    out = ctypes.c_uint64()
    assert lib.fw2_workspace_bytes(None, ctypes.byref(out)) == 1
    assert lib.fw2_step(None, 1) == 4
    assert lib.fw2_current_step(None) == -1
    lib.fw2_destroy_domain(None)
    d, keep = fw2.make_desc(W.plain_2d())
    h = ctypes.c_void_p()
    assert lib.fw2_create_domain(ctypes.byref(d), None, 0, ctypes.byref(h)) == 1
    assert b"workspace" in lib.fw2_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; there is no CPU
    fallback of any step."""
    monkeypatch.setattr(fw2, "LIB_PATH", str(tmp_path / "libfw2.so"))
    monkeypatch.setattr(fw2, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        fw2.lib()


def test_product_package_does_not_import_the_oracle():
    """The oracle is test infrastructure: no module of the package refers to it."""
    pkg = os.path.join(ROOT, "paper_2106_11476_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            src = open(os.path.join(pkg, name)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", src, re.M), name
            assert "from oracle" not in src and "import oracle" not in src, name


def test_two_dimensional_grids_just_below_the_offset_limit_are_accepted():
    """(nx + 72)(ny + 8) < 2^30 is the 2D limit; only scalars are read."""
    prob = W.plain_2d()
    prob.shape = (32000, 33000)
    assert fw2.workspace_bytes(prob) > 32000 * 33000 * 4
    prob.shape = (32697, 32759)                     # (nx + 72)(ny + 8) = 2^30 - 1: the largest accepted
    assert fw2.workspace_bytes(prob) > 32697 * 32759 * 4
    for shape in ((32698, 32759), (32697, 32760)):  # one column or one row more
        prob.shape = shape
        with pytest.raises(fw2.Fw2Error, match="2\\^30"):
            fw2.workspace_bytes(prob)


def _slab_problem(**kw):
    prob = W.homogeneous((24, 20, 16), L=2, nb=(4, 4, 4))
    prob.slab_z0, prob.slab_nz = 8, 40
    prob.fd_r, prob.pml_cp = 0.4, 1540.0
    for k, v in kw.items():
        setattr(prob, k, v)
    return prob


def test_slab_descriptors_are_validated():
    assert fw2.workspace_bytes(_slab_problem()) > 0
    for kw, msg in [(dict(slab_z0=30), "slab_z0"), (dict(slab_z0=-1), "slab_z0"),
                    (dict(fd_r=0.0), "fd_r"), (dict(pml_cp=0.0), "pml_cp"),
                    (dict(shape=(24, 20, 3), slab_z0=0), "4 planes"),
                    (dict(bound_cells=(4, 4, 21), trans_cells=(3, 3, 3)), "wider")]:
        with pytest.raises(fw2.Fw2Error) as e:
            fw2.workspace_bytes(_slab_problem(**kw))
        assert e.value.status == 1 and msg in str(e.value), (kw, str(e.value))
    # a slab's boundary layers may exceed its own planes (they follow the whole grid)
    assert fw2.workspace_bytes(_slab_problem(bound_cells=(4, 4, 12), trans_cells=(3, 3, 9))) > 0


def test_halo_and_phase_calls_reject_null_domains():
    lib = fw2.lib()
    n = ctypes.c_uint64()
    assert lib.fw2_halo_bytes(None, 0, ctypes.byref(n)) == 4
    assert lib.fw2_halo_pack(None, 0, 0, None) == 4
    assert lib.fw2_halo_unpack(None, 0, 0, None) == 4
    assert lib.fw2_step_phase(None, 0) == 4


def test_desc_layout_matches_the_c_compiler():
    """Every field offset of the ctypes descriptor equals offsetof() in a C
    program built from include/fw2.h."""
    import subprocess
    import tempfile
    fields = [f[0] for f in fw2.DomainDesc._fields_]
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "layout.c")
        with open(src, "w") as fh:
            fh.write('#include <stdio.h>\n#include <stddef.h>\n#include "fw2.h"\nint main(void){\n')
            for f in fields:
                fh.write('printf("%%s %%zu\\n", "%s", offsetof(fw2_domain_desc, %s));\n' % (f, f))
            fh.write('printf("sizeof %zu\\n", sizeof(fw2_domain_desc));\nreturn 0;}\n')
        exe = os.path.join(td, "layout")
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", exe, src])
        out = subprocess.check_output([exe]).decode().split("\n")
    got = dict(line.split() for line in out if line.strip())
    for f in fields:
        assert int(got[f]) == getattr(fw2.DomainDesc, f).offset, f
    assert int(got["sizeof"]) == ctypes.sizeof(fw2.DomainDesc)


def test_relaxation_maps_become_labels_and_a_table():
    """fw2_label_relaxation_map (host only): the returned table indexed by the
    labels reproduces every dense map bitwise, rows appear in order of first
    appearance, and more than 256 distinct tuples are refused."""
    rng = np.random.default_rng(7)
    L = 3
    rows = rng.uniform(0.5, 2.0, (11, 2 + 4 * L))
    lab = rng.integers(0, 9, (37, 53))                 # rows 9, 10 unused
    maps = np.moveaxis(rows[lab], -1, 0)              # [2 + 4L] + grid
    got_lab, table = fw2.label_relaxation_map(maps, L)
    assert got_lab.shape == lab.shape and table.shape[1] == 2 + 4 * L
    assert np.array_equal(np.moveaxis(table[got_lab], -1, 0), maps)
    first = [int(x) for x in dict.fromkeys(lab.reshape(-1).tolist())]
    assert np.array_equal(table, rows[first])
    assert len(table) == len(set(lab.reshape(-1).tolist()))
    many = np.moveaxis(rng.uniform(1, 2, (300, 2 + 4 * L)), -1, 0)[:, :, None]
    with pytest.raises(fw2.Fw2Error, match="256"):
        fw2.label_relaxation_map(many, L)
    with pytest.raises(ValueError):
        fw2.label_relaxation_map(maps[:-1], L)
