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
