"""The C-ABI library loads and exports every symbol the header declares
(no compute call: these run without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0810_1648_amd", "libgabp_svm.so")


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(gabp_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_0810_1648_amd import build
        build.build()
    return ct.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared_functions()
    for n in ["gabp_svm_create", "gabp_svm_solve", "gabp_svm_query", "gabp_svm_destroy",
              "gabp_svm_predict", "gabp_svm_solve_kernel", "gabp_svm_params_default"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_default_and_layout(lib):
    from paper_0810_1648_amd import gabp
    p = gabp.default_params()
    assert p.struct_size == ct.sizeof(gabp.Params)
    assert p.precision == gabp.PREC["mixed"] and p.diag_mode == gabp.DIAG["dominant_row"]
    assert p.diag_delta == 0.1 and p.lambda_aug < 0 and p.tol_rel == 1e-7
    assert gabp.lib().gabp_abi_version() == gabp.ABI_VERSION == 9
    assert gabp.lib().gabp_status_string(4) == b"diverged"


def test_create_rejects_bad_params_without_device(lib):
    from paper_0810_1648_amd import gabp
    for bad in ({"C": 0.0}, {"gamma": -1.0}, {"max_sweeps": 0}, {"precision": 7}):
        p = gabp.make_params(**bad)
        h = ct.c_void_p()
        assert gabp.lib().gabp_svm_create(ct.byref(p), ct.byref(h)) == gabp.E_INVALID
        assert not h.value
    p = gabp.make_params()
    p.struct_size = 8
    h = ct.c_void_p()
    assert gabp.lib().gabp_svm_create(ct.byref(p), ct.byref(h)) == gabp.E_INVALID


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_0810_1648_amd import gabp
    monkeypatch.setattr(gabp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gabp, "_lib", None)
    with pytest.raises(RuntimeError):
        gabp.lib()
