"""The C-ABI library loads (no GPU needed) and exports every symbol include/cpm.h declares."""
import ctypes
import os
import re

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(REPO, "include", "cpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("cpm_build_band", "cpm_apply", "cpm_vcycle", "cpm_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1307_4354_amd as cpm

    lib = ctypes.CDLL(cpm.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    import paper_1307_4354_amd as cpm
    from paper_1307_4354_amd.binding import _lib

    assert _lib.cpm_status_string(cpm.CPM_OK) == b"ok"
    assert _lib.cpm_status_string(cpm.CPM_E_BAND) == b"stencil leaves the band"


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    """Without the native library the package does not import (no fallback path)."""
    import importlib.util
    import sys

    spec = importlib.util.spec_from_file_location(
        "cpm_binding_probe", os.path.join(REPO, "paper_1307_4354_amd", "binding.py"))
    mod = importlib.util.module_from_spec(spec)
    monkeypatch.setattr(os.path, "exists", lambda p: False if p.endswith("libcpm.so") else os.path.isfile(p))
    try:
        spec.loader.exec_module(mod)
    except ImportError:
        return
    raise AssertionError("binding imported without libcpm.so")
