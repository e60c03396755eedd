"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/hns.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hns.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hns_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libhns():
    from paper_1207_0486_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1207_0486_amd import build
        build.build()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hns_assemble", "hns_solve", "hns_solve_batched", "hns_footprint_bytes",
                     "hns_operator_destroy", "hns_status_string", "hns_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(libhns):
    missing = [n for n in declared_functions() if not hasattr(libhns, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1207_0486_amd import _lib
    assert set(declared_functions()) <= set(_lib.exported_names())


def test_status_strings_without_gpu(libhns):
    libhns.hns_status_string.restype = ctypes.c_char_p
    libhns.hns_status_string.argtypes = [ctypes.c_int]
    assert libhns.hns_status_string(0) == b"ok"
    assert libhns.hns_status_string(-5) == b"CG breakdown"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1207_0486_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.LibraryMissing):
        _lib.lib()
