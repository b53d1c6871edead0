"""The C-ABI library loads and exports every entry point include/matsgw.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "matsgw.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(msgw_[a-zA-Z0-9_]+)\s*\(", txt)))


def test_header_declares_the_hot_path():
    names = declared()
    for n in ["msgw_polarization", "msgw_screen", "msgw_self_energy", "msgw_tau_to_iw",
              "msgw_iw_to_tau", "msgw_dyson", "msgw_sigma_x", "msgw_green0", "msgw_screened_tau"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1602_02313_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmatsgw.so not built")
    _lib.load_library()                      # loads torch's HIP runtime first
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == declared()
    # the binding declares a signature for each
    _lib.load_library()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1602_02313_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load_library()
