"""CPU checks of the C-ABI library: it loads and exports every symbol that
include/tn.h declares (no GPU work is issued)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "tn.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tn_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_core_entry_points():
    names = _declared()
    for n in ("tn_mpo_build", "tn_dmrg_sweep", "tn_energy", "tn_lbo_step", "tn_sample"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2410_18740_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string():
    from paper_2410_18740_amd import _lib
    assert _lib.lib().tn_version().decode().startswith("tn-gfx950")


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2410_18740_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    try:
        _lib.lib()
    except RuntimeError as e:
        assert "no CPU fallback" in str(e)
    else:
        raise AssertionError("expected a loud failure")
