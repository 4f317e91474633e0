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


def test_binding_structs_match_the_header(tmp_path):
    """Every structure the binding mirrors has the header's size and field
    offsets: a small C program built with gcc from include/tn.h prints
    sizeof and offsetof, compared with ctypes'."""
    import shutil
    import subprocess
    import pytest
    from paper_2410_18740_amd import _lib as L
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    structs = [getattr(L, n) for n in dir(L)
               if n.startswith("tn_") and isinstance(getattr(L, n), type) and issubclass(getattr(L, n), ctypes.Structure)]
    assert len(structs) >= 7
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HDR}"', "int main(void) {"]
    for S in structs:
        lines.append(f'  printf("{S.__name__} size %zu\\n", sizeof({S.__name__}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{S.__name__} {f} %zu\\n", offsetof({S.__name__}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True, capture_output=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, val = ln.split()
        got[(name, field)] = int(val)
    for S in structs:
        assert got[(S.__name__, "size")] == ctypes.sizeof(S), S.__name__
        for f, _ in S._fields_:
            assert got[(S.__name__, f)] == getattr(S, f).offset, (S.__name__, f)
