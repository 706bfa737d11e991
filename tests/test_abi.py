"""The C-ABI library loads and exports every function include/hcurl_amg.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hcurl_amg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hcurl_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2506_08284_amd as P
    lib = ctypes.CDLL(P.library_path)
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.EXPORTED_SYMBOLS) == names


def test_error_strings_without_gpu():
    import paper_2506_08284_amd as P
    assert P.hcurl_error_string(P.HCURL_EREDUCIBLE).startswith("disconnected")
    assert P.hcurl_error_string(0) == "ok"
