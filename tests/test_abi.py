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


def test_options_struct_matches_header_and_rejects_unknown_names():
    """The ctypes mirror of hcurl_amg_opts has the header's fields in the
    header's order (a missing or misplaced field would shift every later
    one), the defaults come from the library, and a misspelt option is an
    error instead of a silently ignored Python attribute."""
    import pytest
    import paper_2506_08284_amd.binding as B
    txt = open(os.path.join(ROOT, "include", "hcurl_amg.h")).read()
    body = txt.split("} hcurl_amg_opts;")[0].rsplit("typedef struct {", 1)[1]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"(\w+)\s*(?:;|\)\s*\()", body)
    assert [f for f, _ in B.hcurl_amg_opts._fields_] == names
    o = B.hcurl_amg_default_opts(emin_iters=4)
    assert o.emin_iters == 4 and o.emin_omega == 0.5 and o.power_iters == 20
    with pytest.raises(TypeError):
        B.hcurl_amg_default_opts(emin_iter=4)


def build_c_demo(out_dir):
    """Compiles tests/c/abi_demo.c as C99 against include/hcurl_amg.h and
    links it to the library: the header is plain C and every symbol the
    program uses resolves."""
    import shutil
    import subprocess
    import paper_2506_08284_amd as P
    cc = shutil.which("gcc") or shutil.which("cc")
    exe = os.path.join(out_dir, "abi_demo")
    libdir = os.path.dirname(P.library_path)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c", "abi_demo.c"), "-L", libdir, "-l:libhcurl_amg.so",
                        "-Wl,-rpath," + libdir, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_caller_compiles_and_links(tmp_path):
    assert os.path.exists(build_c_demo(str(tmp_path)))
