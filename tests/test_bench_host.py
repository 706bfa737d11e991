"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the
fingerprint of the code that decides the dominant kernel's traffic, and the
reading of the stored counter summary."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_fingerprint_follows_the_fingerprinted_functions_only(tmp_path, monkeypatch):
    for path, _ in bench.TRAFFIC_CODE:
        dst = tmp_path / path
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, path), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    f0 = bench.code_fingerprint()
    assert len(f0) == 16 and all(ch in "0123456789abcdef" for ch in f0)
    src = tmp_path / bench.TRAFFIC_CODE[0][0]
    text = src.read_text()
    # a change outside the fingerprinted functions keeps the fingerprint
    src.write_text(text + "\n// trailing comment\n")
    assert bench.code_fingerprint() == f0
    # a change inside one of them changes it
    sig = bench.TRAFFIC_CODE[0][1]
    a = text.index(sig)
    b = text.index("{", a) + 1
    src.write_text(text[:b] + "\n  // changed\n" + text[b:])
    assert bench.code_fingerprint() != f0
    # a missing function is reported as such
    src.write_text(text.replace(sig, "void renamed("))
    assert bench.code_fingerprint() == "missing"


def test_stored_traffic_is_used_only_for_its_kernel_workload_and_code(monkeypatch):
    kv = {}
    for line in open(bench.PMC_SUMMARY):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    stored = kv["code_fingerprint"]
    monkeypatch.setattr(bench, "code_fingerprint", lambda: stored)
    t = bench.pmc_traffic(kv["tag"], kv["workload"])
    assert t == pytest.approx(float(kv["traffic_bytes_per_launch"]))
    assert bench.pmc_traffic("another_kernel", kv["workload"]) is None
    assert bench.pmc_traffic(kv["tag"], "another_workload") is None
    monkeypatch.setattr(bench, "code_fingerprint", lambda: "0" * 16)
    assert bench.pmc_traffic(kv["tag"], kv["workload"]) is None
