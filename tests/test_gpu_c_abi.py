"""The library from a plain C program (tests/c/abi_demo.c), without Python
in the process: host arrays in, setup, solve, the commuting-relation check
on every level; the solution matches the Python binding's and the oracle's."""
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import hcurl_oracle as O
from tests.test_abi import build_c_demo

pytestmark = pytest.mark.gpu


def test_c_program_solves_like_the_binding(tmp_path):
    import paper_2506_08284_amd as P
    pr = synth.problem(8, jitter=0.1, jitter_seed=3, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=4)
    m = 729
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    agg = pr["aggregates"][0]
    n = pr["A"][0].shape[0] - 1
    d = str(tmp_path)
    np.array([n, m, pr["A"][0][-1], agg.max() + 1], np.int64).tofile(os.path.join(d, "meta.bin"))
    for name, a in (("A_rowptr", pr["A"][0].astype(np.int64)), ("A_col", pr["A"][1].astype(np.int32)),
                    ("A_val", pr["A"][2].astype(np.float64)), ("D_rowptr", Dh[0]), ("D_col", Dh[1]),
                    ("D_val", Dh[2]), ("agg", agg.astype(np.int32)), ("f", pr["f"])):
        np.ascontiguousarray(a).tofile(os.path.join(d, name + ".bin"))
    exe = build_c_demo(d)
    print("running", exe, flush=True)
    r = subprocess.run([exe, d], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    levels, it_c, rel_c, commute = r.stdout.split()
    u_c = np.fromfile(os.path.join(d, "u.bin"), np.float64)
    H = P.Hierarchy(pr["A"], Dh, [agg], n_nodes=m)
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u)
    assert int(levels) == H.num_levels() == 2
    H.close()
    levels_o = O.setup(pr["A"], pr["tail"], pr["head"], m, [agg])
    uo, ito, _, _ = O.pcg(levels_o, pr["f"])
    assert abs(int(it_c) - it) <= 1 and abs(int(it_c) - ito) <= 1 and float(rel_c) <= 1e-8
    assert float(commute) <= 1e-12
    assert np.linalg.norm(u_c - u) <= 1e-9 * np.linalg.norm(u)
    assert np.linalg.norm(u_c - uo) <= 1e-6 * np.linalg.norm(uo)
