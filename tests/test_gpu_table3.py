"""The 3D model problems of Table 3 (Sec. 6.1) on the GPU: unit cube, n^3
nodes (n = 10, 28, 82), constant sigma, random right-hand side, tolerances
as the table lists them; tetrahedral (six-tet split, Whitney elements) and
hexahedral (lowest-order Nedelec elements) meshes.

The library's default form (box aggregates, smoothed-aggregation P^(n) from
D^T A D, ten projected-CG energy-minimisation iterations, multicolour
symmetric Hiptmair) is not the paper's exact configuration (aggregates from
its SA package, one projected-Jacobi step, lexicographic Gauss-Seidel), so
the counts are compared loosely:
* for sigma <= 10 the iterations vary by at most 3 over the three meshes and
  lie within 3 of the paper's count;
* for sigma = 1e2 the default form needs 8-12 iterations where the paper
  reports 4-9; that row may grow over the meshes by no more than the
  paper's own row does (5)."""
import os

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_tet_iterations.txt")
GOLDEN_HEX = os.path.join(os.path.dirname(__file__), "golden", "table3_hex_iterations.txt")


def _table(path=GOLDEN):
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            n, s, it, tol = line.split()
            rows.append((int(n), float(s), int(it), float(tol)))
    return rows


def test_table3_tet_iterations():
    import paper_2506_08284_amd as P
    its = {}
    for n, sigma, paper_it, tol in _table():
        pr = synth.problem(n - 1, sigma=("const", sigma), f_seed=11)
        assert pr["A"][0].shape[0] - 1 == {10: 5859, 28: 144423, 82: 3779379}[n]
        H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=n ** 3)
        it, rel, rc = H.solve(pr["f"], np.empty(pr["A"][0].shape[0] - 1), tol, 300)
        H.close()
        assert rc == 0
        its[(n, sigma)] = (it, paper_it)
        print("nodal %d^3 sigma %g: %d iterations (paper %d)" % (n, sigma, it, paper_it))
    for sigma in sorted({s for _, s in its}):
        got = [its[(n, sigma)][0] for n in (10, 28, 82)]
        paper = [its[(n, sigma)][1] for n in (10, 28, 82)]
        assert max(got) - min(got) <= max(3, max(paper) - min(paper)), (sigma, got)
        if sigma <= 10:
            for n in (10, 28, 82):
                it, paper_it = its[(n, sigma)]
                assert abs(it - paper_it) <= 3, (n, sigma, it, paper_it)


def test_table3_hex_iterations():
    """Hex column: for sigma <= 10 every count within 2 of the paper's (the
    default form gives 5-7 where the paper lists 4-6); for sigma = 1e2, where
    the paper needs 3, within 3; every row varies by at most 2 over the
    meshes; the operator complexity within 0.01 of the table's (1.09, 1.06,
    1.05)."""
    import paper_2506_08284_amd as P
    its = {}
    oc_paper = {10: 1.09, 28: 1.06, 82: 1.05}
    rows = _table(GOLDEN_HEX)
    for n in (10, 28, 82):
        mesh = synth.hex_mesh(n - 1)
        one = np.ones((n - 1) ** 3)
        S = synth.assemble_hex(mesh, one, "S")
        M = synth.assemble_hex(mesh, one, "M")
        assert np.array_equal(S[0], M[0]) and np.array_equal(S[1], M[1])
        assert S[0].shape[0] - 1 == {10: 2700, 28: 63504, 82: 1633932}[n]
        maps, _ = synth.box_aggregates(n)
        f = synth.rhs(S[0].shape[0] - 1, 11)
        Dh = synth.gradient_csr(mesh["tail"], mesh["head"])
        for nn, sigma, paper_it, tol in rows:
            if nn != n:
                continue
            A = (S[0], S[1], S[2] + sigma * M[2])
            H = P.Hierarchy(A, Dh, maps, n_nodes=n ** 3)
            it, rel, rc = H.solve(f, np.empty_like(f), tol, 300)
            oc = H.stats()["operator_complexity"]
            H.close()
            assert rc == 0
            assert abs(oc - oc_paper[n]) <= 0.01, (n, oc)
            its[(n, sigma)] = (it, paper_it)
            print("hex nodal %d^3 sigma %g: %d iterations (paper %d), o.c. %.3f" % (n, sigma, it, paper_it, oc))
    for (n, sigma), (it, paper_it) in its.items():
        assert abs(it - paper_it) <= (2 if sigma <= 10 else 3), (n, sigma, it, paper_it)
    for sigma in sorted({s for _, s in its}):
        got = [its[(n, sigma)][0] for n in (10, 28, 82)]
        assert max(got) - min(got) <= 2, (sigma, got)
