"""The 2D model problems of Tables 1 and 2 (Sec. 6.1) on the GPU: unit square,
n^2 nodes (n = 28, 82, 244, 730), constant sigma, random right-hand side,
tolerances as the tables list them; triangles (each square split in two,
Whitney elements) and squares (lowest-order Nedelec elements).

The library's default form (3-wide box aggregates, smoothed-aggregation
P^(n) from D^T A D, ten projected-CG iterations, multicolour symmetric
Hiptmair) is not the paper's exact configuration, so the counts are compared
loosely: for sigma <= 10 within 3 of the paper's; every row varies over the
meshes by no more than 3 or the paper's own row; the operator complexity
within 0.1 of the table's."""
import os

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table12_2d_iterations.txt")


def _table():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            kind, n, s, it, tol, edges, oc = line.split()
            rows.append((kind, int(n), float(s), int(it), float(tol), int(edges), float(oc)))
    return rows


@pytest.mark.parametrize("kind", ["tri", "quad"])
def test_tables_1_2_iterations(kind):
    import paper_2506_08284_amd as P
    rows = [r for r in _table() if r[0] == kind]
    its = {}
    for n in sorted({r[1] for r in rows}):
        N = n - 1
        mesh = synth.tri_mesh(N) if kind == "tri" else synth.quad_mesh(N)
        asm = synth.assemble_tri if kind == "tri" else synth.assemble_quad
        ncell = mesh["tris"].shape[0] if kind == "tri" else N * N
        one = np.ones(ncell)
        S, M = asm(mesh, one, "S"), asm(mesh, one, "M")
        assert np.array_equal(S[0], M[0]) and np.array_equal(S[1], M[1])
        maps, _ = synth.box_aggregates_2d(n)
        f = synth.rhs(S[0].shape[0] - 1, 11)
        Dh = synth.gradient_csr(mesh["tail"], mesh["head"])
        for _, nn, sigma, paper_it, tol, edges, oc_paper in rows:
            if nn != n:
                continue
            assert S[0].shape[0] - 1 == edges
            A = (S[0], S[1], S[2] + sigma * M[2])
            H = P.Hierarchy(A, Dh, maps, n_nodes=n * n)
            it, rel, rc = H.solve(f, np.empty_like(f), tol, 300)
            oc = H.stats()["operator_complexity"]
            H.close()
            assert rc == 0
            assert abs(oc - oc_paper) <= 0.1, (n, oc)
            its[(n, sigma)] = (it, paper_it)
            print("%s nodal %d^2 sigma %g: %d iterations (paper %d), o.c. %.3f (paper %.2f)"
                  % (kind, n, sigma, it, paper_it, oc, oc_paper))
    ns = sorted({n for n, _ in its})
    for sigma in sorted({s for _, s in its}):
        got = [its[(n, sigma)][0] for n in ns]
        paper = [its[(n, sigma)][1] for n in ns]
        assert max(got) - min(got) <= max(3, max(paper) - min(paper)), (sigma, got)
        if sigma <= 10:
            for n in ns:
                it, paper_it = its[(n, sigma)]
                assert abs(it - paper_it) <= 3, (n, sigma, it, paper_it)
