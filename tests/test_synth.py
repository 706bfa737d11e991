"""Pins of the synthetic problem generator (not of the method)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_edge_counts():
    rows = []
    for line in open(os.path.join(GOLDEN, "table3_edge_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, kind, cnt = line.split()
        rows.append((int(n), kind, int(cnt)))
    return rows


@pytest.mark.parametrize("n,kind,count", _golden_edge_counts())
def test_edge_counts_table3(n, kind, count):
    """#edges of Table 3 for n^3 nodal meshes (tets: six-tet split)."""
    N = n - 1
    if kind == "tet":
        assert synth.edge_count(N) == count
        eptr = np.empty(n ** 3 + 1, np.int64)
        assert synth._lib().synth_edge_ptr(N, synth._p(eptr)) == count
    else:
        assert 3 * N * (N + 1) ** 2 == count
        if n <= 28:
            assert len(synth.hex_mesh(N)["tail"]) == count


def _grad(tail, head, m):
    n = len(tail)
    return sp.csr_matrix((np.tile([-1.0, 1.0], n), (np.repeat(np.arange(n), 2), np.stack([tail, head], 1).ravel())),
                         shape=(n, m))


def _mat(t):
    rowptr, col, val = t
    return sp.csr_matrix((val, col, rowptr), shape=(len(rowptr) - 1, len(rowptr) - 1))


@pytest.mark.parametrize("N,jit", [(3, 0.0), (5, 0.2)])
def test_curl_grad_null_space(N, jit):
    """S D_h = 0 (Sec. 1, eq. "discrete null space condition")."""
    mesh = synth.kuhn_mesh(N, jit, 7)
    sig = synth.sigma_lognormal(mesh, 3, 1.0)
    S = _mat(synth.assemble(mesh, sig, "S"))
    D = _grad(mesh["tail"], mesh["head"], mesh["n"] ** 3)
    assert abs(S @ D).max() <= 1e-13 * abs(S).max()


def _p1_stiffness(mesh, sig):
    """Independent P1 assembly: sum over tets of sigma |T| grad(l_a).grad(l_b)."""
    X = mesh["coords"]
    m = X.shape[0]
    rows, cols, vals = [], [], []
    for t, tv in enumerate(mesh["tets"]):
        M = np.ones((4, 4))
        M[:, 1:] = X[tv]
        C = np.linalg.inv(M)  # columns: coefficients of barycentric functions
        grads = C[1:, :].T  # row a = grad lambda_a
        vol = abs(np.linalg.det(M)) / 6.0
        K = sig[t] * vol * grads @ grads.T
        for a in range(4):
            for b in range(4):
                rows.append(tv[a]); cols.append(tv[b]); vals.append(K[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m))


def test_mass_of_gradients_is_p1_stiffness():
    """D^T M D equals the sigma-weighted P1 stiffness: gradients of nodal hat
    functions lie in the lowest-order edge space (Sec. 1)."""
    mesh = synth.kuhn_mesh(3, 0.15, 11)
    sig = synth.sigma_lognormal(mesh, 5, 1.5)
    M = _mat(synth.assemble(mesh, sig, "M"))
    D = _grad(mesh["tail"], mesh["head"], mesh["n"] ** 3)
    K = _p1_stiffness(mesh, sig)
    assert abs(D.T @ M @ D - K).max() <= 1e-12 * abs(K).max()


def test_operator_symmetric_positive_definite():
    mesh = synth.kuhn_mesh(4, 0.2, 3)
    sig = synth.sigma_inclusions(mesh, 1, 1.0, 1e-3)
    A = _mat(synth.assemble(mesh, sig, "A")).toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-14 * abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0


def test_jitter_keeps_orientation():
    mesh = synth.kuhn_mesh(16, 0.2, 303)
    ref = synth.tet_volumes(synth.kuhn_mesh(16))
    v = synth.tet_volumes(mesh)
    assert np.all(np.sign(v) == np.sign(ref))
    assert abs(abs(v).sum() - 1.0) < 1e-12


def test_box_aggregates_levels():
    """3-wide box coarsening: sides and level counts of the named workloads."""
    assert synth.box_aggregates(9)[1] == [9, 3]
    assert synth.box_aggregates(33)[1] == [33, 11, 4, 2]
    assert synth.box_aggregates(65)[1] == [65, 22, 8, 3]
    assert synth.box_aggregates(129)[1] == [129, 43, 15, 5, 2]
    maps, sides = synth.box_aggregates(33)
    for agg, nc in zip(maps, sides[1:]):
        assert agg.max() + 1 == nc ** 3
        assert np.all(np.bincount(agg) > 0)


# ---------------------------------------------------------------------------
# hexahedral Nedelec elements (the hex column of Table 3)
# ---------------------------------------------------------------------------
def _q1_stiffness(N):
    """Trilinear (Q1) stiffness of N^3 cubes, by its own quadrature: the
    gradients of the Q1 basis lie in the Nedelec space, so D^T M D equals it."""
    g = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) * 0.5 + 0.5
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    K = np.zeros((8, 8))
    corners = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
    f = lambda s, t: t if s else 1.0 - t
    df = lambda s: 1.0 if s else -1.0
    for x, wx in zip(g, w):
        for y, wy in zip(g, w):
            for z, wz in zip(g, w):
                G = np.array([[df(a) * f(b, y) * f(c, z), f(a, x) * df(b) * f(c, z), f(a, x) * f(b, y) * df(c)]
                              for a, b, c in corners])
                K += wx * wy * wz * G @ G.T
    n = N + 1
    h = 1.0 / N
    rows, cols, vals = [], [], []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                ids = [(i + a) + n * (j + b) + n * n * (k + c) for a, b, c in corners]
                for p_, u in enumerate(ids):
                    for q_, v in enumerate(ids):
                        rows.append(u); cols.append(v); vals.append(h * K[p_, q_])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n ** 3, n ** 3))


@pytest.mark.parametrize("N", [2, 4])
def test_hex_elements_null_space_and_gradient_mass(N):
    """S_h D_h = 0 (the curl of a gradient) and D^T M D = sigma K_Q1."""
    p = synth.hex_problem(N, sigma=0.7)
    n = N + 1
    D = _grad(p["tail"], p["head"], n ** 3)
    S = _mat(synth.assemble_hex(p["mesh"], p["sigma"], "S"))
    M = _mat(synth.assemble_hex(p["mesh"], p["sigma"], "M"))
    assert abs(S @ D).max() <= 1e-13 * abs(S).max()
    K = _q1_stiffness(N)
    assert abs(D.T @ M @ D - 0.7 * K).max() <= 1e-13 * abs(K).max()
    A = _mat(p["A"])
    assert abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


# ---------------------------------------------------------------------------
# 2D elements (Tables 1 and 2)
# ---------------------------------------------------------------------------
def _table12():
    rows = {}
    for line in open(os.path.join(GOLDEN, "table12_2d_iterations.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, n, _, _, _, edges, _ = line.split()
        rows[(kind, int(n))] = int(edges)
    return sorted(rows.items())


@pytest.mark.parametrize("key,edges", _table12())
def test_2d_edge_counts_tables_1_2(key, edges):
    """#edges of Tables 1 and 2 (generated meshes up to 244^2, closed forms
    above)."""
    kind, n = key
    N = n - 1
    closed = 2 * n * N + (N * N if kind == "tri" else 0)
    assert closed == edges
    if n <= 244:
        mesh = synth.tri_mesh(N) if kind == "tri" else synth.quad_mesh(N)
        assert len(mesh["tail"]) == edges


def _p1_stiffness_2d(mesh):
    """P1 stiffness by the per-triangle gradient formula."""
    X = mesh["coords"][mesh["tris"]]
    rows, cols, vals = [], [], []
    for t in range(X.shape[0]):
        B = np.array([X[t, 1] - X[t, 0], X[t, 2] - X[t, 0]]).T
        Gr = np.linalg.inv(B).T @ np.array([[-1.0, 1.0, 0.0], [-1.0, 0.0, 1.0]])
        area = 0.5 * abs(np.linalg.det(B))
        K = area * Gr.T @ Gr
        for a in range(3):
            for b in range(3):
                rows.append(mesh["tris"][t, a]); cols.append(mesh["tris"][t, b]); vals.append(K[a, b])
    m = mesh["coords"].shape[0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m))


def _q1_stiffness_2d(N):
    g = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) * 0.5 + 0.5
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    corners = [(a, b) for b in (0, 1) for a in (0, 1)]
    f = lambda s, t: t if s else 1.0 - t
    df = lambda s: 1.0 if s else -1.0
    K = np.zeros((4, 4))
    for x, wx in zip(g, w):
        for y, wy in zip(g, w):
            G = np.array([[df(a) * f(b, y), f(a, x) * df(b)] for a, b in corners])
            K += wx * wy * G @ G.T
    n = N + 1
    rows, cols, vals = [], [], []
    for j in range(N):
        for i in range(N):
            ids = [(i + a) + n * (j + b) for a, b in corners]
            for p_, u in enumerate(ids):
                for q_, v in enumerate(ids):
                    rows.append(u); cols.append(v); vals.append(K[p_, q_])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


@pytest.mark.parametrize("kind", ["tri", "quad"])
def test_2d_elements_null_space_and_gradient_mass(kind):
    """S_h D_h = 0 and D^T M D = sigma times the P1 (triangles) or Q1
    (squares) stiffness, each formed independently here."""
    N = 4
    p = synth.problem_2d(kind, N, sigma=0.7)
    n = N + 1
    D = _grad(p["tail"], p["head"], n * n)
    asm = synth.assemble_tri if kind == "tri" else synth.assemble_quad
    S = _mat(asm(p["mesh"], p["sigma"], "S"))
    M = _mat(asm(p["mesh"], p["sigma"], "M"))
    assert abs(S @ D).max() <= 1e-13 * abs(S).max()
    K = _p1_stiffness_2d(p["mesh"]) if kind == "tri" else _q1_stiffness_2d(N)
    assert abs(D.T @ M @ D - 0.7 * K).max() <= 1e-13 * abs(K).max()
    A = _mat(p["A"])
    assert abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_random_aggregates_are_connected_and_numbered():
    """synth.random_aggregates: every id used, every aggregate connected in
    the mesh graph with at least two nodes, and the same map for the same seed."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    pr = synth.problem(6)
    m = 343
    agg = synth.random_aggregates(pr["tail"], pr["head"], m, 9, 4)
    assert np.array_equal(agg, synth.random_aggregates(pr["tail"], pr["head"], m, 9, 4))
    K = int(agg.max()) + 1
    assert np.array_equal(np.unique(agg), np.arange(K))
    assert np.bincount(agg).min() >= 2
    G = sp.coo_matrix((np.ones(len(pr["tail"])), (pr["tail"], pr["head"])), shape=(m, m)).tocsr()
    for k in range(K):
        idx = np.nonzero(agg == k)[0]
        ncomp, _ = connected_components(G[idx][:, idx], directed=False)
        assert ncomp == 1, k
