"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names what it pins.  None of them re-types the oracle's own formula:
they use printed values (tests/golden), closed forms, library routines on the
same definition (dense solves, null spaces, triangular solves, eigensolvers) or
invariants that a dropped term, wrong sign or transposed operand would break.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components

import synth
from oracle import hcurl_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    p = synth.workload("cube8_const", with_S=True)
    levels = O.setup(p["A"], p["tail"], p["head"], 9 ** 3, p["aggregates"])
    return p, levels


# --------------------------------------------------------------------------
# symbolic setup: Table 4 (exact), coarse gradient closed form
# --------------------------------------------------------------------------

def _table4():
    out = {}
    for line in open(os.path.join(GOLDEN, "table4_ls_histogram.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, J, lo, hi, cnt = line.split()
        out.setdefault(kind, []).append((int(J), int(lo), int(hi), int(cnt)))
    return out


@pytest.mark.parametrize("kind", ["tet", "hex"])
def test_table4_least_squares_histogram(kind):
    """Level-0 row of Table 4 on the 82^3 nodal mesh: the number of rows with
    each column dimension |J| is reproduced exactly, and every row's n_p lies in
    the printed range.  Inputs: vertex-centred 3-wide aggregates and a nodal
    prolongator with the pattern of a 27-point nodal operator times P-bar."""
    n = 82
    mesh = synth.kuhn_mesh(n - 1)
    tail, head = mesh["tail"], mesh["head"]
    if kind == "hex":
        d = head - tail
        keep = (d == 1) | (d == n) | (d == n * n)
        tail, head = tail[keep], head[keep]
    agg, a = synth.vertex_centred_aggregates(n)
    T1 = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    A27 = sp.kron(T1, sp.kron(T1, T1, format="csr"), format="csr")
    Pn = O.symbolic_product(A27, O.tentative_prolongator(agg, a ** 3))
    D = O.gradient_matrix(tail, head, n ** 3)
    th, hd = O.coarse_gradient(D, agg, a ** 3)
    DH = O.gradient_matrix(th, hd, a ** 3)
    N, T, R = O.emin_pattern(D, Pn, DH)
    J = np.diff(T.indptr)
    npv = np.diff(N.indptr)
    expect = _table4()[kind]
    assert sum(c for _, _, _, c in expect) == D.shape[0]
    for Jv, lo, hi, cnt in expect:
        sel = J == Jv
        assert int(sel.sum()) == cnt
        assert npv[sel].min() >= lo and npv[sel].max() <= hi
    assert set(np.unique(J)) == {e[0] for e in expect}


@pytest.mark.parametrize("n", [9, 33])
def test_coarse_gradient_is_coarse_kuhn_lattice(n):
    """With box aggregates the RS rule (eq. "revised RS DH") connects exactly
    the aggregates joined by a fine edge; for the Kuhn lattice that is again a
    Kuhn lattice on the coarse nodes, in lexicographic order."""
    mesh = synth.kuhn_mesh(n - 1)
    maps, sides = synth.box_aggregates(n)
    D = O.gradient_matrix(mesh["tail"], mesh["head"], n ** 3)
    th, hd = O.coarse_gradient(D, maps[0], sides[1] ** 3)
    ref = synth.kuhn_mesh(sides[1] - 1)
    assert np.array_equal(th, ref["tail"]) and np.array_equal(hd, ref["head"])


def test_c1_pattern_counts(c1):
    """nnz(P^(e)_0) and level sizes of the 8^3 workload (lattice counts)."""
    p, levels = c1
    assert levels[0]["N"].nnz == 19566
    assert len(levels[0]["DH_tail"]) == synth.edge_count(2)
    assert levels[1]["A"].shape[0] == 98


# --------------------------------------------------------------------------
# local systems: Sec. 4.2 figures, projector properties, min-norm solution
# --------------------------------------------------------------------------

def _fig_matrices():
    mats, cur, name = {}, None, None
    for line in open(os.path.join(GOLDEN, "fig_local_submatrices.txt")):
        if line.startswith("#") or not line.strip():
            continue
        if line.startswith("matrix") or line.startswith("reducible"):
            name = line.strip()
            mats[name] = []
            continue
        mats[name].append([int(v) for v in line.split()])
    return {k: np.array(v, float) for k, v in mats.items()}


def _one_row_system(G, r):
    """Wrap one transposed sub-matrix G (edges x nodes) as a single-row pattern."""
    n_p, nJ = G.shape
    tail = np.array([np.nonzero(G[e] < 0)[0][0] for e in range(n_p)])
    head = np.array([np.nonzero(G[e] > 0)[0][0] for e in range(n_p)])
    N = sp.csr_matrix((np.ones(n_p), np.arange(n_p), [0, n_p]), shape=(1, n_p))
    T = sp.csr_matrix((np.ones(nJ), np.arange(nJ), [0, nJ]), shape=(1, nJ))
    R = sp.csr_matrix((r, np.arange(nJ), [0, nJ]), shape=(1, nJ))
    lt, lh = O.local_graphs(N, T, tail, head)
    return N, T, R, lt, lh


def test_figure_submatrices_rank_and_min_norm():
    """Sec. 4.2 figure: every drawn sub-matrix has rank |J| - 1 (constant null
    vector); the local solve returns the min-norm solution of G^T p = r, the
    same vector as the pseudo-inverse (library routine) of G^T."""
    rng = np.random.default_rng(1)
    for name, G in _fig_matrices().items():
        if name.startswith("reducible"):
            continue
        n_p, nJ = G.shape
        assert np.linalg.matrix_rank(G) == nJ - 1
        r = rng.standard_normal(nJ)
        r -= r.mean()  # consistent right-hand side (rows of P^(n) sum to 1)
        N, T, R, lt, lh = _one_row_system(G, r)
        assert len(O.disconnected_rows(N, T, lt, lh)) == 0
        loc = O.LocalSystems(N, T, R, lt, lh)
        p = loc.make_feasible(np.zeros(n_p))
        assert np.allclose(p, np.linalg.pinv(G.T) @ r, atol=1e-13)
        x = rng.standard_normal(n_p)
        q = loc.make_feasible(x)
        assert np.allclose(G.T @ q, r, atol=1e-12)
        # closest feasible point: the correction is orthogonal to the null space
        Z = sla.null_space(G.T)
        assert np.allclose(Z.T @ (q - x), 0, atol=1e-12)


def test_figure_reducible_graph_detected():
    """Sec. 4.2 reducible example: null space of dimension two, flagged."""
    G = _fig_matrices()["reducible 2x4"]
    assert 4 - np.linalg.matrix_rank(G) == 2
    N, T, R, lt, lh = _one_row_system(G, np.zeros(4))
    assert list(O.disconnected_rows(N, T, lt, lh)) == [0]


def test_projector_properties(c1):
    """Pi is the orthogonal projector onto {x : G~_i^T x = 0} for every row:
    idempotent, symmetric, kills G~ y, output satisfies the homogeneous
    constraint; and it does not depend on which column is dropped."""
    p, levels = c1
    lvl = levels[0]
    loc = lvl["loc"]
    rng = np.random.default_rng(2)
    x = rng.standard_normal(lvl["N"].nnz)
    y = rng.standard_normal(lvl["N"].nnz)
    px = loc.project(x)
    assert np.allclose(loc.project(px), px, atol=1e-12)
    assert abs(np.dot(px, y) - np.dot(x, loc.project(y))) < 1e-10
    DH = O.gradient_matrix(lvl["DH_tail"], lvl["DH_head"], lvl["Pn"].shape[1])
    assert abs(O.with_values(lvl["N"], px) @ DH).max() < 1e-12
    for g in loc.groups:
        if g["n_p"] == 0:
            continue
        b = len(g["rows"])
        v = np.zeros(lvl["N"].nnz)
        yk = rng.standard_normal((b, g["k"]))
        v[g["pos"]] = np.einsum("bpk,bk->bp", g["G"][:, :, 1:], yk)  # drop column 0 instead
        assert abs(loc.project(v)).max() < 1e-12


def test_single_coarse_edge_rows(c1):
    """Rows with n_p = 1 have the unique solution p = r_K = -r_I (Sec. 4.2)."""
    p, levels = c1
    lvl = levels[0]
    Pe = lvl["Pe"]
    N, T, R = lvl["N"], lvl["T"], lvl["R"]
    one = np.nonzero(np.diff(N.indptr) == 1)[0]
    assert len(one) == 1170
    j = N.indices[N.indptr[one]]
    K = lvl["DH_head"][j]
    I = lvl["DH_tail"][j]
    rK = np.array([R[i, k] for i, k in zip(one, K)])
    rI = np.array([R[i, k] for i, k in zip(one, I)])
    assert np.allclose(Pe.data[N.indptr[one]], rK, atol=1e-14)
    assert np.allclose(rK, -rI, atol=1e-14)


def test_rs_special_case():
    """P^(n) = P-bar (no smoothing) gives the Reitzinger-Schoeberl prolongator
    (Sec. 2): +1 on fine edges from aggregate I to K > I, -1 on edges from K to
    I, empty rows inside aggregates; energy minimisation cannot change it."""
    pr = synth.workload("cube8_const")
    agg = pr["aggregates"][0]
    Pbar = O.tentative_prolongator(agg, 27)
    lvl, _ = O.build_level(O.csr(pr["A"]), pr["tail"], pr["head"], 729, agg, dict(Pn=Pbar))
    Pe = lvl["Pe"].toarray()
    ia, ib = agg[pr["tail"]], agg[pr["head"]]
    edge_index = {(a, b): e for e, (a, b) in enumerate(zip(lvl["DH_tail"], lvl["DH_head"]))}
    ref = np.zeros_like(Pe)
    for e in range(len(ia)):
        if ia[e] < ib[e]:
            ref[e, edge_index[(ia[e], ib[e])]] = 1.0
        elif ia[e] > ib[e]:
            ref[e, edge_index[(ib[e], ia[e])]] = -1.0
    assert np.array_equal(Pe, ref)


# --------------------------------------------------------------------------
# energy minimisation: dense KKT brute force, monotone energy
# --------------------------------------------------------------------------

def _kkt_dense(lvl):
    """Minimise sum_j 1/2 P_:j^T A P_:j over the pattern subject to the
    commuting constraint, by a null-space basis of the stacked constraint
    matrix and a dense solve (eq. KKT, eliminated)."""
    A = lvl["A"].toarray()
    N = lvl["N"]
    rows = np.repeat(np.arange(N.shape[0]), np.diff(N.indptr))
    cols = N.indices
    nz = N.nnz
    Ahat = np.zeros((nz, nz))
    for a in range(nz):
        same = np.nonzero(cols == cols[a])[0]
        Ahat[a, same] = A[rows[a], rows[same]]
    DH = O.gradient_matrix(lvl["DH_tail"], lvl["DH_head"], lvl["Pn"].shape[1]).toarray()
    C, rhs = [], []
    Rd = (lvl["D"] @ lvl["Pn"]).toarray()
    for i in range(N.shape[0]):
        sel = np.nonzero(rows == i)[0]
        Tn = lvl["T"].indices[lvl["T"].indptr[i]:lvl["T"].indptr[i + 1]]
        for I in Tn:
            row = np.zeros(nz)
            row[sel] = DH[cols[sel], I]
            C.append(row)
            rhs.append(Rd[i, I])
    C = np.array(C)
    rhs = np.array(rhs)
    p0 = np.linalg.lstsq(C, rhs, rcond=None)[0]
    Z = sla.null_space(C)
    y = np.linalg.solve(Z.T @ Ahat @ Z, -Z.T @ Ahat @ p0)
    return p0 + Z @ y


@pytest.mark.parametrize("N,width", [(3, 2), (5, 3)])
def test_projected_cg_reaches_dense_kkt_solution(N, width):
    """Many projected-CG iterations converge to the dense KKT minimiser."""
    pr = synth.problem(N, jitter=0.1, jitter_seed=4, sigma=("lognormal", 9, 1.0), agg_width=width)
    m = (N + 1) ** 3
    lvl, _ = O.build_level(O.csr(pr["A"]), pr["tail"], pr["head"], m, pr["aggregates"][0], dict(emin_iters=400))
    ref = _kkt_dense(lvl)
    assert np.max(abs(lvl["Pe"].data - ref)) <= 1e-8 * np.max(abs(ref))


def test_energy_monotone_and_cg_decrement(c1):
    """Energy never increases and drops by rho^2 / (2 gamma) per CG step (the
    CG minimisation property)."""
    p, levels = c1
    lvl = levels[0]
    E = np.array(lvl["energies"])
    assert np.all(np.diff(E) < 0)
    rho = np.array(lvl["cg"]["rho"][:-1])
    gam = np.array(lvl["cg"]["gamma"])
    assert np.allclose(E[:-1] - E[1:], rho ** 2 / (2 * gam), rtol=1e-8)


# --------------------------------------------------------------------------
# structure preservation (eq. "commute" and the Galerkin identities)
# --------------------------------------------------------------------------

def test_commuting_relation_and_coarse_null_space(c1):
    """P^(e) D_H = D_h P^(n) at rounding; S_H D_H = 0 (Sec. 2); the nodal
    operator of the coarse level equals P^(n)T A^(n) P^(n)."""
    p, levels = c1
    lvl = levels[0]
    assert O.commuting_residual(lvl) <= 1e-12 * abs(lvl["D"] @ lvl["Pn"]).max()
    S = O.csr(p["S"])
    SH = O.galerkin(lvl["Pe"], S)
    DH = O.gradient_matrix(lvl["DH_tail"], lvl["DH_head"], 27)
    assert abs(SH @ DH).max() <= 1e-12 * abs(SH).max()
    AnH = levels[1]["An"]
    ref = lvl["Pn"].T @ lvl["An"] @ lvl["Pn"]
    assert abs(AnH - ref).max() <= 1e-11 * abs(ref).max()


def test_nodal_operator_is_p1_laplacian():
    """A^(n) = D^T (S + M) D = D^T M D: the sigma-weighted P1 stiffness."""
    from tests.test_synth import _p1_stiffness
    mesh = synth.kuhn_mesh(3, 0.1, 5)
    sig = synth.sigma_lognormal(mesh, 6, 1.0)
    A = O.csr(synth.assemble(mesh, sig, "A"))
    D = O.gradient_matrix(mesh["tail"], mesh["head"], 64)
    An = O.nodal_operator(A, D)
    K = _p1_stiffness(mesh, sig)
    assert abs(An - K).max() <= 1e-12 * abs(K).max()


def test_sa_prolongator_properties():
    """SA: rows sum to one; rho close to the largest eigenvalue of D^-1 A^(n)
    (library eigensolver); P-bar pattern contained."""
    pr = synth.workload("cube8_const")
    D = O.gradient_matrix(pr["tail"], pr["head"], 729)
    An = O.nodal_operator(O.csr(pr["A"]), D)
    Pn, info = O.sa_prolongator(An, pr["aggregates"][0], 27)
    assert np.allclose(np.asarray(Pn.sum(axis=1)).ravel(), 1.0, atol=1e-14)
    dm = sp.diags(1 / np.sqrt(An.diagonal()))
    lam = spla.eigsh(dm @ An @ dm, k=1, which="LA")[0][0]
    assert 0.9 * lam <= info["rho"] <= lam * (1 + 1e-12)
    assert np.allclose(info["row_sums_before"], 1.0, atol=1e-12)


# --------------------------------------------------------------------------
# smoother / V-cycle / PCG
# --------------------------------------------------------------------------

def test_coloring_valid(c1):
    p, levels = c1
    for key, A in (("colors_A", levels[0]["A"]), ("colors_An", levels[0]["An"])):
        c = levels[0][key]
        co = A.tocoo()
        off = co.row != co.col
        assert np.all(c[co.row[off]] != c[co.col[off]])
        assert np.all(c >= 0)


def test_sgs_equals_triangular_solves(c1):
    """Multicolour SGS equals forward then backward Gauss-Seidel on the matrix
    permuted to colour order (library triangular solves)."""
    p, levels = c1
    A = levels[0]["A"]
    col = levels[0]["colors_A"]
    perm = np.argsort(col, kind="stable")
    Ap = A[perm][:, perm].tocsr()
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    L = sp.tril(Ap, 0, format="csr")
    U = sp.triu(Ap, 0, format="csr")
    bp, xp = b[perm], x0[perm]
    xp = xp + spla.spsolve_triangular(L, bp - Ap @ xp, lower=True)
    xp = xp + spla.spsolve_triangular(U, bp - Ap @ xp, lower=False)
    ref = np.empty_like(xp)
    ref[perm] = xp
    assert np.allclose(O.sgs(A, col, x0, b), ref, rtol=0, atol=1e-10 * abs(ref).max())


def test_vcycle_symmetric_positive_definite(c1):
    p, levels = c1
    n = levels[0]["A"].shape[0]
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    vx, vy = O.vcycle(levels, x), O.vcycle(levels, y)
    assert abs(np.dot(vx, y) - np.dot(x, vy)) <= 1e-10 * abs(np.dot(vx, y))
    assert np.dot(x, vx) > 0


def test_pcg_matches_dense_solve(c1):
    p, levels = c1
    f = p["f"]
    u, it, rel, hist = O.pcg(levels, f)
    A = levels[0]["A"].toarray()
    ustar = np.linalg.solve(A, f)
    assert rel <= 1e-8
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(u - ustar) / np.linalg.norm(ustar) <= kappa * 1e-8
    assert it <= 20


def test_fp32_vcycle_pcg_reaches_tolerance(c1):
    p, levels = c1
    l32 = O.fp32_levels(levels)
    u, it, rel, _ = O.pcg(levels, p["f"], precond=lambda r: O.vcycle_fp32(l32, r), flexible=True)
    assert rel <= 1e-8
    assert it <= 25


def test_fp32_form_needs_fp64_residuals_at_high_contrast():
    """Contrast 1e6 on an 8^3 mesh (sigma h^2 = 1.6e-8, below FP32 epsilon):
    with residuals formed from the FP32 copy of A the FP32 V-cycle stalls
    (D^T of the rounding noise drives the nodal correction); with the FP64
    operator in the residuals it converges.  Pins the precision layout of
    vcycle_fp32 against a plausible simplification."""
    p = synth.problem(8, sigma=("inclusions", 8, 1.0, 1e-6), f_seed=3)
    levels = O.setup(p["A"], p["tail"], p["head"], 9 ** 3, p["aggregates"])
    l32 = O.fp32_levels(levels)
    _, it, rel, _ = O.pcg(levels, p["f"], precond=lambda r: O.vcycle_fp32(l32, r), flexible=True, maxit=200)
    # converged (recursive residual 1e-8 before maxit); the true residual is
    # limited near eps64 times the cancellation ratio, as for the FP64 form
    assert it < 150 and rel < 1e-6
    bad = [dict(lv, A=lv["A32"]) for lv in l32[:-1]] + [l32[-1]]
    _, it_b, rel_b, _ = O.pcg(levels, p["f"], precond=lambda r: O.vcycle_fp32(bad, r), flexible=True, maxit=200)
    assert rel_b > 1e-3


@pytest.mark.slow
def test_mesh_independent_iterations():
    """PCG iterations stay within 2 over a 2x refinement (Sec. 6.1 behaviour;
    larger meshes are covered by the GPU tests)."""
    its = []
    for N in (8, 16):
        pr = synth.problem(N, sigma=("const", 1.0), f_seed=7)
        lv = O.setup(pr["A"], pr["tail"], pr["head"], (N + 1) ** 3, pr["aggregates"])
        its.append(O.pcg(lv, pr["f"])[1])
    assert max(its) - min(its) <= 2, its


# --------------------------------------------------------------------------
# make_irreducible (reading R15), forced with irregular aggregates
# --------------------------------------------------------------------------

def test_make_irreducible_restores_feasibility():
    """A nodal prolongator whose row reaches a far aggregate makes the local
    graph of the fine edges at that node disconnected (Sec. 4.2, figure of the
    reducible case); make_irreducible adds coarse edges until every row is
    connected and the commuting relation holds again."""
    pr = synth.problem(6, sigma=("const", 1.0))
    agg = pr["aggregates"][0]  # 3 x 3 x 3 box aggregates of the 7^3 nodes
    Pn = O.tentative_prolongator(agg, 27).tolil()
    Pn[0, 26] = 0.25  # node 0 sits in aggregate 0 = (0,0,0); 26 = (2,2,2) is far
    Pn[0, 0] = 0.75
    Pn = O.csr(Pn.tocsr())
    D = O.gradient_matrix(pr["tail"], pr["head"], 343)
    th, hd = O.coarse_gradient(D, agg, 27)
    N, T, R = O.emin_pattern(D, Pn, O.gradient_matrix(th, hd, 27))
    lt, lh = O.local_graphs(N, T, th, hd)
    assert len(O.disconnected_rows(N, T, lt, lh)) > 0
    lvl, _ = O.build_level(O.csr(pr["A"]), pr["tail"], pr["head"], 343, agg, dict(Pn=Pn))
    assert lvl["irreducible_added"] > 0
    assert len(lvl["DH_tail"]) == len(th) + lvl["irreducible_added"]
    assert len(O.disconnected_rows(lvl["N"], lvl["T"], lvl["lt"], lvl["lh"])) == 0
    assert O.commuting_residual(lvl) <= 1e-12


# ---------------------------------------------------------------------------
# Alg. 1: piecewise-constant interpolation from a given P^(n) (reading R5)
# ---------------------------------------------------------------------------
def test_alg1_recovers_piecewise_constant_prolongator():
    """A P^(n) that is already piecewise constant (one unit entry per row) is
    mapped back to exactly its aggregates, whatever the number of passes."""
    agg = synth.box_aggregates(9)[0][0]
    mH = int(agg.max()) + 1
    Pbar = O.tentative_prolongator(agg, mH)
    for passes in (1, 2, 3):
        assert np.array_equal(O.piecewise_constant_assignment(Pbar, passes), agg)


def test_alg1_on_smoothed_aggregation_prolongator():
    """On a smoothed P^(n) the assignment is a partition that uses every
    coarse node, takes only columns where the row of P^(n) is non-zero, and
    returns most rows to the aggregate they came from (smoothing only adds
    smaller entries around each aggregate)."""
    p = synth.problem(8, sigma=("const", 1.0))
    A = O.csr(p["A"])
    D = O.gradient_matrix(p["tail"], p["head"], 9 ** 3)
    agg = p["aggregates"][0]
    mH = int(agg.max()) + 1
    Pn, _ = O.sa_prolongator(O.nodal_operator(A, D), agg, mH)
    a = O.piecewise_constant_assignment(Pn, 2)
    assert a.shape == agg.shape and a.min() >= 0 and np.all(np.bincount(a, minlength=mH) > 0)
    Pn = O.csr(Pn)
    for i in range(Pn.shape[0]):
        assert a[i] in Pn.indices[Pn.indptr[i]:Pn.indptr[i + 1]]
    assert np.mean(a == agg) > 0.8


def test_hierarchy_from_given_nodal_prolongator():
    """Setup from a given level-0 P^(n) instead of aggregates (the boundary
    takes either): aggregates for P-bar and D_H come from Alg. 1, the
    commuting relation holds and PCG converges like the aggregate path."""
    p = synth.problem(8, sigma=("const", 1.0), f_seed=5)
    m = 9 ** 3
    A = O.csr(p["A"])
    D = O.gradient_matrix(p["tail"], p["head"], m)
    agg = p["aggregates"][0]
    Pn, _ = O.sa_prolongator(O.nodal_operator(A, D), agg, int(agg.max()) + 1)
    ref = O.setup(p["A"], p["tail"], p["head"], m, p["aggregates"])
    lv = O.setup(p["A"], p["tail"], p["head"], m, [None] + list(p["aggregates"][1:]), dict(Pn=Pn))
    assert np.array_equal(lv[0]["agg"], O.piecewise_constant_assignment(O.scale_rows_to_one(Pn), 2))
    assert O.commuting_residual(lv[0]) <= 1e-12
    _, it_ref, _, _ = O.pcg(ref, p["f"])
    _, it, rel, _ = O.pcg(lv, p["f"])
    assert rel <= 1e-8 and abs(it - it_ref) <= 3


def _dense_csr(rows):
    return sp.csr_matrix(np.array(rows, dtype=float))


def test_alg1_rules_on_hand_worked_example():
    """Worked by hand from Alg. 1 with reading R5 (4 fine nodes, 2 coarse).
    nnz = 8, so both targets are ceil(4 * 4 / 8) = 2.  One pass (2 rows per
    column): column 0 ranks rows 2 (0.9), 0, 1 (0.5, tie -> row 0) and takes
    {2, 0}; column 1 then takes the free rows {3, 1}.  Two passes (1 row per
    column per pass): 2, 3, then 0 (tie -> smaller row), then 1."""
    P = _dense_csr([[0.5, 0.5], [0.5, 0.5], [0.9, 0.1], [0.1, 0.9]])
    for passes in (1, 2):
        assert np.array_equal(O.piecewise_constant_assignment(P, passes), [0, 1, 0, 1])
    # rows scaled by positive factors: the same assignment once rows sum to one
    Q = sp.diags([4.0, 0.25, 3.0, 7.0]) @ P
    assert np.array_equal(O.piecewise_constant_assignment(O.scale_rows_to_one(Q), 1), [0, 1, 0, 1])
    assert np.allclose(O.scale_rows_to_one(Q).toarray(), P.toarray(), rtol=1e-15, atol=0)


def test_alg1_passes_greedy_and_safeguard_by_hand():
    """Rows [1.2, -0.2], [1.2, -0.2], [1.0, 0]: nnz = 5, targets ceil(9/5) = 2
    and ceil(6/5) = 2.  One pass: column 0 takes rows 0 and 1 (1.2), column 1
    finds no free row; row 2 is left over and goes to column 0; column 1 is
    empty, rows 0 and 1 may move (column 0 keeps 3), |-0.2| ties -> row 0.
    Two passes: column 0 takes row 0, column 1 row 1, then column 0 row 2."""
    P = _dense_csr([[1.2, -0.2], [1.2, -0.2], [1.0, 0.0]])
    assert np.array_equal(O.piecewise_constant_assignment(P, 1), [1, 0, 0])
    assert np.array_equal(O.piecewise_constant_assignment(P, 2), [0, 1, 0])


def test_alg1_empty_column_without_movable_row_is_an_error():
    """Column 1 meets only row 0, which column 0 takes first and which is
    column 0's only row: the safeguard cannot fill column 1."""
    P = _dense_csr([[1.2, -0.2, 0.0], [0.0, 0.0, 1.0]])
    with pytest.raises(ValueError):
        O.piecewise_constant_assignment(P, 1)
    with pytest.raises(ValueError):
        O.scale_rows_to_one(_dense_csr([[1.0, -1.0], [0.5, 0.5]]))


def test_pbar_from_alg1_on_smoothed_prolongator():
    """P-bar from Alg. 1 on the smoothed P^(n) (the paper's own configuration,
    Sec. 4.1): the hierarchy keeps the commuting relation and converges like
    the aggregate-P-bar one; P^(n) itself is unchanged."""
    p = synth.problem(8, jitter=0.2, jitter_seed=3, sigma=("lognormal", 4, 1.0), f_seed=5)
    m = 9 ** 3
    ref = O.setup(p["A"], p["tail"], p["head"], m, p["aggregates"])
    lv = O.setup(p["A"], p["tail"], p["head"], m, p["aggregates"], dict(pbar_alg1=True))
    assert abs(lv[0]["Pn"] - ref[0]["Pn"]).max() == 0.0
    assert np.array_equal(lv[0]["agg"], O.piecewise_constant_assignment(ref[0]["Pn"], 2))
    for l in lv[:-1]:
        assert O.commuting_residual(l) <= 1e-12
    _, it_ref, _, _ = O.pcg(ref, p["f"])
    _, it, rel, _ = O.pcg(lv, p["f"])
    assert rel <= 1e-8 and abs(it - it_ref) <= 3


# ---------------------------------------------------------------------------
# setup reuse for a sequence of systems (Sec. 3; remarks after Table 4)
# ---------------------------------------------------------------------------
def _sequence_pair():
    """Two systems on one mesh: lognormal sigma from two seeds (same pattern)."""
    p1 = synth.problem(8, jitter=0.1, jitter_seed=2, sigma=("lognormal", 4, 1.0), f_seed=5)
    p2 = synth.problem(8, jitter=0.1, jitter_seed=2, sigma=("lognormal", 9, 1.0), f_seed=5)
    return p1, p2, 9 ** 3


def test_update_with_the_same_matrix_reproduces_the_setup():
    p1, _, m = _sequence_pair()
    lv = O.setup(p1["A"], p1["tail"], p1["head"], m, p1["aggregates"])
    u = O.update(lv, p1["A"], "transfers")
    for a, b in zip(lv, u):
        assert np.array_equal(O.csr(a["A"]).data, O.csr(b["A"]).data)
        assert np.array_equal(O.csr(a["An"]).data, O.csr(b["An"]).data)
    # a feasible P^(e) is a fixed point of the min-norm correction, and CG
    # continued from the minimiser cannot raise the energy
    w = O.update(lv, p1["A"], "warm", iters=4)
    for a, b in zip(lv[:-1], w[:-1]):
        assert abs(b["p0"] - a["Pe"].data).max() <= 1e-13 * abs(a["Pe"].data).max()
        assert abs(b["energies"][0] - a["energies"][-1]) <= 1e-12 * a["energies"][-1]
        assert b["energies"][-1] <= b["energies"][0] * (1 + 1e-14)


def test_update_transfers_keeps_the_nodal_galerkin_identity():
    """With P^(e) D_H = D_h P^(n), re-projecting any matrix gives
    D_H^T (P^T A P) D_H = P^(n)T (D_h^T A D_h) P^(n): the kept transfers stay
    structure preserving for the new sigma on every level."""
    p1, p2, m = _sequence_pair()
    lv = O.setup(p1["A"], p1["tail"], p1["head"], m, p1["aggregates"])
    u = O.update(lv, p2["A"], "transfers")
    assert abs(O.csr(u[0]["A"]) - O.csr(p2["A"])).max() == 0.0
    for l, lvl in enumerate(u[:-1]):
        DH = O.gradient_matrix(lvl["DH_tail"], lvl["DH_head"], lvl["Pn"].shape[1])
        left = DH.T @ u[l + 1]["A"] @ DH
        right = lvl["Pn"].T @ lvl["An"] @ lvl["Pn"]
        assert abs(left - right).max() <= 1e-10 * abs(right).max(), l
    _, it, rel, _ = O.pcg(u, p2["f"])
    assert rel <= 1e-8


def test_update_warm_start_meets_the_new_constraints():
    """Warm mode: P^(n) rebuilt from the new A^(n), the previous P^(e) moved
    onto the new constraints, then projected CG; the commuting relation holds,
    energies decrease, and the solve converges like a fresh setup."""
    p1, p2, m = _sequence_pair()
    lv = O.setup(p1["A"], p1["tail"], p1["head"], m, p1["aggregates"])
    fresh = O.setup(p2["A"], p2["tail"], p2["head"], m, p2["aggregates"])
    w = O.update(lv, p2["A"], "warm", iters=10)
    for a, b in zip(fresh[:-1], w[:-1]):
        assert abs(O.csr(a["Pn"]) - O.csr(b["Pn"])).max() <= 1e-13
        assert O.commuting_residual(b) <= 1e-12
        assert np.all(np.diff(b["energies"]) <= 1e-12 * b["energies"][0])
    _, it_f, _, _ = O.pcg(fresh, p2["f"])
    _, it_w, rel, _ = O.pcg(w, p2["f"])
    assert rel <= 1e-8 and it_w <= it_f + 2


# ---------------------------------------------------------------------------
# MIS-2 aggregation when the caller gives no aggregates (reading R26)
# ---------------------------------------------------------------------------
def _graph_lists(An):
    An = O.csr(An)
    return [[int(j) for j in An.indices[An.indptr[i]:An.indptr[i + 1]] if j != i] for i in range(An.shape[0])]


def _mis2_by_hand(An):
    """Sequential definition: nodes in decreasing key order, a node becomes a
    root unless a root lies within two steps; then the two attachment rules."""
    nb = _graph_lists(An)
    n = len(nb)
    key = [((int(O.splitmix64(np.array([i]))[0]) >> 34) << 32) | i for i in range(n)]
    dist2 = [set(nb[i]) | {k for j in nb[i] for k in nb[j]} for i in range(n)]
    roots = []
    taken = set()
    for i in sorted(range(n), key=lambda v: -key[v]):
        if not (dist2[i] & taken):
            taken.add(i)
    roots = sorted(taken)
    rid = {r: a for a, r in enumerate(roots)}
    agg = [-1] * n
    for r in roots:
        agg[r] = rid[r]
    first = list(agg)
    for i in range(n):
        if agg[i] < 0:
            near = [j for j in nb[i] if j in rid]
            if near:
                assert len(near) == 1
                first[i] = rid[near[0]]
    out = list(first)
    for i in range(n):
        if first[i] < 0:
            cand = [j for j in nb[i] if first[j] >= 0 and j not in rid]
            out[i] = first[max(cand, key=lambda j: key[j])]
    return np.array(out), roots


@pytest.mark.parametrize("N,jit", [(4, 0.0), (6, 0.2)])
def test_mis2_aggregates_match_the_sequential_definition(N, jit):
    """The Luby rounds choose the roots a sequential sweep in decreasing key
    order chooses (distance-2 greedy); both attachment steps by hand."""
    p = synth.problem(N, jitter=jit, jitter_seed=3, sigma=("lognormal", 2, 1.0))
    m = (N + 1) ** 3
    An = O.nodal_operator(O.csr(p["A"]), O.gradient_matrix(p["tail"], p["head"], m))
    ref, roots = _mis2_by_hand(An)
    got = O.mis2_aggregates(An)
    assert np.array_equal(got, ref)
    # roots three or more steps apart, every node within two steps of one
    nb = _graph_lists(An)
    rs = set(roots)
    for r in roots:
        assert not ((set(nb[r]) | {k for j in nb[r] for k in nb[j]}) - {r}) & rs
    for i in range(m):
        assert i in rs or (set(nb[i]) | {k for j in nb[i] for k in nb[j]}) & rs


def test_mis2_hierarchy_converges():
    """Setup with no aggregates at all: MIS-2 on every level's nodal graph
    down to coarse_max_rows; aggregates are connected in the nodal graph, the
    commuting relation holds and PCG converges."""
    p = synth.problem(12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7)
    m = 13 ** 3
    lv = O.setup(p["A"], p["tail"], p["head"], m, [], dict(aggregation="mis2", coarse_max_rows=200))
    assert len(lv) >= 3 and lv[-1]["A"].shape[0] <= 200
    for l in lv[:-1]:
        assert O.commuting_residual(l) <= 1e-12
        assert l["irreducible_added"] == 0
        a = l["agg"]
        G = O.csr(l["An"])
        same = a[np.repeat(np.arange(len(a)), np.diff(G.indptr))] == a[G.indices]
        sub = sp.csr_matrix((same.astype(float), G.indices, G.indptr), shape=G.shape)
        sub.eliminate_zeros()
        ncomp, lab = connected_components(sub, directed=False)
        assert ncomp == a.max() + 1
    _, it, rel, _ = O.pcg(lv, p["f"])
    assert rel <= 1e-8 and it < 60


# ---------------------------------------------------------------------------
# Sec. 5: ideal interpolation on refined triangles
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("M", [4, 6])
def test_ideal_interpolation_is_a_fixed_point_on_refined_triangles(M):
    """Sec. 5: with P^(n) the linear interpolation of a uniform refinement, the
    coarse Whitney basis sampled on the fine edges is feasible (it lies in the
    pattern of Alg. 2 and meets P^(e) D_H = D_h P^(n)), and the curl-curl
    energy has no projected gradient there (delta P = 0 solves the KKT
    system), so projected CG from it does not move."""
    r = synth.refined_triangles(M)
    f, c = r["fine"], r["coarse"]
    nf, nc = 2 * M + 1, M + 1
    D = O.gradient_matrix(f["tail"], f["head"], nf * nf)
    th, hd = O.coarse_gradient(D, r["agg"], nc * nc)
    assert np.array_equal(th, c["tail"]) and np.array_equal(hd, c["head"])
    DH = O.gradient_matrix(th, hd, nc * nc)
    assert abs(r["Pe"] @ DH - D @ r["Pn"]).max() <= 1e-14
    N, T, R = O.emin_pattern(D, r["Pn"], DH)
    assert abs(O.on_pattern(N, r["Pe"]) - r["Pe"]).max() == 0.0
    lt, lh = O.local_graphs(N, T, th, hd)
    loc = O.LocalSystems(N, T, R, lt, lh)
    p = O.on_pattern(N, r["Pe"]).data
    assert abs(loc.make_feasible(p) - p).max() <= 1e-14
    S = O.csr(synth.assemble_tri(f, np.ones(f["tris"].shape[0]), "S"))
    g = O.masked_product(S, O.with_values(N, p), N)
    assert abs(g).max() > 1.0
    assert abs(loc.project(g)).max() <= 1e-12 * abs(g).max()
    q, E, _ = O.projected_cg(S, N, loc, p, 5)
    assert abs(q - p).max() <= 1e-12 and abs(E[-1] - E[0]) <= 1e-12 * E[0]


# ---------------------------------------------------------------------------
# Dirichlet (single-node) edges: Sec. 2 and Alg. 2 (reading R27)
# ---------------------------------------------------------------------------
def _dirichlet(N, **kw):
    p = synth.dirichlet_problem(N, **kw)
    return p, O.gradient_matrix(p["tail"], p["head"], p["m"])


def test_dirichlet_problem_keeps_the_null_space():
    """With boundary nodes and boundary edges eliminated, S D = 0 still holds
    on the kept edges (Sec. 2), and rows of D have one or two entries."""
    p, D = _dirichlet(6, sigma=("lognormal", 3, 1.0))
    full = synth.problem(6, sigma=("lognormal", 3, 1.0), with_S=True)
    S = sp.csr_matrix((full["S"][2], full["S"][1], full["S"][0]))[p["kept_edges"]][:, p["kept_edges"]]
    assert abs(S @ D).max() <= 1e-13 * abs(S).max()
    cnt = np.diff(D.indptr)
    assert set(np.unique(cnt)) == {1, 2}


def test_dirichlet_rs_special_case():
    """P^(n) = P-bar: the RS prolongator (a Dirichlet fine edge to the
    single-node coarse edge of its interior node's aggregate, with the sign
    of its D row; two-node edges as before) meets the commuting relation with
    the single-node coarse edges; the single-node edges of Alg. 2's pattern
    (W = 2) give rows near the boundary free entries, so the energy minimiser
    may differ from it but has no more energy."""
    p, D = _dirichlet(8)
    agg = p["aggregates"][0]
    mH = int(agg.max()) + 1
    Pbar = O.tentative_prolongator(agg, mH)
    lvl, _ = O.build_level(O.csr(p["A"]), p["tail"], p["head"], p["m"], agg, dict(Pn=Pbar))
    th, hd = lvl["DH_tail"], lvl["DH_head"]
    two = {(a, b): e for e, (a, b) in enumerate(zip(th, hd)) if a >= 0}
    one = {b: e for e, (a, b) in enumerate(zip(th, hd)) if a < 0}
    Pe = lvl["Pe"].toarray()
    ref = np.zeros_like(Pe)
    t, h = p["tail"], p["head"]
    for e in range(len(t)):
        if t[e] < 0 or h[e] < 0:
            node, sgn = (h[e], 1.0) if t[e] < 0 else (t[e], -1.0)
            ref[e, one[agg[node]]] = sgn
        elif agg[t[e]] < agg[h[e]]:
            ref[e, two[(agg[t[e]], agg[h[e]])]] = 1.0
        elif agg[t[e]] > agg[h[e]]:
            ref[e, two[(agg[h[e]], agg[t[e]])]] = -1.0
    DH = O.gradient_matrix(th, hd, mH)
    assert abs(ref @ DH - (D @ Pbar).toarray()).max() == 0.0
    A = O.csr(p["A"])
    assert O.energy(A, lvl["N"], lvl["Pe"].data) <= O.energy(A, lvl["N"], O.on_pattern(lvl["N"], sp.csr_matrix(ref)).data)
    assert abs(O.on_pattern(lvl["N"], sp.csr_matrix(ref)) - sp.csr_matrix(ref)).max() == 0.0


@pytest.mark.parametrize("N", [4, 5])
def test_dirichlet_projected_cg_reaches_dense_kkt_solution(N):
    """With Dirichlet edges in the pattern the local systems keep every
    column (full rank); many projected-CG iterations reach the dense KKT
    minimiser, and the commuting relation holds."""
    p, D = _dirichlet(N, jitter=0.1, jitter_seed=4, sigma=("lognormal", 9, 1.0))
    agg = p["aggregates"][0]
    lvl, _ = O.build_level(O.csr(p["A"]), p["tail"], p["head"], p["m"], agg, dict(emin_iters=400))
    assert np.any(lvl["lt"] == O.MISSING)
    ref = _kkt_dense(lvl)
    assert np.max(abs(lvl["Pe"].data - ref)) <= 1e-8 * np.max(abs(ref))
    assert O.commuting_residual(lvl) <= 1e-12 * abs(lvl["D"] @ lvl["Pn"]).max()


def test_dirichlet_hierarchy_converges():
    p, D = _dirichlet(10, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=9)
    lv = O.setup(p["A"], p["tail"], p["head"], p["m"], p["aggregates"], dict(aggregation="mis2", coarse_max_rows=150))
    assert len(lv) >= 3
    for l in lv[:-1]:
        assert O.commuting_residual(l) <= 1e-12 * max(1.0, abs(l["D"] @ l["Pn"]).max())
        assert np.all(np.diff(l["energies"]) <= 1e-12 * l["energies"][0])
    _, it, rel, _ = O.pcg(lv, p["f"])
    assert rel <= 1e-8 and it < 80


# --------------------------------------------------------------------------
# hand-worked pins of smoothed aggregation and of the colouring rule
# --------------------------------------------------------------------------

def _complete_graph_operator(n, c):
    """(n + c) I - J: the Laplacian of the complete graph K_n plus c I.  Its
    Jacobi-scaled form D^-1 A has the eigenvalue c / (n - 1 + c) on constants
    and (n + c) / (n - 1 + c) on every vector of mean zero."""
    return O.csr(sp.csr_matrix((n + c) * np.eye(n) - np.ones((n, n))))


@pytest.mark.parametrize("c,expect", [
    # K_6, aggregates {0,1} and {2,3,4,5}; rho = 6/5, omega = 4/(3 rho) = 10/9,
    # omega / d = 2/9; (A Pbar) rows (4, -4) and (-2, 2):
    # P = Pbar - 2/9 A Pbar, rows already sum to one
    (0.0, [[1 / 9, 8 / 9], [4 / 9, 5 / 9]]),
    # K_6 + I: rho = 7/6, omega = 8/7, omega / d = 4/21; (A Pbar) rows (5, -4)
    # and (-2, 3): rows (1/21, 16/21) and (8/21, 9/21) sum to 17/21 and are
    # scaled to one (Sec. 4.2)
    (1.0, [[1 / 17, 16 / 17], [8 / 17, 9 / 17]]),
])
def test_sa_prolongator_hand_worked(c, expect):
    """Smoothed aggregation with omega = 4 / (3 rho(D^-1 A^(n))) (Sec. 3,
    reading R12), worked by hand on K_6: the power iteration reaches the
    closed-form rho and every entry of P^(n) matches.  A damping of 1/rho, a
    dropped D^-1 or a missing row scaling each change these values."""
    An = _complete_graph_operator(6, c)
    agg = np.array([0, 0, 1, 1, 1, 1], np.int32)
    Pn, info = O.sa_prolongator(An, agg, 2)
    rho = (6 + c) / (5 + c)
    assert abs(info["rho"] - rho) <= 1e-14 * rho
    assert abs(info["omega"] - 4 / (3 * rho)) <= 1e-14
    P = Pn.toarray()
    want = np.array([expect[0]] * 2 + [expect[1]] * 4)
    assert np.max(np.abs(P - want)) <= 1e-14
    assert Pn.nnz == 12  # pattern of Pbar union A^(n) Pbar: every entry


def _greedy_by_priority(A):
    """Sequential restatement of the colouring rule: visit the vertices in
    decreasing priority (splitmix64(i), i) and give each the smallest colour
    none of its already coloured neighbours has.  Jones-Plassmann rounds
    colour a vertex exactly when all its neighbours of higher priority are
    coloured and none of lower priority is, so the two agree vertex by
    vertex."""
    A = O.csr(A)
    n = A.shape[0]
    h = [int(v) for v in O.splitmix64(np.arange(n))]
    order = sorted(range(n), key=lambda i: (h[i], i), reverse=True)
    color = [-1] * n
    for v in order:
        used = {color[w] for w in A.indices[A.indptr[v]:A.indptr[v + 1]] if w != v and color[w] >= 0}
        k = 0
        while k in used:
            k += 1
        color[v] = k
    return np.array(color)


def test_coloring_is_greedy_in_priority_order(c1):
    """Jones-Plassmann colouring (reading R18) equals the sequential greedy
    colouring in decreasing priority on the level-0 edge and nodal graphs of
    the 8^3 cube, its coarse level and a random graph.  The greedy colouring
    in increasing priority, a different rule, differs on each."""
    p, levels = c1
    rng = np.random.default_rng(8)
    R = sp.random(400, 400, density=0.02, random_state=rng)
    graphs = [levels[0]["A"], levels[0]["An"], levels[1]["A"], O.csr(R + R.T + sp.eye(400))]
    for G in graphs:
        want = _greedy_by_priority(G)
        assert np.array_equal(O.color_graph(G), want)
        # discriminating: the reversed priority order gives another colouring
        Gr = O.csr(G)
        n = Gr.shape[0]
        rev = np.empty(n, np.int64)
        h = [int(v) for v in O.splitmix64(np.arange(n))]
        col = [-1] * n
        for v in sorted(range(n), key=lambda i: (h[i], i)):
            used = {col[w] for w in Gr.indices[Gr.indptr[v]:Gr.indptr[v + 1]] if w != v and col[w] >= 0}
            k = 0
            while k in used:
                k += 1
            col[v] = k
        rev[:] = col
        assert not np.array_equal(rev, want)


# ---------------------------------------------------------------------------
# attainable accuracy: Lanczos estimate from the CG coefficients, stagnation
# (Sec. 6.1 relaxes its tolerance by a condition estimate; Sec. 6.2 stops on
# two consecutive equal iterates)
# ---------------------------------------------------------------------------
def test_lanczos_extremes_exact_for_few_distinct_eigenvalues():
    """CG on diag(1, 2, 5, 2, 1) with the identity preconditioner ends after
    three iterations (three distinct eigenvalues, equal weights); the Lanczos
    matrix of those coefficients has exactly the eigenvalues 1, 2, 5."""
    A = sp.diags([1.0, 2.0, 5.0, 2.0, 1.0]).tocsr()
    info = {}
    x, it, rel, _ = O.pcg([dict(A=A)], np.ones(5), tol=1e-14, maxit=10, precond=lambda r: r, info=info)
    assert it == 3 and not info["stagnated"]
    lo, hi = O.lanczos_extremes(info["alpha"], info["beta"])
    assert abs(lo - 1.0) <= 1e-14 and abs(hi - 5.0) <= 1e-14


def test_lanczos_extremes_inside_and_at_the_ends_of_the_v_cycle_spectrum():
    """On a 4^3 mesh the V-cycle is formed column by column and the spectrum
    of V A computed densely: the Lanczos extremes lie inside it and, at
    PCG tolerance 1e-12, reach its smallest eigenvalue to 1e-6 and its
    largest to 1e-3 (the top end is a cluster near 1)."""
    pr = synth.problem(4, jitter=0.1, jitter_seed=1, sigma=("lognormal", 2, 1.0), f_seed=3)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], 125, pr["aggregates"])
    A = levels[0]["A"]
    n = A.shape[0]
    V = np.column_stack([O.vcycle(levels, e) for e in np.eye(n)])
    w = np.sort(np.linalg.eigvals(V @ A.toarray()).real)
    info = {}
    O.pcg(levels, pr["f"], tol=1e-12, info=info)
    lo, hi = O.lanczos_extremes(info["alpha"], info["beta"])
    assert w[0] * (1 - 1e-10) <= lo <= hi <= w[-1] * (1 + 1e-10)
    assert lo <= w[0] * (1 + 1e-6)
    assert hi >= w[-1] * (1 - 1e-3)


def test_pcg_stops_on_stagnation_below_rounding():
    """With tolerance 0 the recursive residual keeps falling, but once the
    updates round away the iterate repeats: the stagnation criterion ends the
    solve well before maxit with the true residual at rounding level."""
    pr = synth.problem(4, jitter=0.1, jitter_seed=1, sigma=("lognormal", 2, 1.0), f_seed=3)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], 125, pr["aggregates"])
    info = {}
    x, it, rel, hist = O.pcg(levels, pr["f"], tol=0.0, maxit=300, info=info)
    assert info["stagnated"] and it < 100
    assert rel <= 1e-12
    assert len(info["alpha"]) == it and len(info["beta"]) == it - 1


def test_lexicographic_sgs_is_the_symmetric_gauss_seidel_preconditioner(c1):
    """From x = 0 one lexicographic SGS sweep returns M^-1 b with the
    textbook M = (D + L) D^-1 (D + U) (dense solve); from any x it is the
    stationary step x + M^-1 (b - A x).  Sweeping forward twice (a wrong
    backward pass) gives a non-symmetric operator and fails the first check."""
    p, levels = c1
    A = O.csr(levels[1]["A"])  # 98 x 98 coarse operator: dense algebra is cheap
    Ad = A.toarray()
    Dg = np.diag(np.diag(Ad))
    M = (np.tril(Ad, -1) + Dg) @ np.linalg.solve(Dg, np.triu(Ad, 1) + Dg)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    ref0 = np.linalg.solve(M, b)
    assert np.allclose(O.sgs_lexicographic(A, np.zeros_like(b), b), ref0, rtol=0, atol=1e-10 * abs(ref0).max())
    ref = x0 + np.linalg.solve(M, b - Ad @ x0)
    assert np.allclose(O.sgs_lexicographic(A, x0, b), ref, rtol=0, atol=1e-10 * abs(ref).max())
    # the lexicographic V-cycle is symmetric like the multicolour one
    n = levels[0]["A"].shape[0]
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    a = np.dot(O.vcycle(levels, u, lex=True), v)
    c = np.dot(u, O.vcycle(levels, v, lex=True))
    assert abs(a - c) <= 1e-10 * abs(a)


def test_full_pattern_level_gives_the_pseudo_inverse_guess_and_a_singular_coarse_operator():
    """A level so small that every fine edge's pattern holds every coarse
    edge (3^3 nodes after 2-wide boxes on a 9^3 cube, coarsened 2-wide to
    2^3): each row's local system then spans all coarse nodes, and the local
    minimum-norm correction of the all-ones start (Sec. 6.1) has the closed
    form  P_0 = 1 1^T (I - D_H D_H^+) + D_h P^(n) D_H^+  (D_H^+ the
    pseudo-inverse).  Its rank is at most m_H = 8 of the 19 coarse edges, so
    the coarse operator P^T A P built from it after the energy minimisation
    is singular to rounding: the reason a six-level box hierarchy whose last
    step coarsens 3^3 nodes to 2^3 cannot be factored on its coarsest level."""
    N = 8
    pr = synth.problem(N, sigma=("const", 1.0), f_seed=1)
    maps, sides = synth.box_aggregates(N + 1, [2, 2, 2])
    assert sides == [9, 5, 3, 2]
    A, t, h, m = O.csr(pr["A"]), pr["tail"], pr["head"], (N + 1) ** 3
    for agg in maps[:2]:
        lv, (A, t, h, m) = O.build_level(A, t, h, m, agg, {})
    lv, (AH, _, _, mH) = O.build_level(A, t, h, m, maps[2], {})
    n, nH = lv["N"].shape
    assert (n, nH, mH) == (98, 19, 8) and lv["N"].nnz == n * nH
    DH = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], mH).toarray()
    Dp = np.linalg.pinv(DH)
    G = (lv["D"] @ lv["Pn"]).toarray()
    closed = np.ones((n, 1)) @ (np.ones((1, nH)) @ (np.eye(nH) - DH @ Dp)) + G @ Dp
    P0 = O.with_values(lv["N"], lv["p0"]).toarray()
    assert np.max(abs(P0 - closed)) <= 1e-13 * np.max(abs(closed))
    assert np.linalg.matrix_rank(P0) == mH
    ev = np.linalg.eigvalsh(O.csr(AH).toarray())
    assert ev[0] <= 1e-12 * ev[-1]
