"""GPU checks of the boundary's reporting and error paths:
* the (|J|, n_p) histogram of the local least-squares problems, counted on
  the device, against the oracle's row by row and against Table 4;
* the curl-curl Galerkin check S_H D_H = 0 formed on the device (Sec. 2);
* the PCG coefficients and their Lanczos eigenvalue estimates against the
  oracle's (reading R20);
* HCURL_ESTAGNATE (Sec. 6.2: two consecutive equal iterates), forced from
  the host by a zero tolerance;
* HCURL_EINFEASIBLE, forced by a caller P^(n) whose rows give a commuting
  constraint without finite solution;
* HCURL_ENOTSPD on a level whose pattern is full (its minimum-norm guess has
  rank m_H, so the coarsest operator is singular), where the oracle's
  Cholesky factorisation fails likewise."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = {
    "cube8_const": dict(N=8, sigma=("const", 1.0), f_seed=101),
    "cube12_jitter_lognormal": dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7),
    "cube10_inclusions": dict(N=10, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=9),
}
_cache = {}


def _case(name):
    if name not in _cache:
        import paper_2506_08284_amd as P
        pr = synth.problem(**CASES[name])
        m = pr["mesh"]["n"] ** 3
        levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"])
        H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m)
        _cache[name] = (pr, m, levels, H)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_ls_histogram_matches_oracle(name):
    pr, m, levels, H = _case(name)
    import paper_2506_08284_amd as P
    st = H.stats()
    mj = mp = 0
    for l, lv in enumerate(levels[:-1]):
        h = H.export_vec(l, "ls_histogram")
        ref = np.zeros_like(h)
        for (J, npv), cnt in lv["loc"].histogram().items():
            ref[min(J, P.LS_HIST_J - 1), min(npv, P.LS_HIST_NP - 1)] += cnt
        assert np.array_equal(h, ref), l
        assert h.sum() == lv["A"].shape[0]
        mj = max(mj, int(np.diff(lv["T"].indptr).max()))
        mp = max(mp, int(np.diff(lv["N"].indptr).max()))
    assert (st["max_local_J"], st["max_local_np"]) == (mj, mp)


def test_ls_histogram_reproduces_table4_tet():
    """Level 0 of Table 4 (tetrahedra, 82^3 nodes, 3,779,379 edges) through
    the library: vertex-centred 3-wide aggregates and a caller P^(n) with the
    pattern of a 27-point nodal operator times P-bar (values: the counts of
    that product, scaled to row sums one by the library), MIS-2 below.  The
    rows per |J| are the table's exactly and every n_p lies in its range."""
    import paper_2506_08284_amd as P
    n = 82
    mesh = synth.kuhn_mesh(n - 1)
    agg, a = synth.vertex_centred_aggregates(n)
    T1 = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    A27 = sp.kron(T1, sp.kron(T1, T1, format="csr"), format="csr")
    Pn = O.csr(A27 @ O.tentative_prolongator(agg, a ** 3))
    sig = synth.sigma_const(mesh, 1.0)
    A = synth.assemble(mesh, sig, "A")
    H = P.Hierarchy(A, synth.gradient_csr(mesh["tail"], mesh["head"]), [agg.astype(np.int32)], n_nodes=n ** 3,
                    nodal_prolongator=(Pn.indptr.astype(np.int64), Pn.indices.astype(np.int32), Pn.data, a ** 3),
                    aggregation="mis2", coarse_max_rows=1024)
    h = H.export_vec(0, "ls_histogram")
    rows = {}
    for line in open(os.path.join(GOLDEN, "table4_ls_histogram.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, J, lo, hi, cnt = line.split()
        if kind == "tet":
            rows[int(J)] = (int(lo), int(hi), int(cnt))
    assert int(h.sum()) == 3779379
    for J in range(h.shape[0]):
        if J in rows:
            lo, hi, cnt = rows[J]
            assert int(h[J].sum()) == cnt, J
            nz = np.nonzero(h[J])[0]
            assert nz.min() >= lo and nz.max() <= hi, J
        else:
            assert h[J].sum() == 0, J
    H.close()


@pytest.mark.parametrize("name", list(CASES))
def test_curl_residual_on_device(name):
    """S_l D_l on every level with S_{l+1} = P^(e)T S_l P^(e) formed on the
    device: at rounding level, and equal (to rounding) to the same quantity
    formed on the host from the exported prolongators."""
    pr, m, levels, H = _case(name)
    S = synth.assemble(pr["mesh"], pr["sigma"], "S")
    a, r = H.curl_residual(S)
    Sl = O.csr(S)
    for l in range(H.num_levels()):
        lv = levels[l]
        D = O.gradient_matrix(lv["tail"], lv["head"], lv["m"])
        ref_a = abs(Sl @ D).max()
        ref_r = abs(Sl).max()
        print("level %d: max|S D| %.3e, max|S| %.3e (host %.3e, %.3e)" % (l, a[l], r[l], ref_a, ref_r))
        assert a[l] <= 1e-11 * r[l]
        assert abs(r[l] - ref_r) <= 1e-12 * ref_r
        assert ref_a <= 1e-11 * ref_r
        if l + 1 < H.num_levels():
            arr, shp = H.export_csr(l, "Pe")
            Pe = sp.csr_matrix((arr[2], arr[1], arr[0]), shape=shp)
            Sl = O.csr(Pe.T @ Sl @ Pe)
    import paper_2506_08284_amd as P
    with pytest.raises(P.HcurlError):
        H.curl_residual(S, H.num_levels() + 1)


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_coefficients_and_lanczos_estimate(name):
    pr, m, levels, H = _case(name)
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    info = {}
    _, ito, _, _ = O.pcg(levels, pr["f"], info=info)
    al, be = H.export_vec(0, "pcg_alpha"), H.export_vec(0, "pcg_beta")
    assert len(al) == it and len(be) == it - 1
    k = min(it, ito)
    assert np.allclose(al[:k], info["alpha"][:k], rtol=1e-8, atol=0)
    assert np.allclose(be[:k - 1], info["beta"][:k - 1], rtol=1e-8, atol=0)
    st = H.stats()
    lo, hi = O.lanczos_extremes(al, be)
    assert abs(st["lanczos_lambda_min"] - lo) <= 1e-10 * lo
    assert abs(st["lanczos_lambda_max"] - hi) <= 1e-10 * hi
    if it == ito:
        lo_o, hi_o = O.lanczos_extremes(info["alpha"], info["beta"])
        assert abs(lo - lo_o) <= 1e-8 * lo_o and abs(hi - hi_o) <= 1e-8 * hi_o
    assert 0 < st["lanczos_lambda_min"] < st["lanczos_lambda_max"] <= 1.0 + 1e-6
    assert st["last_stagnated"] == 0


def test_stagnation_forced_by_zero_tolerance():
    """rtol = 0 cannot be met: the recursive residual keeps falling until the
    updates no longer change the iterate, and the solve returns
    HCURL_ESTAGNATE with u, iters and relres written, before maxit; the
    oracle stops the same way."""
    import paper_2506_08284_amd as P
    pr, m, levels, H = _case("cube8_const")
    n = pr["A"][0].shape[0] - 1
    u = np.full(n, np.nan)
    it, rel, rc = H.solve(pr["f"], u, 0.0, 400)
    info = {}
    _, ito, relo, _ = O.pcg(levels, pr["f"], tol=0.0, maxit=400, info=info)
    print("stagnation after %d iterations (oracle %d), relres %.2e (oracle %.2e)" % (it, ito, rel, relo))
    assert rc == P.HCURL_ESTAGNATE
    assert info["stagnated"]
    assert it < 400 and rel <= 1e-12 and np.all(np.isfinite(u))
    assert H.stats()["last_stagnated"] == 1
    # the same handle solves normally afterwards
    it2, rel2, rc2 = H.solve(pr["f"], u, 1e-8, 400)
    assert rc2 == 0 and rel2 <= 1e-8 and H.stats()["last_stagnated"] == 0


def test_infeasible_constraint_is_reported():
    """A caller P^(n) row with entries +-1e308 keeps a finite, non-zero row
    sum (the validation passes) but the commuting right-hand side of the
    edges at that node overflows: no finite P^(e) row meets it, and the
    setup fails with HCURL_EINFEASIBLE instead of returning non-finite
    values."""
    import paper_2506_08284_amd as P
    pr = synth.problem(5, sigma=("const", 1.0), f_seed=3)
    m = 216
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"])
    Pn = O.csr(levels[0]["Pn"]).copy()
    node = 3 * 36 + 3 * 6 + 3  # an interior node
    a, b = Pn.indptr[node], Pn.indptr[node + 1]
    assert b - a >= 3
    Pn.data[a] += 1e308
    Pn.data[a + 1] -= 1e308
    kw = dict(nodal_prolongator=(Pn.indptr.astype(np.int64), Pn.indices.astype(np.int32), Pn.data, Pn.shape[1]))
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m, **kw)
    assert e.value.code == P.HCURL_EINFEASIBLE
    # the unmodified prolongator is accepted
    Pn0 = O.csr(levels[0]["Pn"])
    kw0 = dict(nodal_prolongator=(Pn0.indptr.astype(np.int64), Pn0.indices.astype(np.int32), Pn0.data, Pn0.shape[1]))
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m, **kw0)
    H.close()


def test_full_pattern_level_makes_the_coarsest_operator_singular():
    """9^3 cube with 2-wide boxes on every level (9 -> 5 -> 3 -> 2 nodes per
    side): the 3^3 level's pattern holds every coarse edge, its guess has
    rank 8 of 19, and the 19-edge coarsest operator is singular to rounding
    (the oracle pins the closed form and the rank).  The library reports it
    at the coarsest factorisation as HCURL_ENOTSPD; the oracle's Cholesky
    factorisation fails on the same hierarchy."""
    import paper_2506_08284_amd as P
    import numpy.linalg as la
    N = 8
    pr = synth.problem(N, sigma=("const", 1.0), f_seed=1)
    maps, sides = synth.box_aggregates(N + 1, [2, 2, 2])
    m = (N + 1) ** 3
    with pytest.raises(la.LinAlgError):
        O.setup(pr["A"], pr["tail"], pr["head"], m, maps, {})
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), maps, n_nodes=m)
    assert e.value.code == P.HCURL_ENOTSPD and "coarsest" in str(e.value)
    # one level fewer: the 3^3 level is the coarsest, its operator is definite
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), maps[:2], n_nodes=m)
    assert H.num_levels() == 3
    H.close()
