"""GPU parity with Dirichlet (single-node) edges: boundary nodes and boundary
edges eliminated, D_h rows with one entry (Sec. 2), single-node coarse edges
weighted W = 2 in Alg. 2, full-rank local systems where they appear
(reading R27).  Coarse gradients, patterns and local pairs bit for bit; values
within the usual tolerances; the solve."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _export(H, level, which):
    arrs, shape = H.export_csr(level, which)
    return sp.csr_matrix((arrs[2], arrs[1], arrs[0]), shape=shape)


def _same_pattern(G, R):
    G, R = O.csr(G), O.csr(R)
    assert G.shape == R.shape
    assert np.array_equal(G.indptr, R.indptr) and np.array_equal(G.indices, R.indices)


def _close(G, R, rtol):
    _same_pattern(G, R)
    G, R = O.csr(G), O.csr(R)
    scale = max(abs(R.data).max(), 1e-300) if R.nnz else 1.0
    assert np.max(abs(G.data - R.data), initial=0.0) <= rtol * scale


CASES = {
    "incl10": dict(N=10, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=9),
    "lognormal12": dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_dirichlet_hierarchy_matches_oracle(name):
    import paper_2506_08284_amd as P
    p = synth.dirichlet_problem(**CASES[name])
    m = p["m"]
    opts = dict(aggregation="mis2", coarse_max_rows=150)
    levels = O.setup(p["A"], p["tail"], p["head"], m, p["aggregates"], dict(opts, record_energy=True))
    Dh = O.gradient_matrix(p["tail"], p["head"], m)
    H = P.Hierarchy(p["A"], (Dh.indptr.astype(np.int64), Dh.indices.astype(np.int32), Dh.data.copy()),
                    p["aggregates"], n_nodes=m, record_energy=1, **opts)
    assert H.num_levels() == len(levels) >= 3
    for l, lv in enumerate(levels[:-1]):
        assert np.array_equal(H.export_vec(l, "aggregates"), lv["agg"]), l
        DH = _export(H, l, "DH")
        ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], lv["Pn"].shape[1])
        _same_pattern(DH, ref)
        assert np.array_equal(O.csr(DH).data, O.csr(ref).data)
        assert np.any(lv["DH_tail"] < 0)
        _same_pattern(_export(H, l, "An"), lv["An"])
        _same_pattern(_export(H, l, "Pe"), lv["N"])
        lp = H.export_vec(l, "local_pairs")
        assert np.array_equal(lp & 255, lv["lt"]) and np.array_equal(lp >> 8, lv["lh"])
        assert np.any(lv["lt"] == O.MISSING)
        # cancellation ratio with one |D| entry on Dirichlet rows; it divides
        # by a diagonal of D^T A D whose own relative error is up to eps times
        # the ratio
        B = abs(lv["D"]).T @ abs(lv["A"]) @ abs(lv["D"])
        kappa_o = float(np.max(np.asarray(B.sum(axis=1)).ravel() / abs(lv["An"].diagonal())))
        kappa = H.level_info(l)["cancellation_ratio"]
        assert abs(kappa - kappa_o) <= max(1e-12, 100 * EPS * kappa_o) * kappa_o
        t_n, t_e = max(1e-11, 100 * EPS * kappa), max(1e-10, 1000 * EPS * kappa)
        _close(_export(H, l, "Pn"), lv["Pn"], t_n)
        _close(_export(H, l, "R"), lv["R"], t_n)
        _close(_export(H, l, "P0"), O.with_values(lv["N"], lv["p0"]), t_e)
        _close(_export(H, l, "Pe"), lv["Pe"], t_e)
        _close(_export(H, l + 1, "A"), levels[l + 1]["A"], t_e)
        E = H.export_vec(l, "energy")
        assert np.all(abs(E - np.array(lv["energies"])) <= t_e * abs(np.array(lv["energies"])))
    D0 = O.gradient_matrix(p["tail"], p["head"], m)
    C = _export(H, 0, "Pe") @ _export(H, 0, "DH") - D0 @ _export(H, 0, "Pn")
    assert abs(C).max() <= 1e-12 * abs(D0 @ _export(H, 0, "Pn")).max()
    # the library's own check, with single-node coarse edges on every level
    for l in range(H.num_levels() - 1):
        a, r = H.commute_residual(l)
        assert a <= 1e-12 * r, (l, a, r)
    n = p["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(p["f"], u, 1e-8, 500)
    uo, ito, _, _ = O.pcg(levels, p["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()


def test_dirichlet_learned_guess_is_refused():
    import paper_2506_08284_amd as P
    p = synth.dirichlet_problem(6)
    Dh = O.gradient_matrix(p["tail"], p["head"], p["m"])
    net = P.Network(np.zeros(P.hcurl_mpnn_num_params(), np.float32))
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(p["A"], (Dh.indptr.astype(np.int64), Dh.indices.astype(np.int32), Dh.data.copy()),
                    p["aggregates"], n_nodes=p["m"], coords=p["coords"], init_guess=2, mpnn=net,
                    aggregation="mis2", coarse_max_rows=100)
    assert e.value.code == P.HCURL_EUNSUPPORTED


def test_dirichlet_update_warm_matches_oracle():
    """Setup reuse on a boundary-eliminated problem: a second sigma field on
    the same mesh (same pattern), warm mode with MIS-2 levels below a box
    map; the rebuilt P^(n), the re-minimised P^(e) with its single-node
    coarse edges, the Galerkin operators and the solve against the oracle."""
    import paper_2506_08284_amd as P
    p1 = synth.dirichlet_problem(10, sigma=("lognormal", 6, 1.5), f_seed=3)
    p2 = synth.dirichlet_problem(10, sigma=("lognormal", 12, 1.5), f_seed=3)
    assert np.array_equal(p1["A"][0], p2["A"][0]) and np.array_equal(p1["A"][1], p2["A"][1])
    m = p1["m"]
    opts = dict(aggregation="mis2", coarse_max_rows=150)
    lv = O.setup(p1["A"], p1["tail"], p1["head"], m, p1["aggregates"], dict(opts, record_energy=True))
    ref = O.update(lv, p2["A"], "warm", iters=4)
    Dh = O.gradient_matrix(p1["tail"], p1["head"], m)
    H = P.Hierarchy(p1["A"], (Dh.indptr.astype(np.int64), Dh.indices.astype(np.int32), Dh.data.copy()),
                    p1["aggregates"], n_nodes=m, record_energy=1, **opts)
    H.update(p2["A"], "warm", 4)
    assert H.num_levels() == len(ref) >= 3
    for l, r in enumerate(ref[:-1]):
        kappa = H.level_info(l)["cancellation_ratio"]
        t_n, t_e = max(1e-11, 100 * EPS * kappa), max(1e-10, 1000 * EPS * kappa)
        _close(_export(H, l, "Pn"), r["Pn"], t_n)
        _close(_export(H, l, "R"), r["R"], t_n)
        _close(_export(H, l, "Pe"), r["Pe"], t_e)
        _close(_export(H, l + 1, "A"), ref[l + 1]["A"], t_e)
        a, rr = H.commute_residual(l)
        assert a <= 1e-12 * rr
    n = p2["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(p2["f"], u, 1e-8, 500)
    uo, ito, _, _ = O.pcg(ref, p2["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()
