"""GPU parity on irregular aggregates: seeded random connected aggregates
grown breadth-first over the mesh graph (synth.random_aggregates) on level
0, MIS-2 below.  Local systems up to |J| = 12 and uneven coarse edges; the
same bar as the other parity cases: structures bit for bit, values within
the cancellation-widened tolerances, the solve."""
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


@pytest.mark.parametrize("seed,size,spec", [
    (1, 10, dict(N=10, jitter=0.15, jitter_seed=2, sigma=("lognormal", 3, 1.5), f_seed=6)),
    (2, 14, dict(N=10, sigma=("inclusions", 7, 1.0, 1e-4), f_seed=8)),
    (3, 6, dict(N=9, sigma=("const", 1.0), f_seed=1)),
])
def test_random_aggregates_match_oracle(seed, size, spec):
    import paper_2506_08284_amd as P
    pr = synth.problem(**spec)
    m = (spec["N"] + 1) ** 3
    agg = synth.random_aggregates(pr["tail"], pr["head"], m, size, seed)
    opts = dict(aggregation="mis2", coarse_max_rows=200)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, [agg], dict(opts, record_energy=True))
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [agg], n_nodes=m, record_energy=1, **opts)
    assert H.num_levels() == len(levels) >= 3
    for l, lv in enumerate(levels[:-1]):
        assert np.array_equal(H.export_vec(l, "aggregates"), lv["agg"]), l
        DH = _export(H, l, "DH")
        ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], lv["Pn"].shape[1])
        _same_pattern(DH, ref)
        assert np.array_equal(O.csr(DH).data, O.csr(ref).data)
        assert H.level_info(l)["irreducible_added"] == lv["irreducible_added"]
        _same_pattern(_export(H, l, "An"), lv["An"])
        _same_pattern(_export(H, l, "R"), lv["R"])
        _same_pattern(_export(H, l, "Pe"), lv["N"])
        lp = H.export_vec(l, "local_pairs")
        assert np.array_equal(lp & 255, lv["lt"]) and np.array_equal(lp >> 8, lv["lh"])
        assert np.array_equal(H.export_vec(l, "colors_A"), lv["colors_A"])
        kappa = H.level_info(l)["cancellation_ratio"]
        t_n, t_e = max(1e-11, 100 * EPS * kappa), max(1e-10, 1000 * EPS * kappa)
        _close(_export(H, l, "Pn"), lv["Pn"], t_n)
        _close(_export(H, l, "R"), lv["R"], t_n)
        _close(_export(H, l, "P0"), O.with_values(lv["N"], lv["p0"]), t_e)
        _close(_export(H, l, "Pe"), lv["Pe"], t_e)
        _close(_export(H, l + 1, "A"), levels[l + 1]["A"], t_e)
        E = H.export_vec(l, "energy")
        assert np.all(abs(E - np.array(lv["energies"])) <= t_e * abs(np.array(lv["energies"])))
        a, r = H.commute_residual(l)
        assert a <= 1e-12 * r
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 300)
    uo, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()
