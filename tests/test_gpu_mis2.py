"""GPU parity of MIS-2 aggregation (no caller aggregates; reading R26): the
aggregate maps of every level bit for bit against the oracle (they depend
only on the symbolic nodal patterns), the hierarchy built on them within the
usual tolerances, and the solve."""
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


@pytest.mark.parametrize("spec,cmr,maps", [
    (dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7), 200, 0),
    (dict(N=10, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=9), 100, 1),
])
def test_mis2_hierarchy_matches_oracle(spec, cmr, maps):
    """maps = number of leading levels with caller (box) aggregates; MIS-2
    takes over below them."""
    import paper_2506_08284_amd as P
    pr = synth.problem(**spec)
    m = (spec["N"] + 1) ** 3
    aggs = list(pr["aggregates"][:maps])
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, aggs, dict(aggregation="mis2", coarse_max_rows=cmr))
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), aggs, n_nodes=m,
                    aggregation="mis2", coarse_max_rows=cmr)
    assert H.num_levels() == len(levels) >= 3
    for l, lv in enumerate(levels[:-1]):
        assert np.array_equal(H.export_vec(l, "aggregates"), lv["agg"]), l
        _same_pattern(_export(H, l, "An"), lv["An"])
        _same_pattern(_export(H, l, "Pe"), lv["N"])
        DH = _export(H, l, "DH")
        ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], lv["Pn"].shape[1])
        _same_pattern(DH, ref)
        assert np.array_equal(O.csr(DH).data, O.csr(ref).data)
        kappa = H.level_info(l)["cancellation_ratio"]
        t_n, t_e = max(1e-11, 100 * EPS * kappa), max(1e-10, 1000 * EPS * kappa)
        _close(_export(H, l, "Pn"), lv["Pn"], t_n)
        _close(_export(H, l, "Pe"), lv["Pe"], t_e)
        _close(_export(H, l + 1, "A"), levels[l + 1]["A"], t_e)
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    uo, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()


def test_mis2_requires_a_map_or_the_option():
    import paper_2506_08284_amd as P
    pr = synth.problem(4)
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    # no maps and no aggregation option: a single level, solved directly
    H = P.Hierarchy(pr["A"], Dh, [], n_nodes=125)
    assert H.num_levels() == 1
    H.close()
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], Dh, [None], n_nodes=125)
    assert e.value.code == P.HCURL_EINVAL
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], Dh, [], n_nodes=125, aggregation=5)
    assert e.value.code == P.HCURL_EINVAL


@pytest.mark.slow
def test_mis2_level0_at_64cubed():
    """The 64^3 jittered lognormal cube (1,872,064 edges): the level-0 MIS-2
    map bit for bit against the oracle's, then setup and solve to 1e-8."""
    import paper_2506_08284_amd as P
    pr = synth.workload("cube64_jitter_lognormal")
    m = 65 ** 3
    A = O.csr(pr["A"])
    An = O.nodal_operator(A, O.gradient_matrix(pr["tail"], pr["head"], m))
    ref = O.mis2_aggregates(An)
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [], n_nodes=m, aggregation="mis2",
                    coarse_max_rows=1024)
    assert np.array_equal(H.export_vec(0, "aggregates"), ref)
    n = A.shape[0]
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    assert rc == 0 and rel <= 1e-8 and it < 80
    H.close()
