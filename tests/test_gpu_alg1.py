"""GPU parity of the Alg. 1 paths.

* Setup from a caller-given level-0 nodal prolongator: rows scaled to sum one,
  aggregates for P-bar and D_H from Alg. 1 (with the details of reading R5),
  everything after that as on the aggregate path.  Inputs come from the
  oracle and synth only: the oracle's smoothed-aggregation P^(n), and two
  variants with its pattern (random positive factors; small integers, which
  make ties everywhere).  Alg. 1's map is compared bit for bit.
* P-bar from Alg. 1 on the library's own smoothed P^(n) (the paper's runs).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps

SPEC = dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7)


def _export(H, level, which):
    arrs, shape = H.export_csr(level, which)
    return sp.csr_matrix((arrs[2], arrs[1], arrs[0]), shape=shape)


def _same_pattern(G, R):
    G, R = O.csr(G), O.csr(R)
    assert G.shape == R.shape
    assert np.array_equal(G.indptr, R.indptr)
    assert np.array_equal(G.indices, R.indices)


def _close(G, R, rtol):
    G, R = O.csr(G), O.csr(R)
    scale = max(abs(R.data).max(), 1e-300) if R.nnz else 1.0
    assert np.max(abs(G.data - R.data), initial=0.0) <= rtol * scale


_cache = {}


def _problem():
    if "pr" not in _cache:
        pr = synth.problem(**SPEC)
        m = pr["mesh"]["n"] ** 3
        A = O.csr(pr["A"])
        D = O.gradient_matrix(pr["tail"], pr["head"], m)
        agg = pr["aggregates"][0]
        Pn, _ = O.sa_prolongator(O.nodal_operator(A, D), agg, int(agg.max()) + 1)
        _cache["pr"] = (pr, m, O.csr(Pn))
    return _cache["pr"]


def _variant(Pn, kind):
    P = Pn.copy()
    rng = np.random.default_rng(3)
    if kind == "factors":
        P.data = abs(P.data) * rng.uniform(0.2, 1.8, P.nnz)
    elif kind == "ties":
        P.data = rng.integers(1, 4, P.nnz).astype(np.float64)
    return P


def _hierarchy(pr, m, P, passes, aggs0=None, **kw):
    import paper_2506_08284_amd as Pk
    P = O.csr(P)
    given = (P.indptr.astype(np.int64), P.indices.astype(np.int32), np.ascontiguousarray(P.data), P.shape[1])
    return Pk.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [aggs0] + list(pr["aggregates"][1:]),
                        n_nodes=m, nodal_prolongator=given, alg1_passes=passes, **kw)


@pytest.mark.parametrize("kind", ["sa", "factors", "ties"])
@pytest.mark.parametrize("passes", [1, 2, 3])
def test_alg1_aggregates_and_scaled_prolongator_bit_exact(kind, passes):
    pr, m, Pn = _problem()
    P = _variant(Pn, kind)
    Ps = O.scale_rows_to_one(P)
    ref = O.piecewise_constant_assignment(Ps, passes)
    H = _hierarchy(pr, m, P, passes)
    assert np.array_equal(H.export_vec(0, "aggregates"), ref)
    G = O.csr(_export(H, 0, "Pn"))
    _same_pattern(G, Ps)
    assert np.array_equal(G.data, Ps.data)
    # D_H from the derived aggregates, bit for bit
    DH_t, DH_h = O.coarse_gradient(O.gradient_matrix(pr["tail"], pr["head"], m), ref, Ps.shape[1])[:2]
    ref_DH = O.gradient_matrix(DH_t, DH_h, Ps.shape[1])
    DH = _export(H, 0, "DH")
    _same_pattern(DH, ref_DH)
    assert np.array_equal(O.csr(DH).data, O.csr(ref_DH).data)
    H.close()


@pytest.mark.parametrize("kind", ["sa", "ties"])
def test_hierarchy_from_given_prolongator_matches_oracle(kind):
    """The whole hierarchy and the solve against the oracle set up from the
    same P^(n) (tolerances as on the aggregate path)."""
    pr, m, Pn = _problem()
    P = _variant(Pn, kind)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, [None] + list(pr["aggregates"][1:]),
                     dict(Pn=P, alg1_passes=2, record_energy=True))
    H = _hierarchy(pr, m, P, 2, record_energy=1)
    assert H.num_levels() == len(levels)
    for l, lv in enumerate(levels[:-1]):
        assert np.array_equal(H.export_vec(l, "aggregates"), lv["agg"])
        _same_pattern(_export(H, l, "An"), lv["An"])
        _same_pattern(_export(H, l, "Pn"), lv["Pn"])
        _same_pattern(_export(H, l, "R"), lv["R"])
        _same_pattern(_export(H, l, "Pe"), lv["N"])
        lp = H.export_vec(l, "local_pairs")
        assert np.array_equal(lp & 255, lv["lt"]) and np.array_equal(lp >> 8, lv["lh"])
        assert np.array_equal(H.export_vec(l, "colors_A"), lv["colors_A"])
        kappa = H.level_info(l)["cancellation_ratio"]
        t_n, t_e = max(1e-11, 100 * EPS * kappa), max(1e-10, 1000 * EPS * kappa)
        _close(_export(H, l, "Pn"), lv["Pn"], t_n)
        _close(_export(H, l, "R"), lv["R"], t_n)
        _close(_export(H, l, "Pe"), lv["Pe"], t_e)
        _close(_export(H, l + 1, "A"), levels[l + 1]["A"], t_e)
        E = H.export_vec(l, "energy")
        assert np.all(abs(E - np.array(lv["energies"])) <= t_e * abs(np.array(lv["energies"])))
    assert H.level_info(0)["rho"] == 0.0
    # commuting relation on the GPU's own level-0 operators
    D = O.gradient_matrix(pr["tail"], pr["head"], m)
    C = _export(H, 0, "Pe") @ _export(H, 0, "DH") - D @ _export(H, 0, "Pn")
    assert abs(C).max() <= 1e-12 * abs(D @ _export(H, 0, "Pn")).max()
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    uo, ito, relo, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()


def test_given_prolongator_with_given_aggregates():
    """P^(n) given together with aggregates: the aggregates feed P-bar as given
    and the prolongator is used as given (rows scaled)."""
    pr, m, Pn = _problem()
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"], dict(Pn=Pn))
    H = _hierarchy(pr, m, Pn, 2, aggs0=pr["aggregates"][0])
    assert np.array_equal(H.export_vec(0, "aggregates"), pr["aggregates"][0])
    DH = _export(H, 0, "DH")
    ref = O.gradient_matrix(levels[0]["DH_tail"], levels[0]["DH_head"], Pn.shape[1])
    _same_pattern(DH, ref)
    assert np.array_equal(O.csr(DH).data, O.csr(ref).data)
    _same_pattern(_export(H, 0, "Pe"), levels[0]["N"])
    H.close()


def test_alg1_safeguard_fills_an_empty_column():
    """Rows 0 and 1 = [1.2, -0.2], every other row [1, 0]: in one pass column 0
    takes its m-1 largest rows including 0 and 1, column 1 finds none free,
    the last row goes to column 0 greedily, and the safeguard moves row 0
    (|-0.2| tie -> smaller row) to column 1.  The two-node coarse level that
    follows is set up and solved like any other."""
    import paper_2506_08284_amd as Pk
    pr, m, _ = _problem()
    rp = np.concatenate([[0, 2], 4 + np.arange(m - 1, dtype=np.int64)])
    col = np.concatenate([[0, 1, 0, 1], np.zeros(m - 2)]).astype(np.int32)
    val = np.concatenate([[1.2, -0.2, 1.2, -0.2], np.ones(m - 2)])
    P = O.csr((rp, col, val), shape=(m, 2))
    ref = O.piecewise_constant_assignment(P, 1)
    assert ref[0] == 1 and np.all(ref[1:] == 0)
    H = Pk.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [None], n_nodes=m,
                     nodal_prolongator=(rp, col, val, 2), alg1_passes=1)
    assert np.array_equal(H.export_vec(0, "aggregates"), ref)
    assert H.num_levels() == 2
    H.close()


def test_given_prolongator_errors():
    import paper_2506_08284_amd as Pk
    pr, m, Pn = _problem()
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    # a row summing to zero
    Z = Pn.copy()
    Z.data[Pn.indptr[0]:Pn.indptr[1]] = 0.0
    with pytest.raises(Pk.HcurlError) as e:
        _hierarchy(pr, m, Z, 2)
    assert e.value.code == Pk.HCURL_EINVAL
    # columns out of order within a row
    if Pn.indptr[1] - Pn.indptr[0] >= 2:
        B = Pn.copy()
        B.indices = B.indices.copy()
        B.indices[[0, 1]] = B.indices[[1, 0]]
        given = (B.indptr.astype(np.int64), B.indices.astype(np.int32), B.data.copy(), B.shape[1])
        with pytest.raises(Pk.HcurlError) as e:
            Pk.Hierarchy(pr["A"], Dh, [None] + list(pr["aggregates"][1:]), n_nodes=m, nodal_prolongator=given)
        assert e.value.code == Pk.HCURL_EINVAL
    # an empty column no row can move to: row 0 = [1.2, -0.2, 0] is column 0's
    # only row and column 1's only row; every other row is [0, 0, 1]
    rp = np.concatenate([[0], 2 + np.arange(m, dtype=np.int64)])
    col = np.concatenate([[0, 1], np.full(m - 1, 2)]).astype(np.int32)
    val = np.concatenate([[1.2, -0.2], np.ones(m - 1)])
    O.csr((rp, col, val), shape=(m, 3))  # well formed
    with pytest.raises(ValueError):
        O.piecewise_constant_assignment(O.csr((rp, col, val), shape=(m, 3)), 2)
    with pytest.raises(Pk.HcurlError) as e:
        Pk.Hierarchy(pr["A"], Dh, [None], n_nodes=m, nodal_prolongator=(rp, col, val, 3))
    assert e.value.code == Pk.HCURL_EINVAL
    # no aggregates and no prolongator
    with pytest.raises(Pk.HcurlError) as e:
        Pk.Hierarchy(pr["A"], Dh, [None], n_nodes=m)
    assert e.value.code == Pk.HCURL_EINVAL


def _rs_edges(tail, head, a):
    """Coarse edges of the RS rule on the map a: every pair (I, K), I < K, of
    aggregates joined by a fine edge, in lexicographic order."""
    I, K = a[tail], a[head]
    cross = I != K
    lo, hi = np.minimum(I, K)[cross], np.maximum(I, K)[cross]
    pairs = np.unique(np.stack([lo, hi], axis=1), axis=0)
    return pairs[:, 0], pairs[:, 1]


def test_pbar_from_alg1_on_smoothed_prolongator():
    """P-bar by Alg. 1 on the smoothed P^(n) of every level.  The GPU's P^(n)
    differs from the oracle's in rounding, which can move near-tied choices
    of Alg. 1, so the map is compared in bulk; what follows from the map (D_H
    by the RS rule, the commuting relation, convergence) is checked exactly
    or against the oracle's solve."""
    import paper_2506_08284_amd as Pk
    pr, m, _ = _problem()
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"], dict(pbar_alg1=True))
    H = Pk.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m, pbar_alg1=1)
    assert H.num_levels() == len(levels)
    tail, head = np.asarray(pr["tail"]), np.asarray(pr["head"])
    for l, lv in enumerate(levels[:-1]):
        a = H.export_vec(l, "aggregates")
        Pn = O.csr(_export(H, l, "Pn"))
        assert np.mean(a == lv["agg"]) >= 0.98, l
        # the map takes a column of the node's own row and covers every column
        for i in range(Pn.shape[0]):
            assert a[i] in Pn.indices[Pn.indptr[i]:Pn.indptr[i + 1]]
        assert np.all(np.bincount(a, minlength=Pn.shape[1]) > 0)
        # D_H is the RS rule on this map, bit for bit
        DH = O.csr(_export(H, l, "DH"))
        t, h = _rs_edges(tail, head, a)
        assert DH.shape[0] == len(t)
        assert np.array_equal(DH.indices[0::2], t) and np.array_equal(DH.indices[1::2], h)
        assert np.all(DH.data[0::2] == -1.0) and np.all(DH.data[1::2] == 1.0)
        # commuting relation on the GPU's own operators
        Dl = O.gradient_matrix(tail, head, Pn.shape[0])
        DPn = Dl @ Pn
        C = _export(H, l, "Pe") @ DH - DPn
        assert abs(C).max() <= 1e-12 * abs(DPn).max(), l
        # next level's endpoints
        tail, head = t, h
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    _, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 2
    H.close()
