"""Degenerate inputs on the GPU: a zero right-hand side, an empty problem, a
single aggregate (no coarse edge), every node its own aggregate (a coarse
level as large as the fine one), and a problem small enough to be the
coarsest level at once."""
import numpy as np
import pytest

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2506_08284_amd as P
    return P


def test_zero_right_hand_side_gives_zero_solution():
    P = _lib()
    pr = synth.problem(6, sigma=("const", 1.0))
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=343)
    u = np.full(pr["A"][0].shape[0] - 1, 7.0)
    it, rel, rc = H.solve(np.zeros_like(u), u)
    assert rc == 0 and it == 0 and rel == 0.0 and np.all(u == 0.0)
    H.close()


def test_empty_problem_is_rejected():
    P = _lib()
    A = (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(A, (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0)), [], n_nodes=0)
    assert e.value.code == P.HCURL_EINVAL


def test_single_aggregate_is_rejected():
    """All nodes in one aggregate: no coarse edge exists, so there is no
    transfer to build."""
    P = _lib()
    pr = synth.problem(4)
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], Dh, [np.zeros(125, np.int32)], n_nodes=125)
    assert e.value.code == P.HCURL_EINVAL


def test_identity_aggregates_against_oracle():
    """Every node its own aggregate: the coarse level has the fine level's
    size, D_H = D_h, P^(n) is the smoothed identity; structures bit for bit,
    the solve against the oracle's."""
    P = _lib()
    pr = synth.problem(4, jitter=0.1, jitter_seed=3, sigma=("lognormal", 4, 1.0), f_seed=2)
    m = 125
    ident = np.arange(m, dtype=np.int32)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, [ident])
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [ident], n_nodes=m)
    arrs, shape = H.export_csr(0, "DH")
    assert np.array_equal(arrs[1], O.gradient_matrix(pr["tail"], pr["head"], m).indices)
    assert H.level_info(1)["n_edges"] == pr["A"][0].shape[0] - 1
    arrs, shape = H.export_csr(0, "Pe")
    assert np.array_equal(arrs[0], levels[0]["N"].indptr) and np.array_equal(arrs[1], levels[0]["N"].indices)
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u)
    uo, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    H.close()


def test_slab_aggregates_long_transposed_rows():
    """Three slabs of 5 x 15 x 15 nodes as the aggregates: the transposes of
    P^(n) and P^(e) get rows of more than 1024 entries (the interface's coarse
    edge lies in the pattern of thousands of fine edges), which the library
    sorts in its long-row path.  Structures bit for bit, the coarse operator
    and the solve against the oracle."""
    P = _lib()
    N = 14
    m = (N + 1) ** 3
    pr = synth.problem(N, sigma=("const", 1.0), f_seed=5)
    agg = ((np.arange(m) % (N + 1)) // 5).astype(np.int32)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, [agg])
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [agg], n_nodes=m)
    assert H.num_levels() == len(levels) == 2
    Pe = O.csr(levels[0]["N"])
    assert np.bincount(Pe.indices).max() > 1024
    arrs, shape = H.export_csr(0, "Pe")
    assert np.array_equal(arrs[0], Pe.indptr) and np.array_equal(arrs[1], Pe.indices)
    ref = O.csr(levels[0]["Pe"])
    assert np.max(abs(arrs[2] - ref.data)) <= 1e-10 * abs(ref.data).max()
    arrs, shape = H.export_csr(0, "DH")
    DH = O.gradient_matrix(levels[0]["DH_tail"], levels[0]["DH_head"], 3)
    assert np.array_equal(arrs[1], DH.indices) and np.array_equal(arrs[2], DH.data)
    a, r = H.commute_residual(0)
    assert a <= 1e-12 * r
    arrs, shape = H.export_csr(1, "A")
    A1 = O.csr(levels[1]["A"])
    assert np.array_equal(arrs[0], A1.indptr) and np.array_equal(arrs[1], A1.indices)
    assert np.max(abs(arrs[2] - A1.data)) <= 1e-10 * abs(A1.data).max()
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u)
    uo, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()


def test_fine_edge_touching_too_many_coarse_nodes_is_refused():
    """A caller P^(n) whose row reaches 40 coarse nodes gives fine edges with
    |T_i| > 32, beyond the library's local-system layouts: HCURL_EUNSUPPORTED,
    not a wrong answer."""
    P = _lib()
    pr = synth.problem(6)
    m = 343
    maps, _ = synth.box_aggregates(7, width=2)
    agg = maps[0]
    mH = int(agg.max()) + 1
    assert mH == 64
    Pn = O.tentative_prolongator(agg, mH).tolil()
    Pn[0, :] = 0.0
    for j in range(40):
        Pn[0, j] = 1.0 / 40
    Pn = O.csr(Pn.tocsr())
    given = (Pn.indptr.astype(np.int64), Pn.indices.astype(np.int32), Pn.data.copy(), mH)
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [agg], n_nodes=m, nodal_prolongator=given)
    assert e.value.code == P.HCURL_EUNSUPPORTED
    assert "32 coarse nodes" in str(e.value)


def test_largest_local_systems_against_oracle():
    """A caller P^(n) whose row 0 spreads over 30 coarse nodes (a 3 x 3 x 3 +
    3 block of aggregates) gives fine edges with |T_i| = 30: the widest
    local-system layout the library has (32).  Pattern, local pairs and D_H
    bit for bit, P^(e) within the usual tolerance (also with the masked
    product searching in every launch: up to 105 pattern entries per row), the
    solve."""
    import scipy.sparse as sp
    P = _lib()
    pr = synth.problem(6, sigma=("const", 1.0), f_seed=2)
    m = 343
    maps, _ = synth.box_aggregates(7, width=2)
    agg = maps[0]
    mH = int(agg.max()) + 1
    Pn = O.tentative_prolongator(agg, mH).tolil()
    cols = [0, 1, 2, 4, 5, 6, 8, 9, 10, 16, 17, 18, 20, 21, 22, 24, 25, 26, 32, 33, 34, 36, 37, 38, 40, 41, 42,
            48, 49, 50]
    Pn[0, :] = 0.0
    for j in cols:
        Pn[0, j] = 1.0 / len(cols)
    Pn = O.csr(Pn.tocsr())
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, [agg], dict(Pn=Pn))
    lv = levels[0]
    assert np.diff(O.csr(lv["R"]).indptr).max() == 30
    given = (Pn.indptr.astype(np.int64), Pn.indices.astype(np.int32), Pn.data.copy(), mH)
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [agg], n_nodes=m, nodal_prolongator=given)
    ex = lambda w: (lambda a: sp.csr_matrix((a[0][2], a[0][1], a[0][0]), shape=a[1]))(H.export_csr(0, w))
    DH = O.csr(ex("DH"))
    ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], mH)
    assert np.array_equal(DH.indptr, ref.indptr) and np.array_equal(DH.indices, ref.indices)
    Pe = O.csr(ex("Pe"))
    N = O.csr(lv["N"])
    assert np.array_equal(Pe.indptr, N.indptr) and np.array_equal(Pe.indices, N.indices)
    lp = H.export_vec(0, "local_pairs")
    assert np.array_equal(lp & 255, lv["lt"]) and np.array_equal(lp >> 8, lv["lh"])
    assert np.max(abs(Pe.data - O.csr(lv["Pe"]).data)) <= 1e-10 * abs(lv["Pe"].data).max()
    # pattern rows of more than 64 entries put the masked product in its wide
    # row blocks; the recorded codes and the searching form agree there too
    assert np.diff(N.indptr).max() > 64
    H0 = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), [agg], n_nodes=m, nodal_prolongator=given,
                     emin_codes=0)
    Pe0 = H0.export_csr(0, "Pe")[0][2]
    H0.close()
    assert np.max(abs(Pe.data - Pe0)) <= 1e-13 * abs(Pe0).max()
    a, r = H.commute_residual(0)
    assert a <= 1e-12 * r
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u)
    uo, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    H.close()
