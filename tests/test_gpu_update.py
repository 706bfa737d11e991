"""GPU parity of setup reuse (hcurl_amg_update) against the oracle's update:
two systems on one mesh (lognormal sigma from two seeds, same pattern).

* transfers mode: every A_l, A^(n)_l of the re-projected hierarchy, the
  V-cycle and the solve;
* warm mode: the rebuilt P^(n), the re-minimised P^(e) and its energies, the
  Galerkin operators and the solve;
* device pointers on a stream (graphs captured before the update are
  dropped and captured again) against the host-pointer run;
* errors: a different pattern is refused and leaves the handle usable;
* updates in a row on one handle (the products' kept patterns reused)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
SPEC1 = dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7)
SPEC2 = dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 11, 2.0), f_seed=7)

_cache = {}


def _pair():
    if "p" not in _cache:
        p1, p2 = synth.problem(**SPEC1), synth.problem(**SPEC2)
        m = 13 ** 3
        lv = O.setup(p1["A"], p1["tail"], p1["head"], m, p1["aggregates"], dict(record_energy=True))
        _cache["p"] = (p1, p2, m, lv)
    return _cache["p"]


def _export(H, level, which):
    arrs, shape = H.export_csr(level, which)
    return sp.csr_matrix((arrs[2], arrs[1], arrs[0]), shape=shape)


def _close(G, R, rtol):
    G, R = O.csr(G), O.csr(R)
    assert np.array_equal(G.indptr, R.indptr) and np.array_equal(G.indices, R.indices)
    scale = max(abs(R.data).max(), 1e-300) if R.nnz else 1.0
    assert np.max(abs(G.data - R.data), initial=0.0) <= rtol * scale


def _hierarchy(p, m, **kw):
    import paper_2506_08284_amd as P
    return P.Hierarchy(p["A"], synth.gradient_csr(p["tail"], p["head"]), p["aggregates"], n_nodes=m, **kw)


def _kappa(lv):
    B = abs(lv["D"]).T @ abs(lv["A"]) @ abs(lv["D"])
    return float(np.max(np.asarray(B.sum(axis=1)).ravel() / abs(lv["An"].diagonal())))


def test_update_transfers_matches_oracle():
    p1, p2, m, lv = _pair()
    ref = O.update(lv, p2["A"], "transfers")
    H = _hierarchy(p1, m)
    H.update(p2["A"], "transfers")
    assert H.num_levels() == len(ref)
    for l, r in enumerate(ref[:-1]):
        t_e = max(1e-10, 1000 * EPS * _kappa(r))
        _close(_export(H, l, "A"), r["A"], t_e)
        _close(_export(H, l, "An"), r["An"], max(1e-12, 10 * EPS * _kappa(r)) if l == 0 else t_e)
        # the transfers are the setup's
        _close(_export(H, l, "Pe"), lv[l]["Pe"], t_e)
        assert len(H.export_vec(l, "energy")) == 0
    _close(_export(H, len(ref) - 1, "A"), ref[-1]["A"], max(1e-10, 1000 * EPS * _kappa(ref[-2])))
    n = p2["A"][0].shape[0] - 1
    r = np.random.default_rng(4).standard_normal(n)
    z = np.empty(n)
    H.vcycle(r, z)
    zo = O.vcycle(ref, r)
    assert np.linalg.norm(z - zo) <= 1e-8 * np.linalg.norm(zo)
    u = np.empty(n)
    it, rel, rc = H.solve(p2["f"], u, 1e-8, 500)
    uo, ito, _, _ = O.pcg(ref, p2["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    assert H.stats()["update_ms"] > 0
    H.close()


def test_update_warm_matches_oracle():
    p1, p2, m, lv = _pair()
    ref = O.update(lv, p2["A"], "warm", iters=4)
    H = _hierarchy(p1, m, record_energy=1)
    H.update(p2["A"], "warm", 4)
    for l, r in enumerate(ref[:-1]):
        kappa = _kappa(r)
        t_n, t_e = max(1e-11, 100 * EPS * kappa), max(1e-10, 1000 * EPS * kappa)
        info = H.level_info(l)
        assert abs(info["rho"] - r["sa"]["rho"]) <= max(1e-10, 100 * EPS * kappa) * r["sa"]["rho"]
        _close(_export(H, l, "Pn"), r["Pn"], t_n)
        _close(_export(H, l, "R"), r["R"], t_n)
        _close(_export(H, l, "P0"), O.with_values(r["N"], r["p0"]), t_e)
        _close(_export(H, l, "Pe"), r["Pe"], t_e)
        _close(_export(H, l + 1, "A"), ref[l + 1]["A"], t_e)
        E = H.export_vec(l, "energy")
        Eo = np.array(r["energies"])
        assert len(E) == 5 and np.all(abs(E - Eo) <= t_e * abs(Eo))
    # the commuting relation for the rebuilt operators
    D = O.gradient_matrix(p2["tail"], p2["head"], m)
    C = _export(H, 0, "Pe") @ _export(H, 0, "DH") - D @ _export(H, 0, "Pn")
    assert abs(C).max() <= 1e-12 * abs(D @ _export(H, 0, "Pn")).max()
    for l in range(H.num_levels() - 1):
        a, r = H.commute_residual(l)
        assert a <= 1e-12 * r
    n = p2["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(p2["f"], u, 1e-8, 500)
    uo, ito, _, _ = O.pcg(ref, p2["f"])
    assert rc == 0 and rel <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)
    H.close()


def test_update_on_a_stream_with_graphs_matches_host_run():
    """Solve (graphs captured), update, solve again: the second solve uses the
    new operators, as the host-pointer hierarchy updated the same way does."""
    import torch
    import paper_2506_08284_amd as P
    p1, p2, m, lv = _pair()
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    with torch.cuda.stream(side):
        A1 = tuple(T(a) for a in p1["A"])
        A2 = tuple(T(a) for a in p2["A"])
        D_t = tuple(T(a) for a in synth.gradient_csr(p1["tail"], p1["head"]))
        aggs = [T(a) for a in p1["aggregates"]]
        f = T(p2["f"])
        u1, u2 = torch.empty_like(f), torch.empty_like(f)
        side.synchronize()
        H = P.Hierarchy(A1, D_t, aggs, n_nodes=m, mem_space="device", stream=side.cuda_stream)
        H.solve(f, u1)
        H.update(A2, "warm", 3)
        it, rel, rc = H.solve(f, u2)
        side.synchronize()
    Hh = _hierarchy(p1, m)
    Hh.update(p2["A"], "warm", 3)
    uh = np.empty_like(p2["f"])
    ith, relh, _ = Hh.solve(p2["f"], uh)
    assert rc == 0 and abs(it - ith) <= 1 and rel <= 1e-8
    assert np.linalg.norm(u2.cpu().numpy() - uh) <= 1e-9 * np.linalg.norm(uh)
    H.close()
    Hh.close()


def test_update_errors_leave_the_handle_usable():
    import paper_2506_08284_amd as P
    p1, p2, m, lv = _pair()
    H = _hierarchy(p1, m)
    rp, col, val = p2["A"]
    bad = (rp, col.copy(), val)
    i = int(np.nonzero(np.diff(rp) >= 2)[0][0])
    a = int(rp[i])
    bad[1][a], bad[1][a + 1] = bad[1][a + 1], bad[1][a]  # unsorted row: malformed
    with pytest.raises(P.HcurlError) as e:
        H.update(bad, "transfers")
    assert e.value.code == P.HCURL_EINVAL
    other = synth.problem(12, sigma=("const", 1.0))  # same mesh size, no jitter: same pattern
    q = synth.problem(11, sigma=("const", 1.0))      # another size: another pattern
    with pytest.raises(P.HcurlError) as e:
        H.update(q["A"], "transfers")
    assert e.value.code == P.HCURL_EINVAL
    with pytest.raises(P.HcurlError) as e:
        H.update(p2["A"], 7)
    assert e.value.code == P.HCURL_EINVAL
    n = p1["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(p1["f"], u)
    assert rc == 0 and rel <= 1e-8
    H.update(other["A"], "transfers")
    it, rel, rc = H.solve(other["f"], u)
    assert rc == 0 and rel <= 1e-8
    H.close()


def test_repeated_updates_reuse_the_kept_product_patterns():
    """Updates in a row on one handle (A1 -> A2 -> A1, transfers kept, then A2
    warm) run only the numeric passes of the products on the patterns kept
    from the setup: going back to A1 gives the setup's operators on every
    level, and the final warm update the operators of a fresh setup on A1
    followed by the same warm update, both to rounding."""
    p1, p2, m, lv = _pair()
    H = _hierarchy(p1, m)
    nl = H.num_levels()
    ref = [(_export(H, l, "A"), _export(H, l, "An") if l + 1 < nl else None) for l in range(nl)]
    H.update(p2["A"], "transfers")
    H.update(p1["A"], "transfers")
    for l in range(nl):
        _close(_export(H, l, "A"), ref[l][0], 1e-12)
        if ref[l][1] is not None:
            _close(_export(H, l, "An"), ref[l][1], 1e-12)
    H.update(p2["A"], "warm", 3)
    H2 = _hierarchy(p1, m)
    H2.update(p2["A"], "warm", 3)
    for l in range(nl):
        _close(_export(H, l, "A"), _export(H2, l, "A"), 1e-12)
    for l in range(nl - 1):
        _close(_export(H, l, "Pe"), _export(H2, l, "Pe"), 1e-12)
    n = p2["A"][0].shape[0] - 1
    u, u2 = np.empty(n), np.empty(n)
    it, rel, rc = H.solve(p2["f"], u)
    it2, rel2, rc2 = H2.solve(p2["f"], u2)
    assert rc == rc2 == 0 and rel <= 1e-8 and abs(it - it2) <= 1
    H.close()
    H2.close()
