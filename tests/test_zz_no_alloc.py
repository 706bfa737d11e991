"""hcurl_amg_solve_noalloc, the solve that allocates no device memory, against
hcurl_amg_solve through the C ABI: the same kernels on the same hierarchy, so
the solutions agree to the last bit and the iteration counts are equal.  Two
calls in a row share the GPU's staging array; the second has a smaller input."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _host_hierarchy(N, sigma, f_seed, **opts):
    import paper_2506_08284_amd as P
    pr = synth.problem(N=N, sigma=sigma, f_seed=f_seed, **({"jitter": 0.2, "jitter_seed": 5} if N > 8 else {}))
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=pr["mesh"]["n"] ** 3, **opts)
    return H, pr


def _check_same(H, f):
    n = f.shape[0]
    u_ref = np.full(n, np.nan)
    it_ref, rel_ref, rc_ref = H.solve(f, u_ref, 1e-8, 300)
    u = np.full(n, np.nan)  # the staging array still holds the previous call's u
    it, rel, rc = H.solve_noalloc(f, u, 1e-8, 300)
    print("n=%d iterations %d / %d, relres %.3e / %.3e" % (n, it, it_ref, rel, rel_ref), flush=True)
    assert rc == rc_ref == 0
    assert it == it_ref
    assert np.array_equal(u, u_ref)
    assert rel == rel_ref and rel <= 1e-8


def test_noalloc_matches_solve_two_calls_smaller_second():
    import paper_2506_08284_amd as P
    H1, pr1 = _host_hierarchy(12, ("lognormal", 6, 2.0), 7)
    H2, pr2 = _host_hierarchy(8, ("const", 1.0), 101)
    try:
        assert pr2["f"].shape[0] < pr1["f"].shape[0]
        _check_same(H1, pr1["f"])
        _check_same(H2, pr2["f"])
        # and back to the larger one: nothing of the smaller call leaks into it
        _check_same(H1, pr1["f"])
        # a zero right-hand side returns u = 0 after no iteration, as solve does
        u = np.full(pr2["f"].shape[0], np.nan)
        it, rel, rc = H2.solve_noalloc(np.zeros_like(pr2["f"]), u)
        assert (it, rc) == (0, 0) and not u.any()
    finally:
        H1.close()
        H2.close()
    assert P.HCURL_NOALLOC_MAX_ROWS == 2097152


def test_noalloc_device_memory_handle():
    import torch
    import paper_2506_08284_amd as P
    pr = synth.problem(N=10, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=9)
    dev = torch.device("cuda:0")
    A = tuple(torch.from_numpy(a).to(dev) for a in pr["A"])
    Dh = tuple(torch.from_numpy(a).to(dev) for a in synth.gradient_csr(pr["tail"], pr["head"]))
    aggs = [torch.from_numpy(a).to(dev) for a in pr["aggregates"]]
    H = P.Hierarchy(A, Dh, aggs, n_nodes=pr["mesh"]["n"] ** 3, mem_space="device")
    try:
        f = torch.from_numpy(pr["f"]).to(dev)
        u_ref = torch.full_like(f, float("nan"))
        u = torch.full_like(f, float("nan"))
        r_ref = H.solve(f, u_ref, 1e-8, 300)
        r = H.solve_noalloc(f, u, 1e-8, 300)
        torch.cuda.synchronize()
        assert r == r_ref and r[2] == 0
        assert torch.equal(u, u_ref)
    finally:
        H.close()


def test_noalloc_rejects_more_rows_than_the_staging_limit():
    import paper_2506_08284_amd as P
    N = 68
    assert synth.edge_count(N) > P.HCURL_NOALLOC_MAX_ROWS
    pr = synth.problem(N=N, sigma=("const", 1.0), f_seed=1)
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=pr["mesh"]["n"] ** 3)
    try:
        u = np.zeros_like(pr["f"])
        with pytest.raises(P.HcurlError) as e:
            H.solve_noalloc(pr["f"], u)
        assert e.value.code == P.HCURL_EUNSUPPORTED
        assert "2097152" in str(e.value)
        # the regular solve still takes it
        it, rel, rc = H.solve(pr["f"], u, 1e-8, 100)
        assert rc == 0 and rel <= 1e-8
    finally:
        H.close()
