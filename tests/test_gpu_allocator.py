"""The caller's device allocator (hcurl_amg_opts.dev_alloc / dev_free): every
buffer of a handle comes from it and goes back to it by hcurl_amg_destroy,
a NULL from it is HCURL_ENOMEM with nothing leaked, and the results match
the default allocator's, on the host path and on a stream with graphs."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu


class Tracker:
    """Python allocator over PyTorch's caching allocator that records every
    live block, and can refuse after a given number of allocations."""

    def __init__(self, limit=None):
        import torch
        self.torch = torch
        self.live = {}
        self.n_alloc = 0
        self.limit = limit
        self.bad_free = 0

    def alloc(self, nbytes, stream):
        if self.limit is not None and self.n_alloc >= self.limit:
            return 0
        p = self.torch.cuda.caching_allocator_alloc(nbytes, stream=stream)
        self.n_alloc += 1
        self.live[p] = nbytes
        return p

    def free(self, ptr, nbytes, stream):
        if self.live.pop(ptr, None) != nbytes:
            self.bad_free += 1
        self.torch.cuda.caching_allocator_delete(ptr)


def _case():
    pr = synth.problem(8, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=4)
    return pr, 729, synth.gradient_csr(pr["tail"], pr["head"])


def test_every_buffer_comes_from_the_callers_allocator():
    import paper_2506_08284_amd as P
    pr, m, Dh = _case()
    n = pr["A"][0].shape[0] - 1
    H0 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m)
    u0 = np.empty(n)
    it0, rel0, rc0 = H0.solve(pr["f"], u0)
    H0.close()
    t = Tracker()
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, allocator=(t.alloc, t.free))
    assert t.n_alloc > 50 and len(t.live) > 0
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u)
    a, r = H.commute_residual(0)
    H.update(pr["A"], "warm", 2)
    H.close()
    assert not t.live and t.bad_free == 0
    assert rc == rc0 == 0 and it == it0
    assert np.linalg.norm(u - u0) <= 1e-10 * np.linalg.norm(u0)
    assert a <= 1e-12 * r


def test_refusing_allocator_gives_enomem_and_leaks_nothing():
    import paper_2506_08284_amd as P
    pr, m, Dh = _case()
    for limit in (0, 5, 40):
        t = Tracker(limit)
        with pytest.raises(P.HcurlError) as e:
            P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, allocator=(t.alloc, t.free))
        assert e.value.code == P.HCURL_ENOMEM
        assert not t.live and t.bad_free == 0 and t.n_alloc == limit


def test_masked_product_codes_fall_back_when_their_allocation_fails():
    """A NULL from the caller's allocator for the masked product's codes (2
    bytes per product a_ik x_kj of A X on the pattern) makes that energy
    minimisation search in every product instead of failing: the setup
    completes, with the P^(e) of the default run to rounding."""
    import paper_2506_08284_amd as P
    pr, m, Dh = _case()
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"])
    A, N = O.csr(levels[0]["A"]), O.csr(levels[0]["N"])
    codes = 2 * int(np.sum(np.diff(N.indptr)[A.indices]))

    class RefuseCodes(Tracker):
        def __init__(self):
            super().__init__()
            self.refused = 0

        def alloc(self, nbytes, stream):
            if nbytes == codes:
                self.refused += 1
                return 0
            return super().alloc(nbytes, stream)

    t = RefuseCodes()
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, allocator=(t.alloc, t.free))
    H0 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m)
    pe, pe0 = H.export_csr(0, "Pe")[0][2], H0.export_csr(0, "Pe")[0][2]
    H.close()
    H0.close()
    assert t.refused == 1 and not t.live and t.bad_free == 0
    assert np.max(np.abs(pe - pe0)) <= 1e-13 * np.max(np.abs(pe0))


def test_torch_allocator_on_a_stream_with_graphs():
    import torch
    import paper_2506_08284_amd as P
    pr, m, Dh = _case()
    n = pr["A"][0].shape[0] - 1
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"])
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A_t = tuple(torch.from_numpy(a).to(dev) for a in pr["A"])
        D_t = tuple(torch.from_numpy(a).to(dev) for a in Dh)
        ag = [torch.from_numpy(a).to(dev) for a in pr["aggregates"]]
        f_t = torch.from_numpy(pr["f"]).to(dev)
        u_t = torch.empty(n, dtype=torch.float64, device=dev)
        H = P.Hierarchy(A_t, D_t, ag, n_nodes=m, mem_space="device", stream=s.cuda_stream, allocator="torch")
        its = []
        for _ in range(3):  # the first solve captures the V-cycle graph, the others replay it
            it, rel, rc = H.solve(f_t, u_t)
            its.append(it)
        u = u_t.cpu().numpy()
        H.close()
    s.synchronize()
    uo, ito, _, _ = O.pcg(levels, pr["f"])
    assert rc == 0 and len(set(its)) == 1 and abs(its[0] - ito) <= 1
    assert np.linalg.norm(u - uo) <= 1e-6 * np.linalg.norm(uo)


def test_allocator_functions_go_together():
    import paper_2506_08284_amd as P
    pr, m, Dh = _case()
    keep = P.DEV_ALLOC_FN(lambda nbytes, stream, ctx: None)
    opts = P.hcurl_amg_default_opts()
    opts.dev_alloc = ctypes.cast(keep, ctypes.c_void_p).value
    with pytest.raises(P.HcurlError) as e:
        P.hcurl_amg_setup(pr["A"], Dh, pr["aggregates"], None, opts, n_nodes=m)
    assert e.value.code == P.HCURL_EINVAL
