"""The trained network on the evaluation mesh of its training law: 96^3
hexes split into tetrahedra (6,276,384 edges), node jitter 0.1 h, lognormal
conductivity with s = 2.  The learned start plus 3 projected-CG iterations
is compared with the plain start plus 10: the final level-0 energy (the
quantity the energy minimisation lowers, Sec. 3) and the PCG iterations of
the resulting hierarchy.  The learned start is always made feasible, so the
commuting relation holds to rounding whatever the network predicts."""
import os

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2506_08284_amd", "weights",
                       "mpnn_lognormal_200.npy")


def test_learned_three_iterations_against_plain_ten_at_96_cubed():
    import torch
    import paper_2506_08284_amd as P
    pr = synth.workload("cube96_eval")
    N = synth.WORKLOADS["cube96_eval"]["N"]
    m = (N + 1) ** 3
    n = pr["A"][0].shape[0] - 1
    assert n == 6276384
    dev = torch.device("cuda:0")
    T_ = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    A_t = tuple(T_(a) for a in pr["A"])
    D_t = tuple(T_(a) for a in synth.gradient_csr(pr["tail"], pr["head"]))
    aggs = [T_(a) for a in pr["aggregates"]]
    coords = T_(pr["coords"])
    f_t = T_(pr["f"])
    u_t = torch.empty_like(f_t)
    net = P.Network(np.load(WEIGHTS))
    res = {}
    for name, opts in (("plain10", dict()), ("learned3", dict(init_guess=2, mpnn=net, emin_iters_given=3))):
        H = P.Hierarchy(A_t, D_t, aggs, n_nodes=m, coords=coords, mem_space="device", record_energy=1,
                        coarse_max_rows=1024, **opts)
        E = H.export_vec(0, "energy")
        it, rel, rc = H.solve(f_t, u_t, 1e-8, 500)
        a, r = H.commute_residual(0)
        res[name] = dict(E=E, it=it, rel=rel, rc=rc, commute=a / r)
        H.close()
    print("final level-0 energy: plain+10 %.6g, learned+3 %.6g; PCG iterations %d / %d; relres %.2e / %.2e" % (
        res["plain10"]["E"][-1], res["learned3"]["E"][-1], res["plain10"]["it"], res["learned3"]["it"],
        res["plain10"]["rel"], res["learned3"]["rel"]))
    assert len(res["plain10"]["E"]) == 11 and len(res["learned3"]["E"]) == 4
    for r in res.values():
        assert r["rc"] == 0 and r["rel"] <= 1e-8
        assert r["commute"] <= 1e-12
        assert np.all(np.diff(r["E"]) <= 0)
    # the learned start plus 3 iterations ends below the plain start plus 10
    assert res["learned3"]["E"][-1] < res["plain10"]["E"][-1]
    # and starts far below the plain start
    assert res["learned3"]["E"][0] < 0.5 * res["plain10"]["E"][0]
    assert res["learned3"]["it"] <= res["plain10"]["it"] + 2
