"""GPU parity at the full sizes of two workloads.

* cube32_incl (32^3, 238,688 edges, inclusions 1 / 1e-3, four levels): the
  whole hierarchy against the FP64 oracle, as in the small-case parity tests.
* cube128_contrast (128^3, 14,827,904 edges, inclusions 1 / 1e-6), in the
  configuration the benchmark times (device memory, a non-null stream, levels
  of at most 1024 edges solved directly):
  - the oracle's A^(n) = D^T A D, rho, P^(n) and D_H of level 0 in full;
  - T and the P^(e) pattern on sampled rows, where the oracle's pattern
    routine applies row by row;
  - properties at any size: the commuting relation on the sampled rows,
    decreasing energies, valid colourings of every level, and the true
    residual of the solve recomputed on the host.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O
from tests.stage_parity import stage_isolated_check

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

EPS = np.finfo(np.float64).eps


def _export(H, level, which):
    arrs, shape = H.export_csr(level, which)
    return sp.csr_matrix((arrs[2], arrs[1], arrs[0]), shape=shape)


def _same_pattern(G, R):
    G, R = O.csr(G), O.csr(R)
    assert G.shape == R.shape
    assert np.array_equal(G.indptr, R.indptr)
    assert np.array_equal(G.indices, R.indices)


def _abs_product(D, A):
    """|D|^T |A| |D| on the symbolic pattern of D^T A D."""
    return O.product_on_symbolic_pattern(abs(D).T.tocsr(), abs(A), abs(D))


def _colouring_valid(A, colors):
    A = O.csr(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    off = rows != A.indices
    return bool(np.all(colors[rows[off]] != colors[A.indices[off]])) and colors.min() >= 0


def _check_true_residual(A, f, u, rel):
    """The library's true residual equals ||f - A u|| / ||f|| formed on the
    host, within the rounding of forming it (eps times |A||u| + |f|)."""
    nf = np.linalg.norm(f)
    true_rel = np.linalg.norm(f - A @ u) / nf
    noise = 64 * EPS * np.linalg.norm(abs(A) @ abs(u) + abs(f)) / nf
    assert abs(true_rel - rel) <= noise + 1e-6 * rel, (true_rel, rel, noise)


def test_cube32_incl_whole_hierarchy():
    pr = synth.workload("cube32_incl")
    m = pr["mesh"]["n"] ** 3
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"], dict(record_energy=True))
    import paper_2506_08284_amd as P
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m, record_energy=1)
    assert H.num_levels() == len(levels) == 4
    for l, lv in enumerate(levels[:-1]):
        An = _export(H, l, "An")
        _same_pattern(An, lv["An"])
        # every entry within a few roundings of the sum of its absolute terms,
        # plus (below level 0) what the two sides' A_l differ by, carried through
        B = O.csr(_abs_product(lv["D"], lv["A"]))
        bound = 64 * EPS * B.data
        if l > 0:
            A_gpu = O.csr(_export(H, l, "A"))
            dA = abs(A_gpu - O.csr(lv["A"]))
            prop = O.csr(O.on_pattern(B, abs(lv["D"]).T @ dA @ abs(lv["D"])))
            bound = bound + prop.data
        assert np.all(abs(O.csr(An).data - O.csr(lv["An"]).data) <= bound + 1e-300), l
        for which, ref in (("Pn", lv["Pn"]), ("R", lv["R"]), ("Pe", lv["N"])):
            _same_pattern(_export(H, l, which), ref)
        DH = _export(H, l, "DH")
        ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], lv["Pn"].shape[1])
        _same_pattern(DH, ref)
        assert np.array_equal(O.csr(DH).data, O.csr(ref).data)
        _same_pattern(_export(H, l + 1, "A"), levels[l + 1]["A"])
        assert np.array_equal(H.export_vec(l, "colors_A"), lv["colors_A"])
        assert np.array_equal(H.export_vec(l, "colors_An"), lv["colors_An"])
        # every stage against the oracle fed the library's inputs of that stage
        err = stage_isolated_check(H, levels, l)["err"]
        # end to end: tolerances from the level's cancellation ratio (as in
        # the small-case parity tests; the largest measured errors there and
        # here are 0.42 eps kappa for P^(e))
        ek = EPS * H.level_info(l)["cancellation_ratio"]
        t_n, t_e, t_h = max(1e-11, 4 * ek), max(1e-10, 4 * ek), max(1e-10, ek)
        for which, ref, tol in (("Pn", lv["Pn"], t_n), ("R", lv["R"], t_n), ("Pe", lv["Pe"], t_e),
                                ("P0", O.with_values(lv["N"], lv["p0"]), t_e)):
            G, Rf = O.csr(_export(H, l, which)), O.csr(ref)
            assert np.max(abs(G.data - Rf.data)) <= tol * abs(Rf.data).max(), (l, which)
        G, Rf = O.csr(_export(H, l + 1, "A")), O.csr(levels[l + 1]["A"])
        assert np.max(abs(G.data - Rf.data)) <= t_h * abs(Rf.data).max()
        E = H.export_vec(l, "energy")
        assert np.all(np.diff(E) <= 1e-12 * abs(E[0]))
        assert np.allclose(E, lv["energies"], rtol=t_h, atol=0)
        print("level %d: stage-isolated P^(e) error %.2e, eps kappa %.2e" % (l, err, ek))
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    assert rc == 0 and rel <= 1e-8
    A = O.csr(pr["A"])
    _check_true_residual(A, pr["f"], u, rel)
    # solve parity (reading R25): iterations within one, the solution within
    # 1e-8 (measured 8.5e-10)
    uo, ito, relo, _ = O.pcg(levels, pr["f"])
    du = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    print("PCG %d / %d iterations, true residual %.2e / %.2e, solution difference %.2e" % (it, ito, rel, relo, du))
    assert abs(it - ito) <= 1
    assert du <= 1e-8
    H.close()


def test_cube128_contrast_bench_configuration():
    import torch
    import paper_2506_08284_amd as P
    pr = synth.workload("cube128_contrast")
    N = synth.WORKLOADS["cube128_contrast"]["N"]
    m = (N + 1) ** 3
    n = pr["A"][0].shape[0] - 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        T_ = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        A_t = tuple(T_(a) for a in pr["A"])
        D_t = tuple(T_(a) for a in synth.gradient_csr(pr["tail"], pr["head"]))
        aggs = [T_(a) for a in pr["aggregates"]]
        f_t = T_(pr["f"])
        u_t = torch.empty_like(f_t)
        torch.cuda.synchronize()
        H = P.Hierarchy(A_t, D_t, aggs, n_nodes=m, mem_space="device", stream=stream.cuda_stream,
                        coarse_max_rows=1024, record_energy=1)
        it, rel, rc = H.solve(f_t, u_t, 1e-8, 600)
        torch.cuda.synchronize()
        u = u_t.cpu().numpy()
    assert rc == 0
    # the true residual, recomputed on the host
    A = O.csr(pr["A"])
    _check_true_residual(A, pr["f"], u, rel)
    assert rel <= 1e-3  # limited near eps times the cancellation ratio (about 2e12 here)

    # level 0 against the oracle
    D = O.gradient_matrix(pr["tail"], pr["head"], m)
    agg = pr["aggregates"][0]
    mH = int(agg.max()) + 1
    An_o = O.nodal_operator(A, D)
    An = _export(H, 0, "An")
    _same_pattern(An, An_o)
    # row sums of |D|^T |A| |D|: every row of D has two entries of size 1
    babs = 2.0 * (abs(D).T @ (abs(A) @ np.ones(n)))
    err = abs(O.csr(An).data - O.csr(An_o).data)
    assert np.all(err <= 64 * EPS * np.repeat(babs, np.diff(O.csr(An_o).indptr)))
    # the ratio divides by a diagonal entry whose own relative error is up to
    # 64 eps times that row's ratio (the entrywise bound above)
    kappa = H.level_info(0)["cancellation_ratio"]
    row_kappa = babs / An_o.diagonal()
    kmax = row_kappa.max()
    assert abs(kappa - kmax) <= 64 * EPS * kmax * kmax
    Pn_o, sa = O.sa_prolongator(An_o, agg, mH)
    info = H.level_info(0)
    # rho of D^-1 A^(n): rows of the low-conductivity region enter with
    # relative errors up to eps times their ratio
    drho = abs(info["rho"] - sa["rho"]) / sa["rho"]
    assert drho <= 100 * EPS * kmax
    Pn = O.csr(_export(H, 0, "Pn"))
    _same_pattern(Pn, Pn_o)
    # per row: relative to the row's largest entry, widened by the row's ratio
    # and by what the difference in rho (hence omega) moves every row by
    scale = np.maximum.reduceat(abs(Pn_o.data), Pn_o.indptr[:-1]) if Pn_o.nnz else np.zeros(0)
    tol_row = (np.maximum(1e-11, 1000 * EPS * row_kappa) + 10 * drho) * scale
    assert np.all(abs(Pn.data - Pn_o.data) <= np.repeat(tol_row, np.diff(Pn_o.indptr)))
    assert np.allclose(np.asarray(Pn.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-12)
    DH_tail, DH_head = O.coarse_gradient(D, agg, mH)[:2]
    DH_o = O.gradient_matrix(DH_tail, DH_head, mH)
    DH = _export(H, 0, "DH")
    _same_pattern(DH, DH_o)
    assert np.array_equal(O.csr(DH).data, O.csr(DH_o).data)

    # pattern rows of T and P^(e) on sampled fine edges (the oracle's routine
    # is row-local: rows of D give the same rows of T, N and R)
    rng = np.random.default_rng(128)
    I = np.sort(rng.choice(n, 4000, replace=False))
    N_o, T_o, R_o = O.emin_pattern(D[I], Pn_o, DH_o)
    Pe = O.csr(_export(H, 0, "Pe"))
    R = O.csr(_export(H, 0, "R"))
    _same_pattern(Pe[I], N_o)
    _same_pattern(R[I], T_o)
    # commuting relation P^(e) D_H = D_h P^(n) on the sampled rows
    C = O.csr(Pe[I] @ DH_o - D[I] @ Pn)
    assert abs(C.data).max(initial=0.0) <= 1e-11 * abs(O.csr(D[I] @ Pn).data).max()
    # stage-isolated (the oracle step on the library's inputs of that step):
    # P^(n) and rho from the library's A^(n) in full, 1e-12; R on the sampled
    # rows from the library's P^(n), bit for bit; the initial guess P_0 of the
    # sampled rows from the library's R (the local systems are row-local),
    # 1e-12; rows of A_1 = P^(e)T A P^(e) from the library's P^(e) and A,
    # within 16 eps of their absolute terms
    Pn_l, sa_l = O.sa_prolongator(O.csr(An), agg, mH)
    assert abs(info["rho"] - sa_l["rho"]) <= 1e-12 * sa_l["rho"]
    assert np.max(abs(Pn.data - O.csr(Pn_l).data)) <= 1e-12 * abs(Pn_l.data).max()
    R_l = O.csr(O.on_pattern(T_o, D[I] @ Pn))
    assert np.array_equal(R[I].data, R_l.data)
    lt, lh = O.local_graphs(N_o, T_o, DH_tail, DH_head)
    loc = O.LocalSystems(N_o, T_o, O.csr(R[I]), lt, lh)
    P0 = O.csr(_export(H, 0, "P0"))
    p0_l = O.initial_guess(N_o, loc)
    assert np.max(abs(P0[I].data - p0_l)) <= 1e-12 * np.max(abs(p0_l))
    A1 = O.csr(_export(H, 1, "A"))
    J = np.sort(rng.choice(A1.shape[0], 200, replace=False))
    PeJ = O.csr(Pe[:, J])
    rows = O.csr(PeJ.T @ A @ Pe)
    rows_abs = O.csr(abs(PeJ).T @ abs(A) @ abs(Pe))
    for k, j in enumerate(J):
        g = A1[j].toarray().ravel()
        o = rows[k].toarray().ravel()
        b = rows_abs[k].toarray().ravel()
        assert np.all(abs(g - o) <= 16 * EPS * b), j
    # the commuting relation over every row of every level, on the device
    for l in range(H.num_levels() - 1):
        a, r = H.commute_residual(l)
        assert a <= 1e-11 * r, (l, a, r)
    # energy decreases over the projected-CG iterations on every level
    for l in range(H.num_levels() - 1):
        E = H.export_vec(l, "energy")
        assert len(E) == 11 and np.all(np.diff(E) <= 1e-12 * abs(E[0]))
    # colourings of every level are proper
    for l in range(H.num_levels() - 1):
        assert _colouring_valid(_export(H, l, "A"), H.export_vec(l, "colors_A"))
        assert _colouring_valid(_export(H, l, "An"), H.export_vec(l, "colors_An"))
    H.close()


def test_cube64_jitter_lognormal_fp32_form():
    """cube64_jitter_lognormal (64^3, 1,872,064 edges, jitter 0.2 h, lognormal
    sigma s = 2, four levels), where the precision guard admits the FP32 form:
    * level 0 stage by stage against the oracle fed the library's inputs:
      A^(n) within 4 eps of its absolute terms, P^(n) and rho 1e-12, R on
      sampled rows bit for bit, P_0 on those rows 1e-12;
    * the FP32 V-cycle inside FP64 PCG against the FP64 form: both reach the
      true residual 1e-8, iterations within one;
    * the FP32 V-cycle against the oracle's FP32 V-cycle applied to the
      library's operators: 1e-5 relative (2-norm), as on the small cases."""
    import paper_2506_08284_amd as P
    from tests.stage_parity import library_hierarchy
    pr = synth.workload("cube64_jitter_lognormal")
    m = pr["mesh"]["n"] ** 3
    n = pr["A"][0].shape[0] - 1
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    H64 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, coarse_max_rows=1024)
    H32 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, coarse_max_rows=1024, vcycle_fp32=1)
    assert H32.stats()["vcycle_fp32"] == 1 and H64.num_levels() == 4
    u64, u32 = np.empty(n), np.empty(n)
    it64, rel64, rc64 = H64.solve(pr["f"], u64, 1e-8, 500)
    it32, rel32, rc32 = H32.solve(pr["f"], u32, 1e-8, 500)
    A = O.csr(pr["A"])
    _check_true_residual(A, pr["f"], u64, rel64)
    _check_true_residual(A, pr["f"], u32, rel32)
    print("FP64 form %d iterations (true relres %.2e), FP32 form %d (%.2e)" % (it64, rel64, it32, rel32))
    assert rc64 == 0 and rc32 == 0 and rel64 <= 1e-8 and rel32 <= 1e-8
    assert abs(it32 - it64) <= 1

    # level 0, stage by stage
    D = O.gradient_matrix(pr["tail"], pr["head"], m)
    agg = pr["aggregates"][0]
    mH = int(agg.max()) + 1
    An = O.csr(_export(H64, 0, "An"))
    B = O.csr(_abs_product(D, A))
    _same_pattern(An, B)
    An_o = O.csr(O.nodal_operator(A, D))
    assert np.all(abs(An.data - An_o.data) <= 4 * EPS * B.data)
    Pn = O.csr(_export(H64, 0, "Pn"))
    Pn_l, sa = O.sa_prolongator(An, agg, mH)
    assert abs(H64.level_info(0)["rho"] - sa["rho"]) <= 1e-12 * sa["rho"]
    assert np.max(abs(Pn.data - O.csr(Pn_l).data)) <= 1e-12 * abs(Pn_l.data).max()
    th, hd = O.coarse_gradient(D, agg, mH)[:2]
    DH_o = O.gradient_matrix(th, hd, mH)
    rng = np.random.default_rng(64)
    I = np.sort(rng.choice(n, 4000, replace=False))
    N_o, T_o, _ = O.emin_pattern(D[I], Pn, DH_o)
    R = O.csr(_export(H64, 0, "R"))
    _same_pattern(O.csr(_export(H64, 0, "Pe"))[I], N_o)
    _same_pattern(R[I], T_o)
    assert np.array_equal(R[I].data, O.csr(O.on_pattern(T_o, D[I] @ Pn)).data)
    lt, lh = O.local_graphs(N_o, T_o, th, hd)
    p0_l = O.initial_guess(N_o, O.LocalSystems(N_o, T_o, O.csr(R[I]), lt, lh))
    P0 = O.csr(_export(H64, 0, "P0"))
    assert np.max(abs(P0[I].data - p0_l)) <= 1e-12 * np.max(abs(p0_l))

    # the FP32 V-cycle on the library's operators
    levels = library_hierarchy(H32, pr["tail"], pr["head"], m)
    l32 = O.fp32_levels(levels)
    r = np.random.default_rng(3).standard_normal(n)
    z = np.empty(n)
    H32.vcycle(r, z)
    zo = O.vcycle_fp32(l32, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    print("FP32 V-cycle relative error %.3e on the library's operators (%d levels)" % (err, len(levels)))
    assert err <= 1e-5
    H64.close()
    H32.close()

