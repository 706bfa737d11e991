"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Patterns, aggregates-derived structures, colours and
local endpoint pairs are compared bit for bit; floating-point results within
the tolerances stated per check (P^(e): 1e-10 relative, solution residual
1e-8)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O
from tests.stage_parity import library_levels, stage_isolated_check

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2506_08284_amd as P
    return P


CASES = {
    "cube8_const": dict(N=8, sigma=("const", 1.0), f_seed=101),
    "cube12_jitter_lognormal": dict(N=12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7),
    "cube10_inclusions": dict(N=10, sigma=("inclusions", 8, 1.0, 1e-3), f_seed=9),
    "cube5_const": dict(N=5, sigma=("const", 0.5), f_seed=3),
    "cube3_width2": dict(N=3, jitter=0.1, jitter_seed=2, sigma=("lognormal", 4, 1.0), f_seed=4, agg_width=2),
}

_cache = {}


def _case(name):
    if name in _cache:
        return _cache[name]
    spec = dict(CASES[name])
    pr = synth.problem(**spec)
    m = pr["mesh"]["n"] ** 3
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"], dict(record_energy=True))
    P = _lib()
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, record_energy=1)
    _cache[name] = (pr, m, levels, H)
    return _cache[name]


def _sp(t, shape):
    (rp, col, val), _ = t, None
    return sp.csr_matrix((val, col, rp), shape=shape)


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


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_structure_bit_exact(name):
    pr, m, levels, H = _case(name)
    assert H.num_levels() == len(levels)
    for l, lv in enumerate(levels[:-1]):
        info = H.level_info(l)
        assert info["n_edges"] == lv["A"].shape[0]
        assert info["n_nodes"] == lv["m"]
        _same_pattern(_export(H, l, "An"), lv["An"])
        _same_pattern(_export(H, l, "Pn"), lv["Pn"])
        _same_pattern(_export(H, l, "R"), lv["R"])
        _same_pattern(_export(H, l, "Pe"), lv["N"])
        DH = _export(H, l, "DH")
        ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], lv["Pn"].shape[1])
        _same_pattern(DH, ref)
        assert np.array_equal(DH.data, O.csr(ref).data)
        lp = H.export_vec(l, "local_pairs")
        assert np.array_equal(lp & 255, lv["lt"]) and np.array_equal(lp >> 8, lv["lh"])
        _same_pattern(_export(H, l + 1, "A"), levels[l + 1]["A"])
        # colourings are bit-identical (same Jones-Plassmann rule and hash)
        assert np.array_equal(H.export_vec(l, "colors_A"), lv["colors_A"])
        assert np.array_equal(H.export_vec(l, "colors_An"), lv["colors_An"])


EPS = np.finfo(np.float64).eps


def _cancellation_ratio(lv):
    """max_u sum_v (|D|^T |A| |D|)_uv / A^(n)_uu: how much of D^T A D cancels.
    The curl-curl part of A is annihilated by D exactly (S D = 0) but not in
    rounding, so every A^(n) entry carries an error of order eps times this
    ratio times its diagonal, whichever order the sums run in."""
    D, A = lv["D"], lv["A"]
    B = abs(D).T @ abs(A) @ abs(D)
    return float(np.max(np.asarray(B.sum(axis=1)).ravel() / abs(lv["An"].diagonal())))


@pytest.mark.parametrize("name", list(CASES))
def test_stage_isolated_parity(name):
    """Each stage of every level against the oracle fed the library's inputs to
    that stage (see stage_isolated_check): P_0, P^(e), P^(n) and the energies
    within 1e-12 relative, R bit for bit, A^(n) and A_H within a few eps of
    their absolute terms."""
    pr, m, levels, H = _case(name)
    for l in range(len(levels) - 1):
        stage_isolated_check(H, levels, l)


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_values_within_tolerance(name):
    """End to end (the oracle's own hierarchy): rounding differences of the
    first stages reach P^(n) through rho and the Jacobi step, and every later
    quantity carries them.  Their size is eps times the level's cancellation
    ratio kappa (the curl-curl part of A cancels in D^T A D only in exact
    arithmetic).  Tolerances relative to the largest entry: A^(n) max(1e-12,
    5 eps kappa), P^(n), R max(1e-11, 4 eps kappa), P_0, P^(e) max(1e-10, 4 eps
    kappa), A_H and energies max(1e-10, eps kappa): ten times the largest
    error measured on these cases and the 32^3 workload, in units of eps
    kappa (A^(n) 0.5, P^(n) 0.41, P^(e) 0.42, A_H 0.045, energies 0.076).
    The stage-isolated test holds every stage to 1e-12 instead."""
    pr, m, levels, H = _case(name)
    for l, lv in enumerate(levels[:-1]):
        info = H.level_info(l)
        ek = EPS * _cancellation_ratio(lv)
        t_n = max(1e-11, 4 * ek)
        t_e = max(1e-10, 4 * ek)
        t_h = max(1e-10, ek)
        if "rho" in lv["sa"]:
            assert abs(info["rho"] - lv["sa"]["rho"]) <= t_n * lv["sa"]["rho"]
        _close(_export(H, l, "An"), lv["An"], max(1e-12, 5 * ek))
        _close(_export(H, l, "Pn"), lv["Pn"], t_n)
        _close(_export(H, l, "R"), lv["R"], t_n)
        _close(_export(H, l, "P0"), O.with_values(lv["N"], lv["p0"]), t_e)
        _close(_export(H, l, "Pe"), lv["Pe"], t_e)
        _close(_export(H, l + 1, "A"), levels[l + 1]["A"], t_h)
        E = H.export_vec(l, "energy")
        Eo = np.array(lv["energies"])
        assert len(E) == len(Eo)
        assert np.all(abs(E - Eo) <= t_h * abs(Eo))
        assert np.all(np.diff(E) <= 0)


@pytest.mark.parametrize("name", list(CASES))
def test_structure_preservation_on_gpu_output(name):
    """Commuting relation P^(e) D_H = D_h P^(n) and S_H D_H = 0 hold for the
    GPU's own operators at rounding level."""
    pr, m, levels, H = _case(name)
    if H.num_levels() < 2:
        pytest.skip("single level")
    Pe = _export(H, 0, "Pe")
    Pn = _export(H, 0, "Pn")
    DH = _export(H, 0, "DH")
    D = O.gradient_matrix(pr["tail"], pr["head"], m)
    E = Pe @ DH - D @ Pn
    assert abs(E).max() <= 1e-12 * abs(D @ Pn).max()
    S = O.csr(synth.assemble(pr["mesh"], pr["sigma"], "S"))
    SH = Pe.T @ S @ Pe
    assert abs(SH @ DH).max() <= 1e-11 * abs(SH).max()
    # the library's own check over every row of every level: its reference
    # maximum is the exported R's exactly, its residual at rounding level like
    # the one formed here from the exports
    for l in range(H.num_levels() - 1):
        a, r = H.commute_residual(l)
        R = O.csr(_export(H, l, "R"))
        assert r == abs(R.data).max()
        Dl = O.gradient_matrix(levels[l]["DH_tail"], levels[l]["DH_head"], levels[l]["Pn"].shape[1])
        Eh = O.csr(_export(H, l, "Pe") @ Dl - R)
        assert a <= 1e-12 * r and abs(Eh.data).max(initial=0.0) <= 1e-12 * r
    P = _lib()
    with pytest.raises(P.HcurlError):
        H.commute_residual(H.num_levels() - 1)


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_and_pcg_parity(name):
    """V-cycle: on the library's own operators the oracle's V-cycle agrees
    entry by entry within max(1e-11, eps kappa_0 / 2) of the largest entry
    (kappa_0: level 0's cancellation ratio; the two sides form the Hiptmair
    nodal right-hand side D^T (b - A x) in different orders, whose rounding
    is of that size; largest measured 0.044 eps kappa_0); end to end within
    1e-8.  PCG: iterations within one, the true residual at 1e-8 and the
    solution within 1e-9 in the 2-norm and entry by entry (largest measured
    difference 1e-10)."""
    pr, m, levels, H = _case(name)
    n = pr["A"][0].shape[0] - 1
    r = np.random.default_rng(11).standard_normal(n)
    z = np.empty(n)
    H.vcycle(r, z)
    zl = O.vcycle(library_levels(H, levels), r)
    err_iso = np.max(abs(z - zl)) / np.max(abs(zl))
    zo = O.vcycle(levels, r)
    err = np.max(abs(z - zo)) / np.max(abs(zo))
    print("%s: V-cycle max error %.2e on the library's operators, %.2e end to end" % (name, err_iso, err))
    assert err_iso <= max(1e-11, 0.5 * EPS * _cancellation_ratio(levels[0]))
    assert err <= 1e-8 and np.linalg.norm(z - zo) <= 1e-8 * np.linalg.norm(zo)
    f = pr["f"]
    u = np.empty(n)
    it, rel, rc = H.solve(f, u, 1e-8, 500)
    uo, ito, relo, _ = O.pcg(levels, f)
    du = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    print("%s: PCG %d / %d iterations, solution difference %.2e" % (name, it, ito, du))
    assert rc == 0 and rel <= 1e-8
    assert abs(it - ito) <= 1
    assert du <= 1e-9
    assert np.max(abs(u - uo)) <= 1e-9 * np.max(abs(uo))


def test_fp32_vcycle_in_fp64_pcg():
    pr, m, levels, H64 = _case("cube12_jitter_lognormal")
    P = _lib()
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, vcycle_fp32=1)
    assert H.stats()["vcycle_fp32"] == 1  # lognormal sigma: the guard admits FP32
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    it64, _, _ = H64.solve(pr["f"], np.empty(n), 1e-8, 500)
    assert rc == 0 and rel <= 1e-8
    assert it <= it64 + 1
    l32 = O.fp32_levels(levels)
    r = np.random.default_rng(1).standard_normal(n)
    z = np.empty(n)
    H.vcycle(r, z)
    zo = O.vcycle_fp32(l32, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    # FP32 sums of the coarse-level smoothers run in different orders on the
    # two sides; level-0 vectors and all residuals are FP64
    assert err <= 1e-5, err


def test_fp32_vcycle_on_launch_swept_levels():
    """33^3 jittered lognormal cube: level 1 has 10,439 edges, more than the
    8,192 rows one workgroup sweeps, so the FP32 sweeps below level 0 run one
    launch per colour (or per run of small colours), and the pre-smoother's
    first colour from x = 0 is written in one pass on FP32 vectors.  The
    V-cycle agrees with the oracle's FP32 V-cycle within 1e-5 and PCG with it
    reaches 1e-8 in at most one iteration more than the FP64 form."""
    pr = synth.problem(33, jitter=0.2, jitter_seed=21, sigma=("lognormal", 22, 2.0), f_seed=23)
    m = 34 ** 3
    P = _lib()
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    H = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, vcycle_fp32=1)
    H64 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m)
    assert H.stats()["vcycle_fp32"] == 1
    assert H.level_info(1)["n_edges"] > 8192
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    it64, rel64, _ = H64.solve(pr["f"], np.empty(n), 1e-8, 500)
    print("FP32 form %d iterations (relres %.2e), FP64 form %d (%.2e)" % (it, rel, it64, rel64))
    assert rc == 0 and rel <= 1e-8
    assert it <= it64 + 1
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"])
    l32 = O.fp32_levels(levels)
    r = np.random.default_rng(2).standard_normal(n)
    z = np.empty(n)
    H.vcycle(r, z)
    zo = O.vcycle_fp32(l32, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    print("FP32 V-cycle relative error %.3e" % err)
    assert err <= 1e-5, err
    H.close()
    H64.close()


@pytest.mark.parametrize("name", list(CASES))
def test_cancellation_ratio(name):
    """The per-level cancellation ratio that guards the FP32 form matches its
    definition evaluated on the oracle's operators."""
    pr, m, levels, H = _case(name)
    for l, lv in enumerate(levels[:-1]):
        k = H.level_info(l)["cancellation_ratio"]
        ko = _cancellation_ratio(lv)
        assert abs(k - ko) <= 1e-10 * ko, (l, k, ko)
    assert H.level_info(len(levels) - 1)["cancellation_ratio"] == 0.0


def test_fp32_guard_keeps_fp64_at_high_contrast():
    """Contrast 1e6 on an 8^3 mesh: FP32 epsilon times the cancellation ratio
    is far above 10, so vcycle_fp32 = 1 keeps the FP64 V-cycle (same
    iterations and solution as the FP64 form), while vcycle_fp32 = 2 forces
    the FP32 form, which still converges through the FP64 residuals."""
    pr = synth.problem(8, sigma=("inclusions", 8, 1.0, 1e-6), f_seed=3)
    m = 9 ** 3
    P = _lib()
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    n = pr["A"][0].shape[0] - 1
    H64 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m)
    H1 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, vcycle_fp32=1)
    H2 = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, vcycle_fp32=2)
    assert 2.0 ** -23 * H1.level_info(0)["cancellation_ratio"] > 10
    assert H1.stats()["vcycle_fp32"] == 0 and H2.stats()["vcycle_fp32"] == 1
    u64, u1, u2 = np.empty(n), np.empty(n), np.empty(n)
    it64, _, rc64 = H64.solve(pr["f"], u64, 1e-8, 500)
    it1, _, rc1 = H1.solve(pr["f"], u1, 1e-8, 500)
    it2, _, rc2 = H2.solve(pr["f"], u2, 1e-8, 500)
    assert rc64 == 0 and rc1 == 0 and rc2 == 0
    assert it1 == it64 and np.array_equal(u1, u64)
    assert it2 > it64


def test_projected_jacobi_variant():
    """One projected Jacobi step with omega = 0.5 (Sec. 3 eq. "emin iteration",
    the setting of Sec. 6.1)."""
    pr = synth.problem(8, jitter=0.1, jitter_seed=3, sigma=("lognormal", 2, 1.0))
    m = 729
    P = _lib()
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m,
                    emin_method=1, emin_iters=1, emin_omega=0.5)
    lvl, _ = O.build_level(O.csr(pr["A"]), pr["tail"], pr["head"], m, pr["aggregates"][0],
                           dict(emin_method="jacobi", emin_iters=1, emin_omega=0.5))
    _close(_export(H, 0, "Pe"), lvl["Pe"], 1e-10)


@pytest.mark.parametrize("method", [0, 1])
def test_masked_product_codes_match_searching_form(method):
    """The masked product A X of the energy minimisation with recorded codes
    (emin_codes = 1, the default: the first product searches and records,
    the later ones read back) and with a search in every product give the
    same P^(e), energies and coarse operators to rounding, CG and Jacobi
    alike, and both agree with the oracle at 1e-10."""
    pr = synth.problem(12, jitter=0.2, jitter_seed=5, sigma=("lognormal", 6, 2.0), f_seed=7)
    m = pr["mesh"]["n"] ** 3
    P = _lib()
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    kw = dict(emin_method=method, emin_iters=10 if method == 0 else 3, emin_omega=0.5, record_energy=1)
    Hc = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, emin_codes=1, **kw)
    Hs = P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, emin_codes=0, **kw)
    levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"],
                     dict(record_energy=True, emin_method="cg" if method == 0 else "jacobi",
                          emin_iters=kw["emin_iters"], emin_omega=0.5))
    assert Hc.num_levels() == Hs.num_levels() == len(levels)
    for l in range(len(levels) - 1):
        Pc, Ps = _export(Hc, l, "Pe"), _export(Hs, l, "Pe")
        _same_pattern(Pc, Ps)
        _close(Pc, Ps, 1e-13)
        _close(Pc, levels[l]["Pe"], 1e-10)
        Ec, Es = Hc.export_vec(l, "energy"), Hs.export_vec(l, "energy")
        assert len(Ec) == len(Es) == kw["emin_iters"] + 1
        assert np.allclose(Ec, Es, rtol=1e-13, atol=0.0)
        _close(_export(Hc, l + 1, "A"), _export(Hs, l + 1, "A"), 1e-13)
    with pytest.raises(P.HcurlError):
        P.Hierarchy(pr["A"], Dh, pr["aggregates"], n_nodes=m, emin_codes=2)


def test_given_initial_guess_is_projected_then_refined():
    """A caller-given level-0 guess is made feasible by the local min-norm
    correction and refined by 3 CG iterations, like the oracle with p_init."""
    pr, m, levels, _ = _case("cube8_const")
    rng = np.random.default_rng(5)
    guess = levels[0]["Pe"].data + 0.1 * rng.standard_normal(levels[0]["N"].nnz)
    P = _lib()
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m,
                    init_guess=1, init_values=guess, emin_iters_given=3, record_energy=1)
    lvl, _ = O.build_level(O.csr(pr["A"]), pr["tail"], pr["head"], m, pr["aggregates"][0],
                           dict(p_init=guess, emin_iters=3))
    _close(_export(H, 0, "P0"), O.with_values(lvl["N"], lvl["p0"]), 1e-10)
    _close(_export(H, 0, "Pe"), lvl["Pe"], 1e-10)
    assert len(H.export_vec(0, "energy")) == 4


def test_device_pointers_and_graph_replay_match_host_run():
    """Device inputs on a side stream: the V-cycle is captured as a HIP graph
    and replayed every PCG iteration (with eager dots and updates between
    replays).  Two solves in a row and the host-pointer run (no graph) agree."""
    import torch
    pr, m, levels, Hh = _case("cube10_inclusions")
    P = _lib()
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        Dh = synth.gradient_csr(pr["tail"], pr["head"])
        A_t = tuple(torch.from_numpy(a).to(dev) for a in pr["A"])
        D_t = tuple(torch.from_numpy(a).to(dev) for a in Dh)
        aggs = [torch.from_numpy(a).to(dev) for a in pr["aggregates"]]
        f = torch.from_numpy(pr["f"]).to(dev)
        u1 = torch.empty_like(f)
        u2 = torch.empty_like(f)
        side.synchronize()
        H = P.Hierarchy(A_t, D_t, aggs, n_nodes=m, mem_space="device", stream=side.cuda_stream)
        it1, rel1, rc1 = H.solve(f, u1)
        it2, rel2, rc2 = H.solve(f, u2)
        side.synchronize()
    un = np.empty_like(pr["f"])
    ith, relh, _ = Hh.solve(pr["f"], un)
    assert rc1 == 0 and rc2 == 0 and it1 == ith and it2 == ith and rel1 <= 1e-8
    a1, a2 = u1.cpu().numpy(), u2.cpu().numpy()
    assert np.array_equal(a1, a2)
    assert np.linalg.norm(a1 - un) <= 1e-9 * np.linalg.norm(un)


def test_profiled_solves_match_unprofiled():
    """Per-kernel events (profile 1), no graphs (2) and sampled events (3) do
    not change the arithmetic: the same solution on a stream, up to the setup's
    unordered LDS atomics (1e-9).  Profile 3 books events only on PCG
    iterations 0, 16, ... (and the setup)."""
    import torch
    pr, m, levels, Hh = _case("cube12_jitter_lognormal")
    P = _lib()
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(side):
        Dh = synth.gradient_csr(pr["tail"], pr["head"])
        A_t = tuple(torch.from_numpy(a).to(dev) for a in pr["A"])
        D_t = tuple(torch.from_numpy(a).to(dev) for a in Dh)
        aggs = [torch.from_numpy(a).to(dev) for a in pr["aggregates"]]
        f = torch.from_numpy(pr["f"]).to(dev)
        for prof in (0, 1, 2, 3):
            u = torch.empty_like(f)
            side.synchronize()
            H = P.Hierarchy(A_t, D_t, aggs, n_nodes=m, mem_space="device", stream=side.cuda_stream, profile=prof)
            it, rel, rc = H.solve(f, u)
            side.synchronize()
            out[prof] = (it, u.cpu().numpy(), H.kernel_stats() if prof else {})
            H.close()
    it0, u0, _ = out[0]
    for prof in (1, 2, 3):
        assert abs(out[prof][0] - it0) <= 1, prof
        assert np.linalg.norm(out[prof][1] - u0) <= 1e-9 * np.linalg.norm(u0), prof
    # the PCG SpMV runs once per iteration plus the final residual
    it1, it3 = out[1][0], out[3][0]
    assert out[1][2]["pcg_spmv"]["launches"] == it1 + 1
    assert out[3][2]["pcg_spmv"]["launches"] == (it3 - 1) // 16 + 1 + 1


def test_invalid_inputs_rejected():
    P = _lib()
    pr = synth.problem(4)
    m = 125
    Dh = synth.gradient_csr(pr["tail"], pr["head"])
    bad = (Dh[0], Dh[1], Dh[2].copy())
    bad[2][0] = 2.0
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], bad, pr["aggregates"], n_nodes=m)
    assert e.value.code == P.HCURL_EINVAL
    agg = pr["aggregates"][0].copy()
    agg[agg == 3] = 0  # aggregate 3 left empty
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(pr["A"], Dh, [agg], n_nodes=m)
    assert e.value.code == P.HCURL_EINVAL
    A = (pr["A"][0], pr["A"][1], pr["A"][2].copy())
    d0 = np.nonzero(A[1][A[0][0]:A[0][1]] == 0)[0][0]
    A[2][d0] = -1.0
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(A, Dh, pr["aggregates"], n_nodes=m)
    assert e.value.code == P.HCURL_EINVAL
    big = synth.problem(8)
    with pytest.raises(P.HcurlError) as e:
        P.Hierarchy(big["A"], synth.gradient_csr(big["tail"], big["head"]), [], n_nodes=729)
    assert e.value.code == P.HCURL_EUNSUPPORTED


def test_single_level_is_direct_solve():
    pr = synth.problem(2, sigma=("const", 1.0), f_seed=1)
    P = _lib()
    H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=27)
    assert H.num_levels() == 1
    n = pr["A"][0].shape[0] - 1
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u)
    assert it == 1 and rel <= 1e-12
