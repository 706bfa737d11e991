"""GPU parity on the other element families of the paper's experiments
(Sec. 6.1): lowest-order Nedelec hexahedra (Table 3, hex column), Whitney
triangles (Table 1) and Nedelec squares (Table 2), against the FP64 oracle on
the same inputs.  The library and the oracle only see A^(e), D_h and the
aggregates, so the checks are those of the tetrahedral parity tests:
* structures bit for bit: patterns of A^(n), P^(n), T, P^(e), A_H; D_H; the
  local endpoint pairs; both colourings;
* every setup stage against the oracle fed the library's inputs of that
  stage (1e-12; R bit for bit; A^(n) and A_H within a few eps of their
  absolute terms);
* end to end within the cancellation-ratio tolerances of the tetrahedral
  cases; the V-cycle on the library's operators within max(1e-11, eps
  kappa_0 / 2); PCG
  iterations within one and the solution within 1e-9."""
import numpy as np
import pytest

import synth
from oracle import hcurl_oracle as O
from tests.stage_parity import EPS, _close, _export, _same_pattern, library_levels, stage_isolated_check

pytestmark = pytest.mark.gpu

CASES = {
    "hex12_sigma1": lambda: synth.hex_problem(12, sigma=1.0, f_seed=21),
    "hex9_sigma0.01": lambda: synth.hex_problem(9, sigma=0.01, f_seed=22),
    "tri27_sigma1": lambda: synth.problem_2d("tri", 27, sigma=1.0, f_seed=23),
    "tri27_sigma100": lambda: synth.problem_2d("tri", 27, sigma=100.0, f_seed=24),
    "quad27_sigma1": lambda: synth.problem_2d("quad", 27, sigma=1.0, f_seed=25),
    "quad27_sigma0.01": lambda: synth.problem_2d("quad", 27, sigma=0.01, f_seed=26),
}
_cache = {}


def _case(name):
    if name not in _cache:
        import paper_2506_08284_amd as P
        pr = CASES[name]()
        m = int(pr["coords"].shape[0])
        levels = O.setup(pr["A"], pr["tail"], pr["head"], m, pr["aggregates"], dict(record_energy=True))
        H = P.Hierarchy(pr["A"], synth.gradient_csr(pr["tail"], pr["head"]), pr["aggregates"], n_nodes=m,
                        record_energy=1)
        _cache[name] = (pr, m, levels, H)
    return _cache[name]


def _cancellation_ratio(lv):
    D, A = lv["D"], lv["A"]
    B = abs(D).T @ abs(A) @ abs(D)
    return float(np.max(np.asarray(B.sum(axis=1)).ravel() / abs(lv["An"].diagonal())))


@pytest.mark.parametrize("name", list(CASES))
def test_structures_bit_exact(name):
    pr, m, levels, H = _case(name)
    assert H.num_levels() == len(levels) >= 2
    for l, lv in enumerate(levels[:-1]):
        info = H.level_info(l)
        assert info["n_edges"] == lv["A"].shape[0] and info["n_nodes"] == lv["m"]
        _same_pattern(_export(H, l, "An"), lv["An"])
        _same_pattern(_export(H, l, "Pn"), lv["Pn"])
        _same_pattern(_export(H, l, "R"), lv["R"])
        _same_pattern(_export(H, l, "Pe"), lv["N"])
        DH = _export(H, l, "DH")
        ref = O.gradient_matrix(lv["DH_tail"], lv["DH_head"], lv["Pn"].shape[1])
        _same_pattern(DH, ref)
        assert np.array_equal(O.csr(DH).data, O.csr(ref).data)
        lp = H.export_vec(l, "local_pairs")
        assert np.array_equal(lp & 255, lv["lt"]) and np.array_equal(lp >> 8, lv["lh"])
        _same_pattern(_export(H, l + 1, "A"), levels[l + 1]["A"])
        assert np.array_equal(H.export_vec(l, "colors_A"), lv["colors_A"])
        assert np.array_equal(H.export_vec(l, "colors_An"), lv["colors_An"])


@pytest.mark.parametrize("name", list(CASES))
def test_stage_isolated_and_end_to_end_values(name):
    pr, m, levels, H = _case(name)
    for l, lv in enumerate(levels[:-1]):
        st = stage_isolated_check(H, levels, l)
        sens = st["sens"]
        ek = EPS * _cancellation_ratio(lv)
        t_n, t_e, t_h = max(1e-11, 4 * ek), max(1e-10, 4 * ek), max(1e-10, ek)
        _close(_export(H, l, "An"), lv["An"], max(1e-12, 5 * ek))
        _close(_export(H, l, "Pn"), lv["Pn"], t_n)
        _close(_export(H, l, "R"), lv["R"], t_n)
        P0g = O.csr(_export(H, l, "P0"))
        _close(P0g, O.with_values(lv["N"], lv["p0"]), t_e)
        if sens is not None:
            # a level whose projected CG moves by `sens` under a one-rounding
            # perturbation of its start (tiny coarse levels) carries the
            # difference of its inputs (P_0 and A_l) amplified by sens / eps
            d_in = max(np.max(abs(P0g.data - lv["p0"])) / np.max(abs(lv["p0"])),
                       np.max(abs(O.csr(_export(H, l, "A")).data - O.csr(lv["A"]).data)) / abs(lv["A"].data).max())
            amp = max(1.0, d_in / EPS)
            t_e = max(t_e, 30 * sens * amp)
            t_h = max(t_h, 2 * t_e, 30 * st["sens_e"] * amp)
        _close(_export(H, l, "Pe"), lv["Pe"], t_e)
        _close(_export(H, l + 1, "A"), levels[l + 1]["A"], t_h)
        E = H.export_vec(l, "energy")
        Eo = np.array(lv["energies"])
        assert np.all(abs(E - Eo) <= t_h * abs(Eo))
        assert np.all(np.diff(E) <= 0)
        a, r = H.commute_residual(l)
        assert a <= 1e-12 * r


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_and_pcg(name):
    pr, m, levels, H = _case(name)
    n = pr["A"][0].shape[0] - 1
    r = np.random.default_rng(12).standard_normal(n)
    z = np.empty(n)
    H.vcycle(r, z)
    zl = O.vcycle(library_levels(H, levels), r)
    err = np.max(abs(z - zl)) / np.max(abs(zl))
    assert err <= max(1e-11, 0.5 * EPS * _cancellation_ratio(levels[0])), err
    u = np.empty(n)
    it, rel, rc = H.solve(pr["f"], u, 1e-8, 500)
    uo, ito, relo, _ = O.pcg(levels, pr["f"])
    du = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    print("%s: %d levels, V-cycle error %.2e, PCG %d / %d, solution difference %.2e" % (
        name, len(levels), err, it, ito, du))
    assert rc == 0 and rel <= 1e-8
    assert abs(it - ito) <= 1
    assert du <= 1e-9
