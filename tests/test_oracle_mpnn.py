"""Pins of the FP64 reference network (the learned initial guess is not in the
paper; its reference is pinned by calculus and by construction)."""
import numpy as np
import pytest

import synth
from oracle import hcurl_oracle as O
from oracle import mpnn_oracle as M


@pytest.fixture(scope="module")
def small():
    pr = synth.problem(4, jitter=0.1, jitter_seed=1, sigma=("lognormal", 2, 1.0))
    A = O.csr(pr["A"])
    lvl, _ = O.build_level(A, pr["tail"], pr["head"], 125, pr["aggregates"][0], {})
    pmin = lvl["loc"].make_feasible(np.zeros(lvl["N"].nnz))
    X = M.features(lvl, pr["coords"], pr["aggregates"][0], A.diagonal(), pmin)
    return pr, lvl, X, M.graph(lvl["N"])


def test_gradient_matches_central_differences(small):
    """Every parameter block: the hand-written backward pass agrees with
    central finite differences (h = 1e-6) to 1e-6 relative."""
    pr, lvl, X, g = small
    p = M.init_params(3)
    loss, grads, _ = M.loss_and_grad(p, X, g, lvl["p0"], lvl["Pe"].data)
    rng = np.random.default_rng(0)
    for k in M.param_order():
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in p[k].shape)
            if k == "W_in" and idx[0] >= 13:
                continue  # zero padding features
            h = 1e-6
            pp = {kk: v.copy() for kk, v in p.items()}
            pp[k][idx] += h
            lp = M.loss_and_grad(pp, X, g, lvl["p0"], lvl["Pe"].data)[0]
            pp[k][idx] -= 2 * h
            lm = M.loss_and_grad(pp, X, g, lvl["p0"], lvl["Pe"].data)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(grads[k][idx] - fd) <= 1e-6 * max(abs(fd), 1e-4), (k, idx)


def test_zero_head_gives_plain_guess(small):
    pr, lvl, X, g = small
    p = M.init_params(5, zero_head=True)
    delta, _ = M.forward(p, X, g)
    assert np.array_equal(delta, np.zeros_like(delta))


def test_features_of_the_lattice(small):
    """Feature sanity on the construction: cosines in [-1, 1], counts match
    the pattern, the min-norm values satisfy the row constraint."""
    pr, lvl, X, g = small
    assert np.all(np.abs(X[:, 2]) <= 1 + 1e-12)
    assert np.allclose(X[:, 5] * 16, np.diff(lvl["N"].indptr)[g["rows"]])
    assert np.allclose(X[:, 6] * 8, np.diff(lvl["T"].indptr)[g["rows"]])
    assert np.array_equal(X[:, 13:], np.zeros((X.shape[0], 3)))
    DH = O.gradient_matrix(lvl["DH_tail"], lvl["DH_head"], lvl["Pn"].shape[1])
    assert abs(O.with_values(lvl["N"], X[:, 1]) @ DH - lvl["D"] @ lvl["Pn"]).max() < 1e-12
