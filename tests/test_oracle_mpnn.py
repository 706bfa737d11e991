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


def test_forward_worked_by_hand_on_three_entries():
    """The reference forward pass on a 2 x 2 pattern with three entries
    e0 = (row 0, col 0), e1 = (row 0, col 1), e2 = (row 1, col 0), hidden
    width 2, one layer, against the network's definition written out entry by
    entry in scalars: h0 = silu(x W_in + b_in); the row and column means
    (row 0 averages two entries, row 1 one; column 0 two, column 1 one);
    z = [h, mean_row, mean_col]; h1 = h0 + silu(z W_0 + b_0); delta =
    h1 . w_out + b_out.  Sums in place of means, swapped row and column
    messages or a dropped residual term each change delta."""
    import math
    import scipy.sparse as sp

    def s(u):
        return u / (1.0 + math.exp(-u))

    N = sp.csr_matrix((np.ones(3), np.array([0, 1, 0]), np.array([0, 2, 3])), shape=(2, 2))
    g = M.graph(N)
    X = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    W0 = np.zeros((6, 2))
    W0[2, 0] = 1.0  # u[0] = first component of the row mean
    W0[5, 1] = 1.0  # u[1] = second component of the column mean
    p = {"W_in": np.eye(2), "b_in": np.array([0.0, -1.0]), "W0": W0, "b0": np.zeros(2),
         "w_out": np.array([1.0, 2.0]), "b_out": np.array([0.5])}
    delta, _ = M.forward(p, X, g, layers=1)
    # by hand: u0 = x + (0, -1)
    h = {0: (s(1.0), s(-1.0)), 1: (s(0.0), s(0.0)), 2: (s(1.0), s(0.0))}
    row_mean = {0: ((h[0][0] + h[1][0]) / 2, (h[0][1] + h[1][1]) / 2), 1: h[2]}
    col_mean = {0: ((h[0][0] + h[2][0]) / 2, (h[0][1] + h[2][1]) / 2), 1: h[1]}
    where = {0: (0, 0), 1: (0, 1), 2: (1, 0)}
    want = []
    for e in range(3):
        r, c = where[e]
        u = (row_mean[r][0], col_mean[c][1])
        h1 = (h[e][0] + s(u[0]), h[e][1] + s(u[1]))
        want.append(h1[0] * 1.0 + h1[1] * 2.0 + 0.5)
    assert np.max(np.abs(delta - np.array(want))) <= 1e-15
    # the same numbers to twelve digits from 40-digit decimal arithmetic
    assert np.allclose(delta, [0.783533156687, 0.715800544717, 1.599107429996], atol=1e-11, rtol=0)
