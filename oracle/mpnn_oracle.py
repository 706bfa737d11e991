"""FP64 reference of the message-passing network that predicts P^(e)'s initial
values on its pattern (the learned initial guess; not part of the paper, which
starts from ones plus the local min-norm correction, Sec. 6.1).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU network's
features, forward pass and gradients.  Shares no code with the GPU library.

Graph: one node per pattern entry e = (i, j) of the level-0 P^(e) pattern
(fine edge i, coarse edge j).  Messages run through the rows (entries of the
same fine edge) and the columns (entries of the same coarse edge).

  h0      = silu(X W_in + b_in)                               X: E x 16 features
  layer l: m_row(i) = mean of h over row i, m_col(j) = mean over column j
           z_e = [h_e, m_row(i(e)), m_col(j(e))]                 E x 192
           h  <- h + silu(z W_l + b_l)                            l = 1..3
  delta_e = h_e . w_out + b_out
  pred_e  = p0_e + delta_e;  loss = mean_e (pred_e - target_e)^2

Every function below is the plain definition; the backward pass is the chain
rule written out and is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

NFEAT = 16
HIDDEN = 64
LAYERS = 3


def silu(u):
    return u / (1.0 + np.exp(-u))


def dsilu(u):
    s = 1.0 / (1.0 + np.exp(-u))
    return s * (1.0 + u * (1.0 - s))


def init_params(seed: int, hidden: int = HIDDEN, layers: int = LAYERS, nfeat: int = NFEAT, zero_head: bool = False):
    """Glorot-uniform weights from numpy's PCG64 generator; zero biases.  The
    output head starts at zero unless told otherwise (then delta = 0 and the
    learned guess equals the plain one)."""
    rng = np.random.default_rng(seed)

    def glorot(a, b):
        lim = np.sqrt(6.0 / (a + b))
        return rng.uniform(-lim, lim, size=(a, b))

    p = {"W_in": glorot(nfeat, hidden), "b_in": np.zeros(hidden)}
    for l in range(layers):
        p["W%d" % l] = glorot(3 * hidden, hidden)
        p["b%d" % l] = np.zeros(hidden)
    if zero_head:
        p["w_out"] = np.zeros(hidden)
    else:
        p["w_out"] = glorot(hidden, 1)[:, 0] * 0.1
    p["b_out"] = np.zeros(1)
    return p


def param_order(layers: int = LAYERS):
    names = ["W_in", "b_in"]
    for l in range(layers):
        names += ["W%d" % l, "b%d" % l]
    return names + ["w_out", "b_out"]


def flatten(p, layers: int = LAYERS):
    return np.concatenate([np.ravel(p[k]) for k in param_order(layers)])


def features(lvl: dict, coords: np.ndarray, agg: np.ndarray, Adiag: np.ndarray, pmin: np.ndarray) -> np.ndarray:
    """Per pattern entry e = (i, j):
      0 p0_e                         plain initial value
      1 pmin_e                       min-norm solution of the row constraint
      2 cos(t_i, T_j)                fine edge vs coarse edge direction
      3 |t_i| / |T_j|
      4 |mid_i - Mid_j| / |T_j|      midpoint distance
      5 n_p(i) / 16                  row length of the pattern
      6 |T_i| / 8                    coarse nodes seen by row i
      7 n_c(j) / 256                 column length of the pattern
      8 r_i(tail_j), 9 r_i(head_j)   row of D_h P^(n) at the coarse end points
      10 [agg(tail_i) in j], 11 [agg(head_i) in j]
      12 log10(A_ii) / 8
      13-15 zero
    Coarse nodes sit at the centroid of their aggregate's fine nodes; t_i and
    T_j run from tail to head."""
    N, T, R = lvl["N"], lvl["T"], lvl["R"]
    tail, head = np.asarray(lvl["tail"]), np.asarray(lvl["head"])
    ct, ch = np.asarray(lvl["DH_tail"]), np.asarray(lvl["DH_head"])
    mH = T.shape[1]
    cnt = np.bincount(agg, minlength=mH).astype(np.float64)
    cen = np.stack([np.bincount(agg, weights=coords[:, d], minlength=mH) for d in range(3)], axis=1) / cnt[:, None]
    rows = np.repeat(np.arange(N.shape[0]), np.diff(N.indptr))
    cols = N.indices
    t = coords[head[rows]] - coords[tail[rows]]
    mid = 0.5 * (coords[head[rows]] + coords[tail[rows]])
    Tv = cen[ch[cols]] - cen[ct[cols]]
    Mid = 0.5 * (cen[ch[cols]] + cen[ct[cols]])
    lt = np.linalg.norm(t, axis=1)
    LT = np.linalg.norm(Tv, axis=1)
    X = np.zeros((N.nnz, NFEAT))
    X[:, 0] = lvl["p0"]
    X[:, 1] = pmin
    X[:, 2] = np.sum(t * Tv, axis=1) / (lt * LT)
    X[:, 3] = lt / LT
    X[:, 4] = np.linalg.norm(mid - Mid, axis=1) / LT
    X[:, 5] = np.diff(N.indptr)[rows] / 16.0
    X[:, 6] = np.diff(T.indptr)[rows] / 8.0
    X[:, 7] = np.bincount(cols, minlength=N.shape[1])[cols] / 256.0
    Rd = R.tocsr()
    X[:, 8] = np.asarray(Rd[rows, ct[cols]]).ravel()
    X[:, 9] = np.asarray(Rd[rows, ch[cols]]).ravel()
    ai, bi = agg[tail[rows]], agg[head[rows]]
    X[:, 10] = ((ai == ct[cols]) | (ai == ch[cols])).astype(np.float64)
    X[:, 11] = ((bi == ct[cols]) | (bi == ch[cols])).astype(np.float64)
    X[:, 12] = np.log10(Adiag[rows]) / 8.0
    return X


def graph(N: sp.csr_matrix):
    """Row and column of every entry and the two averaging operators."""
    rows = np.repeat(np.arange(N.shape[0]), np.diff(N.indptr))
    cols = N.indices.astype(np.int64)
    E = N.nnz
    one = np.ones(E)
    Rsum = sp.csr_matrix((one, (rows, np.arange(E))), shape=(N.shape[0], E))
    Csum = sp.csr_matrix((one, (cols, np.arange(E))), shape=(N.shape[1], E))
    rcnt = np.maximum(np.asarray(Rsum.sum(axis=1)).ravel(), 1.0)
    ccnt = np.maximum(np.asarray(Csum.sum(axis=1)).ravel(), 1.0)
    return dict(rows=rows, cols=cols, Rmean=sp.diags(1.0 / rcnt) @ Rsum, Cmean=sp.diags(1.0 / ccnt) @ Csum)


def forward(p, X, g, layers: int = LAYERS):
    cache = {}
    u0 = X @ p["W_in"] + p["b_in"]
    h = silu(u0)
    cache["u0"] = u0
    for l in range(layers):
        mr = g["Rmean"] @ h
        mc = g["Cmean"] @ h
        z = np.concatenate([h, mr[g["rows"]], mc[g["cols"]]], axis=1)
        u = z @ p["W%d" % l] + p["b%d" % l]
        cache["z%d" % l] = z
        cache["u%d" % (l + 1)] = u
        h = h + silu(u)
    cache["h"] = h
    delta = h @ p["w_out"] + p["b_out"][0]
    return delta, cache


def loss_and_grad(p, X, g, p0, target, layers: int = LAYERS):
    """Mean squared error of p0 + delta against target and its gradient."""
    delta, c = forward(p, X, g, layers)
    E = X.shape[0]
    res = p0 + delta - target
    loss = float(np.mean(res ** 2))
    dd = 2.0 * res / E
    grads = {"w_out": c["h"].T @ dd, "b_out": np.array([dd.sum()])}
    dh = np.outer(dd, p["w_out"])
    H = p["w_out"].shape[0]
    for l in reversed(range(layers)):
        du = dh * dsilu(c["u%d" % (l + 1)])
        z = c["z%d" % l]
        grads["W%d" % l] = z.T @ du
        grads["b%d" % l] = du.sum(axis=0)
        dz = du @ p["W%d" % l].T
        dzh, dzr, dzc = dz[:, :H], dz[:, H:2 * H], dz[:, 2 * H:]
        # m_row = (Rmean h)[rows] and m_col = (Cmean h)[cols]: their adjoints
        # sum over each segment, then apply the transposed averaging operator
        dh = dh + dzh + _adj_mean(dzr, g["rows"], g["Rmean"]) + _adj_mean(dzc, g["cols"], g["Cmean"])
    du0 = dh * dsilu(c["u0"])
    grads["W_in"] = X.T @ du0
    grads["b_in"] = du0.sum(axis=0)
    return loss, grads, delta


def _seg_sum(v, seg, n):
    out = np.zeros((n, v.shape[1]))
    np.add.at(out, seg, v)
    return out


def _adj_mean(dv, seg, M):
    """Adjoint of h -> (M h)[seg]: first sum dv over each segment, then apply M^T."""
    s = _seg_sum(dv, seg, M.shape[0])
    return M.T @ s
