"""Plain FP64 CPU checker for structure-preserving H(curl) algebraic multigrid.

TEST INFRASTRUCTURE ONLY.  This module is the oracle that the GPU library is
checked against.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product path never calls it.  It shares no
code with the GPU library: it takes its inputs from the ``synth`` generator and
computes everything with numpy/scipy primitives in double precision, following
the paper (Tuminaro & Glusa, "A structure preserving H-curl algebraic multigrid
method for the eddy current equations").

Paper references in docstrings name the section, equation, algorithm or table.

Readings where the paper is silent or garbled (the library follows the same ones):
  R1  coarse edges of D_H are ordered lexicographically by (I, K), I < K, with
      -1 at I and +1 at K (Sec. 2, eq. "RS coarse gradient" only says "strictly
      upper triangular").
  R3  the weight of Alg. 2 is W = Diag(3 - |D_H| 1) over coarse edges (the
      printed |D_h| has the wrong dimension for B = |T| |D_H|^T W).
  R4  Alg. 2 loops over fine edges (rows of P^(e)).
  R5  Alg. 1 (piecewise-constant interpolation from a given P^(n)): column
      target t_j = ceil(nnz(P_:j) m_h / nnz(P)); in each pass the columns in
      order take their ceil(t_j / passes) unassigned rows of largest |p_ij|
      (ties: smaller row); a row left over goes to the column of its largest
      |p_ij| (ties: smaller column); the unstated safeguard: an empty column,
      in column order, takes its row of largest |p_ij| (ties: smaller row)
      among rows whose column keeps another row, else it is an error.  A given
      P^(n) is scaled to row sums one first (sums in column order).  P-bar
      comes from the aggregates unless ``pbar_alg1`` asks for Alg. 1 on the
      smoothed P^(n), as in the paper's runs (Sec. 4.1).
  R6  Reduce_Dimension drops the column of the largest coarse node id of T_i.
  R25 setup reuse (suggested in Sec. 3 and after Table 4): see ``update``.
  R26 aggregates when the caller gives none: see ``mis2_aggregates``.
  R27 Dirichlet edges (one entry in D_h): one single-node coarse edge, +1 at
      the node, for every coarse node their remaining node is aggregated to,
      after the two-node edges in node order; W = 2 in Alg. 2; a row holding
      one keeps every column of its local system; 255 marks the absent end.
  R8  sparsity patterns are symbolic: products of absolute values, structural
      zeros kept (Alg. 2 uses |.|).
  R9  the energy is measured in A^(e) (footnote to eq. min2_hcurl allows it).
  R10 P_0 = ones on the pattern, then the local min-norm correction (Sec. 6.1).
  R11 projected CG is unpreconditioned CG with the Frobenius inner product on
      the pattern, a fixed number of iterations (Sec. 3); once <R, R> has
      fallen to 1e-24 of its first value the iterate is kept as it is.
  R12 smoothed aggregation uses omega = 4 / (3 rho(D^-1 A^(n))), rho from 20
      power iterations, no dropping (Sec. 3, eq. "emin iteration"; drop tol 0
      in Sec. 6.1).
  R13 the nodal operator is A^(n) = D_h^T A^(e) D_h (the Hiptmair smoother of
      Sec. 6.1 applies exactly this product).
  R15 make_irreducible: two-phase, new edges merged into the order of R1;
      see ``make_irreducible``.
  R18 Gauss-Seidel runs in a multicolour order (Jones-Plassmann, hashed
      priorities) shared with the GPU path.
  R19 PCG stops on the recursive residual, ||r|| <= tol ||b||; the FP32 V-cycle
      uses the flexible (Polak-Ribiere) beta.

The FP32 V-cycle form is not in the paper: its precision layout is pinned by
a high-contrast test against the plausible simplification (FP32 residuals).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

MASK64 = (1 << 64) - 1
MISSING = 255  # local index of the absent end of a Dirichlet coarse edge


# ---------------------------------------------------------------------------
# small helpers
# ---------------------------------------------------------------------------

def csr(A, shape=None) -> sp.csr_matrix:
    """(rowptr, col, val) -> scipy CSR with sorted indices, duplicates summed."""
    if sp.issparse(A):
        M = A.tocsr()
    else:
        rowptr, col, val = A
        n = len(rowptr) - 1
        if shape is None:
            shape = (n, n)
        M = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col, np.int64), np.asarray(rowptr, np.int64)),
                          shape=shape)
    M = M.copy()
    M.sum_duplicates()
    M.sort_indices()
    return M


def gradient_matrix(tail, head, m: int) -> sp.csr_matrix:
    """Discrete gradient D (n x m): row e has -1 at its tail node and +1 at its
    head node (Sec. 1, the discrete gradient has at most two +-1 per row).  An
    endpoint -1 marks a Dirichlet edge whose other node was eliminated: its row
    keeps one entry (Sec. 2)."""
    n = len(tail)
    rows = np.repeat(np.arange(n), 2)
    cols = np.stack([np.asarray(tail, np.int64), np.asarray(head, np.int64)], axis=1).ravel()
    vals = np.tile([-1.0, 1.0], n)
    keep = cols >= 0
    return csr(sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, m)))


def symbolic_product(*mats) -> sp.csr_matrix:
    """Pattern of |M1| |M2| ... as a 0/1 CSR (reading R8: no cancellation)."""
    out = abs(mats[0]).astype(np.float64)
    out.data[:] = 1.0
    for M in mats[1:]:
        B = abs(M).astype(np.float64)
        B.data[:] = 1.0
        out = out @ B
        out.data[:] = 1.0
    out = csr(out)
    out.data[:] = 1.0
    return out


def on_pattern(pattern: sp.csr_matrix, M: sp.csr_matrix) -> sp.csr_matrix:
    """Values of M placed on `pattern` (entries of M outside it are dropped,
    pattern entries absent from M are explicit zeros)."""
    pattern = csr(pattern)
    M = csr(M)
    ncol = pattern.shape[1]
    prow = np.repeat(np.arange(pattern.shape[0], dtype=np.int64), np.diff(pattern.indptr))
    pkey = prow * ncol + pattern.indices.astype(np.int64)
    mrow = np.repeat(np.arange(M.shape[0], dtype=np.int64), np.diff(M.indptr))
    mkey = mrow * ncol + M.indices.astype(np.int64)
    pos = np.searchsorted(mkey, pkey)
    pos = np.minimum(pos, max(len(mkey) - 1, 0))
    hit = (len(mkey) > 0) & (mkey[pos] == pkey) if len(mkey) else np.zeros(len(pkey), bool)
    vals = np.where(hit, M.data[pos] if len(mkey) else 0.0, 0.0)
    return sp.csr_matrix((vals, pattern.indices.copy(), pattern.indptr.copy()), shape=pattern.shape)


def product_on_symbolic_pattern(*mats) -> sp.csr_matrix:
    """Numeric product placed on the symbolic pattern of the product."""
    pat = symbolic_product(*mats)
    num = mats[0]
    for M in mats[1:]:
        num = num @ M
    return on_pattern(pat, num)


def splitmix64(i: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied to state i + golden-gamma (Steele, Lea and
    Flood, 2014); one 64-bit output per integer i."""
    with np.errstate(over="ignore"):
        z = (np.asarray(i, np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def hash_unit(i: np.ndarray) -> np.ndarray:
    """Uniform double in [0, 1) from the top 53 bits of splitmix64(i)."""
    return (splitmix64(i) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---------------------------------------------------------------------------
# nodal hierarchy pieces (Sec. 2, Sec. 4.1, Alg. 3 first lines)
# ---------------------------------------------------------------------------

def nodal_operator(A: sp.csr_matrix, D: sp.csr_matrix) -> sp.csr_matrix:
    """A^(n) = D^T A D on its symbolic pattern (reading R13)."""
    return product_on_symbolic_pattern(D.T.tocsr(), A, D)


def tentative_prolongator(agg: np.ndarray, m_coarse: int) -> sp.csr_matrix:
    """Piecewise-constant P-bar: one 1 per row, in the column of the node's
    aggregate (Sec. 2)."""
    m = len(agg)
    return csr(sp.csr_matrix((np.ones(m), (np.arange(m), np.asarray(agg, np.int64))), shape=(m, m_coarse)))


def mis2_aggregates(An: sp.csr_matrix) -> np.ndarray:
    """Aggregates of the nodes of a level from its nodal graph (the pattern of
    A^(n), diagonal aside) when the caller gives none -- not in the paper,
    which takes aggregates from its smoothed-aggregation package (Sec. 6.1);
    reading R26.  Roots form a distance-2 maximal independent set chosen in
    Luby rounds with priority key(i) = (bits 30..63 of splitmix64(i), i); every
    other node joins the root next to it, or, two steps away, the aggregate of
    its neighbour of largest key among those next to a root.  Aggregate ids
    follow the roots' node order."""
    A = csr(An)
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices.astype(np.int64)
    key = ((splitmix64(np.arange(n)) >> np.uint64(34)) << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    UND, IN, OUT = 1, 2, 0
    state = np.full(n, UND, np.int64)

    def closed_max(v):
        # max over i and its neighbours
        m = v.copy()
        np.maximum.at(m, rows, v[cols])
        return m

    while np.any(state == UND):
        t = (state.astype(np.uint64) << np.uint64(62)) | key
        m2 = closed_max(closed_max(t))
        und = state == UND
        win = und & (m2 == t)
        lose = und & ~win & ((m2 >> np.uint64(62)) == np.uint64(IN))
        state[win] = IN
        state[lose] = OUT
    roots = np.nonzero(state == IN)[0]
    agg = np.full(n, -1, np.int64)
    agg[roots] = np.arange(len(roots))
    # next to a root (roots are at least three steps apart: one root each)
    adj_root = (state[cols] == IN) & (rows != cols)
    first = agg.copy()
    first[rows[adj_root]] = agg[cols[adj_root]]
    # two steps away: the neighbour of largest key among those next to a root
    near = (first >= 0) & (agg < 0)  # assigned in the first step, not roots
    cand = (first[rows] < 0) & near[cols]
    best = np.zeros(n, np.uint64)
    np.maximum.at(best, rows[cand], key[cols[cand]] + np.uint64(1))
    second = first.copy()
    todo = (first < 0) & (best > 0)
    owner = (best[todo] - np.uint64(1)) & np.uint64(0xFFFFFFFF)
    second[np.nonzero(todo)[0]] = first[owner.astype(np.int64)]
    if np.any(second < 0):
        raise ValueError("a node is more than two steps from every root (isolated node?)")
    return second.astype(np.int32)


def power_rho(An: sp.csr_matrix, iters: int = 20) -> float:
    """Largest eigenvalue of D^-1 A^(n) by power iteration (reading R12);
    start vector x_i = hash_unit(i); returns ||y|| / ||x|| of the last step."""
    d = An.diagonal()
    x = hash_unit(np.arange(An.shape[0]))
    rho = 0.0
    for _ in range(iters):
        y = (An @ x) / d
        nx = np.sqrt(np.dot(x, x))
        ny = np.sqrt(np.dot(y, y))
        rho = ny / nx
        x = y / ny
    return rho


def sa_prolongator(An: sp.csr_matrix, agg: np.ndarray, m_coarse: int, power_iters: int = 20):
    """Smoothed aggregation P^(n) = (I - omega D^-1 A^(n)) P-bar (the one-step
    Jacobi view of Sec. 3, eq. "emin iteration", omega = 4/(3 rho)), then each
    row scaled to sum 1 (Sec. 4.2, constant preservation)."""
    Pbar = tentative_prolongator(agg, m_coarse)
    rho = power_rho(An, power_iters)
    omega = 4.0 / (3.0 * rho)
    d = An.diagonal()
    AP = product_on_symbolic_pattern(An, Pbar)
    pat = symbolic_product(An, Pbar)
    Pb = on_pattern(pat, Pbar)
    P = Pb - sp.diags(omega / d) @ AP
    P = on_pattern(pat, P)
    rs = np.asarray(P.sum(axis=1)).ravel()
    P.data = P.data / np.repeat(rs, np.diff(P.indptr))  # in place: keeps structural zeros
    return P, dict(rho=rho, omega=omega, row_sums_before=rs)


def scale_rows_to_one(P: sp.csr_matrix) -> sp.csr_matrix:
    """Each row of a nodal prolongator scaled to sum one, structural zeros
    kept (Sec. 4.2: constants must be preserved for the commuting relation)."""
    P = csr(P).copy()
    lens = np.diff(P.indptr)
    rs = np.zeros(P.shape[0])
    for k in range(int(lens.max(initial=0))):      # in index order, one term at a time
        on = lens > k
        rs[on] += P.data[P.indptr[:-1][on] + k]
    if np.any(rs == 0) or not np.all(np.isfinite(rs)):
        raise ValueError("a row of P^(n) is empty or sums to zero")
    P.data = P.data / np.repeat(rs, lens)
    return P


def piecewise_constant_assignment(P: sp.csr_matrix, passes: int = 2) -> np.ndarray:
    """Alg. 1 (Gen_Piecewise_Const) with the details of reading R5: assigns
    every fine node (row of P^(n)) to one coarse node (column); the map is the
    piecewise-constant P-bar that the coarse gradient is built from
    (Sec. 4.1).  Steps in the order of Alg. 1: per-column targets; ``passes``
    sweeps over the columns in order, each column taking its
    ceil(target / passes) unassigned rows of largest |p_ij|; greedy
    assignment of the rows left; then the safeguard for empty columns."""
    P = csr(P)
    mh, mH = P.shape
    C = P.tocsc()
    C.sort_indices()
    ncol = np.diff(C.indptr)
    target = -(-ncol * mh // max(P.nnz, 1))            # ceil(nnz_j m_h / nnz)
    n_assign = -(-target // passes)                     # ceil(target_j / passes)
    assign = np.full(mh, -1, np.int64)
    for _ in range(passes):
        for j in range(mH):
            rows = C.indices[C.indptr[j]:C.indptr[j + 1]]
            mag = np.abs(C.data[C.indptr[j]:C.indptr[j + 1]])
            free = assign[rows] < 0
            r, v = rows[free], mag[free]
            take = r[np.lexsort((r, -v))][:n_assign[j]]   # largest |p| first, ties: smaller row
            assign[take] = j
    # greedy: a row left over goes to the column of its largest |p| (ties: smaller column)
    for i in np.nonzero(assign < 0)[0]:
        cols = P.indices[P.indptr[i]:P.indptr[i + 1]]
        if len(cols) == 0:
            raise ValueError("a fine node has no coarse node in P^(n)")
        assign[i] = cols[np.argmax(np.abs(P.data[P.indptr[i]:P.indptr[i + 1]]))]
    # safeguard, columns in order: an empty column takes its row of largest |p|
    # (ties: smaller row) among rows whose column keeps at least one other row
    cnt = np.bincount(assign, minlength=mH)
    for j in np.nonzero(cnt == 0)[0]:
        rows = C.indices[C.indptr[j]:C.indptr[j + 1]]
        mag = np.abs(C.data[C.indptr[j]:C.indptr[j + 1]])
        ok = cnt[assign[rows]] >= 2
        if not np.any(ok):
            raise ValueError("Alg. 1 left a coarse node without fine nodes and no row can move to it")
        r, v = rows[ok], mag[ok]
        pick = r[np.lexsort((r, -v))][0]
        cnt[assign[pick]] -= 1
        assign[pick] = j
        cnt[j] += 1
    return assign.astype(np.int32)


def coarse_gradient(D: sp.csr_matrix, agg: np.ndarray, m_coarse: int):
    """Coarse discrete gradient by the Reitzinger-Schoeberl rule with the
    tentative prolongator (Sec. 2 eq. "RS coarse gradient", Sec. 4.1 eq.
    "revised RS DH"): Z = Pbar^T D^T D Pbar, one coarse edge per nonzero of the
    strictly upper triangle, ordered lexicographically (reading R1)."""
    Pbar = tentative_prolongator(agg, m_coarse)
    DP = csr(D @ Pbar)
    DP.eliminate_zeros()
    Z = csr(DP.T @ DP)
    Z.eliminate_zeros()
    U = csr(sp.triu(Z, k=1))
    rows = np.repeat(np.arange(m_coarse), np.diff(U.indptr))
    tail = rows.astype(np.int32)
    head = U.indices.astype(np.int32)
    # Dirichlet edges (one entry in D): every coarse node that the interior
    # node of one interpolates to gets one single-node coarse edge (Sec. 2),
    # +1 at that node (reading R27), after the two-node edges in node order
    D = csr(D)
    single = np.nonzero(np.diff(D.indptr) == 1)[0]
    if len(single):
        nodes = np.unique(np.asarray(agg)[D.indices[D.indptr[single]]]).astype(np.int32)
        tail = np.r_[tail, np.full(len(nodes), -1, np.int32)]
        head = np.r_[head, nodes]
    return tail, head


# ---------------------------------------------------------------------------
# Emin_Setup (Alg. 2) and the local constraint systems (Sec. 4.2)
# ---------------------------------------------------------------------------

class Pattern:
    """Sparsity pattern N of P^(e) and the per-row constraint data.

    Rows are fine edges i; T_i = pattern of row i of |D_h||P^(n)| (coarse
    nodes, sorted); N_i = coarse edges j with B_ij = 2, B = |T| |D_H|^T W."""

    def __init__(self, N: sp.csr_matrix, T: sp.csr_matrix, R: sp.csr_matrix, DH_tail, DH_head):
        self.N = N
        self.T = T
        self.R = R
        self.tail = np.asarray(DH_tail)
        self.head = np.asarray(DH_head)


def emin_pattern(D: sp.csr_matrix, Pn: sp.csr_matrix, DH: sp.csr_matrix) -> Pattern:
    """Alg. 2 first block: T, W, B and the initial pattern N (readings R3, R4)."""
    T = symbolic_product(D, Pn)
    absDH = abs(DH)
    W = sp.diags(3.0 - np.asarray(absDH.sum(axis=1)).ravel())
    B = csr(T @ absDH.T @ W)
    N = B.copy()
    N.data = (B.data == 2.0).astype(np.float64)  # N_ij = 1 if B_ij = 2
    N.eliminate_zeros()
    N = csr(N)
    R = on_pattern(T, D @ Pn)  # r_i, the row of D_h P^(n) on T_i (eq. "one row")
    return N, T, R


def gradient_from_pairs(tail, head, m: int) -> sp.csr_matrix:
    return gradient_matrix(np.asarray(tail), np.asarray(head), m)


def local_graphs(N: sp.csr_matrix, T: sp.csr_matrix, tail, head):
    """Local endpoint indices: for entry (i, j) of N, the positions of the tail
    and head of coarse edge j inside T_i (sorted)."""
    nrow = N.shape[0]
    mH = T.shape[1]
    nrow_of = np.repeat(np.arange(nrow, dtype=np.int64), np.diff(N.indptr))
    trow_of = np.repeat(np.arange(nrow, dtype=np.int64), np.diff(T.indptr))
    tkey = trow_of * mH + T.indices.astype(np.int64)
    j = N.indices
    out = []
    for ends in (tail, head):
        e = np.asarray(ends, np.int64)[j]
        k = nrow_of * mH + np.maximum(e, 0)
        pos = np.searchsorted(tkey, k)
        ok = e >= 0
        assert np.all(tkey[pos[ok]] == k[ok])
        # a Dirichlet coarse edge has no node at this end: local index 255
        out.append(np.where(ok, pos - T.indptr[nrow_of], MISSING).astype(np.int64))
    return out[0], out[1]


def disconnected_rows(N, T, lt, lh):
    """Rows whose local graph (T_i nodes, N_i edges) is not connected (Sec. 4.2,
    irreducibility).  Returns the row ids."""
    bad = []
    J = np.diff(T.indptr)
    for i in np.nonzero(J > 1)[0]:
        a, b = N.indptr[i], N.indptr[i + 1]
        nJ = J[i]
        if b == a:
            bad.append(i)
            continue
        two = (lt[a:b] != MISSING) & (lh[a:b] != MISSING)
        G = sp.csr_matrix((np.ones(int(two.sum())), (lt[a:b][two], lh[a:b][two])), shape=(nJ, nJ))
        nc, _ = connected_components(G, directed=False)
        if nc > 1:
            bad.append(i)
    return np.array(bad, np.int64)


class LocalSystems:
    """Per-row factors of the transposed constraint sub-matrix G~_i (Sec. 4.2:
    QR of the D_H sub-matrix, min-norm solution Q~ R~^-T r~).

    Rows are grouped by shape (n_p, |J|) so that the independent small QRs run
    as stacked numpy calls; the arithmetic per row is the plain definition."""

    def __init__(self, N, T, R, lt, lh):
        self.nrow = N.shape[0]
        npv = np.diff(N.indptr)
        Jv = np.diff(T.indptr)
        self.groups = []
        # rows holding a Dirichlet coarse edge have a full-rank G (Alg. 2:
        # no Reduce_Dimension)
        nrow_of = np.repeat(np.arange(self.nrow), npv)
        dirich = np.zeros(self.nrow, np.int64)
        np.add.at(dirich, nrow_of, ((lt == MISSING) | (lh == MISSING)).astype(np.int64))
        hasd = (dirich > 0).astype(np.int64)
        shapes = np.stack([npv, Jv, hasd], axis=1)
        keys, inv = np.unique(shapes, axis=0, return_inverse=True)
        inv = inv.ravel()
        for g, (n_p, nJ, hd) in enumerate(keys):
            rows = np.nonzero(inv == g)[0]
            if n_p == 0:
                # no pattern entry (|T_i| = 1 without a Dirichlet edge): an empty
                # row of P^(e); the constraint needs r_i = 0
                r = R.data[T.indptr[rows]] if nJ == 1 else np.zeros(0)
                self.groups.append(dict(rows=rows, n_p=0, k=0, nJ=int(nJ), r_empty=r))
                continue
            k = nJ if hd else nJ - 1  # reading R6: else drop the last (largest) coarse node
            pos = N.indptr[rows][:, None] + np.arange(n_p)[None, :]
            G = np.zeros((len(rows), n_p, nJ + 1))  # column nJ collects the missing ends
            bidx = np.repeat(np.arange(len(rows)), n_p)
            eidx = np.tile(np.arange(n_p), len(rows))
            ltp = np.minimum(lt[pos].ravel(), nJ)
            lhp = np.minimum(lh[pos].ravel(), nJ)
            G[bidx, eidx, ltp] = -1.0
            G[bidx, eidx, lhp] = 1.0
            G = G[:, :, :nJ]
            Gt = G[:, :, :k]
            Q, Rr = np.linalg.qr(Gt, mode="reduced")
            rpos = T.indptr[rows][:, None] + np.arange(nJ)[None, :]
            rfull = R.data[rpos]
            self.groups.append(dict(rows=rows, n_p=n_p, k=k, nJ=int(nJ), pos=pos, G=G, Gt=Gt, Q=Q, R=Rr,
                                    rt=rfull[:, :k], rfull=rfull))

    def project(self, x: np.ndarray) -> np.ndarray:
        """Pi(x) = x - Q~ Q~^T x row by row: the orthogonal projection onto the
        null space of the constraints (Sec. 3, projected CG; Sec. 4.2)."""
        y = x.copy()
        for g in self.groups:
            if g["n_p"] == 0:
                continue
            xv = x[g["pos"]]
            c = np.einsum("bpk,bp->bk", g["Q"], xv)
            y[g["pos"]] = xv - np.einsum("bpk,bk->bp", g["Q"], c)
        return y

    def make_feasible(self, x: np.ndarray) -> np.ndarray:
        """x + Q~ R~^-T (r~ - G~^T x): the closest point to x satisfying the
        commuting constraint of every row (Sec. 4.2 min-norm solution)."""
        y = x.copy()
        for g in self.groups:
            if g["n_p"] == 0:
                continue
            xv = x[g["pos"]]
            res = g["rt"] - np.einsum("bpk,bp->bk", g["Gt"], xv)
            z = np.linalg.solve(np.transpose(g["R"], (0, 2, 1)), res[:, :, None])[:, :, 0]
            y[g["pos"]] = xv + np.einsum("bpk,bk->bp", g["Q"], z)
        return y

    def histogram(self):
        """(|J|, n_p) -> number of rows (the least-squares sub-problem sizes of
        Tables 2 and 4)."""
        h = {}
        for g in self.groups:
            key = (g["nJ"], int(g["n_p"]))
            h[key] = h.get(key, 0) + len(g["rows"])
        return h


def make_irreducible(D, Pn, DH_tail, DH_head, mH):
    """Reading R15 of make_irreducible (Alg. 2): while some row's local graph is
    disconnected, collect for every such row one new coarse edge (I, K), I in
    the component holding the row's smallest coarse node, K outside it, chosen
    by the largest |(P^T D^T D P)_IK| (ties: smallest (min, max) pair); merge
    the deduplicated new edges into the lexicographic edge order of reading R1;
    rebuild N."""
    tail = np.asarray(DH_tail, np.int32)
    head = np.asarray(DH_head, np.int32)
    added_total = 0
    Zs = csr(Pn.T @ D.T @ D @ Pn)
    for _ in range(64):
        DH = gradient_matrix(tail, head, mH)
        N, T, R = emin_pattern(D, Pn, DH)
        lt, lh = local_graphs(N, T, tail, head)
        bad = disconnected_rows(N, T, lt, lh)
        if len(bad) == 0:
            return tail, head, added_total
        new = set()
        for i in bad:
            nodes = T.indices[T.indptr[i]:T.indptr[i + 1]]
            a, b = N.indptr[i], N.indptr[i + 1]
            nJ = len(nodes)
            two = (lt[a:b] != MISSING) & (lh[a:b] != MISSING)
            G = sp.csr_matrix((np.ones(int(two.sum())), (lt[a:b][two], lh[a:b][two])), shape=(nJ, nJ))
            _, lab = connected_components(G, directed=False)
            c0 = lab[0]
            best = None
            for p in np.nonzero(lab == c0)[0]:
                for q in np.nonzero(lab != c0)[0]:
                    I, K = int(nodes[p]), int(nodes[q])
                    lo, hi = min(I, K), max(I, K)
                    w = abs(Zs[lo, hi])
                    cand = (-w, lo, hi)
                    if best is None or cand < best:
                        best = cand
            new.add((best[1], best[2]))
        two = tail >= 0
        edges = sorted(set(zip(tail[two].tolist(), head[two].tolist())) | new)
        # Dirichlet (single-node) coarse edges stay after the two-node ones
        tail = np.r_[np.array([e[0] for e in edges], np.int32), tail[~two]]
        head = np.r_[np.array([e[1] for e in edges], np.int32), head[~two]]
        added_total += len(new)
    raise RuntimeError("make_irreducible did not converge")


# ---------------------------------------------------------------------------
# energy minimisation (Sec. 3, eq. KKT and projected CG; Sec. 4)
# ---------------------------------------------------------------------------

def masked_product(A: sp.csr_matrix, X: sp.csr_matrix, N: sp.csr_matrix) -> np.ndarray:
    """Values of A X on the pattern N (the sparsity projection of Sec. 3)."""
    return on_pattern(N, A @ X).data


def with_values(N: sp.csr_matrix, v: np.ndarray) -> sp.csr_matrix:
    return sp.csr_matrix((v, N.indices, N.indptr), shape=N.shape)


def energy(A, N, p) -> float:
    """sum_j 1/2 ||P_:j||_A^2 = 1/2 <P, A P>_F over the pattern (eq. min_problem)."""
    return 0.5 * float(np.dot(p, masked_product(A, with_values(N, p), N)))


def initial_guess(N, loc: LocalSystems) -> np.ndarray:
    """P_0: every pattern entry set to one, then the local least-squares (min-norm)
    correction onto the commuting constraint (Sec. 6.1, reading R10)."""
    return loc.make_feasible(np.ones(N.nnz))


def projected_cg(A, N, loc: LocalSystems, p0: np.ndarray, iters: int):
    """Projected conjugate gradients on the KKT system (Sec. 3): CG on
    Pi A-hat Pi with the Frobenius inner product on the pattern (reading R11).
    Once <R, R> has fallen to 1e-24 of its first value the minimiser is
    reached to rounding and the remaining iterations leave the iterate as it
    is (the curvature would be rounding noise of either sign).  Returns the
    final values and the energy after every iteration."""
    p = p0.copy()
    g = masked_product(A, with_values(N, p), N)
    r = -loc.project(g)
    d = r.copy()
    rho = float(np.dot(r, r))
    rho0 = rho
    energies = [0.5 * float(np.dot(p, g))]
    info = dict(rho=[rho], gamma=[])
    for _ in range(iters):
        if rho <= 1e-24 * rho0:
            energies.append(energies[-1])
            continue
        q = loc.project(masked_product(A, with_values(N, d), N))
        gamma = float(np.dot(d, q))
        alpha = rho / gamma
        p = p + alpha * d
        r = r - alpha * q
        rho_new = float(np.dot(r, r))
        d = r + (rho_new / rho) * d
        rho = rho_new
        info["rho"].append(rho)
        info["gamma"].append(gamma)
        energies.append(energy(A, N, p))
    p = loc.make_feasible(p)  # rounding cleanup: re-apply the affine step
    return p, energies, info


def projected_jacobi(A, N, loc: LocalSystems, p0: np.ndarray, iters: int, omega: float):
    """The projected Jacobi emin iteration of Sec. 3 (eq. "emin iteration"):
    P <- P - omega Pi(mask(D^-1 A P))."""
    p = p0.copy()
    dinv = 1.0 / A.diagonal()
    for _ in range(iters):
        dp = on_pattern(N, sp.diags(dinv) @ (A @ with_values(N, p))).data
        p = p - omega * loc.project(dp)
    return loc.make_feasible(p)


# ---------------------------------------------------------------------------
# Galerkin and the hierarchy (Sec. 2, Alg. 3)
# ---------------------------------------------------------------------------

def galerkin(P: sp.csr_matrix, A: sp.csr_matrix) -> sp.csr_matrix:
    """A_H = P^T A P on its symbolic pattern (Sec. 2)."""
    return product_on_symbolic_pattern(P.T.tocsr(), A, P)


def build_level(A, tail, head, m, agg, opts):
    """One coarsening step of Alg. 3 with smoothed aggregation from the given
    aggregates (or a given P^(n)); returns the level record and the coarse
    (A, tail, head, m).  ``agg`` in the record is the map of P-bar, the one
    the coarse gradient is built from."""
    D = gradient_matrix(tail, head, m)
    An = nodal_operator(A, D)
    if opts.get("Pn") is not None:
        Pn = scale_rows_to_one(opts["Pn"])
        sa = {}
        if agg is None:
            agg = piecewise_constant_assignment(Pn, opts.get("alg1_passes", 2))
        mH = Pn.shape[1]
    else:
        mH = int(agg.max()) + 1
        Pn, sa = sa_prolongator(An, agg, mH, opts.get("power_iters", 20))
        sa["agg"] = agg
        if opts.get("pbar_alg1"):
            # Sec. 4.1: the paper's own runs take P-bar from Alg. 1 applied to
            # the smoothed P^(n), not from the aggregates
            agg = piecewise_constant_assignment(Pn, opts.get("alg1_passes", 2))
    cth, chd = coarse_gradient(D, agg, mH)
    DH = gradient_matrix(cth, chd, mH)
    N, T, R = emin_pattern(D, Pn, DH)
    lt, lh = local_graphs(N, T, cth, chd)
    bad = disconnected_rows(N, T, lt, lh)
    added = 0
    if len(bad):
        cth, chd, added = make_irreducible(D, Pn, cth, chd, mH)
        DH = gradient_matrix(cth, chd, mH)
        N, T, R = emin_pattern(D, Pn, DH)
        lt, lh = local_graphs(N, T, cth, chd)
    loc = LocalSystems(N, T, R, lt, lh)
    p0 = opts.get("p_init")
    if p0 is None:
        p0 = initial_guess(N, loc)
    else:
        p0 = loc.make_feasible(np.asarray(p0, np.float64))
    if opts.get("emin_method", "cg") == "cg":
        p, energies, info = projected_cg(A, N, loc, p0, opts.get("emin_iters", 10))
    else:
        p = projected_jacobi(A, N, loc, p0, opts.get("emin_iters", 1), opts.get("emin_omega", 0.5))
        energies, info = [energy(A, N, p0), energy(A, N, p)], {}
    Pe = with_values(N, p)
    AH = galerkin(Pe, A)
    lvl = dict(A=A, D=D, An=An, tail=np.asarray(tail), head=np.asarray(head), m=m, agg=agg, Pn=Pn, sa=sa, Pe=Pe, N=N, T=T,
               R=R, lt=lt, lh=lh, loc=loc, p0=p0, energies=energies, cg=info, DH_tail=cth, DH_head=chd,
               irreducible_added=added)
    return lvl, (AH, cth, chd, mH)


def setup(A, tail, head, m: int, aggregates, opts=None):
    """The whole hierarchy (Alg. 3 per level): returns a list of levels; the
    last one holds the coarsest operator and its Cholesky factor."""
    opts = dict(opts or {})
    levels = []
    A = csr(A)
    li = 0
    while True:
        if opts.get("max_levels") and li + 1 >= opts["max_levels"]:
            break
        if opts.get("coarse_max_rows") and A.shape[0] <= opts["coarse_max_rows"]:
            break
        agg = aggregates[li] if li < len(aggregates) else None
        if agg is None and not (li == 0 and opts.get("Pn") is not None):
            if opts.get("aggregation") != "mis2":
                if li < len(aggregates):
                    raise ValueError("aggregates missing for a level")
                break
            # reading R26: aggregates from the level's nodal graph; a level
            # whose aggregation does not reduce it stays the coarsest
            agg = mis2_aggregates(nodal_operator(A, gradient_matrix(tail, head, m)))
            if int(agg.max()) + 1 >= m:
                break
        li += 1
        lopts = dict(opts)
        if li > 1:
            lopts.pop("Pn", None)
            lopts.pop("p_init", None)
        lvl, (A, tail, head, m) = build_level(A, tail, head, m, None if agg is None else np.asarray(agg), lopts)
        levels.append(lvl)
    D = gradient_matrix(tail, head, m)
    coarse = dict(A=A, D=D, An=nodal_operator(A, D), tail=np.asarray(tail), head=np.asarray(head), m=m,
                  chol=sla.cho_factor(A.toarray(), lower=True))
    levels.append(coarse)
    for lvl in levels[:-1]:
        lvl["colors_A"] = color_graph(lvl["A"])
        lvl["colors_An"] = color_graph(lvl["An"])
    return levels


def update(levels, A_new, mode: str, iters: int = 10, power_iters: int = 20):
    """Setup reuse for a sequence of related systems whose edge matrix keeps
    its sparsity pattern (the shortcuts the paper suggests in Sec. 3 and in
    the remarks after Table 4).  Every pattern (T, N, D_H, the local graphs)
    and every colouring is kept.
      mode "transfers": P^(n), P^(e) and D_H are kept; the new matrix is
        re-projected, A_{l+1} = P^(e)T A_l P^(e), with A^(n)_l = D_l^T A_l D_l.
      mode "warm": on every level the smoothed-aggregation P^(n) is rebuilt
        from the new A^(n) (a caller-given P^(n) is kept), the constraint rows
        R = D P^(n) on T follow it, and the previous P^(e) values, corrected
        onto the new constraints, start ``iters`` projected-CG iterations.
    Returns a new list of levels; the given one is left unchanged."""
    A = csr(A_new)
    old = csr(levels[0]["A"])
    if not (np.array_equal(A.indptr, old.indptr) and np.array_equal(A.indices, old.indices)):
        raise ValueError("the new matrix must keep the sparsity pattern")
    out = []
    for lvl in levels[:-1]:
        new = dict(lvl)
        D = lvl["D"]
        new["A"] = A
        new["An"] = nodal_operator(A, D)
        if mode == "transfers":
            new["energies"] = []
        elif mode == "warm":
            mH = lvl["Pn"].shape[1]
            if lvl["sa"]:
                Pn, sa = sa_prolongator(new["An"], lvl["sa"]["agg"], mH, power_iters)
                sa["agg"] = lvl["sa"]["agg"]
                new["Pn"], new["sa"] = Pn, sa
            DH = gradient_matrix(lvl["DH_tail"], lvl["DH_head"], mH)
            N, T, R = emin_pattern(D, new["Pn"], DH)
            loc = LocalSystems(N, T, R, lvl["lt"], lvl["lh"])
            p0 = loc.make_feasible(lvl["Pe"].data.copy())
            p, energies, info = projected_cg(A, N, loc, p0, iters)
            new.update(N=N, T=T, R=R, loc=loc, p0=p0, energies=energies, cg=info, Pe=with_values(N, p))
        else:
            raise ValueError(mode)
        out.append(new)
        A = galerkin(new["Pe"], A)
    coarse = dict(levels[-1])
    coarse["A"] = A
    coarse["An"] = nodal_operator(A, coarse["D"])
    coarse["chol"] = sla.cho_factor(A.toarray(), lower=True)
    out.append(coarse)
    return out


def commuting_residual(lvl) -> float:
    """max |P^(e) D_H - D_h P^(n)| (eq. "commute")."""
    DH = gradient_matrix(lvl["DH_tail"], lvl["DH_head"], lvl["Pn"].shape[1])
    E = lvl["Pe"] @ DH - lvl["D"] @ lvl["Pn"]
    return float(abs(E).max()) if E.nnz else 0.0


def operator_complexity(levels) -> float:
    """sum of nnz(A_l) over levels / nnz(A_0) (Sec. 6.1)."""
    return sum(l["A"].nnz for l in levels) / levels[0]["A"].nnz


# ---------------------------------------------------------------------------
# smoother, V-cycle and PCG (Sec. 6.1)
# ---------------------------------------------------------------------------

def color_graph(A: sp.csr_matrix) -> np.ndarray:
    """Jones-Plassmann colouring of the graph of A (reading R18): priority of
    vertex i is (splitmix64(i), i); every round, each uncoloured vertex whose
    priority exceeds that of all its uncoloured neighbours takes the smallest
    colour absent from its coloured neighbours."""
    n = A.shape[0]
    A = csr(A)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices.astype(np.int64)
    off = rows != cols
    rows, cols = rows[off], cols[off]
    h = splitmix64(np.arange(n))
    order = np.lexsort((np.arange(n), h))  # ascending (h, i)
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    color = np.full(n, -1, np.int64)
    while np.any(color < 0):
        unc = color < 0
        e = unc[rows] & unc[cols]
        mx = np.full(n, -1, np.int64)
        np.maximum.at(mx, rows[e], rank[cols[e]])
        sel = unc & (rank > mx)
        sidx = np.nonzero(sel)[0]
        pos = np.full(n, -1, np.int64)
        pos[sidx] = np.arange(len(sidx))
        e2 = sel[rows] & (color[cols] >= 0)
        cmax = int(color.max()) + 2 if np.any(color >= 0) else 1
        used = np.zeros((len(sidx), cmax + 1), bool)
        used[pos[rows[e2]], color[cols[e2]]] = True
        color[sidx] = np.argmin(used, axis=1)
    return color


def sgs(A: sp.csr_matrix, colors: np.ndarray, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One symmetric Gauss-Seidel sweep, forward over colours then backward
    (Sec. 6.1; order by reading R18).  Rows of one colour are not coupled, so
    updating them together is Gauss-Seidel."""
    x = x.copy()
    d = A.diagonal()
    nc = int(colors.max()) + 1 if len(colors) else 0
    groups = [np.nonzero(colors == c)[0] for c in range(nc)]
    for rows in groups + groups[::-1]:
        Ar = A[rows]
        x[rows] = x[rows] + (b[rows] - Ar @ x) / d[rows]
    return x


def sgs_lexicographic(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One symmetric Gauss-Seidel sweep in the natural row order, forward then
    backward, the smoother of the paper's runs (Sec. 6.1): with A = L + D + U,
    x <- x + (D + L)^-1 (b - A x), then x <- x + (D + U)^-1 (b - A x).  The
    triangular solves are the row-by-row sweeps."""
    import scipy.sparse.linalg as spla
    A = csr(A)
    x = x + spla.spsolve_triangular(sp.tril(A, 0, format="csr"), b - A @ x, lower=True)
    return x + spla.spsolve_triangular(sp.triu(A, 0, format="csr"), b - A @ x, lower=False)


def hiptmair(lvl, x, b, lex: bool = False):
    """Hiptmair sweep (Sec. 6.1): SGS on A; SGS on D^T A D c = D^T r from c = 0;
    x += D c; SGS on A.  ``lex``: lexicographic SGS (the paper's order) in
    place of the multicolour order of reading R18."""
    A, D = lvl["A"], lvl["D"]
    smooth = (lambda M, cols, y, rhs: sgs_lexicographic(M, y, rhs)) if lex else sgs
    x = smooth(A, lvl["colors_A"], x, b)
    r = b - A @ x
    c = smooth(lvl["An"], lvl["colors_An"], np.zeros(D.shape[1], x.dtype), D.T @ r)
    x = x + D @ c
    x = smooth(A, lvl["colors_A"], x, b)
    return x


def vcycle(levels, b, li: int = 0, lex: bool = False):
    """V-cycle: Hiptmair pre/post on every level, direct solve on the coarsest."""
    if li == len(levels) - 1:
        return sla.cho_solve(levels[-1]["chol"], b)
    lvl = levels[li]
    x = hiptmair(lvl, np.zeros_like(b), b, lex)
    r = b - lvl["A"] @ x
    xc = vcycle(levels, lvl["Pe"].T @ r, li + 1, lex)
    x = x + lvl["Pe"] @ xc
    return hiptmair(lvl, x, b, lex)


def pcg(levels, f, tol: float = 1e-8, maxit: int = 500, precond=None, flexible: bool = False, info=None):
    """CG preconditioned by one V-cycle, x0 = 0, stop at ||r|| <= tol ||f||
    (Sec. 6.1; reading R19), or when an iteration leaves the iterate unchanged
    in every entry (the stagnation of Sec. 6.2: two consecutive iterates
    equal).  ``info``, if a dict, receives the step lengths ``alpha``, the
    coefficients ``beta`` and ``stagnated``."""
    A = levels[0]["A"]
    M = precond or (lambda r: vcycle(levels, r))
    x = np.zeros_like(f)
    r = f.copy()
    z = M(r)
    p = z.copy()
    rz = float(np.dot(r, z))
    nf = float(np.linalg.norm(f))
    hist = [1.0]
    alphas, betas, stagnated = [], [], False
    it = 0
    while it < maxit and nf > 0.0:
        q = A @ p
        alpha = rz / float(np.dot(p, q))
        alphas.append(alpha)
        x_new = x + alpha * p
        r_new = r - alpha * q
        it += 1
        rel = float(np.linalg.norm(r_new)) / nf
        hist.append(rel)
        if rel <= tol:
            x, r = x_new, r_new
            break
        if np.array_equal(x_new, x):
            stagnated = True
            break
        x = x_new
        z_new = M(r_new)
        if flexible:
            beta = float(np.dot(r_new, z_new - z)) / rz
        else:
            beta = float(np.dot(r_new, z_new)) / rz
        betas.append(beta)
        rz = float(np.dot(r_new, z_new))
        p = z_new + beta * p
        r, z = r_new, z_new
    true_rel = float(np.linalg.norm(f - A @ x)) / nf if nf > 0.0 else 0.0
    if info is not None:
        info.update(alpha=alphas, beta=betas, stagnated=stagnated)
    return x, it, true_rel, hist


def lanczos_extremes(alpha, beta):
    """Smallest and largest eigenvalue of the Lanczos tridiagonal matrix that
    CG's coefficients define for the preconditioned operator (the CG-Lanczos
    relation): diagonal 1/alpha_0 and 1/alpha_j + beta_{j-1}/alpha_{j-1},
    off-diagonal sqrt(beta_j)/alpha_j.  Their ratio estimates the condition
    number that bounds the attainable accuracy (Sec. 6.1 relaxes its tolerance
    by such an estimate; reading R20)."""
    a = np.asarray(alpha, np.float64)
    b = np.asarray(beta, np.float64)[: len(a) - 1]
    d = 1.0 / a
    d[1:] += b / a[:-1]
    e = np.sqrt(b) / a[:-1]
    w = sla.eigvalsh_tridiagonal(d, e)
    return float(w[0]), float(w[-1])


def fp32_levels(levels):
    """Operators of the FP32 V-cycle: FP32 copies of A_l, A^(n)_l, D_l^T and
    P^(e)_l for smoothers and transfers, and A_l itself (FP64) for residuals;
    the coarsest Cholesky stays FP64."""
    out = []
    for lvl in levels[:-1]:
        out.append(dict(A=lvl["A"], A32=lvl["A"].astype(np.float32), An32=lvl["An"].astype(np.float32),
                        DT32=lvl["D"].T.tocsr().astype(np.float32), Pe32=lvl["Pe"].astype(np.float32),
                        dA=lvl["A"].diagonal(), dAn=lvl["An"].diagonal(),
                        colors_A=lvl["colors_A"], colors_An=lvl["colors_An"], tail=lvl["tail"], head=lvl["head"]))
    out.append(levels[-1])
    return out


def _sgs_f32op(A32, d, colors, x, b):
    """SGS sweep with FP32 operator values; products and sums in the precision
    of x, the update rounded to it."""
    x = x.copy()
    nc = int(colors.max()) + 1 if len(colors) else 0
    groups = [np.nonzero(colors == c)[0] for c in range(nc)]
    for rows in groups + groups[::-1]:
        x[rows] = (x[rows] + (b[rows] - A32[rows] @ x) / d[rows]).astype(x.dtype)
    return x


def _f64_product(M, x, t):
    """M x with every product and sum in FP64, rounded to type t."""
    return (M.astype(np.float64) @ x.astype(np.float64)).astype(t)


def _hiptmair_fp32(lvl, x, b):
    t = x.dtype
    x = _sgs_f32op(lvl["A32"], lvl["dA"], lvl["colors_A"], x, b)
    r = (b.astype(np.float64) - lvl["A"] @ x.astype(np.float64)).astype(t)
    rn = _f64_product(lvl["DT32"], r, t)
    c = _sgs_f32op(lvl["An32"], lvl["dAn"], lvl["colors_An"], np.zeros(len(rn), t), rn)
    x = x + (c[lvl["head"]] - c[lvl["tail"]])
    return _sgs_f32op(lvl["A32"], lvl["dA"], lvl["colors_A"], x, b)


def vcycle_fp32(levels32, b):
    """V-cycle of the FP32 form: smoothers and transfers use FP32 operator
    values; vectors are FP64 on the finest level and FP32 below; the coarsest
    solve is FP64 and the output is FP64.

    Residuals b - A x are formed with the FP64 operator.  In a region of small
    conductivity a gradient field x = D phi carries energy of relative size
    sigma h^2 only (S D = 0 leaves the sigma M part), while an FP32 copy of A
    breaks S D = 0 at FP32 epsilon times |S||x|.  Once sigma h^2 falls below
    that epsilon, a residual formed with the FP32 copy is rounding noise, D^T
    of it drives the nodal correction and the cycle diverges.  Rounding the
    finest-level vectors to FP32 adds the same kind of noise to the output
    (slower PCG), so they stay FP64."""
    def rec(li, bb):
        if li == len(levels32) - 1:
            return sla.cho_solve(levels32[-1]["chol"], bb.astype(np.float64)).astype(np.float32)
        lvl = levels32[li]
        t = bb.dtype
        x = _hiptmair_fp32(lvl, np.zeros_like(bb), bb)
        r = (bb.astype(np.float64) - lvl["A"] @ x.astype(np.float64)).astype(t)
        xc = rec(li + 1, _f64_product(lvl["Pe32"].T.tocsr(), r, np.float32))
        x = (x.astype(np.float64) + _f64_product(lvl["Pe32"], xc, np.float64)).astype(t)
        return _hiptmair_fp32(lvl, x, bb)
    return rec(0, np.asarray(b, dtype=np.float64))
