"""Seeded synthetic inputs for the eddy-current model problem.

The model problems of the paper's numerical section (Sec. 6.1) are unit cubes
meshed by N^3 hexahedra, each split into six tetrahedra, discretised by
lowest-order edge elements with natural boundary conditions.  This module builds
those problems at any size, with the conductivity fields and node jitter used by
the workloads of this project:

* ``kuhn_mesh``      lattice nodes, Kuhn tetrahedra, oriented sorted edges
* ``sigma_*``        constant, spherical inclusions, per-element lognormal
* ``assemble``       Whitney curl-curl S, mass M or A = S + M (CSR)
* ``box_aggregates`` per-level node aggregates (3-wide boxes, or vertex-centred)
* ``rhs``            uniform[-1, 1] right-hand side
* ``problem``        the named workloads

Nothing here belongs to the multigrid method: the CPU checker and the GPU path
both take their inputs from this module.  Random numbers come from numpy's
PCG64 ``default_rng`` with the seeds given by the caller.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "meshgen.c")
_SO = os.path.join(_HERE, "libsynth.so")
_lock = threading.Lock()
_lib_handle = None


def build(force: bool = False) -> str:
    """Compile the C mesh generator (gcc, OpenMP) next to its source."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    with _lock:
        if _lib_handle is None:
            build()
            L = ctypes.CDLL(_SO)
            P = ctypes.c_void_p
            i64 = ctypes.c_int64
            L.synth_edge_ptr.argtypes = [ctypes.c_int, P]
            L.synth_edge_ptr.restype = i64
            L.synth_edges.argtypes = [ctypes.c_int, P, P, P]
            L.synth_tets.argtypes = [ctypes.c_int, P, P, P]
            L.synth_edge_tets.argtypes = [i64, i64, P, P, P]
            L.synth_row_counts.argtypes = [i64, P, P, P, P]
            L.synth_assemble.argtypes = [i64, P, P, P, P, P, P, ctypes.c_int, P, P, P]
            L.synth_tet_volumes.argtypes = [i64, P, P, P]
            _lib_handle = L
    return _lib_handle


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def edge_count(N: int) -> int:
    """Closed-form edge count of the six-tet split of an N^3 hex lattice:
    axis edges 3N(N+1)^2, face diagonals 3N^2(N+1), body diagonals N^3."""
    return 3 * N * (N + 1) ** 2 + 3 * N * N * (N + 1) + N ** 3


def kuhn_mesh(N: int, jitter: float = 0.0, seed: int | None = None) -> dict:
    """Unit-cube lattice with N^3 hexes split into Kuhn tets.

    jitter: interior nodes move by uniform[-jitter*h, jitter*h] per coordinate.
    """
    L = _lib()
    n = N + 1
    nn = n ** 3
    eptr = np.empty(nn + 1, np.int64)
    ne = int(L.synth_edge_ptr(N, _p(eptr)))
    tail = np.empty(ne, np.int32)
    head = np.empty(ne, np.int32)
    L.synth_edges(N, _p(eptr), _p(tail), _p(head))
    ntet = 6 * N ** 3
    tets = np.empty((ntet, 4), np.int32)
    tet_edges = np.empty((ntet, 6), np.int32)
    L.synth_tets(N, _p(eptr), _p(tets), _p(tet_edges))
    h = 1.0 / N
    ax = np.arange(n, dtype=np.float64) * h
    kk, jj, ii = np.meshgrid(ax, ax, ax, indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).copy()
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        lat = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), axis=-1).reshape(-1, 3)[:, ::-1]
        interior = np.all((lat > 0) & (lat < N), axis=1)
        coords[interior] += d[interior]
    return dict(N=N, n=n, coords=coords, tets=tets, tet_edges=tet_edges, tail=tail, head=head, eptr=eptr)


def tet_volumes(mesh: dict) -> np.ndarray:
    vol = np.empty(mesh["tets"].shape[0], np.float64)
    _lib().synth_tet_volumes(mesh["tets"].shape[0], _p(mesh["tets"]), _p(mesh["coords"]), _p(vol))
    return vol


def tet_centroids(mesh: dict) -> np.ndarray:
    return mesh["coords"][mesh["tets"]].mean(axis=1)


def sigma_const(mesh: dict, value: float = 1.0) -> np.ndarray:
    return np.full(mesh["tets"].shape[0], float(value))


def sigma_inclusions(mesh: dict, seed: int, inside: float = 1.0, background: float = 1e-3,
                     count: int = 32, rmin: float = 0.05, rmax: float = 0.15) -> np.ndarray:
    """Spherical inclusions: `count` centres ~U[0,1]^3, radii ~U[rmin,rmax]; a tet
    belongs to an inclusion when its centroid lies inside the sphere."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(count, 3))
    radii = rng.uniform(rmin, rmax, size=count)
    c = tet_centroids(mesh)
    inside_any = np.zeros(c.shape[0], bool)
    for s in range(count):
        d2 = ((c - centres[s]) ** 2).sum(axis=1)
        inside_any |= d2 <= radii[s] ** 2
    return np.where(inside_any, inside, background).astype(np.float64)


def sigma_lognormal(mesh: dict, seed: int, s: float = 2.0, mu: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.exp(mu + s * rng.standard_normal(mesh["tets"].shape[0]))


_EDGE_TET_CACHE: dict = {}


def _edge_tets(mesh: dict):
    key = id(mesh["tet_edges"])
    hit = _EDGE_TET_CACHE.get(key)
    if hit is not None and hit[0] is mesh["tet_edges"]:
        return hit[1], hit[2]
    ne = mesh["tail"].shape[0]
    ntet = mesh["tets"].shape[0]
    etp = np.empty(ne + 1, np.int64)
    etl = np.empty(6 * ntet, np.int32)
    _lib().synth_edge_tets(ne, ntet, _p(mesh["tet_edges"]), _p(etp), _p(etl))
    _EDGE_TET_CACHE.clear()
    _EDGE_TET_CACHE[key] = (mesh["tet_edges"], etp, etl)
    return etp, etl


def assemble(mesh: dict, sigma: np.ndarray, which: str = "A"):
    """Whitney edge-element operator in CSR (int64 rowptr, int32 col, f64 val).

    which: "A" = S + M, "S" = curl-curl part, "M" = sigma-weighted mass part.
    Element matrices: with g_a the gradient of barycentric lambda_a and local
    edge (a,b) oriented tail a -> head b,
      S[(ab),(cd)] = 4|T| (g_a x g_b).(g_c x g_d)
      M[(ab),(cd)] = sigma_T [ (g_b.g_d) m_ac - (g_b.g_c) m_ad - (g_a.g_d) m_bc + (g_a.g_c) m_bd ],
      m_xy = |T| (1 + delta_xy) / 20.
    """
    L = _lib()
    code = {"A": 0, "S": 1, "M": 2}[which]
    ne = mesh["tail"].shape[0]
    etp, etl = _edge_tets(mesh)
    cnt = np.empty(ne, np.int64)
    L.synth_row_counts(ne, _p(etp), _p(etl), _p(mesh["tet_edges"]), _p(cnt))
    rowptr = np.zeros(ne + 1, np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    sig = np.ascontiguousarray(sigma, np.float64)
    L.synth_assemble(ne, _p(etp), _p(etl), _p(mesh["tets"]), _p(mesh["tet_edges"]), _p(mesh["coords"]), _p(sig),
                     code, _p(rowptr), _p(col), _p(val))
    return rowptr, col, val


def box_aggregates(n: int, width=3, max_maps: int | None = None):
    """Per-level node aggregates of an n^3 node lattice.

    Level l has n_l nodes per side; its aggregates are boxes along each axis,
    agg(i) = floor(i * a / n_l) with a = ceil(n_l / w_l) coarse nodes per side,
    numbered like lattice nodes; w_l = width, or width[l] for a list of widths
    (its last entry repeating).  Levels are added while a >= 2.
    Returns a list of int32 maps (one per coarsening) and the per-level sides.
    """
    maps, sides = [], [n]
    nl = n
    widths = list(width) if isinstance(width, (list, tuple)) else [width]
    while True:
        w = widths[min(len(maps), len(widths) - 1)]
        a = -(-nl // w)
        if a < 2 or (max_maps is not None and len(maps) >= max_maps):
            break
        f = (np.arange(nl, dtype=np.int64) * a) // nl
        agg = (f[None, None, :] + a * f[None, :, None] + a * a * f[:, None, None]).ravel().astype(np.int32)
        maps.append(agg)
        sides.append(a)
        nl = a
    return maps, sides


def vertex_centred_aggregates(n: int):
    """Aggregates {3m-1, 3m, 3m+1} per axis around every third lattice point
    (two wide at the boundary); one coarsening step."""
    f = (np.arange(n, dtype=np.int64) + 1) // 3
    a = int(f[-1]) + 1
    agg = (f[None, None, :] + a * f[None, :, None] + a * a * f[:, None, None]).ravel().astype(np.int32)
    return agg, a


def random_aggregates(tail: np.ndarray, head: np.ndarray, m: int, size: int, seed: int) -> np.ndarray:
    """Irregular connected aggregates of the graph with edges (tail, head):
    seeds are taken in a seeded random node order; each unassigned seed
    grows breadth-first over unassigned nodes until it holds `size` nodes or
    cannot grow; a node left in an aggregate smaller than 2 joins the
    aggregate of its first assigned neighbour.  Ids follow the seeds' order
    (every id used).  Input data only: no step of the method."""
    rng = np.random.default_rng(seed)
    nbr = [[] for _ in range(m)]
    for a, b in zip(tail.tolist(), head.tolist()):
        if a >= 0 and b >= 0:
            nbr[a].append(b)
            nbr[b].append(a)
    agg = np.full(m, -1, np.int64)
    members = []
    for s in rng.permutation(m).tolist():
        if agg[s] >= 0:
            continue
        k = len(members)
        agg[s] = k
        grp, q = [s], [s]
        while q and len(grp) < size:
            u = q.pop(0)
            for v in nbr[u]:
                if agg[v] < 0 and len(grp) < size:
                    agg[v] = k
                    grp.append(v)
                    q.append(v)
        members.append(grp)
    # singletons join a neighbour's aggregate (their ids are then unused)
    for k, grp in enumerate(members):
        if len(grp) == 1:
            u = grp[0]
            for v in nbr[u]:
                if agg[v] != k:
                    agg[u] = agg[v]
                    break
    # drop the ids of the absorbed singletons; the rest keep the seed order
    _, ids = np.unique(agg, return_inverse=True)
    return ids.astype(np.int32)


def rhs(n_edges: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n_edges)


# Named workloads.  "agg_width" 3 gives the box coarsening used throughout.
WORKLOADS = {
    "cube8_const": dict(N=8, jitter=0.0, sigma=("const", 1.0), f_seed=101),
    "cube32_incl": dict(N=32, jitter=0.0, sigma=("inclusions", 202, 1.0, 1e-3), f_seed=102),
    "cube64_jitter_lognormal": dict(N=64, jitter=0.2, jitter_seed=303, sigma=("lognormal", 304, 2.0), f_seed=103),
    "cube96_eval": dict(N=96, jitter=0.1, jitter_seed=404, sigma=("lognormal", 405, 2.0), f_seed=104),
    "cube128_contrast": dict(N=128, jitter=0.0, sigma=("inclusions", 505, 1.0, 1e-6), f_seed=105),
}


def make_sigma(mesh: dict, spec) -> np.ndarray:
    kind = spec[0]
    if kind == "const":
        return sigma_const(mesh, spec[1])
    if kind == "inclusions":
        return sigma_inclusions(mesh, spec[1], inside=spec[2], background=spec[3])
    if kind == "lognormal":
        return sigma_lognormal(mesh, spec[1], s=spec[2])
    raise ValueError(kind)


def problem(N: int, jitter: float = 0.0, jitter_seed: int | None = None, sigma=("const", 1.0), f_seed: int = 0,
            with_S: bool = False, agg_width: int = 3, max_maps: int | None = None) -> dict:
    """Everything the solver boundary consumes, plus the mesh for checks."""
    mesh = kuhn_mesh(N, jitter, jitter_seed)
    sig = make_sigma(mesh, sigma)
    A = assemble(mesh, sig, "A")
    out = dict(mesh=mesh, sigma=sig, A=A, tail=mesh["tail"], head=mesh["head"], coords=mesh["coords"])
    if with_S:
        out["S"] = assemble(mesh, sig, "S")
    maps, sides = box_aggregates(mesh["n"], agg_width, max_maps)
    out["aggregates"] = maps
    out["sides"] = sides
    out["f"] = rhs(mesh["tail"].shape[0], f_seed)
    return out


def workload(name: str, **kw) -> dict:
    spec = dict(WORKLOADS[name])
    spec.update(kw)
    return problem(**spec)


def gradient_csr(tail: np.ndarray, head: np.ndarray):
    """D_h as CSR arrays (int64 rowptr, int32 col, f64 val): -1 at the tail
    node and +1 at the head node of every edge, columns sorted."""
    n = tail.shape[0]
    lo = np.minimum(tail, head).astype(np.int32)
    hi = np.maximum(tail, head).astype(np.int32)
    col = np.stack([lo, hi], axis=1).ravel()
    up = tail < head
    val = np.stack([np.where(up, -1.0, 1.0), np.where(up, 1.0, -1.0)], axis=1).ravel()
    rowptr = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    return rowptr, np.ascontiguousarray(col), np.ascontiguousarray(val)


# ---------------------------------------------------------------------------
# Hexahedral meshes with lowest-order Nedelec (first kind) edge elements: the
# hex column of the 3D model problems (Sec. 6.1, Table 3).  Unit cube, N^3
# axis-aligned cubes of side h = 1/N, natural boundary conditions.
# ---------------------------------------------------------------------------
def hex_mesh(N: int) -> dict:
    """Lattice nodes (id = i + n j + n^2 k, n = N+1) and the axis edges,
    oriented low -> high id and sorted by (tail, head); hex_edges[h, e] is the
    global edge of local edge e of hex h (local order: x-edges at (y, z) =
    (0,0), (1,0), (0,1), (1,1), then y-edges at (x, z), then z-edges at (x, y))."""
    n = N + 1
    v = np.arange(n ** 3, dtype=np.int64)
    i, j, k = v % n, (v // n) % n, v // (n * n)
    tails, dirs = [], []
    for d, (ok, step) in enumerate(((i < N, 1), (j < N, n), (k < N, n * n))):
        tails.append(v[ok])
        dirs.append(np.full(int(ok.sum()), d, np.int64))
    tail = np.concatenate(tails)
    dirv = np.concatenate(dirs)
    key = tail * 3 + dirv  # for one tail, +1 < +n < +n^2
    order = np.argsort(key, kind="stable")
    tail, dirv, key = tail[order], dirv[order], key[order]
    head = tail + np.array([1, n, n * n])[dirv]
    c = np.arange(N, dtype=np.int64)
    hk, hj, hi = np.meshgrid(c, c, c, indexing="ij")
    base = (hi + n * hj + n * n * hk).ravel()
    loc = []
    for d, step in ((0, 1), (1, n), (2, n * n)):
        others = [s for s in (1, n, n * n) if s != step]
        for c2 in (0, 1):
            for c1 in (0, 1):
                loc.append(base * 3 + d * 1 + 3 * (c1 * others[0] + c2 * others[1]))
    hex_edges = np.searchsorted(key, np.stack(loc, axis=1)).astype(np.int32)
    ax = np.arange(n, dtype=np.float64) / N
    kk, jj, ii = np.meshgrid(ax, ax, ax, indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).copy()
    return dict(N=N, n=n, coords=coords, hex_edges=hex_edges, tail=tail.astype(np.int32), head=head.astype(np.int32))


def hex_reference_matrices():
    """12 x 12 mass and curl-curl matrices of the unit cube.  Basis of the
    x-edge at (y, z) = (b, c): phi_b(y) phi_c(z) e_x with phi_0 = 1 - t,
    phi_1 = t (tangential moment one along +x); y- and z-edges alike.  Exact
    3-point Gauss quadrature per direction (the integrands are quadratic)."""
    g = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) * 0.5 + 0.5
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    phi = lambda b, t: t if b else 1.0 - t
    dphi = lambda b: 1.0 if b else -1.0
    vals, curls = [], []
    for d in range(3):
        o1, o2 = [a for a in range(3) if a != d]
        for c2 in (0, 1):
            for c1 in (0, 1):
                u = np.zeros((len(W), 3))
                u[:, d] = phi(c1, P[:, o1]) * phi(c2, P[:, o2])
                # curl of f(x_o1, x_o2) e_d: component o2 gets d f / d x_o1 with
                # the sign of the cyclic order, o1 gets -d f / d x_o2
                df1 = dphi(c1) * phi(c2, P[:, o2])
                df2 = phi(c1, P[:, o1]) * dphi(c2)
                cu = np.zeros((len(W), 3))
                eps = lambda a, b, cc: np.linalg.det(np.eye(3)[[a, b, cc]])
                # (curl F)_i = sum_jk eps_ijk d_j F_k with F_k = f delta_kd
                cu[:, o2] += eps(o2, o1, d) * df1
                cu[:, o1] += eps(o1, o2, d) * df2
                vals.append(u)
                curls.append(cu)
    V = np.stack(vals)   # 12 x q x 3
    C = np.stack(curls)
    M = np.einsum("iqa,jqa,q->ij", V, V, W)
    S = np.einsum("iqa,jqa,q->ij", C, C, W)
    return M, S


def assemble_hex(mesh: dict, sigma: np.ndarray, which: str = "A"):
    """Nedelec hex operator in CSR: S / h + sigma_h h M per cube (which = "A",
    "S" or "M")."""
    import scipy.sparse as sp
    N = mesh["N"]
    h = 1.0 / N
    M, S = hex_reference_matrices()
    ne = mesh["tail"].shape[0]
    E = mesh["hex_edges"].astype(np.int64)
    sig = np.asarray(sigma, np.float64)
    rows = np.repeat(E, 12, axis=1).ravel()
    cols = np.tile(E, (1, 12)).ravel()
    parts = []
    if which in ("A", "S"):
        parts.append(np.broadcast_to((S / h).ravel(), (E.shape[0], 144)))
    if which in ("A", "M"):
        parts.append((sig * h)[:, None] * M.ravel()[None, :])
    vals = sum(parts).ravel()
    A = sp.csr_matrix((vals, (rows, cols)), shape=(ne, ne))
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)


def hex_problem(N: int, sigma: float = 1.0, f_seed: int = 0, agg_width: int = 3) -> dict:
    """The hexahedral constant-sigma model problem on N^3 cubes."""
    mesh = hex_mesh(N)
    sig = np.full(N ** 3, float(sigma))
    out = dict(mesh=mesh, sigma=sig, A=assemble_hex(mesh, sig, "A"), tail=mesh["tail"], head=mesh["head"],
               coords=mesh["coords"])
    maps, sides = box_aggregates(mesh["n"], agg_width)
    out["aggregates"] = maps
    out["sides"] = sides
    out["f"] = rhs(mesh["tail"].shape[0], f_seed)
    return out


# ---------------------------------------------------------------------------
# Two-dimensional model problems (Sec. 6.1, Tables 1 and 2): the unit square
# with N^2 squares, each split into two triangles along (i, j) -> (i+1, j+1)
# (lowest-order Whitney elements) or kept as squares (lowest-order Nedelec
# elements); natural boundary conditions.  Node id = i + n j, n = N + 1.
# ---------------------------------------------------------------------------
def _edges_2d(N: int, diagonals: bool):
    n = N + 1
    v = np.arange(n * n, dtype=np.int64)
    i, j = v % n, v // n
    steps = [(i < N, 1, 0), (j < N, n, 1)]
    if diagonals:
        steps.append(((i < N) & (j < N), n + 1, 2))
    tail = np.concatenate([v[ok] for ok, _, _ in steps])
    dirv = np.concatenate([np.full(int(ok.sum()), d, np.int64) for ok, _, d in steps])
    key = tail * 3 + dirv  # for one tail: +1 < +n < +n+1
    order = np.argsort(key, kind="stable")
    tail, dirv, key = tail[order], dirv[order], key[order]
    head = tail + np.array([1, n, n + 1])[dirv]
    ax = np.arange(n, dtype=np.float64) / N
    jj, ii = np.meshgrid(ax, ax, indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel()], axis=1).copy()
    return tail, head, key, coords


def tri_mesh(N: int) -> dict:
    n = N + 1
    tail, head, key, coords = _edges_2d(N, True)
    c = np.arange(N, dtype=np.int64)
    cj, ci = np.meshgrid(c, c, indexing="ij")
    v = (ci + n * cj).ravel()
    tris = np.concatenate([np.stack([v, v + 1, v + n + 1], 1), np.stack([v, v + n, v + n + 1], 1)])
    return dict(N=N, n=n, coords=coords, tris=tris, tail=tail.astype(np.int32), head=head.astype(np.int32), key=key)


def _edge_id(mesh, a, b):
    """Global id of the edge between nodes a and b (any order)."""
    n = mesh["n"]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    d = hi - lo
    dirv = np.where(d == 1, 0, np.where(d == n, 1, 2))
    return np.searchsorted(mesh["key"], lo * 3 + dirv)


def assemble_tri(mesh: dict, sigma: np.ndarray, which: str = "A"):
    """Whitney triangle operator in CSR.  With g_a the gradient of lambda_a and
    local edge (a, b) oriented a -> b: curl N_ab = 2 g_a x g_b (a scalar in 2D),
    S[(ab),(cd)] = |T| curl N_ab curl N_cd,
    M[(ab),(cd)] = sigma_T [(g_b.g_d) m_ac - (g_b.g_c) m_ad - (g_a.g_d) m_bc + (g_a.g_c) m_bd],
    m_xy = |T| (1 + delta_xy) / 12."""
    import scipy.sparse as sp
    X = mesh["coords"][mesh["tris"]]                        # t x 3 x 2
    e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * np.abs(det)
    # gradients of the barycentric coordinates
    inv = np.stack([np.stack([e2[:, 1], -e2[:, 0]], 1), np.stack([-e1[:, 1], e1[:, 0]], 1)], 1) / det[:, None, None]
    g1, g2 = inv[:, 0], inv[:, 1]
    G = np.stack([-(g1 + g2), g1, g2], 1)                  # t x 3 x 2
    T = mesh["tris"].astype(np.int64)
    pairs = [(0, 1), (0, 2), (1, 2)]
    ids, loc = [], []
    for a, b in pairs:
        swap = T[:, a] > T[:, b]
        la = np.where(swap, b, a)
        lb = np.where(swap, a, b)
        ids.append(_edge_id(mesh, T[:, a], T[:, b]))
        loc.append((la, lb))
    t = np.arange(T.shape[0])
    g = lambda l: G[t, l]
    sig = np.asarray(sigma, np.float64)
    blocks_r, blocks_c, blocks_v = [], [], []
    for p, (a, b) in enumerate(loc):
        cab = 2.0 * (g(a)[:, 0] * g(b)[:, 1] - g(a)[:, 1] * g(b)[:, 0])
        for q, (cc, d) in enumerate(loc):
            ccd = 2.0 * (g(cc)[:, 0] * g(d)[:, 1] - g(cc)[:, 1] * g(d)[:, 0])
            v = np.zeros(T.shape[0])
            if which in ("A", "S"):
                v = v + area * cab * ccd
            if which in ("A", "M"):
                m = lambda x, y: area * (1.0 + (x == y)) / 12.0
                dot = lambda x, y: (g(x) * g(y)).sum(1)
                v = v + sig * (dot(b, d) * m(a, cc) - dot(b, cc) * m(a, d) - dot(a, d) * m(b, cc) + dot(a, cc) * m(b, d))
            blocks_r.append(ids[p]); blocks_c.append(ids[q]); blocks_v.append(v)
    ne = mesh["tail"].shape[0]
    A = sp.csr_matrix((np.concatenate(blocks_v), (np.concatenate(blocks_r), np.concatenate(blocks_c))), shape=(ne, ne))
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)


def quad_mesh(N: int) -> dict:
    n = N + 1
    tail, head, key, coords = _edges_2d(N, False)
    c = np.arange(N, dtype=np.int64)
    cj, ci = np.meshgrid(c, c, indexing="ij")
    v = (ci + n * cj).ravel()
    # local edges: x-edges at y = 0, 1, then y-edges at x = 0, 1
    quad_edges = np.stack([np.searchsorted(key, v * 3), np.searchsorted(key, (v + n) * 3),
                           np.searchsorted(key, v * 3 + 1), np.searchsorted(key, (v + 1) * 3 + 1)], 1)
    return dict(N=N, n=n, coords=coords, quad_edges=quad_edges.astype(np.int32), tail=tail.astype(np.int32),
                head=head.astype(np.int32), key=key)


def quad_reference_matrices():
    """4 x 4 mass and curl-curl matrices of the unit square for the basis
    phi_c(y) e_x (x-edge at y = c) and phi_c(x) e_y (y-edge at x = c); curl
    = d(u_y)/dx - d(u_x)/dy.  Exact 3-point Gauss quadrature per direction."""
    g = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) * 0.5 + 0.5
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    X, Y = np.meshgrid(g, g, indexing="ij")
    W = (w[:, None] * w[None, :]).ravel()
    x, y = X.ravel(), Y.ravel()
    phi = lambda c, t: t if c else 1.0 - t
    dphi = lambda c: 1.0 if c else -1.0
    U, C = [], []
    for c in (0, 1):
        U.append(np.stack([phi(c, y), 0 * y], 1)); C.append(-dphi(c) + 0 * y)
    for c in (0, 1):
        U.append(np.stack([0 * x, phi(c, x)], 1)); C.append(dphi(c) + 0 * x)
    U, C = np.stack(U), np.stack(C)
    M = np.einsum("iqa,jqa,q->ij", U, U, W)
    S = np.einsum("iq,jq,q->ij", C, C, W)
    return M, S


def assemble_quad(mesh: dict, sigma: np.ndarray, which: str = "A"):
    """Nedelec square operator in CSR: S / h^2 + sigma M per square."""
    import scipy.sparse as sp
    h = 1.0 / mesh["N"]
    M, S = quad_reference_matrices()
    E = mesh["quad_edges"].astype(np.int64)
    sig = np.asarray(sigma, np.float64)
    vals = np.zeros((E.shape[0], 16))
    if which in ("A", "S"):
        vals = vals + (S / h ** 2).ravel()[None, :]
    if which in ("A", "M"):
        vals = vals + sig[:, None] * M.ravel()[None, :]
    ne = mesh["tail"].shape[0]
    A = sp.csr_matrix((vals.ravel(), (np.repeat(E, 4, axis=1).ravel(), np.tile(E, (1, 4)).ravel())), shape=(ne, ne))
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)


def box_aggregates_2d(n: int, width: int = 3):
    """box_aggregates for an n^2 node lattice."""
    maps, sides = [], [n]
    nl = n
    while True:
        a = -(-nl // width)
        if a < 2:
            break
        f = (np.arange(nl, dtype=np.int64) * a) // nl
        maps.append((f[None, :] + a * f[:, None]).ravel().astype(np.int32))
        sides.append(a)
        nl = a
    return maps, sides


def problem_2d(kind: str, N: int, sigma: float = 1.0, f_seed: int = 0) -> dict:
    """The 2D constant-sigma model problem on N^2 squares ("tri" or "quad")."""
    mesh = tri_mesh(N) if kind == "tri" else quad_mesh(N)
    ncell = mesh["tris"].shape[0] if kind == "tri" else N * N
    sig = np.full(ncell, float(sigma))
    A = (assemble_tri if kind == "tri" else assemble_quad)(mesh, sig, "A")
    out = dict(mesh=mesh, sigma=sig, A=A, tail=mesh["tail"], head=mesh["head"], coords=mesh["coords"])
    maps, sides = box_aggregates_2d(mesh["n"])
    out["aggregates"] = maps
    out["sides"] = sides
    out["f"] = rhs(mesh["tail"].shape[0], f_seed)
    return out


def refined_triangles(M: int) -> dict:
    """A coarse triangle mesh of M^2 squares and its uniform refinement by two
    (N = 2M, the same diagonals), for the ideal-interpolation case of Sec. 5:
      Pn     linear (P1) interpolation from coarse to fine nodes;
      Pe     the ideal edge prolongator: the tangential moment of every coarse
             Whitney basis function along every fine edge (exact at the
             fine edge's midpoint, the basis being affine in each triangle);
      agg    fine node (x, y) -> coarse node (x // 2, y // 2), whose RS coarse
             gradient is the coarse mesh's own."""
    import scipy.sparse as sp
    fine, coarse = tri_mesh(2 * M), tri_mesh(M)
    nf, nc = 2 * M + 1, M + 1
    v = np.arange(nf * nf)
    x, y = v % nf, v // nf
    # P1 interpolation: a fine node at a coarse vertex copies it, a midpoint
    # (odd coordinates) averages the two ends of the coarse edge it lies on
    rows, cols, vals = [], [], []
    xl, yl = x // 2, y // 2
    ox, oy = x % 2, y % 2
    rows.append(v); cols.append(xl + nc * yl); vals.append(np.where((ox == 0) & (oy == 0), 1.0, 0.5))
    mid = (ox == 1) | (oy == 1)
    rows.append(v[mid]); cols.append((xl + ox + nc * (yl + oy))[mid]); vals.append(np.full(int(mid.sum()), 0.5))
    Pn = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nf * nf, nc * nc))
    Pn.sort_indices()
    # ideal edge prolongator
    X = fine["coords"]
    pm = 0.5 * (X[fine["tail"]] + X[fine["head"]])
    tvec = X[fine["head"]] - X[fine["tail"]]
    # coarse triangle containing each fine midpoint: square (floor) and the
    # side of its diagonal (y - y0 > x - x0: the upper triangle)
    h = 1.0 / M
    sx = np.minimum((pm[:, 0] / h).astype(np.int64), M - 1)
    sy = np.minimum((pm[:, 1] / h).astype(np.int64), M - 1)
    upper = (pm[:, 1] - sy * h) > (pm[:, 0] - sx * h)
    t = (sx + M * sy) + np.where(upper, M * M, 0)  # tri_mesh order: lower triangles, then upper
    T = coarse["tris"][t]
    Xc = coarse["coords"]
    P0 = Xc[T[:, 0]]
    e1, e2 = Xc[T[:, 1]] - P0, Xc[T[:, 2]] - P0
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    g1 = np.stack([e2[:, 1], -e2[:, 0]], 1) / det[:, None]
    g2 = np.stack([-e1[:, 1], e1[:, 0]], 1) / det[:, None]
    G = np.stack([-(g1 + g2), g1, g2], 1)
    d = pm - P0
    l1 = (d * g1).sum(1)
    l2 = (d * g2).sum(1)
    lam = np.stack([1.0 - l1 - l2, l1, l2], 1)
    r, c, w = [], [], []
    for aa, bb in ((0, 1), (0, 2), (1, 2)):
        ga, gb = T[:, aa], T[:, bb]
        lo_is_a = ga < gb
        la = np.where(lo_is_a, aa, bb)
        lb = np.where(lo_is_a, bb, aa)
        idx = np.arange(len(t))
        Nv = lam[idx, la][:, None] * G[idx, lb] - lam[idx, lb][:, None] * G[idx, la]
        r.append(idx); c.append(_edge_id(coarse, ga, gb)); w.append((Nv * tvec).sum(1))
    Pe = sp.csr_matrix((np.concatenate(w), (np.concatenate(r), np.concatenate(c))),
                       shape=(len(fine["tail"]), len(coarse["tail"])))
    Pe.data[np.abs(Pe.data) < 1e-12] = 0.0  # zeros that the evaluation left at rounding level
    Pe.eliminate_zeros()
    Pe.sort_indices()
    agg = (xl + nc * yl).astype(np.int32)
    return dict(fine=fine, coarse=coarse, Pn=Pn, Pe=Pe, agg=agg)


def dirichlet_problem(N: int, sigma=("const", 1.0), f_seed: int = 0, jitter: float = 0.0,
                      jitter_seed: int | None = None) -> dict:
    """The Kuhn-tet problem with Dirichlet conditions on the whole boundary:
    boundary nodes are eliminated and so is every edge with both ends on the
    boundary; an edge with one boundary end keeps one entry in D_h (a
    Dirichlet edge, Sec. 2).  A is the kept principal submatrix; tail/head
    hold -1 for an eliminated end.  Interior nodes keep their lattice order;
    the level-0 aggregates are the box aggregates restricted to them and
    renumbered in order."""
    pr = problem(N, jitter=jitter, jitter_seed=jitter_seed, sigma=sigma, f_seed=f_seed)
    n = N + 1
    v = np.arange(n ** 3)
    i, j, k = v % n, (v // n) % n, v // (n * n)
    interior = (i > 0) & (i < N) & (j > 0) & (j < N) & (k > 0) & (k < N)
    new_id = np.full(n ** 3, -1, np.int64)
    new_id[interior] = np.arange(int(interior.sum()))
    t, h = pr["tail"].astype(np.int64), pr["head"].astype(np.int64)
    keep = interior[t] | interior[h]
    kept = np.nonzero(keep)[0]
    import scipy.sparse as sp
    A = sp.csr_matrix((pr["A"][2], pr["A"][1], pr["A"][0]), shape=(len(t), len(t)))
    Ak = A[kept][:, kept].tocsr()
    Ak.sort_indices()
    agg0 = pr["aggregates"][0][interior]
    _, agg0 = np.unique(agg0, return_inverse=True)
    out = dict(mesh=pr["mesh"], sigma=pr["sigma"], A=(Ak.indptr.astype(np.int64), Ak.indices.astype(np.int32),
                                                      Ak.data.astype(np.float64)),
               tail=new_id[t[kept]].astype(np.int32), head=new_id[h[kept]].astype(np.int32),
               coords=pr["coords"][interior], m=int(interior.sum()), kept_edges=kept,
               aggregates=[agg0.astype(np.int32)])
    out["f"] = rhs(len(kept), f_seed)
    return out
