"""ctypes marshalling for include/hcurl_amg.h (argument conversion only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libhcurl_amg.so")

HCURL_OK = 0
HCURL_EINVAL = -1
HCURL_EHIP = -2
HCURL_ENOMEM = -3
HCURL_EREDUCIBLE = -4
HCURL_ENOTSPD = -5
HCURL_EMAXIT = -6
HCURL_EUNSUPPORTED = -7
HCURL_ESTAGNATE = -8
HCURL_EINFEASIBLE = -9
HCURL_NOALLOC_MAX_ROWS = 2097152  # staging limit of hcurl_amg_solve_noalloc (host-memory handles)

MEM = {"host": 0, "device": 1}
EXPORT = {"A": 0, "An": 1, "Pn": 2, "Pe": 3, "R": 4, "DH": 5, "P0": 6}
VEC = {"colors_A": 0, "colors_An": 1, "energy": 2, "local_pairs": 3, "pcg_history": 4, "aggregates": 5,
       "ls_histogram": 6, "pcg_alpha": 7, "pcg_beta": 8}
LS_HIST_J, LS_HIST_NP = 32, 512  # HCURL_LS_HIST_J, HCURL_LS_HIST_NP

# every function declared in include/hcurl_amg.h
EXPORTED_SYMBOLS = [
    "hcurl_amg_default_opts", "hcurl_amg_setup", "hcurl_amg_solve", "hcurl_amg_solve_noalloc", "hcurl_amg_vcycle", "hcurl_amg_update",
    "hcurl_amg_destroy", "hcurl_amg_num_levels", "hcurl_amg_level_info", "hcurl_amg_commute_residual",
    "hcurl_amg_curl_residual",
    "hcurl_amg_export_csr", "hcurl_amg_export_vec",
    "hcurl_amg_stats", "hcurl_amg_kernel_stats", "hcurl_amg_reset_kernel_stats", "hcurl_last_error",
    "hcurl_error_string", "hcurl_mpnn_num_params", "hcurl_mpnn_create", "hcurl_mpnn_get_params", "hcurl_mpnn_destroy",
    "hcurl_mpnn_set_fp32_products",
    "hcurl_amg_mpnn_sample", "hcurl_mpnn_sample_entries", "hcurl_mpnn_sample_export", "hcurl_mpnn_sample_destroy",
    "hcurl_mpnn_forward", "hcurl_mpnn_loss_grad", "hcurl_mpnn_train_step",
]


class hcurl_csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class hcurl_amg_opts(ctypes.Structure):
    _fields_ = [("max_levels", ctypes.c_int), ("coarse_max_rows", ctypes.c_int), ("emin_iters", ctypes.c_int),
                ("emin_method", ctypes.c_int), ("emin_omega", ctypes.c_double), ("init_guess", ctypes.c_int),
                ("init_values", ctypes.c_void_p), ("emin_iters_given", ctypes.c_int), ("mpnn", ctypes.c_void_p),
                ("vcycle_fp32", ctypes.c_int), ("nodal_prolongator", ctypes.c_void_p), ("alg1_passes", ctypes.c_int),
                ("pbar_alg1", ctypes.c_int), ("aggregation", ctypes.c_int),
                ("power_iters", ctypes.c_int), ("record_energy", ctypes.c_int), ("emin_codes", ctypes.c_int),
                ("profile", ctypes.c_int),
                ("mem_space", ctypes.c_int), ("stream", ctypes.c_void_p), ("dev_alloc", ctypes.c_void_p),
                ("dev_free", ctypes.c_void_p), ("alloc_ctx", ctypes.c_void_p)]

# device-memory callbacks of hcurl_amg_opts (dev_alloc, dev_free)
DEV_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
DEV_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


def _allocator_callbacks(allocator):
    """(dev_alloc, dev_free) ctypes callbacks for `allocator`: "torch" (the
    PyTorch caching allocator, stream-ordered on the handle's stream) or a
    pair of Python callables alloc(nbytes, stream) -> int pointer (0 on
    failure) and free(ptr, nbytes, stream)."""
    if allocator == "torch":
        import torch

        def alloc(nbytes, stream):
            return torch.cuda.caching_allocator_alloc(nbytes, stream=stream or 0)

        def free(ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(ptr)
    else:
        alloc, free = allocator

    def c_alloc(nbytes, stream, ctx):
        try:
            return alloc(int(nbytes), stream or 0) or None
        except Exception:
            return None

    def c_free(ptr, nbytes, stream, ctx):
        free(ptr, int(nbytes), stream or 0)

    return DEV_ALLOC_FN(c_alloc), DEV_FREE_FN(c_free)


class hcurl_level_info(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("nnz_A", ctypes.c_int64),
                ("nnz_An", ctypes.c_int64), ("nnz_Pe", ctypes.c_int64), ("nnz_Pn", ctypes.c_int64),
                ("nnz_T", ctypes.c_int64), ("n_coarse_edges", ctypes.c_int64), ("n_colors_A", ctypes.c_int32),
                ("n_colors_An", ctypes.c_int32), ("rho", ctypes.c_double), ("omega", ctypes.c_double),
                ("cancellation_ratio", ctypes.c_double), ("irreducible_added", ctypes.c_int64)]


class hcurl_amg_stats_t(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int), ("operator_complexity", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("last_iters", ctypes.c_int), ("last_relres", ctypes.c_double),
                ("vcycle_fp32", ctypes.c_int), ("update_ms", ctypes.c_double),
                ("lanczos_lambda_min", ctypes.c_double), ("lanczos_lambda_max", ctypes.c_double),
                ("last_stagnated", ctypes.c_int), ("max_local_J", ctypes.c_int), ("max_local_np", ctypes.c_int)]


class HcurlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("hcurl_amg error %d: %s" % (code, msg))
        self.code = code


def _load():
    # PyTorch ships its own HIP runtime with the same soname as /opt/rocm's.
    # Loading torch first makes the library bind to that runtime, so a single
    # HIP/HSA runtime serves the process and torch device pointers are valid.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(library_path):
        raise ImportError("libhcurl_amg.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2506_08284_amd.build); there is no CPU fallback")
    L = ctypes.CDLL(library_path)
    P = ctypes.c_void_p
    L.hcurl_amg_default_opts.argtypes = [ctypes.POINTER(hcurl_amg_opts)]
    L.hcurl_amg_default_opts.restype = None
    L.hcurl_amg_setup.argtypes = [ctypes.POINTER(hcurl_csr), ctypes.POINTER(hcurl_csr), P, P, ctypes.c_int,
                                  ctypes.POINTER(hcurl_amg_opts), ctypes.POINTER(P)]
    L.hcurl_amg_setup.restype = ctypes.c_int
    L.hcurl_amg_solve.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_double)]
    L.hcurl_amg_solve.restype = ctypes.c_int
    L.hcurl_amg_solve_noalloc.argtypes = L.hcurl_amg_solve.argtypes
    L.hcurl_amg_solve_noalloc.restype = ctypes.c_int
    L.hcurl_amg_vcycle.argtypes = [P, P, P]
    L.hcurl_amg_vcycle.restype = ctypes.c_int
    L.hcurl_amg_update.argtypes = [P, ctypes.POINTER(hcurl_csr), ctypes.c_int, ctypes.c_int]
    L.hcurl_amg_update.restype = ctypes.c_int
    L.hcurl_amg_destroy.argtypes = [P]
    L.hcurl_amg_destroy.restype = None
    L.hcurl_amg_num_levels.argtypes = [P]
    L.hcurl_amg_num_levels.restype = ctypes.c_int
    L.hcurl_amg_level_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(hcurl_level_info)]
    L.hcurl_amg_level_info.restype = ctypes.c_int
    L.hcurl_amg_commute_residual.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]
    L.hcurl_amg_commute_residual.restype = ctypes.c_int
    L.hcurl_amg_curl_residual.argtypes = [P, ctypes.POINTER(hcurl_csr), ctypes.c_int, P, P]
    L.hcurl_amg_curl_residual.restype = ctypes.c_int
    L.hcurl_amg_export_csr.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P]
    L.hcurl_amg_export_csr.restype = ctypes.c_int
    L.hcurl_amg_export_vec.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int64]
    L.hcurl_amg_export_vec.restype = ctypes.c_int
    L.hcurl_amg_stats.argtypes = [P, ctypes.POINTER(hcurl_amg_stats_t)]
    L.hcurl_amg_stats.restype = ctypes.c_int
    L.hcurl_amg_kernel_stats.argtypes = [P, ctypes.c_int, P, P, P, P]
    L.hcurl_amg_kernel_stats.restype = ctypes.c_int
    L.hcurl_amg_reset_kernel_stats.argtypes = [P]
    L.hcurl_amg_reset_kernel_stats.restype = None
    L.hcurl_last_error.argtypes = []
    L.hcurl_last_error.restype = ctypes.c_char_p
    L.hcurl_error_string.argtypes = [ctypes.c_int]
    L.hcurl_error_string.restype = ctypes.c_char_p
    L.hcurl_mpnn_num_params.argtypes = []
    L.hcurl_mpnn_num_params.restype = ctypes.c_int64
    L.hcurl_mpnn_create.argtypes = [P, P, ctypes.POINTER(P)]
    L.hcurl_mpnn_create.restype = ctypes.c_int
    L.hcurl_mpnn_get_params.argtypes = [P, P]
    L.hcurl_mpnn_get_params.restype = ctypes.c_int
    L.hcurl_mpnn_set_fp32_products.argtypes = [P, ctypes.c_int]
    L.hcurl_mpnn_set_fp32_products.restype = ctypes.c_int
    L.hcurl_mpnn_destroy.argtypes = [P]
    L.hcurl_mpnn_destroy.restype = None
    L.hcurl_amg_mpnn_sample.argtypes = [P, ctypes.POINTER(P)]
    L.hcurl_amg_mpnn_sample.restype = ctypes.c_int
    L.hcurl_mpnn_sample_entries.argtypes = [P]
    L.hcurl_mpnn_sample_entries.restype = ctypes.c_int64
    L.hcurl_mpnn_sample_export.argtypes = [P, P, P, P]
    L.hcurl_mpnn_sample_export.restype = ctypes.c_int
    L.hcurl_mpnn_sample_destroy.argtypes = [P]
    L.hcurl_mpnn_sample_destroy.restype = None
    L.hcurl_mpnn_forward.argtypes = [P, P, P]
    L.hcurl_mpnn_forward.restype = ctypes.c_int
    L.hcurl_mpnn_loss_grad.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), P]
    L.hcurl_mpnn_loss_grad.restype = ctypes.c_int
    L.hcurl_mpnn_train_step.argtypes = [P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.hcurl_mpnn_train_step.restype = ctypes.c_int
    return L


lib = _load()


def hcurl_last_error() -> str:
    return lib.hcurl_last_error().decode()


def hcurl_error_string(code: int) -> str:
    return lib.hcurl_error_string(code).decode()


def _check(rc: int, allow=()):
    if rc != HCURL_OK and rc not in allow:
        raise HcurlError(rc, hcurl_last_error() or hcurl_error_string(rc))
    return rc


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        assert a.is_contiguous()
        return a.data_ptr()
    if isinstance(a, int):
        return a
    raise TypeError(type(a))


def _csr(rowptr, col, val, nrows, ncols) -> hcurl_csr:
    nnz = int(col.shape[0])
    return hcurl_csr(nrows, ncols, nnz, _ptr(rowptr), _ptr(col), _ptr(val))


def hcurl_amg_default_opts(**overrides) -> hcurl_amg_opts:
    o = hcurl_amg_opts()
    lib.hcurl_amg_default_opts(ctypes.byref(o))
    names = {f for f, _ in hcurl_amg_opts._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError("hcurl_amg_opts has no field %r" % k)
        if k == "mem_space" and isinstance(v, str):
            v = MEM[v]
        if k == "init_values":
            v = _ptr(v)
        if k == "aggregation" and isinstance(v, str):
            v = {"given": 0, "mis2": 1}[v]
        if k == "mpnn" and v is not None and not isinstance(v, (int, ctypes.c_void_p)):
            v = v.h  # a Network
        if k == "nodal_prolongator" and v is not None:
            # (rowptr int64, col int32, val f64, ncols): the struct lives as long as the opts
            rowptr, col, val, ncols = v
            o._nodal_prolongator = _csr(rowptr, col, val, int(rowptr.shape[0]) - 1, int(ncols))
            v = ctypes.addressof(o._nodal_prolongator)
        setattr(o, k, v)
    return o


def hcurl_amg_setup(A, Dh, aggregates, coords=None, opts: hcurl_amg_opts | None = None, n_nodes: int | None = None):
    """A = (rowptr int64, col int32, val f64); Dh = (rowptr, col, val) n x m.
    aggregates: list of int32 maps (host or device arrays per opts.mem_space)."""
    opts = opts or hcurl_amg_default_opts()
    n = int(A[0].shape[0]) - 1
    m = int(n_nodes) if n_nodes is not None else int(aggregates[0].shape[0])
    cA = _csr(*A, n, n)
    cD = _csr(*Dh, n, m)
    arr = (ctypes.c_void_p * max(1, len(aggregates)))(*[_ptr(a) for a in aggregates])
    h = ctypes.c_void_p()
    _check(lib.hcurl_amg_setup(ctypes.byref(cA), ctypes.byref(cD), _ptr(coords), arr, len(aggregates),
                               ctypes.byref(opts), ctypes.byref(h)))
    return h


def hcurl_amg_solve(h, f, u, rtol: float = 1e-8, maxit: int = 500):
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = _check(lib.hcurl_amg_solve(h, _ptr(f), _ptr(u), rtol, maxit, ctypes.byref(it), ctypes.byref(rel)),
                allow=(HCURL_EMAXIT, HCURL_ESTAGNATE))
    return it.value, rel.value, rc


def hcurl_amg_solve_noalloc(h, f, u, rtol: float = 1e-8, maxit: int = 500):
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = _check(lib.hcurl_amg_solve_noalloc(h, _ptr(f), _ptr(u), rtol, maxit, ctypes.byref(it), ctypes.byref(rel)),
                allow=(HCURL_EMAXIT, HCURL_ESTAGNATE))
    return it.value, rel.value, rc


def hcurl_amg_vcycle(h, r, z):
    _check(lib.hcurl_amg_vcycle(h, _ptr(r), _ptr(z)))


REUSE = {"transfers": 0, "warm": 1}


def hcurl_amg_update(h, A, mode="transfers", iters: int = -1):
    """A = (rowptr int64, col int32, val f64) with the setup's pattern."""
    n = int(A[0].shape[0]) - 1
    cA = _csr(*A, n, n)
    _check(lib.hcurl_amg_update(h, ctypes.byref(cA), REUSE[mode] if isinstance(mode, str) else int(mode), int(iters)))


def hcurl_amg_destroy(h):
    lib.hcurl_amg_destroy(h)


def hcurl_amg_num_levels(h) -> int:
    return lib.hcurl_amg_num_levels(h)


def hcurl_amg_level_info(h, level: int) -> dict:
    info = hcurl_level_info()
    _check(lib.hcurl_amg_level_info(h, level, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def hcurl_amg_commute_residual(h, level: int):
    """(max |P^(e) D_H - D_h P^(n)|, max |D_h P^(n)|) over every row of the level."""
    a, r = ctypes.c_double(), ctypes.c_double()
    _check(lib.hcurl_amg_commute_residual(h, level, ctypes.byref(a), ctypes.byref(r)))
    return a.value, r.value


def hcurl_amg_export_csr(h, level: int, which: str):
    """Copies level data to new host arrays: (rowptr int64, col int32, val f64), shape."""
    info = hcurl_amg_level_info(h, level)
    n, m = info["n_edges"], info["n_nodes"]
    if which == "A":
        nr, nc, nnz = n, n, info["nnz_A"]
    elif which == "An":
        nr, nc, nnz = m, m, info["nnz_An"]
    else:
        nxt = hcurl_amg_level_info(h, level + 1)
        if which == "Pn":
            nr, nc, nnz = m, nxt["n_nodes"], info["nnz_Pn"]
        elif which in ("Pe", "P0"):
            nr, nc, nnz = n, nxt["n_edges"], info["nnz_Pe"]
        elif which == "R":
            nr, nc, nnz = n, nxt["n_nodes"], info["nnz_T"]
        elif which == "DH":
            nr, nc = nxt["n_edges"], nxt["n_nodes"]
            rp = np.empty(nr + 1, np.int64)  # Dirichlet coarse edges hold one entry: count first
            _check(lib.hcurl_amg_export_csr(h, level, EXPORT[which], _ptr(rp), None, None))
            nnz = int(rp[-1])
        else:
            raise ValueError(which)
    rowptr = np.empty(nr + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    _check(lib.hcurl_amg_export_csr(h, level, EXPORT[which], _ptr(rowptr), _ptr(col), _ptr(val)))
    return (rowptr, col, val), (nr, nc)


def hcurl_amg_export_vec(h, level: int, which: str, count: int | None = None):
    info = hcurl_amg_level_info(h, level)
    if which == "colors_A":
        out = np.empty(info["n_edges"], np.int32)
    elif which == "colors_An":
        out = np.empty(info["n_nodes"], np.int32)
    elif which == "energy":
        out = np.empty(count or 1024, np.float64)
    elif which == "local_pairs":
        out = np.empty(info["nnz_Pe"], np.uint16)
    elif which == "aggregates":
        out = np.empty(info["n_nodes"], np.int32)
    elif which == "pcg_history":
        out = np.empty(count or (hcurl_amg_stats(h)["last_iters"] + 1), np.float64)
    elif which in ("pcg_alpha", "pcg_beta"):
        out = np.empty(count or max(hcurl_amg_stats(h)["last_iters"], 1), np.float64)
    elif which == "ls_histogram":
        out = np.empty((LS_HIST_J, LS_HIST_NP), np.int64)
    else:
        raise ValueError(which)
    rc = lib.hcurl_amg_export_vec(h, level, VEC[which], _ptr(out), out.nbytes)
    if rc < 0:
        _check(rc)
    if which in ("energy", "pcg_history", "pcg_alpha", "pcg_beta"):
        return out[:rc]
    return out


def hcurl_amg_curl_residual(h, S, nlev: int | None = None):
    """Per level l: (max |S_l D_l|, max |S_l|) with S_0 = S (rowptr int64, col
    int32, val f64; host or device per the handle) and S_{l+1} = P^(e)T S_l P^(e)."""
    nlev = nlev or hcurl_amg_num_levels(h)
    n = int(S[0].shape[0]) - 1
    cS = _csr(*S, n, n)
    a = np.zeros(nlev)
    r = np.zeros(nlev)
    _check(lib.hcurl_amg_curl_residual(h, ctypes.byref(cS), nlev, _ptr(a), _ptr(r)))
    return a, r


def hcurl_amg_stats(h) -> dict:
    s = hcurl_amg_stats_t()
    _check(lib.hcurl_amg_stats(h, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in s._fields_}


def hcurl_amg_kernel_stats(h, max_kernels: int = 256) -> dict:
    names = (ctypes.c_char * 48 * max_kernels)()
    launches = np.zeros(max_kernels, np.int64)
    ms = np.zeros(max_kernels, np.float64)
    by = np.zeros(max_kernels, np.float64)
    n = lib.hcurl_amg_kernel_stats(h, max_kernels, ctypes.addressof(names), _ptr(launches), _ptr(ms), _ptr(by))
    if n < 0:
        _check(n)
    out = {}
    for k in range(min(n, max_kernels)):
        out[bytes(names[k]).split(b"\0", 1)[0].decode()] = dict(launches=int(launches[k]), ms=float(ms[k]),
                                                                 bytes=float(by[k]))
    return out


def hcurl_amg_reset_kernel_stats(h):
    lib.hcurl_amg_reset_kernel_stats(h)


def hcurl_mpnn_num_params() -> int:
    return int(lib.hcurl_mpnn_num_params())


def hcurl_mpnn_create(params: np.ndarray, stream=None):
    params = np.ascontiguousarray(params, np.float32)
    assert params.size == hcurl_mpnn_num_params()
    h = ctypes.c_void_p()
    _check(lib.hcurl_mpnn_create(_ptr(params), stream, ctypes.byref(h)))
    return h


def hcurl_mpnn_get_params(net) -> np.ndarray:
    out = np.empty(hcurl_mpnn_num_params(), np.float32)
    _check(lib.hcurl_mpnn_get_params(net, _ptr(out)))
    return out


def hcurl_mpnn_destroy(net):
    lib.hcurl_mpnn_destroy(net)


def hcurl_amg_mpnn_sample(h):
    s = ctypes.c_void_p()
    _check(lib.hcurl_amg_mpnn_sample(h, ctypes.byref(s)))
    return s


def hcurl_mpnn_sample_entries(s) -> int:
    return int(lib.hcurl_mpnn_sample_entries(s))


def hcurl_mpnn_sample_export(s):
    E = hcurl_mpnn_sample_entries(s)
    X = np.empty((E, 16), np.float32)
    p0 = np.empty(E)
    tg = np.empty(E)
    _check(lib.hcurl_mpnn_sample_export(s, _ptr(X), _ptr(p0), _ptr(tg)))
    return X, p0, tg


def hcurl_mpnn_sample_destroy(s):
    lib.hcurl_mpnn_sample_destroy(s)


def hcurl_mpnn_forward(net, s) -> np.ndarray:
    out = np.empty(hcurl_mpnn_sample_entries(s))
    _check(lib.hcurl_mpnn_forward(net, s, _ptr(out)))
    return out


def hcurl_mpnn_loss_grad(net, s):
    loss = ctypes.c_double()
    g = np.empty(hcurl_mpnn_num_params(), np.float32)
    _check(lib.hcurl_mpnn_loss_grad(net, s, ctypes.byref(loss), _ptr(g)))
    return loss.value, g


def hcurl_mpnn_train_step(net, s, lr, step, beta1=0.9, beta2=0.999, eps=1e-8) -> float:
    loss = ctypes.c_double()
    _check(lib.hcurl_mpnn_train_step(net, s, lr, beta1, beta2, eps, step, ctypes.byref(loss)))
    return loss.value


class Network:
    """Owns a network handle."""

    def __init__(self, params: np.ndarray, stream=None):
        self.h = hcurl_mpnn_create(params, stream)

    def params(self):
        return hcurl_mpnn_get_params(self.h)

    def set_fp32_products(self, on: bool = True):
        """Debug: FP32-operand dense products (hcurl_mpnn_set_fp32_products)."""
        _check(lib.hcurl_mpnn_set_fp32_products(self.h, 1 if on else 0))

    def close(self):
        if self.h:
            hcurl_mpnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    """Owns a handle; methods map one to one onto the C calls."""

    def __init__(self, A, Dh, aggregates, n_nodes, coords=None, allocator=None, **opts):
        """allocator: None (the library's stream-ordered hipMallocAsync), "torch"
        (PyTorch's caching allocator) or (alloc(nbytes, stream) -> ptr,
        free(ptr, nbytes, stream)); the callbacks live as long as the handle."""
        self.h = None
        self._cbs = _allocator_callbacks(allocator) if allocator is not None else None
        self.opts = hcurl_amg_default_opts(**opts)
        if self._cbs:
            self.opts.dev_alloc = ctypes.cast(self._cbs[0], ctypes.c_void_p).value
            self.opts.dev_free = ctypes.cast(self._cbs[1], ctypes.c_void_p).value
        self._keep = (A, Dh, aggregates, opts.get("init_values"), opts.get("mpnn"), opts.get("nodal_prolongator"), coords)
        self.h = hcurl_amg_setup(A, Dh, aggregates, coords, self.opts, n_nodes=n_nodes)

    def solve(self, f, u, rtol=1e-8, maxit=500):
        return hcurl_amg_solve(self.h, f, u, rtol, maxit)

    def solve_noalloc(self, f, u, rtol=1e-8, maxit=500):
        return hcurl_amg_solve_noalloc(self.h, f, u, rtol, maxit)

    def vcycle(self, r, z):
        hcurl_amg_vcycle(self.h, r, z)

    def update(self, A, mode="transfers", iters=-1):
        hcurl_amg_update(self.h, A, mode, iters)

    def num_levels(self):
        return hcurl_amg_num_levels(self.h)

    def level_info(self, level):
        return hcurl_amg_level_info(self.h, level)

    def commute_residual(self, level):
        return hcurl_amg_commute_residual(self.h, level)

    def curl_residual(self, S, nlev=None):
        return hcurl_amg_curl_residual(self.h, S, nlev)

    def export_csr(self, level, which):
        return hcurl_amg_export_csr(self.h, level, which)

    def export_vec(self, level, which, count=None):
        return hcurl_amg_export_vec(self.h, level, which, count)

    def stats(self):
        return hcurl_amg_stats(self.h)

    def kernel_stats(self):
        return hcurl_amg_kernel_stats(self.h)

    def reset_kernel_stats(self):
        hcurl_amg_reset_kernel_stats(self.h)

    def mpnn_sample(self):
        return hcurl_amg_mpnn_sample(self.h)

    def close(self):
        if self.h:
            hcurl_amg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
