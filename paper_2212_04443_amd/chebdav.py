"""ctypes binding of libchebdav.so (include/chebdav.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory and the current HIP stream.  Dense blocks are
row-major torch tensors whose last dimension is contiguous; the leading
dimension passed to the library is the tensor's row stride.

The library must be built (python -m paper_2212_04443_amd.build); importing
this module raises if it is missing, and there is no fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchebdav.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
ORTH_CHOLQR, ORTH_TSQR = 0, 1
_ORTH = {"cholqr": ORTH_CHOLQR, "tsqr": ORTH_TSQR}
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOCONV", -5: "EBREAKDOWN",
           -6: "EUNSUPPORTED"}

EXPORTED = [
    "chebdav_build_laplacian", "chebdav_graph_info", "chebdav_graph_export", "chebdav_graph_free",
    "chebdav_graph_row_split",
    "chebdav_spmm", "chebdav_filter_workspace_size", "chebdav_filter",
    "chebdav_orthonormalize_workspace_size", "chebdav_orthonormalize",
    "chebdav_solve_workspace_size", "chebdav_solve", "chebdav_small_eig_workspace_size",
    "chebdav_small_eig", "chebdav_philox_fill", "chebdav_dinv", "chebdav_last_error",
    "chebdav_gcn_workspace_size", "chebdav_gcn_forward", "chebdav_gcn_backward", "chebdav_gcn_features",
    "chebdav_subspace_loss_workspace_size", "chebdav_subspace_loss", "chebdav_adam_step",
    "chebdav_rayleigh_ritz_workspace_size", "chebdav_rayleigh_ritz",
    "chebdav_cluster_workspace_size", "chebdav_cluster",
    "chebdav_lanczos_bounds_workspace_size", "chebdav_lanczos_bounds",
    "chebdav_tsqr_workspace_size", "chebdav_tsqr", "chebdav_filter_noalloc",
    "chebdav_probe_gather", "chebdav_probe_gather_out_len",
]


class ChebdavError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, msg))
        self.status = status


class IterRecord(ctypes.Structure):
    _fields_ = [
        ("iteration", ctypes.c_int), ("kc", ctypes.c_int), ("kact", ctypes.c_int), ("ksub", ctypes.c_int),
        ("n_locked", ctypes.c_int), ("n_unlocked", ctypes.c_int), ("inner_restart", ctypes.c_int),
        ("outer_restart", ctypes.c_int), ("filter_f32", ctypes.c_int), ("low_nwb", ctypes.c_double),
        ("min_residual", ctypes.c_double), ("max_residual", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


LOG_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(IterRecord), ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [
        ("k_want", ctypes.c_int), ("kb", ctypes.c_int), ("m", ctypes.c_int), ("itmax", ctypes.c_int),
        ("tol", ctypes.c_double), ("act_max", ctypes.c_int), ("dim_max", ctypes.c_int),
        ("k_ri", ctypes.c_int), ("upperb", ctypes.c_double), ("lowb", ctypes.c_double),
        ("low_nwb0", ctypes.c_double), ("filter_dtype", ctypes.c_int),
        ("f32_switch_tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("timing", ctypes.c_int),
        ("orth", ctypes.c_int), ("k_ro", ctypes.c_int), ("refine_sweeps", ctypes.c_int),
        ("certify_tol", ctypes.c_double), ("log_cb", LOG_FN), ("log_user", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("n_spmm_filter", ctypes.c_int),
        ("n_spmm_filter_f32", ctypes.c_int), ("n_spmm_other", ctypes.c_int),
        ("n_random", ctypes.c_int), ("n_replaced", ctypes.c_int), ("max_residual", ctypes.c_double),
        ("t_total_ms", ctypes.c_double), ("t_filter_ms", ctypes.c_double),
        ("n_filter_launches", ctypes.c_int), ("used_fallback", ctypes.c_int), ("n_unlocked", ctypes.c_int),
        ("n_inner_restarts", ctypes.c_int), ("n_outer_restarts", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libchebdav.so is not built: run `python -m paper_2212_04443_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    p, i64, i32, d, u64, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                               ctypes.c_uint64, ctypes.c_size_t)
    P = ctypes.POINTER
    sig = {
        "chebdav_build_laplacian": [p, i64, i64, i32, p, P(p)],
        "chebdav_graph_info": [p, P(i64), P(i64), P(i64), P(ctypes.c_int32)],
        "chebdav_graph_export": [p, p, p, p, p, p],
        "chebdav_graph_row_split": [p, P(i64)],
        "chebdav_spmm": [p, d, d, d, p, p, p, i64, i32, i32, p],
        "chebdav_filter_workspace_size": [p, i32, i32, P(sz)],
        "chebdav_filter": [p, p, i64, p, i64, i32, i32, d, d, d, i32, p, sz, p],
        "chebdav_filter_noalloc": [p, p, i64, p, i64, i32, i32, d, d, d, i32, p],
        "chebdav_orthonormalize_workspace_size": [i64, i32, i32, i32, P(sz)],
        "chebdav_orthonormalize": [p, i64, i32, p, i64, i32, i64, u64, u64, i32, P(i32), p, sz, p],
        "chebdav_tsqr_workspace_size": [i64, i32, P(sz)],
        "chebdav_tsqr": [p, i64, i64, i32, p, i64, p, i64, p, sz, p],
        "chebdav_solve_workspace_size": [p, P(Params), P(sz)],
        "chebdav_solve": [p, P(Params), p, i32, p, p, P(Stats), p, sz, p],
        "chebdav_small_eig_workspace_size": [i32, P(sz)],
        "chebdav_small_eig": [p, i64, i32, p, p, i64, p, sz, p],
        "chebdav_philox_fill": [p, i64, i32, i64, u64, u64, p],
        "chebdav_dinv": [p, p, i64, p],
        "chebdav_gcn_workspace_size": [p, P(i32), P(sz)],
        "chebdav_gcn_forward": [p, P(i32), p, P(p), p, p, p, sz, p],
        "chebdav_gcn_backward": [p, P(i32), p, P(p), p, p, P(p), p, sz, p],
        "chebdav_gcn_features": [p, u64, i32, p, i64, p],
        "chebdav_subspace_loss_workspace_size": [i64, i32, i32, P(sz)],
        "chebdav_subspace_loss": [p, i64, p, i64, i64, i32, i32, P(d), p, i64, p, sz, p],
        "chebdav_adam_step": [p, p, p, p, i64, d, d, d, d, i32, p],
        "chebdav_rayleigh_ritz_workspace_size": [p, i32, P(sz)],
        "chebdav_rayleigh_ritz": [p, p, i64, i32, u64, p, i64, p, p, sz, p],
        "chebdav_cluster_workspace_size": [i64, i32, i32, P(sz)],
        "chebdav_cluster": [p, i64, i64, i32, i32, i32, u64, p, p, P(i32), P(d), p, sz, p],
        "chebdav_lanczos_bounds_workspace_size": [p, i32, P(sz)],
        "chebdav_lanczos_bounds": [p, i32, u64, P(d), P(d), P(d), P(d), P(i32), p, sz, p],
        "chebdav_probe_gather": [p, i64, i32, i64, u64, p, P(i64), p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.chebdav_graph_free.argtypes = [p]
    L.chebdav_graph_free.restype = None
    L.chebdav_probe_gather_out_len.argtypes = []
    L.chebdav_probe_gather_out_len.restype = ctypes.c_int64
    L.chebdav_last_error.argtypes = []
    L.chebdav_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()


def lib_path() -> str:
    return _LIB_PATH


def last_error() -> str:
    return _lib.chebdav_last_error().decode()


def _check(st: int):
    if st != OK:
        raise ChebdavError(st, last_error())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("expected a 2-D tensor with contiguous rows")
    return t.stride(0)


def _block(t, name: str, rows: int, dtypes, cols: int | None = None, device=None):
    """Checks a device block before its pointer crosses the ABI: 2-D, `rows` rows
    with contiguous rows (leading dimension >= width), one of `dtypes`, on the
    CUDA device (`device` if given), `cols` columns if given.  The library reads
    and writes through raw pointers, so a wrong shape would run off the buffer."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.dim() != 2 or t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError("%s must be 2-D with contiguous rows" % name)
    if t.shape[0] != rows:
        raise ValueError("%s has %d rows, expected %d" % (name, t.shape[0], rows))
    if cols is not None and t.shape[1] != cols:
        raise ValueError("%s has %d columns, expected %d" % (name, t.shape[1], cols))
    if t.dtype not in dtypes:
        raise ValueError("%s must be %s" % (name, " or ".join(str(d) for d in dtypes)))
    if device is not None and not _same_device(t.device, device):
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    return t


def _same_device(a, b) -> bool:
    da, db = torch.device(a), torch.device(b)
    if da.type != db.type:
        return False
    cur = torch.cuda.current_device() if da.type == "cuda" else 0
    return (da.index if da.index is not None else cur) == (db.index if db.index is not None else cur)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Graph:
    """Device CSR of S with its degree scaling; frees itself when collected."""

    def __init__(self, handle: ctypes.c_void_p, device):
        self._h = handle
        self.device = device
        n, nnz, iso, mx = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(_lib.chebdav_graph_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(iso),
                                       ctypes.byref(mx)))
        self.n, self.nnz, self.n_isolated, self.max_deg = n.value, nnz.value, iso.value, mx.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib.chebdav_graph_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_laplacian(edges, n_nodes: int, device="cuda", stream=None) -> Graph:
    """chebdav_build_laplacian from an (E, 2) int64 edge list (NumPy array or
    torch tensor; a CUDA tensor is read in place)."""
    if isinstance(edges, torch.Tensor):
        e = edges.to(torch.int64).contiguous()
        on_dev = 1 if e.is_cuda else 0
        if not on_dev:
            e = e.numpy()
    else:
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
        on_dev = 0
    n_edges = int(e.shape[0]) if e.ndim == 2 else 0
    ptr = ctypes.c_void_p(e.data_ptr()) if on_dev else ctypes.c_void_p(e.ctypes.data)
    h = ctypes.c_void_p()
    with torch.cuda.device(torch.device(device)):
        _check(_lib.chebdav_build_laplacian(ptr, n_edges, int(n_nodes), on_dev, _stream(stream),
                                            ctypes.byref(h)))
    return Graph(h, torch.device(device))


def probe_gather(table: torch.Tensor, row_bytes: int, gathers: int, seed: int = 0, stream=None):
    """chebdav_probe_gather: `gathers` random whole-row reads of `row_bytes` bytes from
    the rows of `table` (a device tensor of rows x row_bytes bytes, any dtype).
    Returns (gathers performed, the device output that keeps the loads live)."""
    nbytes = table.numel() * table.element_size()
    if not table.is_contiguous() or nbytes % row_bytes:
        raise ValueError("table must be contiguous and a whole number of rows")
    out = torch.empty(int(_lib.chebdav_probe_gather_out_len()), dtype=torch.float64, device=table.device)
    done = ctypes.c_int64()
    _check(_lib.chebdav_probe_gather(_ptr(table), nbytes // row_bytes, row_bytes, gathers, seed, _ptr(out),
                                     ctypes.byref(done), _stream(stream)))
    return done.value, out


def graph_row_split(g: Graph):
    """chebdav_graph_row_split: the nine row boundaries of the per-XCD ranges."""
    b = (ctypes.c_int64 * 9)()
    _check(_lib.chebdav_graph_row_split(g.handle, b))
    return [int(x) for x in b]


def graph_export(g: Graph, stream=None):
    """Returns (row_ptr int64[n+1], col int32[nnz], deg int32[n], dinv float64[n]) on the device."""
    dev = g.device
    rp = torch.empty(g.n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    deg = torch.empty(g.n, dtype=torch.int32, device=dev)
    dinv = torch.empty(g.n, dtype=torch.float64, device=dev)
    _check(_lib.chebdav_graph_export(g.handle, _ptr(rp), _ptr(col), _ptr(deg), _ptr(dinv), _stream(stream)))
    return rp, col[: g.nnz], deg, dinv


def spmm(g: Graph, alpha: float, beta: float, gamma: float, U: torch.Tensor, Z, Y: torch.Tensor,
         stream=None):
    """Y = alpha D^{-1/2} S D^{-1/2} U + beta U + gamma Z (float64 or float32)."""
    _block(U, "U", g.n, (torch.float64, torch.float32), device=g.device)
    _block(Y, "Y", g.n, (U.dtype,), U.shape[1], g.device)
    if Z is not None:
        _block(Z, "Z", g.n, (U.dtype,), U.shape[1], g.device)
    dt = {torch.float64: F64, torch.float32: F32}[U.dtype]
    ld = _ld(U)
    if _ld(Y) != ld or (Z is not None and _ld(Z) != ld):
        raise ValueError("U, Z and Y must share the leading dimension")
    _check(_lib.chebdav_spmm(g.handle, alpha, beta, gamma, _ptr(U), _ptr(Z), _ptr(Y), ld,
                             U.shape[1], dt, _stream(stream)))
    return Y


def filter(g: Graph, X: torch.Tensor, m: int, cut: float, upper: float = 2.0, scale_pt: float = 0.0,
           dtype: int = F64, Y: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
           stream=None) -> torch.Tensor:
    """chebdav_filter: Y = p_m(A) X (X float64, n x kb)."""
    _block(X, "X", g.n, (torch.float64,), device=g.device)
    kb = X.shape[1]
    if Y is None:
        Y = torch.empty_like(X)
    _block(Y, "Y", g.n, (torch.float64,), kb, g.device)
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_filter_workspace_size(g.handle, kb, dtype, ctypes.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = _workspace(nb.value, X.device)
    _check(_lib.chebdav_filter(g.handle, _ptr(X), _ld(X), _ptr(Y), _ld(Y), kb, m, cut, upper, scale_pt,
                               dtype, _ptr(workspace), workspace.numel(), _stream(stream)))
    return Y


def filter_noalloc(g: Graph, X: torch.Tensor, m: int, cut: float, upper: float = 2.0, scale_pt: float = 0.0,
                   dtype: int = F64, Y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """chebdav_filter_noalloc: chebdav_filter on the library's static scratch
    (no workspace; Y must be given by callers that cannot allocate)."""
    _block(X, "X", g.n, (torch.float64,), device=g.device)
    kb = X.shape[1]
    if Y is None:
        Y = torch.empty_like(X)
    _block(Y, "Y", g.n, (torch.float64,), kb, g.device)
    _check(_lib.chebdav_filter_noalloc(g.handle, _ptr(X), _ld(X), _ptr(Y), _ld(Y), kb, m, cut, upper, scale_pt,
                                       dtype, _stream(stream)))
    return Y


def orthonormalize(V, X: torch.Tensor, seed: int = 0, first_random_col: int = 0, method: str = "cholqr",
                   stream=None) -> int:
    """chebdav_orthonormalize, in place on X; returns the number of replaced columns.
    method: "cholqr" (Cholesky QR twice) or "tsqr" (Householder TSQR)."""
    _block(X, "X", X.shape[0] if X.dim() == 2 else -1, (torch.float64,))
    n, kb = X.shape
    ksub = 0 if V is None else V.shape[1]
    if ksub:
        _block(V, "V", n, (torch.float64,), device=X.device)
    meth = _ORTH[method]
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_orthonormalize_workspace_size(n, ksub, kb, meth, ctypes.byref(nb)))
    ws = _workspace(nb.value, X.device)
    rep = ctypes.c_int(0)
    _check(_lib.chebdav_orthonormalize(_ptr(V) if ksub else ctypes.c_void_p(0), _ld(V) if ksub else 1,
                                       ksub, _ptr(X), _ld(X), kb, n, seed, first_random_col, meth,
                                       ctypes.byref(rep), _ptr(ws), ws.numel(), _stream(stream)))
    return rep.value


def tsqr(X: torch.Tensor, Q: torch.Tensor | None = None, stream=None):
    """chebdav_tsqr: X = Q R (thin QR, R with a non-negative diagonal).  Q may be X
    itself (in place).  Returns (Q, R)."""
    _block(X, "X", X.shape[0] if X.dim() == 2 else -1, (torch.float64,))
    n, kb = X.shape
    if Q is None:
        Q = torch.empty((n, kb), dtype=torch.float64, device=X.device)
    _block(Q, "Q", n, (torch.float64,), kb, X.device)
    R = torch.empty((kb, kb), dtype=torch.float64, device=X.device)
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_tsqr_workspace_size(n, kb, ctypes.byref(nb)))
    ws = _workspace(nb.value, X.device)
    _check(_lib.chebdav_tsqr(_ptr(X), _ld(X), n, kb, _ptr(Q), _ld(Q), _ptr(R), _ld(R), _ptr(ws), ws.numel(),
                             _stream(stream)))
    return Q, R


def make_params(k_want, kb, m, tol=1e-8, itmax=0, act_max=0, dim_max=0, k_ri=0, upperb=2.0,
                lowb=0.0, low_nwb0=math.nan, filter_dtype=F64, f32_switch_tol=0.0, seed=0,
                timing=False, orth="cholqr", k_ro=0, refine_sweeps=0, certify_tol=0.0,
                log=None) -> Params:
    """chebdav_params.  `log`, if given, is a list that receives one dict per
    Davidson iteration (chebdav_iter_record) through log_cb."""
    cb = LOG_FN()
    if log is not None:
        def _cb(rec, user):
            log.append(rec.contents.as_dict())
        cb = LOG_FN(_cb)
    p = Params(k_want, kb, m, itmax, tol, act_max, dim_max, k_ri, upperb, lowb, low_nwb0,
               filter_dtype, f32_switch_tol, seed, 1 if timing else 0, _ORTH[orth], k_ro, refine_sweeps,
               certify_tol, cb, None)
    p._cb_ref = cb  # the callback object lives as long as the parameters
    return p


def solve_workspace_size(g: Graph, params: Params) -> int:
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_solve_workspace_size(g.handle, ctypes.byref(params), ctypes.byref(nb)))
    return nb.value


@dataclass
class SolveResult:
    evals: torch.Tensor
    evecs: torch.Tensor
    stats: dict
    status: int


def solve(g: Graph, params: Params, V_init: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None, stream=None, allow_noconv: bool = False) -> SolveResult:
    """chebdav_solve.  Returns evals (k_want,), evecs (n, k_want) and the stats."""
    need = solve_workspace_size(g, params)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, g.device)
    evals = torch.empty(params.k_want, dtype=torch.float64, device=g.device)
    evecs = torch.empty(g.n, params.k_want, dtype=torch.float64, device=g.device)
    st = Stats()
    k_init = 0
    vptr = ctypes.c_void_p(0)
    if V_init is not None:
        _block(V_init, "V_init", g.n, (torch.float64,), device=g.device)
        if not V_init.is_contiguous():
            raise ValueError("V_init must be a contiguous float64 (n, k_init) tensor")
        k_init = V_init.shape[1]
        vptr = _ptr(V_init)
    rc = _lib.chebdav_solve(g.handle, ctypes.byref(params), vptr, k_init, _ptr(evals), _ptr(evecs),
                            ctypes.byref(st), _ptr(workspace), workspace.numel(), _stream(stream))
    if rc != OK and not (allow_noconv and rc == ENOCONV):
        raise ChebdavError(rc, last_error())
    return SolveResult(evals, evecs, st.as_dict(), rc)


def small_eig(H: torch.Tensor, stream=None):
    """chebdav_small_eig: (ascending eigenvalues, eigenvectors as columns)."""
    n = H.shape[0]
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_small_eig_workspace_size(n, ctypes.byref(nb)))
    ws = _workspace(nb.value, H.device)
    w = torch.empty(n, dtype=torch.float64, device=H.device)
    Y = torch.empty(n, n, dtype=torch.float64, device=H.device)
    _check(_lib.chebdav_small_eig(_ptr(H), _ld(H), n, _ptr(w), _ptr(Y), _ld(Y), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return w, Y


def philox_fill(n: int, w: int, seed: int, first_col: int = 0, device="cuda", stream=None):
    X = torch.empty(n, w, dtype=torch.float64, device=device)
    _check(_lib.chebdav_philox_fill(_ptr(X), n, w, w, seed, first_col, _stream(stream)))
    return X


def dinv(deg: torch.Tensor, stream=None) -> torch.Tensor:
    """chebdav_dinv on an int32 device tensor."""
    out = torch.empty(deg.shape[0], dtype=torch.float64, device=deg.device)
    _check(_lib.chebdav_dinv(_ptr(deg), _ptr(out), deg.shape[0], _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# Learned warm start (graph-convolution network) building blocks
# ---------------------------------------------------------------------------
def _dims(dims):
    return (ctypes.c_int * 4)(*[int(x) for x in dims])


def _ptr_array(ts):
    return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])


def _gcn_args(g: Graph, dims, X0, W):
    _block(X0, "X0", g.n, (torch.float32,), dims[0], g.device)
    for l in range(3):
        _block(W[l], "W[%d]" % l, dims[l], (torch.float32,), dims[l + 1], g.device)
        if not W[l].is_contiguous():
            raise ValueError("W[%d] must be contiguous" % l)


def gcn_workspace(g: Graph, dims) -> torch.Tensor:
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_gcn_workspace_size(g.handle, _dims(dims), ctypes.byref(nb)))
    return _workspace(nb.value, g.device)


def gcn_forward(g: Graph, dims, X0: torch.Tensor, W, acts=None, out=None, workspace=None, stream=None):
    """chebdav_gcn_forward.  W: three float32 tensors (d_l x d_{l+1}).  Returns (out, acts)."""
    n = g.n
    _gcn_args(g, dims, X0, W)
    if acts is None:
        acts = torch.empty(n * (dims[1] + dims[2]), dtype=torch.float32, device=g.device)
    if out is None:
        out = torch.empty(n, dims[3], dtype=torch.float32, device=g.device)
    ws = workspace if workspace is not None else gcn_workspace(g, dims)
    _check(_lib.chebdav_gcn_forward(g.handle, _dims(dims), _ptr(X0), _ptr_array(W), _ptr(acts), _ptr(out),
                                    _ptr(ws), ws.numel(), _stream(stream)))
    return out, acts


def gcn_backward(g: Graph, dims, X0, W, acts, d_out, dW=None, workspace=None, stream=None):
    """chebdav_gcn_backward.  Returns the three weight gradients."""
    _gcn_args(g, dims, X0, W)
    _block(d_out, "d_out", g.n, (torch.float32,), dims[3], g.device)
    if not acts.is_cuda or acts.dtype != torch.float32 or acts.numel() < g.n * (dims[1] + dims[2]):
        raise ValueError("acts must be the float32 activations of gcn_forward")
    if dW is None:
        dW = [torch.empty_like(w) for w in W]
    ws = workspace if workspace is not None else gcn_workspace(g, dims)
    _check(_lib.chebdav_gcn_backward(g.handle, _dims(dims), _ptr(X0), _ptr_array(W), _ptr(acts), _ptr(d_out),
                                     _ptr_array(dW), _ptr(ws), ws.numel(), _stream(stream)))
    return dW


def gcn_features(g: Graph, seed: int, n_gauss: int = 16, stream=None) -> torch.Tensor:
    X = torch.empty(g.n, n_gauss + 1, dtype=torch.float32, device=g.device)
    _check(_lib.chebdav_gcn_features(g.handle, seed, n_gauss, _ptr(X), n_gauss + 1, _stream(stream)))
    return X


def subspace_loss(X: torch.Tensor, U: torch.Tensor, grad: bool = True, workspace=None, stream=None):
    """chebdav_subspace_loss: (loss, dL/dX or None)."""
    _block(X, "X", X.shape[0] if X.dim() == 2 else -1, (torch.float32,))
    _block(U, "U", X.shape[0], (torch.float64,), device=X.device)
    n, kx = X.shape
    ku = U.shape[1]
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_subspace_loss_workspace_size(n, kx, ku, ctypes.byref(nb)))
    ws = workspace if workspace is not None and workspace.numel() >= nb.value else _workspace(nb.value, X.device)
    dX = torch.empty_like(X) if grad else None
    loss = ctypes.c_double()
    _check(_lib.chebdav_subspace_loss(_ptr(X), _ld(X), _ptr(U), _ld(U), n, kx, ku, ctypes.byref(loss),
                                      _ptr(dX), _ld(dX) if grad else kx, _ptr(ws), ws.numel(), _stream(stream)))
    return loss.value, dX


def adam_step(params, grads, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=1, stream=None):
    _check(_lib.chebdav_adam_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), lr, beta1, beta2,
                                  eps, step, _stream(stream)))


def rayleigh_ritz(g: Graph, X: torch.Tensor, seed: int = 0, stream=None):
    """chebdav_rayleigh_ritz: (V float64 n x k, ritz values ascending)."""
    _block(X, "X", g.n, (torch.float32,), device=g.device)
    n, k = X.shape
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_rayleigh_ritz_workspace_size(g.handle, k, ctypes.byref(nb)))
    ws = _workspace(nb.value, X.device)
    V = torch.empty(n, k, dtype=torch.float64, device=X.device)
    ritz = torch.empty(k, dtype=torch.float64, device=X.device)
    _check(_lib.chebdav_rayleigh_ritz(g.handle, _ptr(X), _ld(X), k, seed, _ptr(V), _ld(V), _ptr(ritz), _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return V, ritz


def cluster(U: torch.Tensor, n_clusters: int, seed: int = 0, max_iter: int = 100, stream=None):
    """chebdav_cluster: row normalization of the eigenvector block U (float64,
    n x k) and K-means.  Returns (labels int32[n], centres n_clusters x k, rounds,
    inertia)."""
    _block(U, "U", U.shape[0] if U.dim() == 2 else -1, (torch.float64,))
    n, k = U.shape
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_cluster_workspace_size(n, k, n_clusters, ctypes.byref(nb)))
    ws = _workspace(nb.value, U.device)
    labels = torch.empty(n, dtype=torch.int32, device=U.device)
    C = torch.empty(n_clusters, k, dtype=torch.float64, device=U.device)
    rounds = ctypes.c_int()
    inertia = ctypes.c_double()
    _check(_lib.chebdav_cluster(_ptr(U), _ld(U), n, k, n_clusters, max_iter, seed, _ptr(labels), _ptr(C),
                                ctypes.byref(rounds), ctypes.byref(inertia), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return labels, C, rounds.value, inertia.value


def lanczos_bounds(g: Graph, steps: int = 10, seed: int = 0, stream=None):
    """chebdav_lanczos_bounds: (lower, upper, alpha, beta) from `steps` Lanczos steps."""
    import numpy as np
    nb = ctypes.c_size_t()
    _check(_lib.chebdav_lanczos_bounds_workspace_size(g.handle, steps, ctypes.byref(nb)))
    ws = _workspace(nb.value, "cuda")
    lo, hi = ctypes.c_double(), ctypes.c_double()
    al = (ctypes.c_double * steps)()
    be = (ctypes.c_double * steps)()
    k = ctypes.c_int()
    _check(_lib.chebdav_lanczos_bounds(g.handle, steps, seed, ctypes.byref(lo), ctypes.byref(hi), al, be,
                                       ctypes.byref(k), _ptr(ws), ws.numel(), _stream(stream)))
    return lo.value, hi.value, np.array(al[:k.value]), np.array(be[:k.value])
