"""s-FairSC on AMD MI355X: Python binding of the HIP library libsfairsc.so.

Scalable fair spectral clustering (Wang, Lu, Davidson and Bai, AISTATS 2023):
the k smallest eigenpairs of the graph Laplacian restricted to the nullspace
of the group-fairness constraint F^T (Alg. 3), computed with the deflated
operator L^sigma = P (L_n - sigma I) P + sigma I (eq. asigma) inside a block
Krylov-Schur eigensolver, then k-means on the rows of H.

This module only marshals arguments (torch tensors -> device pointers and
the current HIP stream); all arithmetic runs in the library's kernels.  It
raises ImportError when the library is missing; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import warnings
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import (  # noqa: F401
    E_ARG,
    E_ASYM,
    E_DEGENERATE,
    E_EMPTY_GROUP,
    E_HIP,
    E_ISOLATED,
    E_NOMEM,
    E_NOT_CONVERGED,
    OK,
    PREC_FP64,
    PREC_MIXED,
    SfairscError,
)

__all__ = [
    "Graph",
    "eigs_batched",
    "autotune",
    "tuning_save",
    "tuning_load",
    "tuning_clear",
    "tuning_size",
    "tuning_lookup",
    "EigsResult",
    "FairEigSum",
    "symeig",
    "SfairscError",
    "version",
    "PREC_FP64",
    "PREC_MIXED",
]

_lib.lib()  # fail loudly at import if the HIP library is missing


def version() -> str:
    return _lib.lib().sfairsc_version().decode()


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _prec(precision) -> int:
    if precision in ("fp64", PREC_FP64):
        return PREC_FP64
    if precision in ("mixed", PREC_MIXED):
        return PREC_MIXED
    raise ValueError(f"unknown precision {precision!r}")


def _dev(x, dtype, device) -> torch.Tensor:
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device=device, dtype=dtype).contiguous()


@dataclass
class EigsResult:
    eigenvalues: np.ndarray  # (k,) ascending
    H: torch.Tensor  # (n, k) float64 on the device (column-major storage)
    info: dict
    status: int


class Graph:
    """A graph handle: CSR of W (both triangles), group labels, variant.

    rowptr/col int32, values float32 or float64, groups int32 in [0, h); numpy
    arrays or torch tensors (copied to the GPU).  normalized selects Alg. 3's
    normalized Laplacian (True) or the unnormalized variant (False).
    """

    def __init__(self, rowptr, col, values, groups, h: int, normalized: bool, device="cuda", stream=None):
        self.device = torch.device(device)
        rp = _dev(rowptr, torch.int32, self.device)
        ci = _dev(col, torch.int32, self.device)
        if isinstance(values, np.ndarray):
            vdt = torch.float32 if values.dtype == np.float32 else torch.float64
        else:
            vdt = values.dtype if values.dtype in (torch.float32, torch.float64) else torch.float64
        va = _dev(values, vdt, self.device)
        gr = _dev(groups, torch.int32, self.device)
        self.n = int(rp.numel() - 1)
        self.nnz = int(ci.numel())
        self.h = int(h)
        self.normalized = bool(normalized)
        self.value_dtype = vdt
        self._rowptr, self._col, self._groups = rp, ci, gr
        handle = ctypes.c_void_p()
        code = _lib.lib().sfairsc_graph_create(
            ctypes.byref(handle),
            self.n,
            self.nnz,
            _ptr(rp),
            _ptr(ci),
            _ptr(va),
            _lib.F32 if vdt == torch.float32 else _lib.F64,
            _ptr(gr),
            self.h,
            int(self.normalized),
            _stream(stream),
        )
        _lib.check(code)
        self._h = handle

    @classmethod
    def from_msbm(cls, g, normalized: bool, device="cuda"):
        """From an sfairsc_inputs.MSBMGraph."""
        return cls(g.rowptr, g.col, g.val, g.groups, g.h, normalized, device=device)

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().sfairsc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        st = _lib.GraphStats()
        _lib.check(_lib.lib().sfairsc_graph_query(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def set_constraint(self, F, center: bool = False, rank_tol: float = 0.0, stream=None) -> int:
        """Constrain by a general n x m matrix F (F^T H = 0) instead of the
        group labels; center=True subtracts the column means first (0/1
        memberships, possibly overlapping).  Returns the rank kept."""
        Ft = torch.as_tensor(F).to(self.device, torch.float64)
        if Ft.dim() == 1:
            Ft = Ft[:, None]
        if Ft.shape[0] != self.n:
            raise ValueError(f"F has {Ft.shape[0]} rows, the graph {self.n} vertices")
        Fc = Ft.t().contiguous()  # column-major storage for the library
        rank = ctypes.c_int32(0)
        _lib.check(
            _lib.lib().sfairsc_graph_set_constraint(
                self._h, _ptr(Fc), self.n, int(Fc.shape[0]), int(bool(center)), float(rank_tol), ctypes.byref(rank),
                _stream(stream)
            )
        )
        self.constraint_rank = int(rank.value)
        return self.constraint_rank

    def set_memberships(self, G, center: bool = True, inner_tol: float = 0.0, max_inner: int = 0, stream=None):
        """Constrain by a sparse 0/1 membership matrix G (scipy sparse or
        dense, n x m; overlapping groups allowed) with the projection
        computed by LSQR inside the eigensolver."""
        import scipy.sparse as sp

        Gc = sp.csr_matrix(G)
        Gc.sort_indices()
        if Gc.shape[0] != self.n:
            raise ValueError(f"G has {Gc.shape[0]} rows, the graph {self.n} vertices")
        rp = torch.from_numpy(Gc.indptr.astype(np.int32)).to(self.device)
        ci = torch.from_numpy(Gc.indices.astype(np.int32)).to(self.device)
        _lib.check(
            _lib.lib().sfairsc_graph_set_memberships(
                self._h, int(Gc.shape[1]), _ptr(rp), _ptr(ci), int(bool(center)), float(inner_tol), int(max_inner),
                _stream(stream)
            )
        )

    def lsqr_stats(self, stream=None) -> dict:
        """LSQR counters of a membership constraint (solves, steps, max
        steps of one solve, unconverged columns)."""
        out = (ctypes.c_int64 * 4)()
        _lib.check(_lib.lib().sfairsc_lsqr_stats(self._h, out, _stream(stream)))
        return {"solves": out[0], "steps": out[1], "max_steps": out[2], "unconverged": out[3]}

    @property
    def sigma(self) -> float:
        return self.stats()["sigma"]

    # -- operator ------------------------------------------------------
    def apply_operator(self, X: torch.Tensor, precision="fp64", sigma: float = 0.0, stream=None) -> torch.Tensor:
        """Y = L^sigma X for X (n x b, b <= 32) float64 on the device."""
        X = X.to(self.device, torch.float64).contiguous()
        if X.dim() == 1:
            X = X[:, None]
        Y = torch.empty_like(X)
        _lib.check(
            _lib.lib().sfairsc_apply_operator(
                self._h, _ptr(X), _ptr(Y), X.shape[1], _prec(precision), float(sigma), _stream(stream)
            )
        )
        return Y

    def apply_operator_noalloc(self, X: torch.Tensor, Y: torch.Tensor, precision="fp64", sigma: float = 0.0,
                               stream=None) -> torch.Tensor:
        """Y = L^sigma X into the caller's Y through the no-allocation entry point.

        X and Y: contiguous float64 (n, b) tensors on the graph's device; the
        library allocates nothing (its scratch is a fixed device array).
        """
        if X.dim() != 2 or Y.shape != X.shape or X.dtype != torch.float64 or Y.dtype != torch.float64:
            raise ValueError("X and Y must be float64 tensors of the same shape (n, b)")
        if not (X.is_contiguous() and Y.is_contiguous()):
            raise ValueError("X and Y must be contiguous")
        _lib.check(
            _lib.lib().sfairsc_apply_operator_noalloc(
                self._h, _ptr(X), _ptr(Y), X.shape[1], _prec(precision), float(sigma), _stream(stream)
            )
        )
        return Y

    def spmm(self, X: torch.Tensor, precision="fp64", stream=None) -> torch.Tensor:
        """T = L X (or L_n X): float32 in and out for 'mixed', float64 for 'fp64'."""
        dt = torch.float32 if _prec(precision) == PREC_MIXED else torch.float64
        X = X.to(self.device, dt).contiguous()
        T = torch.empty_like(X)
        _lib.check(_lib.lib().sfairsc_spmm(self._h, _ptr(X), _ptr(T), X.shape[1], _prec(precision), _stream(stream)))
        return T

    # -- eigensolver -----------------------------------------------------
    def eigs(
        self,
        k: int,
        tol: float = 1e-8,
        precision="fp64",
        block_width: int = 0,
        max_basis: int = 0,
        max_restarts: int = 0,
        keep: int = 0,
        seed: int = 0,
        sigma: float = 0.0,
        certify: bool = True,
        time_kernels: bool = False,
        x0: Optional[torch.Tensor] = None,
        H_out: Optional[torch.Tensor] = None,
        raise_not_converged: bool = True,
        raise_degenerate: bool = False,
        stream=None,
    ) -> EigsResult:
        """The k smallest fair eigenpairs (Alg. 3 step 3).

        A converged solve whose theta_k and theta_{k+1} coincide to the
        tolerance returns with `code == E_DEGENERATE` and a warning (or raises
        with raise_degenerate=True): the k-dimensional subspace is then not
        determined."""
        opts = _lib.EigsOpts()
        _lib.lib().sfairsc_eigs_opts_init(ctypes.byref(opts))
        opts.block_width = block_width
        opts.max_basis = max_basis
        opts.max_restarts = max_restarts
        opts.keep = keep
        opts.seed = seed
        opts.sigma = sigma
        opts.certify = int(certify)
        opts.time_kernels = int(time_kernels)
        if x0 is not None:
            x0 = x0.to(self.device, torch.float64).contiguous()
            opts.x0 = x0.data_ptr()
            opts.b0 = x0.shape[1]
        ev = (ctypes.c_double * k)()
        if H_out is None:
            buf = torch.empty((k, self.n), dtype=torch.float64, device=self.device)
        else:
            buf = H_out
        info = _lib.EigsInfo()
        code = _lib.lib().sfairsc_eigs(
            self._h, k, float(tol), _prec(precision), ctypes.byref(opts), ev, _ptr(buf), ctypes.byref(info),
            _stream(stream)
        )
        allow = _allowed(raise_not_converged, raise_degenerate)
        _lib.check(code, allow=allow)
        if code == E_DEGENERATE:
            warnings.warn(_lib.lib().sfairsc_last_error().decode(errors="replace"), RuntimeWarning, stacklevel=2)
        return EigsResult(np.array(ev[:]), buf.t(), info.as_dict(), code)

    # -- clustering ------------------------------------------------------
    def labels(self, H: torch.Tensor, n_clusters: int, n_restarts: int = 10, seed: int = 0, max_iter: int = 300,
               stream=None):
        """k-means on the rows of H (n x kdim) -> (labels int32 tensor, inertia)."""
        Hc = H.to(self.device, torch.float64).t().contiguous()  # column-major storage
        lab = torch.empty(self.n, dtype=torch.int32, device=self.device)
        inertia = ctypes.c_double()
        _lib.check(
            _lib.lib().sfairsc_labels(
                self._h, _ptr(Hc), Hc.shape[0], n_clusters, n_restarts, seed, max_iter, _ptr(lab),
                ctypes.byref(inertia), _stream(stream)
            )
        )
        return lab, inertia.value

    # -- differentiation -------------------------------------------------
    def eigsum_backward(self, H: torch.Tensor, eigenvalues=None, stream=None) -> torch.Tensor:
        """Gradient of the sum of the k smallest fair eigenvalues w.r.t. the
        stored weights, per stored entry (i, j):
        0.5 * ||H_i - H_j||^2 (unnormalized), or
        0.5 * sum_l [(H_il - H_jl)^2 - lambda_l (H_il^2 + H_jl^2)]
        (normalized; `eigenvalues` = the lambda_l matching H's columns)."""
        Hc = H.to(self.device, torch.float64).t().contiguous()
        k = Hc.shape[0]
        lam = None
        if eigenvalues is not None:
            lam_np = np.ascontiguousarray(np.asarray(eigenvalues, dtype=np.float64).reshape(-1))
            if lam_np.size != k:
                raise ValueError(f"{lam_np.size} eigenvalues for {k} columns")
            lam = lam_np.ctypes.data_as(ctypes.c_void_p)
        grad = torch.empty(self.nnz, dtype=self.value_dtype, device=self.device)
        _lib.check(_lib.lib().sfairsc_eigsum_backward(self._h, _ptr(Hc), k, lam, _ptr(grad), _stream(stream)))
        return grad


# -- batched solves ---------------------------------------------------------
def symeig(T: torch.Tensor, m: Optional[int] = None, stream=None):
    """Eigenvalues (ascending) and the eigenvectors of the m smallest of a
    small symmetric matrix (order <= 192) with the Rayleigh-Ritz kernel of the
    eigensolver (diagnostic) -> (w, Z), Z of shape (c, m)."""
    if T.dim() != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    c = T.shape[0]
    m = c if m is None else int(m)
    Td = T.to(torch.float64).contiguous()
    if not Td.is_cuda:
        raise ValueError("T must be a device tensor")
    w = torch.empty(c, dtype=torch.float64, device=Td.device)
    Z = torch.empty((c, max(m, 1)), dtype=torch.float64, device=Td.device)
    _lib.check(_lib.lib().sfairsc_symeig(_ptr(Td), c, c, m, _ptr(w), _ptr(Z), _stream(stream)))
    return w, Z[:, :m]


def _allowed(raise_not_converged: bool, raise_degenerate: bool):
    allow = ()
    if not raise_not_converged:
        allow += (E_NOT_CONVERGED,)
    if not raise_degenerate:
        allow += (E_DEGENERATE,)
    return allow


def _handles(graphs):
    arr = (ctypes.c_void_p * len(graphs))()
    for i, g in enumerate(graphs):
        arr[i] = g._h
    return arr


def eigs_batched(
    graphs,
    k,
    tol: float = 1e-6,
    precision="mixed",
    block_width: int = 0,
    max_basis: int = 0,
    max_restarts: int = 0,
    seed: int = 0,
    sigma: float = 0.0,
    certify: bool = True,
    H_out=None,
    raise_not_converged: bool = True,
    raise_degenerate: bool = False,
    stream=None,
):
    """The k[i] smallest fair eigenpairs of every graph in one persistent
    launch -> list of EigsResult (info: the per-graph batch record; a graph
    with theta_k ~ theta_{k+1} has status E_DEGENERATE)."""
    graphs = list(graphs)
    cnt = len(graphs)
    if isinstance(k, int):
        k = [k] * cnt
    k = [int(x) for x in k]
    if len(k) != cnt:
        raise ValueError("k must have one entry per graph")
    opts = _lib.EigsOpts()
    _lib.lib().sfairsc_eigs_opts_init(ctypes.byref(opts))
    opts.block_width = block_width
    opts.max_basis = max_basis
    opts.max_restarts = max_restarts
    opts.seed = seed
    opts.sigma = sigma
    opts.certify = int(certify)
    karr = (ctypes.c_int32 * cnt)(*k)
    evs = [(ctypes.c_double * kk)() for kk in k]
    evp = (ctypes.c_void_p * cnt)(*[ctypes.cast(e, ctypes.c_void_p) for e in evs])
    if H_out is None:
        H_out = [torch.empty((kk, g.n), dtype=torch.float64, device=g.device) for g, kk in zip(graphs, k)]
    Hp = (ctypes.c_void_p * cnt)(*[h.data_ptr() for h in H_out])
    infos = (_lib.BatchInfo * cnt)()
    code = _lib.lib().sfairsc_eigs_batched(
        _handles(graphs), cnt, karr, float(tol), _prec(precision), ctypes.byref(opts), evp, Hp, infos,
        _stream(stream)
    )
    allow = _allowed(raise_not_converged, raise_degenerate)
    _lib.check(code, allow=allow)
    if code == E_DEGENERATE:
        warnings.warn(_lib.lib().sfairsc_last_error().decode(errors="replace"), RuntimeWarning, stacklevel=2)
    return [
        EigsResult(np.array(evs[i][:]), H_out[i].t(), infos[i].as_dict(), infos[i].status) for i in range(cnt)
    ]


def autotune(graphs, k, tol: float = 1e-6, precision="mixed", per_bucket: int = 2, stream=None) -> int:
    """Time candidate batched configurations per graph bucket and fill the
    tuning table; returns the number of table entries."""
    graphs = list(graphs)
    cnt = len(graphs)
    if isinstance(k, int):
        k = [k] * cnt
    karr = (ctypes.c_int32 * cnt)(*[int(x) for x in k])
    _lib.check(
        _lib.lib().sfairsc_autotune(
            _handles(graphs), cnt, karr, float(tol), _prec(precision), int(per_bucket), _stream(stream)
        )
    )
    return tuning_size()


def tuning_save(path: str) -> None:
    _lib.check(_lib.lib().sfairsc_tuning_save(str(path).encode()))


def tuning_load(path: str) -> None:
    _lib.check(_lib.lib().sfairsc_tuning_load(str(path).encode()))


def tuning_clear() -> None:
    _lib.check(_lib.lib().sfairsc_tuning_clear())


def tuning_size() -> int:
    return int(_lib.lib().sfairsc_tuning_size())


def tuning_lookup(n: int, nnz: int, k: int, precision="mixed", normalized: bool = False, tol: float = 1e-6):
    """(block_width, max_basis, spmm_rows, from_table) a batched solve would use."""
    b, m, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    code = _lib.lib().sfairsc_tuning_lookup(
        int(n), int(nnz), int(k), _prec(precision), int(normalized), float(tol), ctypes.byref(b), ctypes.byref(m),
        ctypes.byref(r)
    )
    if code < 0:
        _lib.check(code)
    return b.value, m.value, r.value, bool(code)


class FairEigSum(torch.autograd.Function):
    """f(w) = sum of the k smallest fair eigenvalues, as a function of the
    stored edge weights w (CSR order).

    forward(values, rowptr, col, groups, h, k, tol, normalized=False) ->
    scalar tensor.  backward: grad_values = grad_out * the per-entry gradient
    of Graph.eigsum_backward (hand-written HIP kernel).  Both stored copies of
    an edge must receive the same perturbation for the result to be a
    directional derivative.
    """

    @staticmethod
    def forward(ctx, values, rowptr, col, groups, h, k, tol=1e-10, normalized=False):
        g = Graph(rowptr, col, values.detach(), groups, h, normalized=bool(normalized), device=values.device)
        res = g.eigs(k, tol=tol, precision="fp64")
        ctx.graph = g
        ctx.eigenvalues = np.asarray(res.eigenvalues, dtype=np.float64).copy()
        ctx.save_for_backward(res.H)
        return torch.tensor(float(res.eigenvalues.sum()), dtype=values.dtype, device=values.device)

    @staticmethod
    def backward(ctx, grad_out):
        (H,) = ctx.saved_tensors
        lam = ctx.eigenvalues if ctx.graph.normalized else None
        grad = ctx.graph.eigsum_backward(H, lam)
        return grad_out * grad, None, None, None, None, None, None, None
