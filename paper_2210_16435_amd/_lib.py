"""ctypes declarations for libsfairsc.so (see include/sfairsc.h).

Only marshalling lives here: every computation runs in the HIP library.
Importing fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfairsc.so")

OK = 0
E_ARG = -1
E_ASYM = -2
E_EMPTY_GROUP = -3
E_ISOLATED = -4
E_NOT_CONVERGED = -5
E_DEGENERATE = -6
E_HIP = -7
E_NOMEM = -8

F32 = 0
F64 = 1
PREC_FP64 = 0
PREC_MIXED = 1

STATUS_NAMES = {
    E_ARG: "E_ARG",
    E_ASYM: "E_ASYM",
    E_EMPTY_GROUP: "E_EMPTY_GROUP",
    E_ISOLATED: "E_ISOLATED",
    E_NOT_CONVERGED: "E_NOT_CONVERGED",
    E_DEGENERATE: "E_DEGENERATE",
    E_HIP: "E_HIP",
    E_NOMEM: "E_NOMEM",
}


class SfairscError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class GraphStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("h", ctypes.c_int32),
        ("normalized", ctypes.c_int32),
        ("value_dtype", ctypes.c_int32),
        ("constraint_rank", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("min_degree", ctypes.c_double),
        ("max_degree", ctypes.c_double),
    ]


class EigsOpts(ctypes.Structure):
    _fields_ = [
        ("block_width", ctypes.c_int32),
        ("max_basis", ctypes.c_int32),
        ("max_restarts", ctypes.c_int32),
        ("keep", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("sigma", ctypes.c_double),
        ("certify", ctypes.c_int32),
        ("time_kernels", ctypes.c_int32),
        ("x0", ctypes.c_void_p),
        ("b0", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class EigsInfo(ctypes.Structure):
    _fields_ = [
        ("restarts", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("block_steps", ctypes.c_int32),
        ("breakdowns", ctypes.c_int32),
        ("operator_applies", ctypes.c_int64),
        ("spmm_launches", ctypes.c_int64 * 2),
        ("spmm_ms", ctypes.c_double * 2),
        ("max_rel_residual", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("gap_ratio", ctypes.c_double),
        ("phase1_ms", ctypes.c_double),
        ("rr_ms", ctypes.c_double),
        ("operator_ms", ctypes.c_double),
        ("ortho_ms", ctypes.c_double),
        ("restart_ms", ctypes.c_double),
        ("degenerate", ctypes.c_int32),
        ("restarts_unpredicted", ctypes.c_int32),
    ]

    def as_dict(self):
        return {
            "restarts": self.restarts,
            "converged": self.converged,
            "block_steps": self.block_steps,
            "breakdowns": self.breakdowns,
            "operator_applies": self.operator_applies,
            "spmm_launches": [self.spmm_launches[0], self.spmm_launches[1]],
            "spmm_ms": [self.spmm_ms[0], self.spmm_ms[1]],
            "max_rel_residual": self.max_rel_residual,
            "sigma": self.sigma,
            "gap_ratio": self.gap_ratio,
            "phase1_ms": self.phase1_ms,
            "rr_ms": self.rr_ms,
            "operator_ms": self.operator_ms,
            "ortho_ms": self.ortho_ms,
            "restart_ms": self.restart_ms,
            "degenerate": self.degenerate,
            "restarts_unpredicted": self.restarts_unpredicted,
        }


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("batch_status", ctypes.c_int32),
        ("block_width", ctypes.c_int32),
        ("max_basis", ctypes.c_int32),
        ("spmm_rows", ctypes.c_int32),
        ("from_table", ctypes.c_int32),
        ("double_spmm", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("block_steps", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("max_rel_residual", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("gap_ratio", ctypes.c_double),
        ("graph_ms", ctypes.c_double),
        ("batch_ms", ctypes.c_double),
        ("phase_ms", ctypes.c_double * 8),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name not in ("reserved", "phase_ms")}
        d["phase_ms"] = [self.phase_ms[i] for i in range(8)]
        return d


# name -> (restype, argtypes); must match include/sfairsc.h
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
PROTOTYPES = {
    "sfairsc_graph_create": (_int, [ctypes.POINTER(_vp), _i64, _i64, _vp, _vp, _vp, _int, _vp, _i32, _int, _vp]),
    "sfairsc_graph_destroy": (None, [_vp]),
    "sfairsc_graph_query": (_int, [_vp, ctypes.POINTER(GraphStats)]),
    "sfairsc_graph_set_constraint": (_int, [_vp, _vp, _i64, _i32, _i32, _dbl, ctypes.POINTER(_i32), _vp]),
    "sfairsc_graph_set_memberships": (_int, [_vp, _i32, _vp, _vp, _i32, _dbl, _i32, _vp]),
    "sfairsc_lsqr_stats": (_int, [_vp, ctypes.POINTER(_i64), _vp]),
    "sfairsc_apply_operator": (_int, [_vp, _vp, _vp, _i32, _int, _dbl, _vp]),
    "sfairsc_apply_operator_noalloc": (_int, [_vp, _vp, _vp, _i32, _int, _dbl, _vp]),
    "sfairsc_spmm": (_int, [_vp, _vp, _vp, _i32, _int, _vp]),
    "sfairsc_eigs_opts_init": (None, [ctypes.POINTER(EigsOpts)]),
    "sfairsc_eigs": (
        _int,
        [_vp, _i32, _dbl, _int, ctypes.POINTER(EigsOpts), ctypes.POINTER(_dbl), _vp, ctypes.POINTER(EigsInfo), _vp],
    ),
    "sfairsc_eigs_batched": (
        _int,
        [_vp, _i32, _vp, _dbl, _int, ctypes.POINTER(EigsOpts), _vp, _vp, ctypes.POINTER(BatchInfo), _vp],
    ),
    "sfairsc_autotune": (_int, [_vp, _i32, _vp, _dbl, _int, _i32, _vp]),
    "sfairsc_tuning_save": (_int, [ctypes.c_char_p]),
    "sfairsc_tuning_load": (_int, [ctypes.c_char_p]),
    "sfairsc_tuning_clear": (_int, []),
    "sfairsc_tuning_size": (_int, []),
    "sfairsc_tuning_lookup": (
        _int,
        [_i64, _i64, _i32, _int, _int, _dbl, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    ),
    "sfairsc_labels": (_int, [_vp, _vp, _i32, _i32, _i32, ctypes.c_uint64, _i32, _vp, ctypes.POINTER(_dbl), _vp]),
    "sfairsc_eigsum_backward": (_int, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "sfairsc_symeig": (_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
    "sfairsc_last_error": (ctypes.c_char_p, []),
    "sfairsc_version": (ctypes.c_char_p, []),
}


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: the HIP library has not been built "
            "(run `python -c 'import __graft_entry__ as g; g.build()'` or "
            "`python paper_2210_16435_amd/build.py`)"
        )
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def check(code: int, allow=()):
    if code == OK or code in allow:
        return code
    msg = lib().sfairsc_last_error().decode(errors="replace")
    raise SfairscError(code, msg)
