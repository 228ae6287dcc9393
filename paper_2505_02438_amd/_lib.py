"""ctypes loader for libsoptx.so (the HIP library).  Argument marshalling only.

The library must have been built in-tree (``__graft_entry__.build()`` or
``python -m paper_2505_02438_amd.build``); there is no fallback: a missing
library raises immediately.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoptx.so")

SOPTX_OK = 0
STATUS = {
    0: "SOPTX_OK", -1: "SOPTX_E_INVALID_ARG", -2: "SOPTX_E_UNSUPPORTED_ELEM", -3: "SOPTX_E_BAD_MESH",
    -4: "SOPTX_E_JACOBIAN", -5: "SOPTX_E_NONAFFINE", -6: "SOPTX_E_OVERFLOW", -7: "SOPTX_E_OOM",
    -8: "SOPTX_E_DEVICE", -9: "SOPTX_E_SCRATCH",
}

FP64, FP32, BF16_FP32ACC = 0, 1, 2
FILTER_CSR_ONLY = 1
REF_SYMBOLIC, REF_QUADRATURE = 0, 1


class SoptxError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}")


class Mesh(ctypes.Structure):
    _fields_ = [("elem", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("n_cells", ctypes.c_int64), ("cells", ctypes.c_void_p)]


class Material(ctypes.Structure):
    _fields_ = [("E0", ctypes.c_double), ("Emin", ctypes.c_double), ("nu", ctypes.c_double),
                ("p", ctypes.c_double), ("plane_strain", ctypes.c_int32)]


class PatternStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("ndof", "nnz", "n_cells", "n_nodes", "n_groups", "n_signatures",
                                               "n_contributions", "plan_bytes", "device_bytes",
                                               "n_groups_diag", "n_groups_ranked")]


class OcParams(ctypes.Structure):
    _fields_ = [("move", ctypes.c_double), ("eta", ctypes.c_double), ("lmax", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_steps", ctypes.c_int32)]


class OcResult(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("volume", ctypes.c_double), ("change", ctypes.c_double),
                ("steps", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsoptx.so not built at {LIB_PATH}: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "soptx_build_pattern": [ctypes.POINTER(Mesh), ctypes.POINTER(_P), _P],
        "soptx_build_pattern_ex": [ctypes.POINTER(Mesh), _I32, ctypes.POINTER(_P), _P],
        "soptx_build_pattern_general": [ctypes.POINTER(Mesh), ctypes.POINTER(_P), _P],
        "soptx_assemble_general": [_P, ctypes.POINTER(Material), _P, _P, _P, _P],
        "soptx_evaluate_general": [_P, ctypes.POINTER(Material), _P, _P, _P, _P, _P, _P],
        "soptx_debug_host_plan_ex": [ctypes.POINTER(Mesh), _I32, ctypes.POINTER(_P)],
        "soptx_pattern_info": [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_P), ctypes.POINTER(_P)],
        "soptx_pattern_stats_get": [_P, ctypes.POINTER(PatternStats)],
        "soptx_assemble": [_P, ctypes.POINTER(Material), _P, _P, _P, _I32, _P],
        "soptx_apply_dirichlet": [_P, _P, _P, _P],
        "soptx_sensitivity": [_P, ctypes.POINTER(Material), _P, _P, _P, _I32, _P],
        "soptx_compliance": [_P, ctypes.POINTER(Material), _P, _P, _P, _P, _I32, _P],
        "soptx_evaluate": [_P, ctypes.POINTER(Material), _P, _P, _P, _P, _P, _I32, _P],
        "soptx_evaluate_noalloc": [_P, ctypes.POINTER(Material), _P, _P, _P, _P, _P, _I32, _P],
        "soptx_build_dirichlet": [_P, _P, ctypes.POINTER(_P), _P],
        "soptx_dirichlet_info": [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
        "soptx_step": [_P, _P, ctypes.POINTER(Material), _P, _P, _P, _P, _P, _P, _I32, _P],
        "soptx_assemble_backward": [_P, ctypes.POINTER(Material), _P, _P, _P, _P, _I32, _P],
        "soptx_spmv": [_P, _P, _P, _P, _P],
        "soptx_pcg": [_P, _P, _P, _P, ctypes.c_double, _I32, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double),
                      _P],
        "soptx_pattern_copy": [_P, _P, _P],
        "soptx_reference_tensor": [_I32, _I32, _P],
        "soptx_validate_mesh": [ctypes.POINTER(Mesh)],
        "soptx_debug_host_plan": [ctypes.POINTER(Mesh), ctypes.POINTER(_P)],
        "soptx_debug_host_plan_array": [_P, ctypes.c_char_p, ctypes.POINTER(_P), ctypes.POINTER(_I64),
                                        ctypes.POINTER(_I32)],
        "soptx_debug_host_plan_scalars": [_P, _P],
        "soptx_debug_fail_workers": [_I32],
        "soptx_debug_set_assembly_variant": [_I32],
        "soptx_debug_set_general_variant": [_I32],
        "soptx_debug_general_path": [_P, ctypes.POINTER(_I32)],
        "soptx_debug_filter_matrix": [ctypes.POINTER(Mesh), ctypes.c_double, ctypes.POINTER(_I64),
                                      ctypes.POINTER(_I64), _P, _P, _P, _P, _P, _P],
        "soptx_oc_update": [_I64, _P, _P, _P, ctypes.c_double, ctypes.POINTER(OcParams), _P,
                            ctypes.POINTER(OcResult), _P],
        "soptx_build_filter": [ctypes.POINTER(Mesh), ctypes.c_double, ctypes.POINTER(_P), _P],
        "soptx_build_filter_ex": [ctypes.POINTER(Mesh), ctypes.c_double, _I32, ctypes.POINTER(_P), _P],
        "soptx_filter_stencil_size": [_P, ctypes.POINTER(_I32)],
        "soptx_debug_filter_stencil": [ctypes.POINTER(Mesh), ctypes.c_double, ctypes.POINTER(_I32), _P],
        "soptx_filter_info": [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)],
        "soptx_filter_copy": [_P, _P, _P, _P, _P],
        "soptx_filter_sensitivity": [_P, _P, _P, _P, _P],
        "soptx_filter_density": [_P, _P, ctypes.c_double, _P, _P, _P],
        "soptx_filter_density_backward": [_P, _P, ctypes.c_double, _P, _P, _P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _I
    L.soptx_destroy_pattern.argtypes = [_P]
    L.soptx_destroy_pattern.restype = None
    L.soptx_destroy_dirichlet.argtypes = [_P]
    L.soptx_destroy_dirichlet.restype = None
    L.soptx_destroy_filter.argtypes = [_P]
    L.soptx_destroy_filter.restype = None
    L.soptx_debug_host_plan_free.argtypes = [_P]
    L.soptx_debug_host_plan_free.restype = None
    L.soptx_status_string.argtypes = [_I]
    L.soptx_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc: int, what: str):
    if rc != SOPTX_OK:
        raise SoptxError(rc, what)
