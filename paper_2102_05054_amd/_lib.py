"""ctypes binding of libfloquet.so (include/floquet.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_longlong, c_ulonglong, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfloquet.so")

FQ_OK, FQ_NOT_CONVERGED, FQ_EINVAL, FQ_ENOMEM, FQ_EDEVICE, FQ_ENUMERIC = 0, 1, -1, -2, -3, -4
FQ_C64, FQ_C128 = 0, 1
FQ_POLICY_AUTO, FQ_POLICY_TILE, FQ_POLICY_PIPE = 0, 1, 2
FQ_KICKED_ISING, FQ_BRICKWORK, FQ_CIRCUIT = 0, 1, 2

STATUS_NAMES = {
    FQ_OK: "FQ_OK", FQ_NOT_CONVERGED: "FQ_NOT_CONVERGED", FQ_EINVAL: "FQ_EINVAL",
    FQ_ENOMEM: "FQ_ENOMEM", FQ_EDEVICE: "FQ_EDEVICE", FQ_ENUMERIC: "FQ_ENUMERIC",
}


class FqModelDesc(ctypes.Structure):
    _fields_ = [
        ("model", c_int), ("L", c_int), ("periodic", c_int),
        ("J", POINTER(c_double)), ("h", POINTER(c_double)), ("g", c_double),
        ("gates", POINTER(c_double)), ("n_gates", c_int),
        ("gate_sites", POINTER(c_int)), ("gate_widths", POINTER(c_int)),
    ]


class FqArnoldiOpts(ctypes.Structure):
    _fields_ = [
        ("k", c_int), ("ncv", c_int), ("tol", c_double), ("max_restarts", c_int),
        ("filter_dtype", c_int), ("refine", c_int), ("seed", c_ulonglong), ("v0_dev", c_void_p),
        ("refine_k", c_int), ("poly_coeffs", POINTER(c_double)), ("block", c_int),
    ]


class FqArnoldiStats(ctypes.Structure):
    _fields_ = [
        ("nconv", c_int), ("n_restarts", c_int), ("n_filter_apps", c_longlong),
        ("n_U_apps", c_longlong), ("n_U_apps_c64", c_longlong),
        ("t_filter", c_double), ("t_orth", c_double), ("t_restart", c_double),
        ("t_refine", c_double), ("t_total", c_double), ("max_residual", c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# (name, restype, argtypes) of every exported entry point of include/floquet.h
SIGNATURES = [
    ("create_floquet_op", c_int, [POINTER(FqModelDesc), POINTER(c_void_p)]),
    ("destroy_floquet_op", c_int, [c_void_p]),
    ("floquet_op_dim", c_longlong, [c_void_p]),
    ("apply_U", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    ("apply_filter", c_int, [c_void_p, c_int, c_double, c_int, c_void_p, c_void_p, c_void_p]),
    ("apply_filter_many", c_int, [c_void_p, c_int, c_double, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    ("apply_filter_many_noalloc", c_int, [c_void_p, c_int, c_double, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    ("apply_polynomial", c_int, [c_void_p, c_int, POINTER(c_double), c_int, c_void_p, c_void_p, c_void_p]),
    ("arnoldi_eigs", c_int, [c_void_p, c_int, c_double, POINTER(FqArnoldiOpts), POINTER(c_double), c_void_p,
                             POINTER(c_double), POINTER(FqArnoldiStats), c_void_p]),
    ("arnoldi_eigs_batched", c_int, [POINTER(c_void_p), c_int, POINTER(c_double), c_int, c_int,
                                     POINTER(FqArnoldiOpts), POINTER(c_int), POINTER(c_double),
                                     POINTER(c_void_p), POINTER(c_double), POINTER(FqArnoldiStats), c_void_p]),
    ("floquet_last_error", ctypes.c_char_p, []),
    ("fq_set_kernel_policy", c_int, [c_int]),
    ("fq_set_graph_capture", c_int, [c_int]),
    ("fq_host_schur", c_int, [c_int, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    ("fq_paper_parameters", c_int, [c_int, c_int, POINTER(c_int), POINTER(c_int)]),
    ("fq_host_eigvalsh", c_int, [c_int, POINTER(c_double), POINTER(c_double)]),
    ("fq_host_bw_schedule", c_int, [c_int, c_int, c_int, POINTER(c_int), POINTER(c_int), c_int, POINTER(c_int),
                                    POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
    ("entanglement_entropy", c_int, [c_void_p, c_int, c_void_p, c_int, POINTER(c_double), c_void_p]),
]

_lib = None


class FloquetError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname (libamdhip64.so.7);
        # importing torch first makes the dynamic linker bind this library to
        # that one copy, so torch tensors and streams and our kernels share a
        # single runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2102_05054_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str, allow=(FQ_OK,)) -> int:
    if status not in allow:
        raise FloquetError(status, where, lib().floquet_last_error().decode(errors="replace"))
    return status
