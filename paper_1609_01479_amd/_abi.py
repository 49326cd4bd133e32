"""ctypes binding of the C ABI in include/lb.h (argument marshalling only).

The shared library is the in-tree ``liblbmi.so`` built for gfx950 by
``paper_1609_01479_amd/build.py``.  There is no fallback: if it is missing or
does not load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmi.so")

NVEL = 19
LB_OK, LB_EINVAL, LB_ESHAPE, LB_EALIGN, LB_EHIP, LB_ESTATE = range(6)
LB_FP64, LB_FP32_DEV = 0, 1
LB_KERNEL_FUSED, LB_KERNEL_TWO_PASS, LB_KERNEL_STREAM = 0, 1, 2
ABI_VERSION = 5
NOALLOC_MAX_PARTIALS = 4096  # LB_NOALLOC_MAX_PARTIALS

# Every symbol include/lb.h declares.
EXPORTS = ("lb_abi_version", "lb_query_sizes", "lb_create", "lb_destroy", "lb_set_stream",
           "lb_init_phi", "lb_step", "lb_step_sums", "lb_step_sums_noalloc", "lb_step_from", "lb_step_from_phi", "lb_moments", "lb_sums", "lb_get_state", "lb_set_state",
           "lb_export_dist", "lb_import_dist", "lb_adjoint_seed", "lb_adjoint_step",
           "lb_adjoint_step_phi", "lb_adjoint_phi0", "lb_adjoint_export", "lb_pack_faces",
           "lb_unpack_faces", "lb_copy_probe",
           "lb_status_string", "lb_last_error")


class LbParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("A", ctypes.c_double), ("B", ctypes.c_double), ("kappa", ctypes.c_double),
                ("gamma", ctypes.c_double), ("tau_f", ctypes.c_double),
                ("tau_g", ctypes.c_double), ("rho0", ctypes.c_double),
                ("precision", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("segment_x", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("aosoa_len", ctypes.c_int32), ("coupling", ctypes.c_int32),
                ("order_param", ctypes.c_int32), ("halo_x", ctypes.c_int32)]


class LbSizes(ctypes.Structure):
    _fields_ = [("elem_bytes", ctypes.c_size_t), ("stride_elems", ctypes.c_size_t),
                ("state_bytes", ctypes.c_size_t), ("phi_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t), ("adj_bytes", ctypes.c_size_t),
                ("adj_scratch_bytes", ctypes.c_size_t), ("face_bytes", ctypes.c_size_t)]


class LbBuffers(ctypes.Structure):
    _fields_ = [("state", ctypes.c_void_p * 2), ("phi", ctypes.c_void_p),
                ("scratch", ctypes.c_void_p), ("adj", ctypes.c_void_p * 2),
                ("adj_scratch", ctypes.c_void_p)]


class LbError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where} failed with status {status}: {detail}")


_lib = None


def lib():
    """Load liblbmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                           "`python -c 'import __graft_entry__ as g; g.build()'` first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p
    P = ctypes.POINTER
    sigs = {
        "lb_abi_version": ([], i32),
        "lb_query_sizes": ([P(LbParams), P(LbSizes)], ctypes.c_int),
        "lb_create": ([P(LbParams), P(LbBuffers), vp, P(vp)], ctypes.c_int),
        "lb_destroy": ([vp], None),
        "lb_set_stream": ([vp, vp], ctypes.c_int),
        "lb_init_phi": ([vp, dp], ctypes.c_int),
        "lb_step": ([vp, i32], ctypes.c_int),
        "lb_step_from": ([vp, vp, vp], ctypes.c_int),
        "lb_step_from_phi": ([vp, vp, vp, dp], ctypes.c_int),
        "lb_step_sums": ([vp, i32, dp], ctypes.c_int),
        "lb_step_sums_noalloc": ([vp, i32, dp], ctypes.c_int),
        "lb_moments": ([vp, dp, dp, dp], ctypes.c_int),
        "lb_sums": ([vp, dp], ctypes.c_int),
        "lb_get_state": ([vp, vp], ctypes.c_int),
        "lb_set_state": ([vp, vp], ctypes.c_int),
        "lb_export_dist": ([vp, dp, dp], ctypes.c_int),
        "lb_import_dist": ([vp, dp, dp], ctypes.c_int),
        "lb_adjoint_seed": ([vp, dp], ctypes.c_int),
        "lb_adjoint_step": ([vp, vp, dp], ctypes.c_int),
        "lb_adjoint_step_phi": ([vp, vp, dp, dp], ctypes.c_int),
        "lb_adjoint_phi0": ([vp, dp], ctypes.c_int),
        "lb_adjoint_export": ([vp, dp, dp], ctypes.c_int),
        "lb_pack_faces": ([vp, vp, vp], ctypes.c_int),
        "lb_unpack_faces": ([vp, vp, vp], ctypes.c_int),
        "lb_copy_probe": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "lb_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "lb_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if L.lb_abi_version() != ABI_VERSION:
        raise RuntimeError("liblbmi.so ABI version mismatch")
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != LB_OK:
        L = lib()
        detail = L.lb_last_error().decode() or L.lb_status_string(status).decode()
        raise LbError(status, where, detail)
