"""ctypes declarations of liblsl's C ABI (include/lsl.h)."""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_float, c_int32, c_int64,
                    c_uint8, c_uint32, c_void_p)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblsl.so")

LSL_OK = 0
LSL_EINVAL = -1
LSL_ENOMEM = -2
LSL_ECAPACITY = -3
LSL_EDEVICE = -4
LSL_EINTERNAL = -5
LSL_F32 = 0
LSL_F64 = 1


LSL_KERNEL_QUARTIC, LSL_KERNEL_GAUSS = 0, 1


class LslLattice(Structure):
    _fields_ = [("n_nodes", c_int64), ("n_edges", c_int64), ("dtype", c_int32),
                ("nodes", c_void_p), ("edges", c_void_p), ("weight", c_void_p),
                ("R", c_double), ("C", c_double), ("support", c_void_p),
                ("kernel", c_int32), ("sigma", c_double), ("keep_zero_weight", c_int32)]


class LslGrid(Structure):
    _fields_ = [("x0", c_double), ("y0", c_double), ("dx", c_double), ("dy", c_double),
                ("W", c_int32), ("H", c_int32), ("z0", c_double), ("dz", c_double),
                ("n_slices", c_int32)]


class LslBinParams(Structure):
    _fields_ = [("tile", c_int32), ("slab", c_int32), ("max_pairs", c_int64)]


class LslBinsInfo(Structure):
    _fields_ = [("n_edges", c_int64), ("n_nodes", c_int64), ("n_binned", c_int64),
                ("total_pairs", c_int64), ("max_group_pairs", c_int64),
                ("device_bytes", c_int64), ("peak_device_bytes", c_int64),
                ("dtype", c_int32), ("tile", c_int32), ("slab", c_int32),
                ("tiles_x", c_int32), ("tiles_y", c_int32), ("n_slabs", c_int32),
                ("n_groups", c_int32), ("current_group", c_int32),
                ("last_field_ms", c_double), ("last_group_bin_ms", c_double),
                ("last_queue_ms", c_double), ("last_contour_ms", c_double),
                ("plane_group", c_int32), ("last_backward_ms", c_double)]


class LslSupport(Structure):
    _fields_ = [("gamma", c_double), ("psi", c_double), ("risky_area", c_double),
                ("area", c_double), ("supported_length", c_double), ("length", c_double),
                ("n_supported", c_int64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "lattice_bin": (c_int32, [POINTER(LslLattice), POINTER(LslGrid), POINTER(LslBinParams),
                              POINTER(c_void_p), c_void_p]),
    "lattice_bins_free": (c_int32, [c_void_p]),
    "lsl_cache_trim": (c_int32, [POINTER(c_int64)]),
    "lsl_graph_cache_stats": (c_int32, [POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "lattice_bins_info": (c_int32, [c_void_p, POINTER(LslBinsInfo)]),
    "lattice_bins_group": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32),
                                     POINTER(c_int64)]),
    "lattice_bins_export": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "lattice_bins_order": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "slice_field": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "slice_field_stats": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int64), c_void_p]),
    "slice_contours": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_void_p,
                                 c_void_p, POINTER(c_int64), c_void_p]),
    "slice_polylines": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_void_p,
                                  c_void_p, c_void_p, POINTER(c_int64), c_void_p]),
    "slice_density": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_int32,
                                c_void_p, c_void_p]),
    "slice_density_loss": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_int32, c_int32,
                                     c_void_p, c_double, c_void_p, c_void_p, c_void_p,
                                     c_void_p]),
    "slice_occupancy_loss": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_double,
                                       c_void_p, c_void_p, c_void_p]),
    "slice_occupancy_loss_static": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_double,
                                              c_void_p, c_void_p, c_void_p]),
    "slice_field_backward": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                       c_void_p, c_int32, c_void_p]),
    "slice_batch": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                              c_int64, c_void_p, POINTER(c_int64), c_void_p]),
    "slice_autotune": (c_int32, [POINTER(LslLattice), POINTER(LslGrid),
                                 POINTER(LslBinParams), c_char_p, c_void_p]),
    "lattice_support": (c_int32, [POINTER(LslLattice), POINTER(c_double), POINTER(LslSupport),
                                  c_void_p, c_void_p]),
    "lsl_status_string": (c_char_p, [c_int32]),
    "lsl_last_error": (c_char_p, []),
    "lsl_version": (c_char_p, []),
    "lsl_probe_valu": (c_int32, [c_int32, c_int32, POINTER(c_float), POINTER(c_double),
                                 c_void_p]),
}

_lib = None


def lib():
    """The loaded native library.  Raises if it has not been built: there is
    no fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"native library {LIB_PATH} is missing; build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class LslError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.lsl_last_error().decode() or L.lsl_status_string(status).decode()
        super().__init__(f"{where}: {L.lsl_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != LSL_OK:
        raise LslError(status, where)
