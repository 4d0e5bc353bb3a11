"""ctypes declarations of the C ABI in include/eik.h (libeik.so, built in-tree).

There is no fallback: if the library is missing or fails to load, every entry
point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeik.so")

EIK_OK = 0
EIK_EINVAL = -1
EIK_EDOMAIN = -2
EIK_ENOMEM = -3
EIK_EHIP = -4
EIK_ELIMIT = -5
EIK_ENOTSUP = -6
EIK_EBADSRC = -7
EIK_EHANG = -8

EIK_SPEED = 0
EIK_SLOWNESS = 1
EIK_FLAG_TIME_KERNELS = 1
EIK_FLAG_TIMELINE = 4
EIK_OP_DBAR = 0
EIK_OP_DHAT = 1
EIK_OP_DTILDE = 2
EIK_OP_NEWTON = 3
EIK_FLAG_TRACK_CHANGE = 8
EIK_FLAG_WARM_START = 16
EIK_FLAG_PACKED = 32

EXPORTED = (
    "eik_solve", "eik_parents", "eik_adjoint", "eik_solve_batched", "eik_adjoint_batched",
    "eik_reserve", "eik_num_tiles", "eik_status", "eik_strerror", "eik_last_error",
    "eik_release", "eik_version", "eik_timeline", "eik_residual", "eik_solve_noalloc", "eik_solve_rect",
)


class eik_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("h", ctypes.c_double), ("field_kind", ctypes.c_int32)]


class eik_opts(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("tile", ctypes.c_int32 * 3),
                ("grid_blocks", ctypes.c_int32), ("max_tile_visits", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("lookahead", ctypes.c_int32), ("horizon", ctypes.c_int32),
                ("op", ctypes.c_int32), ("work_ref", ctypes.c_void_p)]


class eik_stats(ctypes.Structure):
    _fields_ = [("tile_visits", ctypes.c_int64), ("point_updates", ctypes.c_int64),
                ("ntiles", ctypes.c_int64), ("relax_passes", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_int64),
                ("phase_us", ctypes.c_double * 4),
                ("workgroups", ctypes.c_int64), ("bucket_advances", ctypes.c_int64),
                ("handoffs", ctypes.c_int64), ("evaluations", ctypes.c_int64), ("improving", ctypes.c_int64),
                ("final_updates", ctypes.c_int64)]


class EikError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"eik error {code}: {msg}")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_gp = ctypes.POINTER(eik_grid)
_op = ctypes.POINTER(eik_opts)


def load() -> ctypes.CDLL:
    """Load libeik.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2103_05694_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.eik_solve.restype = _i32
    L.eik_solve.argtypes = [_gp, _vp, _i64, _vp, _vp, _vp, _vp, _op, _vp]
    L.eik_solve_rect.restype = _i32
    L.eik_solve_rect.argtypes = [_gp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _op, _vp]
    L.eik_solve_noalloc.restype = _i32
    L.eik_solve_noalloc.argtypes = [_gp, _vp, _i64, _vp, _vp, _vp, _vp, _op, _vp]
    L.eik_parents.restype = _i32
    L.eik_parents.argtypes = [_gp, _vp, _i64, _vp, _vp, _vp]
    L.eik_adjoint.restype = _i32
    L.eik_adjoint.argtypes = [_gp, _vp, _vp, _vp, _vp, _vp, _vp, _op, _vp]
    L.eik_solve_batched.restype = _i32
    L.eik_solve_batched.argtypes = [_i32, _gp, ctypes.POINTER(_i64), _vp, ctypes.POINTER(_i64), _vp, _vp,
                                    _vp, _vp, _op, _vp]
    L.eik_adjoint_batched.restype = _i32
    L.eik_adjoint_batched.argtypes = [_i32, _gp, ctypes.POINTER(_i64), _vp, _vp, _vp, _vp, _vp, _vp,
                                      _op, _vp]
    L.eik_reserve.restype = _i32
    L.eik_reserve.argtypes = [_i64, _i64, _vp]
    L.eik_num_tiles.restype = _i64
    L.eik_num_tiles.argtypes = [_gp, _op]
    L.eik_status.restype = _i32
    L.eik_status.argtypes = [_vp, ctypes.POINTER(eik_stats)]
    L.eik_residual.restype = _i32
    L.eik_residual.argtypes = [_gp, _vp, _i64, _vp, _vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                               _vp]
    L.eik_timeline.restype = _i32
    L.eik_timeline.argtypes = [_vp, _i32, _vp, _vp, _vp]
    L.eik_strerror.restype = ctypes.c_char_p
    L.eik_strerror.argtypes = [_i32]
    L.eik_last_error.restype = ctypes.c_char_p
    L.eik_last_error.argtypes = []
    L.eik_release.restype = None
    L.eik_release.argtypes = []
    L.eik_version.restype = ctypes.c_char_p
    L.eik_version.argtypes = []
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != EIK_OK:
        L = load()
        msg = L.eik_last_error().decode() or L.eik_strerror(rc).decode()
        raise EikError(rc, msg)
