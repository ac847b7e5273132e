"""ctypes loader of libftle.so (the HIP library built from csrc/).

Loading never falls back to anything else: if the library is missing and
cannot be built, or a symbol is absent, an ImportError/RuntimeError is raised.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftle.so")

STATUS_NAMES = {0: "FTLE_OK", 1: "FTLE_ERR_INVALID_ARG", 2: "FTLE_ERR_BAD_MESH", 3: "FTLE_ERR_DTYPE",
                4: "FTLE_ERR_UNSUPPORTED", 5: "FTLE_ERR_OOM", 6: "FTLE_ERR_DEVICE"}

F32, F64 = 0, 1
STENCIL_RING1, STENCIL_AXIS = 0, 1
NO_REORDER = 1 << 4
HOST_ONLY = 1 << 5
ELL_DIRECT, ELL_STAGED = 0, 1


def tile_flag(k: int) -> int:
    return (k & 0xFF) << 8


class FTLEError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_vp, _i64, _i32, _int, _dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_double
_P = ctypes.POINTER

# name -> (restype, argtypes); every name here is declared in include/ftle.h
SIGNATURES = {
    "ftle_create_mesh": (_int, [_int, _i64, _vp, _int, _i64, _vp, ctypes.c_uint, _P(_vp)]),
    "ftle_create_mesh_from_csr": (_int, [_int, _i64, _vp, _int, _vp, _vp, ctypes.c_uint, _P(_vp)]),
    "ftle_create_mesh_device": (_int, [_int, _i64, _vp, _int, _i64, _vp, ctypes.c_uint, _vp, _P(_vp)]),
    "ftle_create_mesh_device_from_csr": (_int, [_int, _i64, _vp, _int, _vp, _vp, ctypes.c_uint, _vp, _P(_vp)]),
    "ftle_ring1_csr": (_int, [_int, _i64, _i64, _vp, _vp, _vp, _i64, _P(_i64), _vp]),
    "ftle_ring1_csr_workspace": (_int, [_int, _i64, _i64, _P(_i64)]),
    "ftle_ring1_csr_ws": (_int, [_int, _i64, _i64, _vp, _vp, _vp, _i64, _P(_i64), _vp, _i64, _vp]),
    "ftle_axis_ell": (_int, [_int, _i64, _vp, _int, _vp, _vp, _vp, _vp]),
    "ftle_forward_ell": (_int, [_int, _i64, _vp, _int, _vp, _vp, _dbl, _vp, ctypes.c_uint, _vp]),
    "ftle_encode_flow_f16": (_int, [_vp, _vp, _vp, _vp]),
    "ftle_forward_f16": (_int, [_vp, _vp, ctypes.c_double, _vp, _vp]),
    "ftle_advect_rk4": (_int, [_int, _vp, _i64, _vp, _int, _vp, _vp, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, _vp, _vp]),
    "ftle_advect_rk4_grid": (_int, [_int, _vp, _vp, _vp, _i64, ctypes.c_double, ctypes.c_double, _vp, _int, _i64,
                                    _vp, _int, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp,
                                    _vp]),
    "ftle_destroy_mesh": (None, [_vp]),
    "ftle_cached_memory_bytes": (_int, [_P(_i64)]),
    "ftle_release_cached_memory": (_int, []),
    "ftle_mesh_info": (_int, [_vp, _P(_int), _P(_i64), _P(_i64), _P(_int)]),
    "ftle_mesh_get_csr": (_int, [_vp, _vp, _vp, _vp]),
    "ftle_mesh_tile_stats": (_int, [_vp, _P(_i64), _P(_i64), _P(_i64), _P(_i64)]),
    "ftle_mesh_get_tiles": (_int, [_vp, _int, _P(_i64), _P(_i64), _vp, _vp]),
    "ftle_mesh_set_blocks": (_int, [_vp, _int, _int]),
    "ftle_mesh_get_blocks": (_int, [_vp, _P(_int), _P(_int)]),
    "ftle_forward": (_int, [_vp, _vp, _int, _dbl, _vp, _vp]),
    "ftle_tape_bytes": (_int, [_vp, _P(_i64)]),
    "ftle_forward_tape": (_int, [_vp, _vp, _int, _dbl, _vp, _vp, _vp]),
    "ftle_backward_tape": (_int, [_vp, _vp, _int, _vp, _vp, _vp]),
    "ftle_backward": (_int, [_vp, _vp, _int, _dbl, _vp, _vp, _vp]),
    "ftle_backward_noalloc": (_int, [_vp, _vp, _int, _dbl, _vp, _vp, _vp]),
    "ftle_batched": (_int, [_int, _vp, _vp, _vp, _vp, _int, _vp]),
    "ftle_batched_config": (_int, [_int, _vp, _P(_int), _P(_int), _P(_int)]),
    "ftle_mesh_fp64_hits": (_int, [_vp, _P(_i64), _int]),
    "ftle_force_wide_offsets": (_int, [_int]),
    "ftle_set_eig_threshold": (_int, [_dbl]),
    "ftle_get_eig_threshold": (_int, [_P(_dbl)]),
    "ftle_batched_pin_config": (_int, [_int, _int, _int]),
    "ftle_last_error": (ctypes.c_char_p, []),
    "ftle_version": (ctypes.c_char_p, []),
}

_lib = None


def load(build_if_missing: bool = True):
    """Load libftle.so, building it first (hipcc, gfx950) if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise ImportError(f"{LIB_PATH} is not built")
        from . import build as _build
        try:
            _build.build()
        except Exception as e:  # noqa: BLE001 - re-raised with context
            raise ImportError(f"libftle.so is missing and could not be built: {e}") from e
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)  # AttributeError if the export is missing
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        raise FTLEError(status, load().ftle_last_error().decode())
