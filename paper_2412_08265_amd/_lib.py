"""ctypes binding of librubix.so (include/rubix.h): structure mirrors and the raw entry points.

torch is imported before the library is opened so that librubix resolves its HIP runtime to the
one torch already loaded (one runtime per process; torch's streams are then valid handles).
The library is built in-tree by paper_2412_08265_amd/build.py; if it is missing this module
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_void_p

import torch  # noqa: F401  (must precede the dlopen below)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librubix.so")

RUBIX_OK, RUBIX_EINVAL, RUBIX_EWORKSPACE, RUBIX_EDEVICE, RUBIX_ERANGE = 0, -1, -2, -3, -4
RUBIX_MAX_JOBS = 64
RUBIX_MAX_AGE_NODES = 256
RUBIX_MAX_MET_NODES = 64
RUBIX_MAX_RADIUS = 64


class RubixGrid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("spaxel_kpc", c_double)]


class RubixLGrid(ctypes.Structure):
    _fields_ = [("start", c_double), ("step", c_double), ("n", c_int32), ("log_spaced", c_int32)]


class RubixSSP(ctypes.Structure):
    _fields_ = [("n_age", c_int32), ("n_met", c_int32),
                ("log_age_nodes", POINTER(c_float)), ("met_nodes", POINTER(c_float)),
                ("lam", RubixLGrid), ("flux", c_void_p)]


class RubixParticles(ctypes.Structure):
    _fields_ = [("n", c_int64)] + [(f, c_void_p) for f in
                                   ("x", "y", "z", "vx", "vy", "vz", "mass", "age", "met")]


class RubixNoise(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("gain", c_double), ("sigma_floor", c_double)]


class RubixJob(ctypes.Structure):
    _fields_ = [("p", RubixParticles), ("angles_rad", c_double * 3), ("grid", RubixGrid),
                ("tel", RubixLGrid), ("z_sys", c_double), ("flux_scale", c_double),
                ("psf_sigma_spx", c_double), ("lsf_sigma_A", c_double),
                ("key", c_void_p), ("perm", c_void_p), ("seg_off", c_void_p),
                ("vlos", c_void_p), ("cube_raw", c_void_p), ("cube", c_void_p),
                ("resample", c_int32), ("reserved", c_int32)]


EXPORTS = ("rubix_workspace_size", "rubix_rotate_bin", "rubix_cube", "rubix_psf_lsf",
           "rubix_cube_backward", "rubix_last_error", "rubix_version", "rubix_table_bytes",
           "rubix_forward_pack", "rubix_forward_packed", "rubix_graph_create",
           "rubix_graph_launch", "rubix_graph_destroy", "rubix_cube_timer",
           "rubix_cube_timer_read", "rubix_add_noise", "rubix_psf_lsf_noalloc")

_lib = None


class RubixError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rubix error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Open librubix.so (once). Raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2412_08265_amd.build` (no fallback path exists)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.rubix_workspace_size.argtypes = [POINTER(RubixJob), c_int, POINTER(RubixSSP),
                                         POINTER(c_size_t)]
    lib.rubix_rotate_bin.argtypes = [POINTER(RubixJob), c_int, c_void_p, c_size_t, c_void_p]
    lib.rubix_cube.argtypes = [POINTER(RubixJob), c_int, POINTER(RubixSSP), c_void_p, c_size_t,
                               c_void_p]
    lib.rubix_psf_lsf.argtypes = [POINTER(RubixJob), c_int, POINTER(c_void_p), POINTER(c_void_p),
                                  c_void_p, c_size_t, c_void_p]
    lib.rubix_psf_lsf_noalloc.argtypes = [POINTER(RubixJob), c_int, POINTER(c_void_p),
                                          POINTER(c_void_p), c_void_p]
    lib.rubix_cube_backward.argtypes = [POINTER(RubixJob), c_int, POINTER(RubixSSP),
                                        POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                        c_void_p, c_void_p, c_size_t, c_void_p]
    lib.rubix_table_bytes.argtypes = [c_int]
    lib.rubix_table_bytes.restype = c_size_t
    lib.rubix_forward_pack.argtypes = [POINTER(RubixJob), c_int, POINTER(RubixSSP), c_void_p,
                                       c_size_t, c_void_p, c_size_t, c_int, c_int]
    lib.rubix_forward_packed.argtypes = [c_void_p, c_int, c_int, c_int, c_void_p]
    lib.rubix_graph_create.argtypes = [c_void_p, c_int, c_int, c_int, POINTER(c_void_p)]
    lib.rubix_graph_launch.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    lib.rubix_graph_destroy.argtypes = [c_void_p]
    lib.rubix_add_noise.argtypes = [POINTER(RubixJob), c_int, POINTER(RubixNoise),
                                    POINTER(c_void_p), c_void_p]
    lib.rubix_cube_timer.argtypes = [c_int]
    lib.rubix_cube_timer_read.argtypes = [POINTER(c_double), POINTER(c_int)]
    for f in ("rubix_workspace_size", "rubix_rotate_bin", "rubix_cube", "rubix_psf_lsf",
              "rubix_cube_backward", "rubix_forward_pack", "rubix_forward_packed",
              "rubix_graph_create", "rubix_graph_launch", "rubix_graph_destroy",
              "rubix_cube_timer", "rubix_cube_timer_read", "rubix_add_noise",
              "rubix_psf_lsf_noalloc"):
        getattr(lib, f).restype = c_int
    lib.rubix_last_error.restype = ctypes.c_char_p
    lib.rubix_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != RUBIX_OK:
        raise RubixError(rc, load().rubix_last_error().decode())


def ptr_array(ptrs) -> ctypes.Array:
    arr = (c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr
