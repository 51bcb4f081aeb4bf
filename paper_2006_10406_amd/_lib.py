"""ctypes view of ``include/eed4.h``.  Loading fails loudly when the HIP
library has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# EED4_LIBRARY names another build of the library (the sanitizer tests use it)
LIB_PATH = os.environ.get("EED4_LIBRARY") or os.path.join(HERE, "lib", "libeed4.so")

EED4_OK = 0
EED4_EINVAL = -1
EED4_EUNSTABLE = -2
EED4_EWORKSPACE = -3
EED4_EHIP = -4
EED4_EDIVERGED = -5
EED4_ETOOLARGE = -6
EED4_STATIC_SCRATCH_BYTES = 64 << 20

EED4_ALLOW_LARGE_TAU = 0x1
EED4_ABS_TOL = 0x2
EED4_NO_GRAPH = 0x4
EED4_TILE_KERNEL = 0x8


def EED4_FORCE_SHAPE(s):
    return ((s + 1) & 0xFF) << 8


# tensor variants (diffusivities of Table 7, mu3 choices of Sec. 3.1)
EED4_CHARBONNIER = 0
EED4_PERONA_MALIK = 1
EED4_PERONA_MALIK_EXP = 2
EED4_GEMAN_REYNOLDS = 3
EED4_MU3_GEOMETRIC = 0
EED4_MU3_ARITHMETIC = 1
EED4_MU3_MAX = 2
DIFFUSIVITY_NAMES = ("charbonnier", "perona_malik", "perona_malik_exp", "geman_reynolds")
MU3_NAMES = ("geometric", "arithmetic", "max")


def EED4_DIFFUSIVITY(d):
    return (d & 0xF) << 16


def EED4_MU3(r):
    return (r & 0x3) << 20


SHAPE_NAMES = ("tile64x32", "tile64x16", "tile32x32", "strip", "strip_tall", "strip_short",
               "strip_tiny", "strip_wide", "strip_wide_short", "tile32x16", "tile16x16")
# shape ids by kernel family (every shape gives bitwise the same result)
TILE_SHAPES = (0, 1, 2, 9, 10)
STRIP_SHAPES = (3, 4, 5, 6, 7, 8)

EED4_OP_INPAINT = 1
EED4_OP_CYCLE = 2
EED4_OP_BACKWARD = 3

EXPORTED = ("eed4_radius", "eed4_workspace_size", "eed4_inpaint", "eed4_fsi_cycle",
            "eed4_fsi_cycle_static", "eed4_fsi_step",
            "eed4_backward", "eed4_batched_workspace_size", "eed4_inpaint_batched",
            "eed4_autotune_batched", "eed4_step_shape", "eed4_strerror")


class eed4_params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_float), ("sigma", ctypes.c_float), ("tau", ctypes.c_float),
                ("cycle_len", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("tol", ctypes.c_float), ("flags", ctypes.c_int)]


class eed4_stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("residual", ctypes.c_double),
                ("rel_residual", ctypes.c_double)]


class eed4_image(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("known", ctypes.c_void_p),
                ("H", ctypes.c_int), ("W", ctypes.c_int), ("lambda_", ctypes.c_float)]


_L = None


def lib():
    global _L
    if _L is None:
        _L = load_library(LIB_PATH)
    return _L


def load_library(path):
    """ctypes handle of a build of the library at path, with the signatures of
    include/eed4.h (the binding uses the one at LIB_PATH)."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(path)
    vp, sz, i, f = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_float
    pp = ctypes.POINTER(eed4_params)
    L.eed4_radius.restype = i
    L.eed4_radius.argtypes = [f]
    L.eed4_workspace_size.restype = sz
    L.eed4_workspace_size.argtypes = [i, i, i, i, pp]
    L.eed4_inpaint.restype = i
    L.eed4_inpaint.argtypes = [vp, vp, vp, i, i, i, pp, vp, vp, sz, vp,
                               ctypes.POINTER(eed4_stats), vp]
    L.eed4_fsi_cycle.restype = i
    L.eed4_fsi_cycle.argtypes = [vp, vp, vp, i, i, i, pp, vp, sz, vp, vp]
    L.eed4_fsi_cycle_static.restype = i
    L.eed4_fsi_cycle_static.argtypes = [vp, vp, vp, i, i, i, pp, vp, vp]
    L.eed4_fsi_step.restype = i
    L.eed4_fsi_step.argtypes = [vp, vp, vp, vp, i, i, i, pp, i, vp]
    L.eed4_backward.restype = i
    L.eed4_backward.argtypes = [vp, vp, vp, i, i, i, pp, i, vp, vp, vp, vp, vp, sz, vp]
    L.eed4_batched_workspace_size.restype = sz
    L.eed4_batched_workspace_size.argtypes = [ctypes.POINTER(eed4_image), i, pp]
    L.eed4_inpaint_batched.restype = i
    L.eed4_inpaint_batched.argtypes = [ctypes.POINTER(eed4_image), i, pp, vp, sz, vp,
                                       ctypes.POINTER(eed4_stats)]
    L.eed4_autotune_batched.restype = i
    L.eed4_autotune_batched.argtypes = [ctypes.POINTER(eed4_image), i, pp, vp, sz, vp]
    L.eed4_step_shape.restype = i
    L.eed4_step_shape.argtypes = [i, i, i, pp]
    L.eed4_strerror.restype = ctypes.c_char_p
    L.eed4_strerror.argtypes = [i]
    return L
