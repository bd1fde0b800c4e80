"""ctypes loader for liblqcd.so (argument marshalling only).

torch is imported first so that the library binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7); two runtimes in one
process would not share streams or allocations.  A missing library is an
error: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library must share)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblqcd.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p


class GeomT(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("bc", ctypes.c_int32 * 4)]


class CGStatsT(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("reliable_updates", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("true_residual", c_double),
        ("iterated_residual", c_double),
        ("seconds", c_double),
    ]


G = ctypes.POINTER(GeomT)

# name -> (restype, argtypes); mirrors include/lqcd.h
SIGNATURES = {
    "lqcd_version": (c_int, []),
    "lqcd_strerror": (ctypes.c_char_p, [c_int]),
    "lqcd_last_hip_error": (ctypes.c_char_p, []),
    "lqcd_spinor_bytes": (c_size_t, [G, c_int, c_int]),
    "lqcd_gauge_bytes": (c_size_t, [G, c_int, c_int]),
    "lqcd_pack_spinor": (c_int, [G, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "lqcd_unpack_spinor": (c_int, [G, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "lqcd_pack_gauge": (c_int, [G, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "lqcd_unpack_gauge": (c_int, [G, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "lqcd_dslash": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double,
                            c_int, c_int, c_void_p]),
    "lqcd_dslash_dagger": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double,
                                   c_int, c_int, c_void_p]),
    "lqcd_meo": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_int,
                         c_int, c_int, c_void_p]),
    "lqcd_moe": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_int,
                         c_int, c_int, c_void_p]),
    "lqcd_face_bytes": (c_size_t, [G, c_int]),
    "lqcd_face_pack": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                               c_void_p]),
    "lqcd_hop_region": (c_int, [G, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_double, c_double, c_int, c_int, c_int, c_void_p]),
    "lqcd_mhat": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int, c_int,
                          c_int, c_void_p]),
    "lqcd_reduce_workspace_bytes": (c_size_t, [G, c_int]),
    "lqcd_dot": (c_int, [G, c_int, c_void_p, c_void_p, c_int, c_void_p,
                         ctypes.POINTER(c_double), c_void_p]),
    "lqcd_dot_noalloc": (c_int, [G, c_int, c_void_p, c_void_p, c_int, ctypes.POINTER(c_double),
                                 c_void_p]),
    "lqcd_norm2": (c_int, [G, c_int, c_void_p, c_int, c_void_p, ctypes.POINTER(c_double),
                           c_void_p]),
    "lqcd_axpby": (c_int, [G, c_int, c_double, c_void_p, c_double, c_void_p, c_int, c_void_p]),
    "lqcd_convert": (c_int, [G, c_int, c_void_p, c_int, c_void_p, c_int, c_void_p]),
    "lqcd_cg_workspace_bytes": (c_size_t, [G, c_int, c_int]),
    "lqcd_cg_solve": (c_int, [G, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_int,
                              c_double, c_double, c_int, c_int, c_void_p, c_size_t,
                              ctypes.POINTER(CGStatsT), c_void_p]),
    "lqcd_fermion_force": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int,
                                   c_int, c_int, c_int, c_void_p]),
    "lqcd_cshift": (c_int, [G, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "lqcd_colour_mul": (c_int, [G, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                                c_void_p]),
    "lqcd_spin_project": (c_int, [G, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p]),
    "lqcd_dslash_generic": (c_int, [G, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                    c_int, c_int, c_void_p]),
    "lqcd_split_rotate": (c_int, [c_void_p, c_void_p, ctypes.c_int64, c_int, c_int, c_int, c_int,
                                  c_void_p]),
    "lqcd_su3_mul": (c_int, [G, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                             c_void_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load liblqcd.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with paper_2001_07557_amd.build.build() "
            "(hipcc for gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
