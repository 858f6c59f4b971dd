"""Build and load the oracle's C loops (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-shared", "-fPIC", "-std=c11", "-D_GNU_SOURCE"]


def build(force=False):
    """Compile oracle.c into liboracle.so with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i = ctypes.c_int


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.orc_assemble_stiffness_2d.argtypes = [_i, _i, _i, _i, _i, _D, _D, _D, _D, _D]
        _lib.orc_assemble_load_2d.argtypes = [_i, _i, _i, _i, _i, _D, _D, _D, _D, _i, _D]
        _lib.orc_gs_lex.argtypes = [_i, _I, _I, _D, _D, _D, _D]
        _lib.orc_gs_lex_backward.argtypes = [_i, _I, _I, _D, _D, _D, _D]
        _lib.orc_gs_colour.argtypes = [_i, _I, _I, _I, _D, _D, _D, _D, _D]
        _lib.orc_residual.argtypes = [_i, _I, _I, _D, _D, _D, _D]
        for f in ("orc_assemble_stiffness_2d", "orc_assemble_load_2d", "orc_gs_lex",
                  "orc_gs_lex_backward", "orc_gs_colour", "orc_residual"):
            getattr(_lib, f).restype = None
    return _lib
