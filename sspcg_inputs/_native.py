"""Builds and loads the C stencil assembler (stencil.c) with gcc."""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "libsspcg_inputs.so")
_handle = None


def build(force: bool = False) -> str:
    """Compile stencil.c into _build/libsspcg_inputs.so (atomic replace)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(_OUT_DIR, exist_ok=True)
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=_OUT_DIR)
    os.close(fd)
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-std=c99", "-fopenmp",
           "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _handle
    if _handle is None:
        L = ctypes.CDLL(build())
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.inp_stencil_nnz.restype = ctypes.c_int64
        L.inp_stencil_nnz.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p]
        L.inp_stencil.restype = ctypes.c_int
        L.inp_stencil.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 5
        L.inp_scaled_matvec.restype = None
        L.inp_diagonal.restype = None
        L.inp_diagonal.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 4
        L.inp_scaled_matvec.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 6
        _handle = L
    return _handle
