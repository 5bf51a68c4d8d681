"""ctypes wrapper of oracle/cbsr.c: a block-CSR 3x3 operator for the oracle.

TEST INFRASTRUCTURE ONLY.  `BsrOperator(row_ptr, col_idx, hblocks) @ X` is
the plain matrix product H X (X an n-vector or row-major n x q block),
computed by the C loop in cbsr.c on all host cores.  The oracle's filter,
Lanczos and subspace iteration accept it wherever they take a scipy matrix.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cbsr.c")
_LIB = os.path.join(_HERE, "libcbsr.so")
_lib = None


def build() -> str:
    """Compile cbsr.c with gcc (OpenMP)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.oracle_bsr3_matmul.argtypes = [C.c_int64] + [C.c_void_p] * 5 + [C.c_int64]
        L.oracle_bsr3_matmul.restype = None
        _lib = L
    return _lib


class BsrOperator:
    def __init__(self, row_ptr, col_idx, hblocks):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int64)
        self.vals = np.ascontiguousarray(hblocks, dtype=np.float64)
        self.n_atoms = self.row_ptr.shape[0] - 1
        self.shape = (3 * self.n_atoms, 3 * self.n_atoms)

    def __matmul__(self, X):
        X = np.asarray(X, dtype=np.float64)
        if X.shape[0] != self.shape[1]:
            raise ValueError(f"operand has {X.shape[0]} rows, the operator {self.shape[1]} columns")
        vec = X.ndim == 1
        Xc = np.ascontiguousarray(X.reshape(X.shape[0], -1))
        Y = np.empty_like(Xc)
        _load().oracle_bsr3_matmul(self.n_atoms, self.row_ptr.ctypes.data, self.col_idx.ctypes.data,
                                   self.vals.ctypes.data, Xc.ctypes.data, Y.ctypes.data,
                                   Xc.shape[1])
        return Y[:, 0] if vec else Y
