"""Accuracy measurements of a QR factorization, on the CPU in binary64 with compensated
(Dot2) inner products: orthogonality ||Q^T Q - I|| (or ||Q^T B Q - I|| for tridiagonal B) and
the relative residual ||X - QR||_F / ||X||_F.  Independent of the oracle and of the GPU
library.  ``scqr_accuracy.c`` holds the arithmetic; this module marshals NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scqr_accuracy.c")
_LIB = os.path.join(_HERE, "libaccuracy.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.acc_gram_dot2.argtypes = [I64, I64, P, I64, P]
        L.acc_gram_dot2.restype = None
        L.acc_gram_dot2_tridiag.argtypes = [I64, I64, P, I64, P, P, P]
        L.acc_gram_dot2_tridiag.restype = None
        L.acc_gram_dot2_csr.argtypes = [I64, I64, P, I64, P, P, P, P]
        L.acc_gram_dot2_csr.restype = None
        L.acc_residual.argtypes = [I64, I64, P, I64, P, I64, P, I64, ctypes.POINTER(D)]
        L.acc_residual.restype = D
        L.acc_residual_rows.argtypes = [I64, P, I64, P, I64, P, I64, P, I64, ctypes.POINTER(D)]
        L.acc_residual_rows.restype = D
        _lib = L
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gram(Q, tridiag=None, csr=None):
    """Compensated Q^T Q, or Q^T B Q for tridiagonal B = (diag, off) or B in compressed sparse
    rows csr = (row_ptr, col, val)."""
    Q = _c(Q)
    m, n = Q.shape
    G = np.empty((n, n))
    if csr is not None:
        rp = np.ascontiguousarray(csr[0], dtype=np.int64)
        col = np.ascontiguousarray(csr[1], dtype=np.int32)
        val = _c(csr[2])
        if rp.size != m + 1 or rp[-1] != col.size or col.size != val.size or \
                (col.size and (col.min() < 0 or col.max() >= m)):
            raise ValueError("malformed compressed sparse rows")
        lib().acc_gram_dot2_csr(m, n, Q.ctypes.data, n, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                                G.ctypes.data)
    elif tridiag is None:
        lib().acc_gram_dot2(m, n, Q.ctypes.data, n, G.ctypes.data)
    else:
        d, o = _c(tridiag[0]), _c(tridiag[1])
        lib().acc_gram_dot2_tridiag(m, n, Q.ctypes.data, n, d.ctypes.data,
                                    (o if o.size else d).ctypes.data, G.ctypes.data)
    return G


def orthogonality(Q, tridiag=None, csr=None):
    """(||G - I||_2, ||G - I||_F) with G the compensated Gram."""
    G = gram(Q, tridiag, csr)
    E = G - np.eye(G.shape[0])
    return float(np.max(np.abs(np.linalg.eigvalsh(E)))), float(np.linalg.norm(E))


def residual(X, Q, R):
    """||X - QR||_F / ||X||_F with compensated dot products (upper triangle of R)."""
    X, Q, R = _c(X), _c(Q), _c(R)
    m, n = X.shape
    xn = ctypes.c_double()
    r = lib().acc_residual(m, n, X.ctypes.data, n, Q.ctypes.data, n, R.ctypes.data, n,
                           ctypes.byref(xn))
    return r / xn.value if xn.value > 0 else r


def residual_rows(X, Q, R, rows):
    """Residual restricted to a sample of rows: ||X_S - Q_S R||_F / ||X_S||_F."""
    X, Q, R = _c(X), _c(Q), _c(R)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n = X.shape[1]
    xn = ctypes.c_double()
    r = lib().acc_residual_rows(rows.size, rows.ctypes.data, n, X.ctypes.data, n, Q.ctypes.data,
                                n, R.ctypes.data, n, ctypes.byref(xn))
    return r / xn.value if xn.value > 0 else r


def cond2(A) -> float:
    """2-norm condition number from singular values (LAPACK SVD; absolute error ~ u ||A||)."""
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1])
