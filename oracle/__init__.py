"""CPU FP64 oracle for shifted Cholesky QR — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU product path never imports, links or calls it, and the two share
no code.  The arithmetic lives in ``scqr_oracle.c`` (plain binary64 loops, no FMA contraction);
this module only marshals NumPy arrays through ctypes.

Functions follow the paper (Fukaya et al., "Shifted CholeskyQR for computing the QR
factorization of ill-conditioned matrices"):

* ``gram``            equation (eq:gram), Algorithm 1 line 1
* ``gram_tridiag``    X^T B X of Algorithm 4 with tridiagonal B
* ``gram_dense``      X^T B X with dense B (Table 3)
* ``gram_f32``        FP32-first Gram emulation (not in the paper; pinned by its error bound,
                      exact small-integer cases and the closed-form condition number of the
                      first factor; the rest is parity unpinned)
* ``chol_upper``      Algorithm 1 line 3, R^T R = A + sI, breakdown report
* ``trsm_rows``       Algorithm 1 line 4, row-wise substitution (equation (eq:backward2))
* ``trmm_upper``      R := R~ R of Algorithms 2 and 3
* ``shift``           equations (eq:finds2) and (eq:finds2B), remark after Table 3
* ``scqr``            Algorithms 2, 3, 5 and CholeskyQR2 drivers.  Where an unshifted Cholesky is
                      borderline (kappa near 1/u, or an input factor with kappa above u^{-1/2}),
                      whether it breaks down, and so the pass count, is parity unpinned: rounding
                      order decides it
* ``qr_backward``     QR adjoint dX = (dQ + Q copyltu(M)) R^{-T}, M = R dR^T - dQ^T Q
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scqr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIXED3, ADAPTIVE, CHOLQR2, ITERATED = 0, 1, 2, 3
SHIFT_PAPER, SHIFT_FRO, SHIFT_SMALL, SHIFT_CUSTOM, SHIFT_DEPTH = 0, 1, 2, 3, 4
OK, INVALID, BREAKDOWN, NOT_CONVERGED, NONFINITE = 0, 1, 5, 6, 7
U = 2.0 ** -53
U32 = 2.0 ** -24


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (binary64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("shift_mode", ctypes.c_int32),
                ("max_passes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("f32_chain", ctypes.c_int32), ("force_breakdown_pass", ctypes.c_int32),
                ("zero_shift", ctypes.c_int32), ("gram_chunk", ctypes.c_int32),
                ("custom_alpha", ctypes.c_double), ("bnorm", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("shifted_mask", ctypes.c_int32), ("breakdown_mask", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("shift", ctypes.c_double * 16), ("norm2sq", ctypes.c_double * 16),
                ("gram_dev", ctypes.c_double * 16)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I64, D, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32
        sig = {
            "orc_gram": (None, [I64, I64, P, I64, P]),
            "orc_gram_tridiag": (None, [I64, I64, P, I64, P, P, P]),
            "orc_gram_dense": (None, [I64, I64, P, I64, P, P]),
            "orc_gram_csr": (None, [I64, I64, P, I64, P, P, P, P]),
            "orc_gershgorin_csr": (D, [I64, P, P]),
            "orc_gram_f32": (None, [I64, I64, P, I64, I64, P]),
            "orc_gram_chunked": (None, [I64, I64, P, I64, I64, P]),
            "orc_gram_depth": (I64, [I64, I64]),
            "orc_shift_depth": (D, [I64, I64, D]),
            "orc_sym_eig": (None, [I64, P, P]),
            "orc_lambda_max": (D, [I64, P]),
            "orc_chol_upper": (ctypes.c_int, [I64, P, D, P]),
            "orc_trsm_rows": (None, [I64, I64, P, I64, P, P, I64]),
            "orc_trmm_upper": (None, [I64, P, P, P]),
            "orc_gershgorin_tridiag": (D, [I64, P, P]),
            "orc_shift": (D, [I64, I64, D, D, ctypes.c_int, ctypes.c_int, D]),
            "orc_shift_f32": (D, [I64, I64, D]),
            "orc_scqr": (ctypes.c_int, [I64, I64, P, I64, I32, P, P, ctypes.POINTER(_Opts), P, P,
                                        ctypes.POINTER(_Info), P, P]),
            "orc_scqr_csr": (ctypes.c_int, [I64, I64, P, I64, P, P, P, ctypes.POINTER(_Opts), P, P,
                                            ctypes.POINTER(_Info), P, P]),
            "orc_qr_backward": (None, [I64, I64, P, P, P, P, P]),
            "orc_num_threads": (ctypes.c_int, []),
            "orc_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


def gram(X):
    X = _c(X)
    m, n = X.shape
    A = np.empty((n, n))
    lib().orc_gram(m, n, _p(X), n, _p(A))
    return A


def gram_tridiag(X, diag, off):
    X, diag, off = _c(X), _c(diag), _c(off)
    m, n = X.shape
    A = np.empty((n, n))
    lib().orc_gram_tridiag(m, n, _p(X), n, _p(diag), _p(off) if off.size else _p(diag), _p(A))
    return A


def gram_dense(X, B):
    X, B = _c(X), _c(B)
    m, n = X.shape
    A = np.empty((n, n))
    lib().orc_gram_dense(m, n, _p(X), n, _p(B), _p(A))
    return A


def _csr(csr, m):
    """(row_ptr int64[m+1], col int32[nnz], val float64[nnz]) as contiguous arrays, checked."""
    rp, col, val = _c(csr[0], np.int64), _c(csr[1], np.int32), _c(csr[2])
    if rp.size != m + 1 or rp[0] != 0 or np.any(np.diff(rp) < 0) or rp[-1] != col.size or col.size != val.size:
        raise ValueError("malformed compressed sparse rows")
    if col.size and (col.min() < 0 or col.max() >= m):
        raise ValueError("column index out of range")
    return rp, col, val


def gram_csr(X, csr):
    """A = X^T B X with B = (row_ptr, col, val) in compressed sparse row form."""
    X = _c(X)
    m, n = X.shape
    rp, col, val = _csr(csr, m)
    A = np.empty((n, n))
    lib().orc_gram_csr(m, n, _p(X), n, _p(rp), _p(col), _p(val), _p(A))
    return A


def gershgorin_csr(csr) -> float:
    rp = _c(csr[0], np.int64)
    m = rp.size - 1
    rp, _, val = _csr(csr, m)
    return lib().orc_gershgorin_csr(m, _p(rp), _p(val))


def gram_f32(X, chain: int):
    X = _c(X)
    m, n = X.shape
    A = np.empty((n, n))
    lib().orc_gram_f32(m, n, _p(X), n, int(chain), _p(A))
    return A


def gram_chunked(X, chunk: int):
    """A = X^T X summed over consecutive chunks of `chunk` rows, then over the chunks."""
    X = _c(X)
    m, n = X.shape
    A = np.empty((n, n))
    lib().orc_gram_chunked(m, n, _p(X), n, int(chunk), _p(A))
    return A


def gram_depth(m: int, chunk: int) -> int:
    """Summation depth of gram_chunked: chunk + ceil(m / chunk) (m when chunk >= m)."""
    return int(lib().orc_gram_depth(int(m), int(chunk)))


def shift_depth(depth: int, n: int, norm2sq: float) -> float:
    """s = 11 (d n + n (n+1)) u ||X||_2^2 for a Gram of summation depth d."""
    return lib().orc_shift_depth(int(depth), int(n), float(norm2sq))


def sym_eig(A):
    A = _c(A)
    n = A.shape[0]
    w = np.empty(n)
    lib().orc_sym_eig(n, _p(A), _p(w))
    return w


def lambda_max(A) -> float:
    A = _c(A)
    return lib().orc_lambda_max(A.shape[0], _p(A))


def chol_upper(A, s: float = 0.0):
    """Returns (R, info): info 0 on success, else 1 + column of breakdown."""
    A = _c(A)
    n = A.shape[0]
    R = np.empty((n, n))
    info = lib().orc_chol_upper(n, _p(A), float(s), _p(R))
    return R, info


def trsm_rows(X, R):
    X, R = _c(X), _c(R)
    m, n = X.shape
    Q = np.empty((m, n))
    lib().orc_trsm_rows(m, n, _p(X), n, _p(R), _p(Q), n)
    return Q


def trmm_upper(Rt, R):
    Rt, R = _c(Rt), _c(R)
    n = R.shape[0]
    out = np.empty((n, n))
    lib().orc_trmm_upper(n, _p(Rt), _p(R), _p(out))
    return out


def gershgorin_tridiag(diag, off) -> float:
    diag, off = _c(diag), _c(off)
    return lib().orc_gershgorin_tridiag(diag.size, _p(diag), _p(off) if off.size else _p(diag))


def shift(m, n, norm2sq, bnorm=1.0, oblique=False, mode=SHIFT_PAPER, alpha=0.0) -> float:
    return lib().orc_shift(int(m), int(n), float(norm2sq), float(bnorm), int(bool(oblique)),
                           int(mode), float(alpha))


def shift_f32(n, chain, norm2sq) -> float:
    return lib().orc_shift_f32(int(n), int(chain), float(norm2sq))


def f32_chain_rows(n: int) -> int:
    """Rows accumulated in one binary32 chain of the FP32-first Gram, as the option defines it
    per padded width (n padded to 16, 32, 64, 128 or 256): 32 up to n = 64, 64 up to n = 128,
    16 beyond.  The chain length k enters the binary32 shift s32 = 11((k+2) n u32 + n(n+1) u)."""
    n = int(n)
    return 32 if n <= 64 else (64 if n <= 128 else 16)


@dataclass
class Result:
    Q: np.ndarray
    R: np.ndarray
    status: int
    passes: int
    shifted_mask: int
    breakdown_mask: int
    fell_back: int
    shifts: list
    norm2sq: list
    gram_dev: list
    grams: list = field(default_factory=list)
    rts: list = field(default_factory=list)


def scqr(X, schedule=FIXED3, shift_mode=SHIFT_PAPER, max_passes=6, B=None, tridiag=None,
         precision=0, f32_chain=None, force_breakdown_pass=0, zero_shift=False, custom_alpha=0.0,
         bnorm=0.0, history=False, gram_chunk=0, csr=None) -> Result:
    """Run the oracle's driver; ``tridiag=(diag, off)``, dense ``B`` or ``csr=(row_ptr, col,
    val)`` select the oblique form.
    ``shift_mode=SHIFT_DEPTH`` sums every Gram in chunks of ``gram_chunk`` rows and shifts with
    the depth of that summation (Euclidean inner product only)."""
    X = _c(X)
    m, n = X.shape
    if f32_chain is None:
        f32_chain = f32_chain_rows(n)
    o = _Opts(schedule, shift_mode, max_passes, precision, f32_chain, force_breakdown_pass,
              int(bool(zero_shift)), int(gram_chunk), custom_alpha, bnorm)
    info = _Info()
    Q = np.empty((m, n))
    R = np.empty((n, n))
    kind, b0, b1 = 0, None, None
    if tridiag is not None:
        kind = 1
        b0, b1 = _c(tridiag[0]), _c(tridiag[1])
        if b1.size == 0:
            b1 = b0
    elif B is not None:
        kind = 2
        b0 = _c(B)
    hp = 16 if history else 0
    gh = np.zeros((hp, n, n)) if history else None
    rh = np.zeros((hp, n, n)) if history else None
    if csr is not None:
        rp, col, val = _csr(csr, m)
        lib().orc_scqr_csr(m, n, _p(X), n, _p(rp), _p(col), _p(val), ctypes.byref(o), _p(Q), _p(R),
                           ctypes.byref(info), _p(gh), _p(rh))
    else:
        lib().orc_scqr(m, n, _p(X), n, kind, _p(b0), _p(b1), ctypes.byref(o), _p(Q), _p(R),
                       ctypes.byref(info), _p(gh), _p(rh))
    p = info.passes
    k = max(p + (1 if info.status == BREAKDOWN else 0), 1)
    res = Result(Q, R, info.status, p, info.shifted_mask, info.breakdown_mask, info.fell_back,
                 list(info.shift[:k]), list(info.norm2sq[:k]), list(info.gram_dev[:k]))
    if history:
        res.grams = [gh[i].copy() for i in range(p)]
        res.rts = [rh[i].copy() for i in range(p)]
    return res


def qr_backward(Q, R, dQ=None, dR=None):
    Q, R = _c(Q), _c(R)
    m, n = Q.shape
    dQc = None if dQ is None else _c(dQ)
    dRc = None if dR is None else _c(dR)
    dX = np.empty((m, n))
    lib().orc_qr_backward(m, n, _p(Q), _p(R), _p(dQc), _p(dRc), _p(dX))
    return dX
