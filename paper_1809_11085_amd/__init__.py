"""Shifted Cholesky QR on AMD MI355X (gfx950).

Thin Python binding of ``libscqr.so`` (see ``include/scqr.h``): it only marshals arguments
between PyTorch device tensors and the C ABI.  Every step of the factorization runs in the
library's HIP kernels; there is no CPU or PyTorch fallback, and the functions raise if the
library has not been built (``python -m paper_1809_11085_amd.build``).

Functions mirror the C entry points:

* ``qr(X, B=None, **opts) -> (Q, R, info)``  Algorithms 1-3 and 5 of Fukaya et al.; B is a
  tridiagonal ``(diag, off)`` or a ``CsrB(row_ptr, col, val)`` in compressed sparse rows
* ``gram(X, B=None) -> G``                   A = X^T X (or X^T B X), equation (eq:gram)
* ``trsm(X, R) -> Q``                        Q = X R^{-1} row by row (Algorithm 1 line 4)
* ``qr_batched(Xs, **opts)``                 independent problems
* ``qr_backward(Q, R, dQ, dR) -> dX``        QR adjoint
* ``QRFunction``                             ``torch.autograd.Function`` using the adjoint
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import NamedTuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscqr.so")

OK, E_INVALID, E_WORKSPACE, E_UNSUPPORTED, E_HIP, E_BREAKDOWN, E_NOT_CONVERGED, E_NONFINITE = range(8)
SCHEDULES = {"fixed3": 0, "adaptive": 1, "cholqr2": 2, "iterated": 3}
SHIFTS = {"paper": 0, "fro": 1, "small": 2, "custom": 3, "depth": 4}
PRECISIONS = {"fp64": 0, "fp32_first": 1}
MAX_PASSES = 16


class ScqrError(RuntimeError):
    """A failed call: ``status`` is the scqr_status code; for a numerical failure reported on
    the device (breakdown, non-convergence, non-finite Gram) ``info`` holds the decoded record
    and ``result`` the outputs as the library left them."""

    def __init__(self, status: int, msg: str, info=None, result=None):
        super().__init__(msg)
        self.status = status
        self.info = info
        self.result = result


CHECK_MODES = (True, False, "raise", "status")


def check_mode(check) -> str:
    """Normalise the ``check`` argument of ``qr`` / ``qr_batched``: "raise" (True, the default:
    synchronize, decode, raise ScqrError on a numerical failure), "status" (synchronize and
    decode, never raise) or "none" (False: return the raw device record, no synchronisation)."""
    if check is True or check == "raise":
        return "raise"
    if check is False or check is None:
        return "none"
    if check == "status":
        return "status"
    raise ValueError(f"check must be one of {CHECK_MODES}, got {check!r}")


class _Opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("shift_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("final_gram", ctypes.c_int32), ("debug_force_breakdown_pass", ctypes.c_int32),
                ("debug_zero_shift", ctypes.c_int32), ("recompute", ctypes.c_int32),
                ("custom_alpha", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("trace", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("shifted_mask", ctypes.c_int32), ("breakdown_mask", ctypes.c_int32),
                ("fell_back_fp64", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("shift", ctypes.c_double * MAX_PASSES), ("norm2sq", ctypes.c_double * MAX_PASSES),
                ("gram_dev", ctypes.c_double * MAX_PASSES), ("omega_fro", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("gram_depth", ctypes.c_double)]


class _SpdOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("diag", ctypes.c_void_p), ("off", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("nnz", ctypes.c_int64)]


class CsrB(NamedTuple):
    """A sparse symmetric positive definite B in compressed sparse rows on the device:
    row_ptr int64 [m + 1], col int32 [nnz], val float64 [nnz] (CUDA tensors, contiguous)."""
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


INFO_BYTES = ctypes.sizeof(_Info)
_lib = None


def lib():
    """Load libscqr.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1809_11085_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        st = ctypes.c_int
        L.scqr_default_opts.argtypes = [ctypes.POINTER(_Opts)]
        L.scqr_default_opts.restype = None
        L.scqr_status_string.argtypes = [st]
        L.scqr_status_string.restype = ctypes.c_char_p
        L.scqr_build_info.argtypes = []
        L.scqr_build_info.restype = ctypes.c_char_p
        L.scqr_workspace_bytes.argtypes = [I64, I64, ctypes.POINTER(_SpdOp), ctypes.POINTER(_Opts), ctypes.POINTER(SZ)]
        L.scqr_workspace_bytes.restype = st
        L.scqr_qr.argtypes = [P, I64, I64, P, I64, ctypes.POINTER(_SpdOp), P, I64, P, I64, P, SZ,
                              ctypes.POINTER(_Opts), P]
        L.scqr_qr.restype = st
        L.scqr_qr_noalloc.argtypes = [P, I64, I64, P, I64, ctypes.POINTER(_SpdOp), P, I64, P, I64,
                                      ctypes.POINTER(_Opts), P]
        L.scqr_qr_noalloc.restype = st
        L.scqr_peak_copy.argtypes = [P, P, P, I64, I32, I32]
        L.scqr_peak_copy.restype = st
        L.scqr_peak_read.argtypes = [P, P, I64, I32, I32, P]
        L.scqr_peak_read.restype = st
        L.scqr_peak_write.argtypes = [P, P, I64, I32, I32]
        L.scqr_peak_write.restype = st
        L.scqr_peak_fp64.argtypes = [P, I32, I32, I32, P]
        L.scqr_peak_fp64.restype = st
        L.scqr_gram.argtypes = [P, I64, I64, P, I64, ctypes.POINTER(_SpdOp), P, I64, P, SZ]
        L.scqr_gram.restype = st
        L.scqr_trsm.argtypes = [P, I64, I64, P, I64, P, I64, P, I64, P, SZ]
        L.scqr_trsm.restype = st
        L.scqr_batched_workspace_bytes.argtypes = [I32, P, P, ctypes.POINTER(_Opts), P, ctypes.POINTER(SZ)]
        L.scqr_batched_workspace_bytes.restype = st
        L.scqr_qr_batched.argtypes = [P, I32, P, P, P, P, P, P, P, P, P, SZ, ctypes.POINTER(_Opts), P, P]
        L.scqr_qr_batched.restype = st
        L.scqr_batched_plan_create.argtypes = [I32, P, P, P, P, P, P, P, P, P, SZ, ctypes.POINTER(_Opts), P, P,
                                               ctypes.POINTER(P)]
        L.scqr_batched_plan_create.restype = st
        L.scqr_batched_plan_upload.argtypes = [P, P]
        L.scqr_batched_plan_upload.restype = st
        L.scqr_batched_plan_run.argtypes = [P, P]
        L.scqr_batched_plan_run.restype = st
        L.scqr_batched_plan_tuning.argtypes = [P, P, P]
        L.scqr_batched_plan_tuning.restype = st
        L.scqr_batched_plan_destroy.argtypes = [P]
        L.scqr_batched_plan_destroy.restype = st
        L.scqr_backward_workspace_bytes.argtypes = [I64, I64, ctypes.POINTER(SZ)]
        L.scqr_backward_workspace_bytes.restype = st
        L.scqr_qr_backward.argtypes = [P, I64, I64, P, I64, P, I64, P, I64, P, I64, P, I64, P, SZ]
        L.scqr_qr_backward.restype = st
        L.scqr_profile_enable.argtypes = [I32]
        L.scqr_profile_enable.restype = st
        L.scqr_profile_read.argtypes = [ctypes.POINTER(_KernelStat), I32, ctypes.POINTER(I32)]
        L.scqr_profile_read.restype = st
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().scqr_status_string(int(s)).decode()


def _check(s: int, what: str):
    if s != OK:
        raise ScqrError(s, f"{what}: {status_string(s)}")


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _mat(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float64 CUDA tensor")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be row-major (stride(1) == 1, stride(0) >= columns)")
    return t.data_ptr(), t.stride(0)


def _workspace(nbytes: int, dev) -> tuple:
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=dev)
    base = buf.data_ptr()
    return buf, base + ((-base) % 256)


def _opts(schedule="adaptive", shift="paper", precision="fp64", max_passes=6, final_gram=False,
          custom_alpha=0.0, bnorm=0.0, trace_ptr=None, debug_force_breakdown_pass=0,
          debug_zero_shift=False, recompute=False) -> _Opts:
    o = _Opts()
    lib().scqr_default_opts(ctypes.byref(o))
    o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.shift_mode = SHIFTS[shift] if isinstance(shift, str) else int(shift)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.max_passes = int(max_passes)
    o.final_gram = int(bool(final_gram))
    o.custom_alpha = float(custom_alpha)
    o.bnorm = float(bnorm)
    o.trace = trace_ptr
    o.debug_force_breakdown_pass = int(debug_force_breakdown_pass)
    o.debug_zero_shift = int(bool(debug_zero_shift))
    o.recompute = int(bool(recompute))
    return o


def _spd(B, m: int):
    if B is None:
        return None
    if isinstance(B, CsrB):
        for t, nm, dt in ((B.row_ptr, "row_ptr", torch.int64), (B.col, "col", torch.int32),
                          (B.val, "val", torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
                raise TypeError(f"CSR {nm} must be a contiguous 1-D {dt} CUDA tensor")
        if B.row_ptr.numel() != m + 1 or B.col.numel() != B.val.numel():
            raise ValueError("CSR B needs row_ptr[m + 1] and col, val of equal length")
        op = _SpdOp()
        op.kind = 2
        op.row_ptr = B.row_ptr.data_ptr()
        op.col = B.col.data_ptr() if B.col.numel() else B.row_ptr.data_ptr()
        op.val = B.val.data_ptr() if B.val.numel() else B.row_ptr.data_ptr()
        op.nnz = B.val.numel()
        return op
    diag, off = B
    for t, nm in ((diag, "B diag"), (off, "B off")):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous float64 CUDA tensor")
    if diag.numel() != m or off.numel() != max(m - 1, 0):
        raise ValueError("tridiagonal B needs diag[m] and off[m-1]")
    op = _SpdOp()
    op.kind = 1
    op.diag = diag.data_ptr()
    op.off = off.data_ptr() if off.numel() else diag.data_ptr()
    return op


@dataclass
class Info:
    status: int
    passes: int
    shifted_mask: int
    breakdown_mask: int
    fell_back_fp64: int
    shift: list
    norm2sq: list
    gram_dev: list
    omega_fro: float
    bnorm: float
    gram_depth: float = 0.0

    @property
    def ok(self) -> bool:
        return self.status == OK


def decode_info(buf: torch.Tensor) -> Info:
    """Copy a device info record (uint8 tensor of INFO_BYTES) to the host and decode it."""
    raw = bytes(buf.detach().to("cpu").numpy().tobytes())
    c = _Info.from_buffer_copy(raw[:INFO_BYTES])
    k = max(c.passes + (1 if c.status == E_BREAKDOWN else 0), 1)
    return Info(c.status, c.passes, c.shifted_mask, c.breakdown_mask, c.fell_back_fp64,
                list(c.shift[:k]), list(c.norm2sq[:k]), list(c.gram_dev[:k]), c.omega_fro, c.bnorm,
                c.gram_depth)


class Plan:
    """Pre-allocated outputs and workspace for repeated factorizations of one shape (the
    timed loop of a benchmark calls ``run`` with no allocation)."""

    def __init__(self, m, n, device="cuda", B=None, inplace=False, **opts):
        self.m, self.n = int(m), int(n)
        self.dev = torch.device(device)
        self.B = B
        self.opts = _opts(**opts)
        self.spd = _spd(B, self.m) if B is not None else None
        sz = ctypes.c_size_t()
        _check(lib().scqr_workspace_bytes(self.m, self.n, ctypes.byref(self.spd) if self.spd else None,
                                          ctypes.byref(self.opts), ctypes.byref(sz)), "scqr_workspace_bytes")
        self.ws_bytes = sz.value
        self._ws_buf, self.ws = _workspace(self.ws_bytes, self.dev)
        self.Q = None if inplace else torch.empty((self.m, self.n), dtype=torch.float64, device=self.dev)
        self.R = torch.empty((self.n, self.n), dtype=torch.float64, device=self.dev)
        self.info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=self.dev)

    def run(self, X: torch.Tensor):
        xp, ldx = _mat(X, "X")
        if X.shape != (self.m, self.n):
            raise ValueError("X shape does not match the plan")
        Q = X if self.Q is None else self.Q
        qp, ldq = _mat(Q, "Q")
        rp, ldr = _mat(self.R, "R")
        st = lib().scqr_qr(_stream(self.dev), self.m, self.n, xp, ldx,
                           ctypes.byref(self.spd) if self.spd else None, qp, ldq, rp, ldr, self.ws,
                           self.ws_bytes, ctypes.byref(self.opts), self.info.data_ptr())
        _check(st, "scqr_qr")
        return Q, self.R

    def read_info(self) -> Info:
        return decode_info(self.info)


def qr(X: torch.Tensor, B=None, *, inplace=False, check=True, trace=False, **opts):
    """Thin QR X = Q R by shifted Cholesky QR.  Returns (Q, R, info).

    ``check`` (see ``check_mode``): True or "raise" (default) synchronizes the stream, decodes
    ``info`` and raises ScqrError when the factorization failed numerically (breakdown,
    max_passes reached, non-finite Gram); "status" decodes without raising, so that the caller
    inspects ``info.status``; False returns the raw device record without synchronizing.
    ``B = (diag, off)`` selects the oblique inner product with a tridiagonal SPD B, ``B = CsrB(row_ptr,
    col, val)`` with a sparse SPD B in compressed sparse rows.
    ``trace=True`` also returns per-pass input Grams and triangular factors in ``info.trace``
    (shape [passes, 2, n, n]).  ``recompute=True`` (n <= 32, B = I) selects the minimum-traffic
    passes: each pass before the last recomputes its input from X instead of reading a stored
    Q, and only the last pass writes Q (same results bit for bit)."""
    mode = check_mode(check)
    m, n = X.shape
    tr = None
    if trace:
        mp = opts.get("max_passes", 6)
        tr = torch.zeros((max(mp, 3), 2, n, n), dtype=torch.float64, device=X.device)
    plan = Plan(m, n, X.device, B=B, inplace=inplace, trace_ptr=tr.data_ptr() if tr is not None else None,
                **opts)
    Q, R = plan.run(X)
    if mode == "none":
        return Q, R, plan.info
    torch.cuda.current_stream(X.device).synchronize()
    info = plan.read_info()
    if tr is not None:
        info.trace = tr[:max(info.passes, 1)]
    if info.status != OK and mode == "raise":
        raise ScqrError(info.status, f"scqr_qr: {status_string(info.status)}", info, (Q, R))
    return Q, R, info


NOALLOC_SCRATCH_BYTES = 16 << 20


def qr_noalloc(X: torch.Tensor, Q: torch.Tensor, R: torch.Tensor, info: torch.Tensor, B=None, **opts):
    """scqr_qr_noalloc: the factorization into caller-allocated Q (may be X), R and a device
    info record (uint8 tensor of INFO_BYTES), with the library's static device scratch as the
    workspace.  Nothing is allocated on the device and nothing is synchronized; decode the
    record with ``decode_info(info)``.  Shapes whose workspace exceeds the scratch
    (NOALLOC_SCRATCH_BYTES) raise ScqrError with SCQR_E_WORKSPACE."""
    m, n = X.shape
    xp, ldx = _mat(X, "X")
    qp, ldq = _mat(Q, "Q")
    rp, ldr = _mat(R, "R")
    if Q.shape != X.shape or R.shape != (n, n):
        raise ValueError("Q must be m x n and R n x n")
    if info.dtype != torch.uint8 or info.numel() < INFO_BYTES or not info.is_cuda:
        raise TypeError(f"info must be a CUDA uint8 tensor of at least {INFO_BYTES} bytes")
    o = _opts(**opts)
    spd = _spd(B, m) if B is not None else None
    _check(lib().scqr_qr_noalloc(_stream(X.device), m, n, xp, ldx, ctypes.byref(spd) if spd else None,
                                 qp, ldq, rp, ldr, ctypes.byref(o), info.data_ptr()), "scqr_qr_noalloc")
    return Q, R


def gram(X: torch.Tensor, B=None) -> torch.Tensor:
    """G = X^T X (or X^T B X) on the device, both triangles."""
    m, n = X.shape
    xp, ldx = _mat(X, "X")
    spd = _spd(B, m) if B is not None else None
    sz = ctypes.c_size_t()
    _check(lib().scqr_workspace_bytes(max(m, n), n, ctypes.byref(spd) if spd else None, None,
                                      ctypes.byref(sz)), "scqr_workspace_bytes")
    buf, ws = _workspace(sz.value, X.device)
    G = torch.empty((n, n), dtype=torch.float64, device=X.device)
    _check(lib().scqr_gram(_stream(X.device), m, n, xp, ldx, ctypes.byref(spd) if spd else None,
                           G.data_ptr(), n, ws, sz.value), "scqr_gram")
    G._scqr_ws = buf  # keep the workspace alive until the stream has used it
    return G


def trsm(X: torch.Tensor, R: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    """Q = X R^{-1} (row-wise forward substitution, R upper triangular)."""
    m, n = X.shape
    xp, ldx = _mat(X, "X")
    rp, ldr = _mat(R, "R")
    Q = torch.empty((m, n), dtype=torch.float64, device=X.device) if out is None else out
    qp, ldq = _mat(Q, "Q")
    sz = ctypes.c_size_t()
    _check(lib().scqr_workspace_bytes(max(m, n), n, None, None, ctypes.byref(sz)), "scqr_workspace_bytes")
    buf, ws = _workspace(sz.value, X.device)
    _check(lib().scqr_trsm(_stream(X.device), m, n, xp, ldx, rp, ldr, qp, ldq, ws, sz.value), "scqr_trsm")
    Q._scqr_ws = buf
    return Q


NUM_CLASSES = 5
CLASS_WIDTHS = (16, 32, 64, 128, 256)


class _Tuning(ctypes.Structure):
    _fields_ = [("rows_per_task", ctypes.c_int64 * NUM_CLASSES), ("panel_rows", ctypes.c_int32 * NUM_CLASSES),
                ("reserved", ctypes.c_int32 * 3)]


def class_of(n: int) -> int:
    """Width class of an instance: index of the padded width 16, 32, 64, 128 or 256."""
    for c, w in enumerate(CLASS_WIDTHS):
        if n <= w:
            return c
    raise ValueError(f"n = {n} exceeds {CLASS_WIDTHS[-1]}")


def _tuning(t):
    """A scqr_batched_tuning from None, a _Tuning, or a dict {"rows_per_task": [5 ints],
    "panel_rows": [5 ints]} (zeros take the library defaults)."""
    if t is None or isinstance(t, _Tuning):
        return t
    tt = _Tuning()
    for c, v in enumerate(t.get("rows_per_task", [0] * NUM_CLASSES)):
        tt.rows_per_task[c] = int(v)
    for c, v in enumerate(t.get("panel_rows", [0] * NUM_CLASSES)):
        tt.panel_rows[c] = int(v)
    return tt


def tuning_dict(t: _Tuning) -> dict:
    return {"rows_per_task": [int(v) for v in t.rows_per_task], "panel_rows": [int(v) for v in t.panel_rows]}


def _batch_arrays(mats):
    b = len(mats)
    ptrs, lds = [], []
    for M in mats:
        p, ld = _mat(M, "batched matrix")
        ptrs.append(p)
        lds.append(ld)
    return (ctypes.c_void_p * b)(*ptrs), (ctypes.c_int64 * b)(*lds)


def _decode_batch(infos, b, mode, what, result):
    dec = [decode_info(infos[i]) for i in range(b)]
    bad = [i for i, inf in enumerate(dec) if inf.status != OK]
    if bad and mode == "raise":
        raise ScqrError(dec[bad[0]].status, f"{what}: instance {bad[0]} (and {len(bad) - 1} more): "
                        f"{status_string(dec[bad[0]].status)}", dec, result)
    return dec


def qr_batched(Xs, *, inplace=False, check=True, tuning=None, **opts):
    """Factor a list of independent X_i (each m_i x n_i, row-major; a leading dimension larger
    than n_i is allowed).  Returns (Qs, Rs, infos).  ``check`` as in ``qr``: "raise" (default)
    raises ScqrError, with every decoded record in ``.info``, when any instance failed
    numerically; "status" returns the decoded records; False the raw device records.
    ``tuning``: None (library defaults) or a dict as taken by ``_tuning``."""
    mode = check_mode(check)
    if len(Xs) == 0:
        return [], [], []
    dev = Xs[0].device
    b = len(Xs)
    xp, ldx = _batch_arrays(Xs)
    ms = (ctypes.c_int64 * b)(*[int(X.shape[0]) for X in Xs])
    ns = (ctypes.c_int64 * b)(*[int(X.shape[1]) for X in Xs])
    o = _opts(**opts)
    tu = _tuning(tuning)
    sz = ctypes.c_size_t()
    _check(lib().scqr_batched_workspace_bytes(b, ms, ns, ctypes.byref(o), ctypes.byref(tu) if tu else None,
                                              ctypes.byref(sz)), "scqr_batched_workspace_bytes")
    buf, ws = _workspace(sz.value, dev)
    Qs = list(Xs) if inplace else [torch.empty((X.shape[0], X.shape[1]), dtype=torch.float64, device=dev) for X in Xs]
    Rs = [torch.empty((X.shape[1], X.shape[1]), dtype=torch.float64, device=dev) for X in Xs]
    infos = torch.zeros((b, INFO_BYTES), dtype=torch.uint8, device=dev)
    qp, ldq = _batch_arrays(Qs)
    rp, ldr = _batch_arrays(Rs)
    _check(lib().scqr_qr_batched(_stream(dev), b, ms, ns, xp, ldx, qp, ldq, rp, ldr, ws, sz.value,
                                 ctypes.byref(o), ctypes.byref(tu) if tu else None, infos.data_ptr()),
           "scqr_qr_batched")
    if mode == "none":
        return Qs, Rs, (infos, buf)
    torch.cuda.current_stream(dev).synchronize()
    return Qs, Rs, _decode_batch(infos, b, mode, "scqr_qr_batched", (Qs, Rs))


class BatchedPlan:
    """The batched factorization of fixed shapes on fixed buffers, for repeated calls and graph
    capture: workspace, outputs, info records and the library's batched plan (its descriptors
    uploaded to the workspace once).  ``run()`` enqueues kernel launches only, so it may be
    captured in a ``torch.cuda.CUDAGraph`` and replayed.

    The inputs are the tensors ``Xs`` given here (new values are copied into them, e.g. with
    ``X.copy_``), or, when ``Xs`` is None, tensors the plan allocates (``plan.Xs``).  Passing
    other tensors to ``run`` re-binds the plan on the host first (not under capture).
    ``tuning``: None (defaults), a dict (see ``_tuning``), or "auto" to pick it with the
    autotuner (``paper_1809_11085_amd.autotune``: timed trials, cached in a JSON file)."""

    def __init__(self, shapes, device="cuda", inplace=False, Xs=None, tuning=None, **opts):
        self.dev = torch.device(device)
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.b = len(self.shapes)
        if self.b == 0:
            raise ValueError("empty batch")
        self.inplace = inplace
        self.opts_kw = dict(opts)
        self.opts = _opts(**opts)
        if isinstance(tuning, str) and tuning == "auto":
            from . import autotune
            tuning = autotune.tune(self.shapes, device=self.dev, **opts)
        self.tuning = _tuning(tuning)
        self.ms = (ctypes.c_int64 * self.b)(*[m for m, _ in self.shapes])
        self.ns = (ctypes.c_int64 * self.b)(*[n for _, n in self.shapes])
        sz = ctypes.c_size_t()
        _check(lib().scqr_batched_workspace_bytes(self.b, self.ms, self.ns, ctypes.byref(self.opts),
                                                  self._tref(), ctypes.byref(sz)), "scqr_batched_workspace_bytes")
        self.ws_bytes = sz.value
        self._ws_buf, self.ws = _workspace(self.ws_bytes, self.dev)
        if Xs is None:
            Xs = [torch.empty((m, n), dtype=torch.float64, device=self.dev) for m, n in self.shapes]
        self.Rs = [torch.empty((n, n), dtype=torch.float64, device=self.dev) for _, n in self.shapes]
        self.infos = torch.zeros((self.b, INFO_BYTES), dtype=torch.uint8, device=self.dev)
        self._plan = None
        self._bind(Xs)

    def _tref(self):
        return ctypes.byref(self.tuning) if self.tuning is not None else None

    def _bind(self, Xs):
        if len(Xs) != self.b:
            raise ValueError("batch size does not match the plan")
        for X, (m, n) in zip(Xs, self.shapes):
            _mat(X, "X")
            if tuple(X.shape) != (m, n):
                raise ValueError("batched X_i must match the plan's shapes")
        self._destroy()
        self.Xs = list(Xs)
        if self.inplace:
            self.Qs = self.Xs
        elif getattr(self, "Qs", None) is None:
            self.Qs = [torch.empty((m, n), dtype=torch.float64, device=self.dev) for m, n in self.shapes]
        xp, ldx = _batch_arrays(self.Xs)
        qp, ldq = _batch_arrays(self.Qs)
        rp, ldr = _batch_arrays(self.Rs)
        h = ctypes.c_void_p()
        _check(lib().scqr_batched_plan_create(self.b, self.ms, self.ns, xp, ldx, qp, ldq, rp, ldr, self.ws,
                                              self.ws_bytes, ctypes.byref(self.opts), self._tref(),
                                              self.infos.data_ptr(), ctypes.byref(h)), "scqr_batched_plan_create")
        self._plan = h
        _check(lib().scqr_batched_plan_upload(self._plan, _stream(self.dev)), "scqr_batched_plan_upload")
        self._key = tuple(X.data_ptr() for X in self.Xs)

    def run(self, Xs=None):
        """Enqueue the factorization on the current stream; returns (Qs, Rs)."""
        if Xs is not None and tuple(X.data_ptr() for X in Xs) != self._key:
            self._bind(Xs)
        _check(lib().scqr_batched_plan_run(self._plan, _stream(self.dev)), "scqr_batched_plan_run")
        return self.Qs, self.Rs

    def tuning_in_effect(self):
        """(tuning dict, tasks per class) that the library planned."""
        t = _Tuning()
        nt = (ctypes.c_int32 * NUM_CLASSES)()
        _check(lib().scqr_batched_plan_tuning(self._plan, ctypes.byref(t), nt), "scqr_batched_plan_tuning")
        return tuning_dict(t), [int(v) for v in nt]

    def read_infos(self):
        return [decode_info(self.infos[i]) for i in range(self.b)]

    def _destroy(self):
        if getattr(self, "_plan", None) is not None:
            lib().scqr_batched_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self._destroy()
        except Exception:
            pass


def qr_backward(Q: torch.Tensor, R: torch.Tensor, dQ: torch.Tensor = None,
                dR: torch.Tensor = None, out: torch.Tensor = None) -> torch.Tensor:
    """dX = (dQ + Q copyltu(M)) R^{-T}, M = R dR^T - dQ^T Q (None gradients count as zero)."""
    m, n = Q.shape
    qp, ldq = _mat(Q, "Q")
    rp, ldr = _mat(R, "R")
    dqp, lddq = (None, n) if dQ is None else _mat(dQ, "dQ")
    drp, lddr = (None, n) if dR is None else _mat(dR, "dR")
    dX = torch.empty((m, n), dtype=torch.float64, device=Q.device) if out is None else out
    dxp, lddx = _mat(dX, "dX")
    sz = ctypes.c_size_t()
    _check(lib().scqr_backward_workspace_bytes(m, n, ctypes.byref(sz)), "scqr_backward_workspace_bytes")
    buf, ws = _workspace(sz.value, Q.device)
    _check(lib().scqr_qr_backward(_stream(Q.device), m, n, qp, ldq, rp, ldr, dqp, lddq, drp, lddr,
                                  dxp, lddx, ws, sz.value), "scqr_qr_backward")
    dX._scqr_ws = buf
    return dX


class QRFunction(torch.autograd.Function):
    """(Q, R) = QRFunction.apply(X[, opts dict]) with the hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx, X, opts=None):
        Q, R, info = qr(X, **(opts or {}))
        if info.status != OK:
            raise ScqrError(info.status, f"scqr_qr: {status_string(info.status)}")
        ctx.save_for_backward(Q, R)
        return Q, R

    @staticmethod
    def backward(ctx, dQ, dR):
        Q, R = ctx.saved_tensors
        dQc = None if dQ is None else dQ.contiguous()
        dRc = None if dR is None else dR.contiguous()
        return qr_backward(Q, R, dQc, dRc), None


def profile_enable(on: bool = True) -> None:
    _check(lib().scqr_profile_enable(1 if on else 0), "scqr_profile_enable")


def profile_read(capacity: int = 1 << 16) -> list:
    """[(kernel name, ms)] per launch, in enqueue order, since the last read (synchronizes)."""
    arr = (_KernelStat * capacity)()
    cnt = ctypes.c_int32()
    _check(lib().scqr_profile_read(arr, capacity, ctypes.byref(cnt)), "scqr_profile_read")
    return [(arr[i].name.decode(), float(arr[i].total_ms)) for i in range(min(cnt.value, capacity))]


def build_info() -> str:
    return lib().scqr_build_info().decode()


def peak(kind: str, *tensors, variant: int = 0, grid: int = 0, iters: int = 0):
    """Enqueue one device-ceiling kernel on the current stream (no part of a factorization):
    kind "copy" (src, dst), "read" (src, sink), "write" (dst), "mfma" / "fma" (sink)."""
    dev = tensors[0].device
    S = _stream(dev)
    L = lib()
    if kind == "copy":
        src, dst = tensors
        st = L.scqr_peak_copy(S, src.data_ptr(), dst.data_ptr(), min(src.numel(), dst.numel()) * src.element_size(),
                              variant, grid)
    elif kind == "read":
        src, sink = tensors
        if sink.numel() < (grid or 2048) * 256:
            raise ValueError("sink too small")
        st = L.scqr_peak_read(S, src.data_ptr(), src.numel() * src.element_size(), variant, grid, sink.data_ptr())
    elif kind == "write":
        (dst,) = tensors
        st = L.scqr_peak_write(S, dst.data_ptr(), dst.numel() * dst.element_size(), variant, grid)
    elif kind in ("mfma", "fma"):
        (sink,) = tensors
        if sink.numel() < grid * 256:
            raise ValueError("sink too small")
        st = L.scqr_peak_fp64(S, 0 if kind == "mfma" else 1, iters, grid, sink.data_ptr())
    else:
        raise ValueError(kind)
    _check(st, f"scqr_peak_{kind}")
