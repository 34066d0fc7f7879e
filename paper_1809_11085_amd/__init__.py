"""Shifted Cholesky QR on AMD MI355X (gfx950).

Thin Python binding of ``libscqr.so`` (see ``include/scqr.h``): it only marshals arguments
between PyTorch device tensors and the C ABI.  Every step of the factorization runs in the
library's HIP kernels; there is no CPU or PyTorch fallback, and the functions raise if the
library has not been built (``python -m paper_1809_11085_amd.build``).

Functions mirror the C entry points:

* ``qr(X, B=None, **opts) -> (Q, R, info)``  Algorithms 1-3 and 5 of Fukaya et al.
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

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscqr.so")

OK, E_INVALID, E_WORKSPACE, E_UNSUPPORTED, E_HIP, E_BREAKDOWN, E_NOT_CONVERGED, E_NONFINITE = range(8)
SCHEDULES = {"fixed3": 0, "adaptive": 1, "cholqr2": 2, "iterated": 3}
SHIFTS = {"paper": 0, "fro": 1, "small": 2, "custom": 3}
PRECISIONS = {"fp64": 0, "fp32_first": 1}
MAX_PASSES = 16


class ScqrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("shift_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("final_gram", ctypes.c_int32), ("debug_force_breakdown_pass", ctypes.c_int32),
                ("debug_zero_shift", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("custom_alpha", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("trace", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("shifted_mask", ctypes.c_int32), ("breakdown_mask", ctypes.c_int32),
                ("fell_back_fp64", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("shift", ctypes.c_double * MAX_PASSES), ("norm2sq", ctypes.c_double * MAX_PASSES),
                ("gram_dev", ctypes.c_double * MAX_PASSES), ("omega_fro", ctypes.c_double),
                ("bnorm", ctypes.c_double)]


class _SpdOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("diag", ctypes.c_void_p), ("off", ctypes.c_void_p)]


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
        L.scqr_gram.argtypes = [P, I64, I64, P, I64, ctypes.POINTER(_SpdOp), P, I64, P, SZ]
        L.scqr_gram.restype = st
        L.scqr_trsm.argtypes = [P, I64, I64, P, I64, P, I64, P, I64, P, SZ]
        L.scqr_trsm.restype = st
        L.scqr_batched_workspace_bytes.argtypes = [I32, P, P, ctypes.POINTER(_Opts), ctypes.POINTER(SZ)]
        L.scqr_batched_workspace_bytes.restype = st
        L.scqr_qr_batched.argtypes = [P, I32, P, P, P, P, P, P, SZ, ctypes.POINTER(_Opts), P]
        L.scqr_qr_batched.restype = st
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
          debug_zero_shift=False) -> _Opts:
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
    return o


def _spd(B, m: int):
    if B is None:
        return None
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

    @property
    def ok(self) -> bool:
        return self.status == OK


def decode_info(buf: torch.Tensor) -> Info:
    """Copy a device info record (uint8 tensor of INFO_BYTES) to the host and decode it."""
    raw = bytes(buf.detach().to("cpu").numpy().tobytes())
    c = _Info.from_buffer_copy(raw[:INFO_BYTES])
    k = max(c.passes + (1 if c.status == E_BREAKDOWN else 0), 1)
    return Info(c.status, c.passes, c.shifted_mask, c.breakdown_mask, c.fell_back_fp64,
                list(c.shift[:k]), list(c.norm2sq[:k]), list(c.gram_dev[:k]), c.omega_fro, c.bnorm)


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
    """Thin QR X = Q R by shifted Cholesky QR.  Returns (Q, R, info); ``info`` is decoded
    (after a stream synchronisation) when ``check`` is true, and raised on a numerical
    failure; otherwise it is the raw device record.  ``B = (diag, off)`` selects the oblique
    inner product with a tridiagonal SPD B.  ``trace=True`` also returns per-pass input Grams
    and triangular factors in ``info.trace`` (shape [passes, 2, n, n])."""
    m, n = X.shape
    tr = None
    if trace:
        mp = opts.get("max_passes", 6)
        tr = torch.zeros((max(mp, 3), 2, n, n), dtype=torch.float64, device=X.device)
    plan = Plan(m, n, X.device, B=B, inplace=inplace, trace_ptr=tr.data_ptr() if tr is not None else None,
                **opts)
    Q, R = plan.run(X)
    if not check:
        return Q, R, plan.info
    torch.cuda.current_stream(X.device).synchronize()
    info = plan.read_info()
    if tr is not None:
        info.trace = tr[:max(info.passes, 1)]
    if info.status not in (OK,) and check == "raise":
        _check(info.status, "scqr_qr")
    return Q, R, info


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


def qr_batched(Xs, *, inplace=False, check=True, **opts):
    """Factor a list of independent X_i (each m_i x n_i, contiguous).  Returns (Qs, Rs, infos)."""
    if len(Xs) == 0:
        return [], [], []
    dev = Xs[0].device
    b = len(Xs)
    for X in Xs:
        _mat(X, "X")
        if not X.is_contiguous():
            raise ValueError("batched X_i must be contiguous")
    ms = (ctypes.c_int64 * b)(*[int(X.shape[0]) for X in Xs])
    ns = (ctypes.c_int64 * b)(*[int(X.shape[1]) for X in Xs])
    o = _opts(**opts)
    sz = ctypes.c_size_t()
    _check(lib().scqr_batched_workspace_bytes(b, ms, ns, ctypes.byref(o), ctypes.byref(sz)),
           "scqr_batched_workspace_bytes")
    buf, ws = _workspace(sz.value, dev)
    Qs = list(Xs) if inplace else [torch.empty_like(X) for X in Xs]
    Rs = [torch.empty((X.shape[1], X.shape[1]), dtype=torch.float64, device=dev) for X in Xs]
    infos = torch.zeros((b, INFO_BYTES), dtype=torch.uint8, device=dev)
    xp = (ctypes.c_void_p * b)(*[X.data_ptr() for X in Xs])
    qp = (ctypes.c_void_p * b)(*[Q.data_ptr() for Q in Qs])
    rp = (ctypes.c_void_p * b)(*[R.data_ptr() for R in Rs])
    _check(lib().scqr_qr_batched(_stream(dev), b, ms, ns, xp, qp, rp, ws, sz.value, ctypes.byref(o),
                                 infos.data_ptr()), "scqr_qr_batched")
    if not check:
        return Qs, Rs, (infos, buf)
    torch.cuda.current_stream(dev).synchronize()
    return Qs, Rs, [decode_info(infos[i]) for i in range(b)]


class BatchedPlan:
    """Pre-allocated workspace, outputs and pointer tables for repeated batched factorizations
    of one list of shapes (``run`` allocates nothing)."""

    def __init__(self, shapes, device="cuda", inplace=False, **opts):
        self.dev = torch.device(device)
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.b = len(self.shapes)
        self.inplace = inplace
        self.opts = _opts(**opts)
        self.ms = (ctypes.c_int64 * self.b)(*[m for m, _ in self.shapes])
        self.ns = (ctypes.c_int64 * self.b)(*[n for _, n in self.shapes])
        sz = ctypes.c_size_t()
        _check(lib().scqr_batched_workspace_bytes(self.b, self.ms, self.ns, ctypes.byref(self.opts),
                                                  ctypes.byref(sz)), "scqr_batched_workspace_bytes")
        self.ws_bytes = sz.value
        self._ws_buf, self.ws = _workspace(self.ws_bytes, self.dev)
        self.Qs = None if inplace else [torch.empty((m, n), dtype=torch.float64, device=self.dev)
                                        for m, n in self.shapes]
        self.Rs = [torch.empty((n, n), dtype=torch.float64, device=self.dev) for _, n in self.shapes]
        self.infos = torch.zeros((self.b, INFO_BYTES), dtype=torch.uint8, device=self.dev)
        self._rp = (ctypes.c_void_p * self.b)(*[R.data_ptr() for R in self.Rs])
        self._qp = None if inplace else (ctypes.c_void_p * self.b)(*[Q.data_ptr() for Q in self.Qs])
        self._xkey = None

    def run(self, Xs):
        if len(Xs) != self.b:
            raise ValueError("batch size does not match the plan")
        key = tuple(X.data_ptr() for X in Xs)
        if key != self._xkey:
            for X, (m, n) in zip(Xs, self.shapes):
                _mat(X, "X")
                if tuple(X.shape) != (m, n) or not X.is_contiguous():
                    raise ValueError("batched X_i must be contiguous and match the plan's shapes")
            self._xp = (ctypes.c_void_p * self.b)(*key)
            self._xkey = key
        qp = self._xp if self.inplace else self._qp
        _check(lib().scqr_qr_batched(_stream(self.dev), self.b, self.ms, self.ns, self._xp, qp, self._rp,
                                     self.ws, self.ws_bytes, ctypes.byref(self.opts), self.infos.data_ptr()),
               "scqr_qr_batched")
        return (Xs if self.inplace else self.Qs), self.Rs

    def read_infos(self):
        return [decode_info(self.infos[i]) for i in range(self.b)]


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
