"""ctypes binding of ``libccg.so`` (the C ABI of include/ccg.h).

Argument marshalling only: every function here checks that the tensors are
complex128 device tensors of the right shape, passes their data pointers and
the current HIP stream to the entry point of the same name, and turns a
negative or HIP error return into an exception.  All arithmetic runs in the
library's HIP kernels.  There is no fallback: when the library is missing the
call fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

OP_N = 0
OP_C = 1
OP_S = 2  # complex symmetric A read from its upper triangle
WS_MATVEC_C = 1
WS_BICGSTAB = 2
WS_CGNR = 3
WS_MATMAT = 4
WS_BICGSTAB_BLOCK = 5
WS_COCG = 6
WS_COCR = 7
WS_BICGSTAB_MIXED = 8
WS_T3_MATVEC = 9
WS_MATMAT_C64 = 10
WS_BICGSTAB_BLOCK_MIXED = 11
WS_MATVEC_S = 12
WS_SYM = 0x100  # added to WS_BICGSTAB / WS_COCG / WS_COCR with A_SYM_UPPER
X0_ZERO = 1
A_SYM_UPPER = 2  # solver flag: products read only the upper triangle of A
SERVER_REJECTED = -1000
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2

INFO_TEXT = {0: "converged", 1: "iteration budget spent",
             2: "breakdown (rho/sigma or |Ap|/|A^H r| zero)",
             3: "breakdown (omega or t^H t zero)", 4: "non-finite value"}


class CcgError(RuntimeError):
    pass


class _Result(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("confirms", ctypes.c_int32),
                ("relres_rec", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


class _MixedResult(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("matvecs64", ctypes.c_int32),
                ("matvecs32", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("relres_true", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("submitted", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("admission_waits", ctypes.c_int64),
                ("active", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("peak_active", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("pool_used", ctypes.c_uint64), ("pool_peak", ctypes.c_uint64)]


class _EventLog(ctypes.Structure):
    _fields_ = [("events", ctypes.POINTER(ctypes.c_void_p)),
                ("capacity", ctypes.c_int32), ("count", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("seen", ctypes.c_int32),
                ("roles", ctypes.c_uint32), ("pad", ctypes.c_int32)]


PROD_SETUP, PROD_V, PROD_T, PROD_W, PROD_Q, PROD_U = 1, 2, 4, 8, 16, 32


@dataclass
class MixedResult:
    info: int
    outer: int
    inner_iters: int
    matvecs64: int
    matvecs32: int
    relres_true: float
    outer_res: np.ndarray = None  # ||r|| / ||y|| at every outer check (NaN past the last)


@dataclass
class Result:
    info: int
    iters: int
    matvecs: int
    confirms: int
    relres_rec: float
    relres_true: float


_lib = None


def lib_path() -> str:
    return _build.LIB


def load() -> ctypes.CDLL:
    """Load the built library (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime (same soname); load it first so that the
    # library binds to the runtime that owns torch's memory and streams
    _torch()
    path = lib_path()
    if not os.path.exists(path):
        raise CcgError("%s is not built; run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I64, I32, U32, D = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                           ctypes.c_uint32, ctypes.c_double)
    S = ctypes.c_size_t
    lib.ccg_matvec.argtypes = [ctypes.c_int, I64, P, I64, P, P, P]
    lib.ccg_matvec_ex.argtypes = [ctypes.c_int, I64, P, I64, P, P, P, S, P]
    lib.ccg_matvec_noalloc.argtypes = [ctypes.c_int, I64, P, I64, P, P, P]
    lib.ccg_read_stream.argtypes = [P, S, P, S, P]
    lib.ccg_solve_small_batched.argtypes = [ctypes.c_int, I64, I64, P, I64, I64, P, I64,
                                            P, I64, D, I32, U32, P, P]
    lib.ccg_set_event_log.argtypes = [ctypes.POINTER(_EventLog)]
    lib.ccg_workspace_bytes.argtypes = [ctypes.c_int, I64, I64]
    lib.ccg_workspace_bytes.restype = S
    for name in ("ccg_bicgstab", "ccg_cgnr", "ccg_cocg", "ccg_cocr"):
        getattr(lib, name).argtypes = [I64, P, I64, P, P, D, I32,
                                       ctypes.POINTER(I32), P]
    for name in ("ccg_bicgstab_ex", "ccg_cgnr_ex", "ccg_cocg_ex", "ccg_cocr_ex"):
        getattr(lib, name).argtypes = [I64, P, I64, P, P, D, I32, U32, P, S,
                                       ctypes.POINTER(_Result), P, P]
    lib.ccg_bicgstab_mixed_ex.argtypes = [I64, P, I64, P, I64, P, P, D, I32, D, I32,
                                          U32, P, S, ctypes.POINTER(_MixedResult), P, P]
    lib.ccg_round_c64.argtypes = [I64, I64, P, I64, P, I64, P]
    lib.ccg_matvec_c64.argtypes = [I64, P, I64, P, P, P]
    lib.ccg_matmat.argtypes = [I64, I64, P, I64, P, I64, P, I64, P]
    lib.ccg_matmat_ex.argtypes = [I64, I64, P, I64, P, I64, P, I64, P, S, P]
    lib.ccg_bicgstab_block.argtypes = [I64, I64, P, I64, P, I64, P, I64, D, I32,
                                       ctypes.POINTER(I32), P]
    lib.ccg_bicgstab_block_ex.argtypes = [I64, I64, P, I64, P, I64, P, I64, D,
                                          I32, U32, P, S, ctypes.POINTER(_Result),
                                          P]
    lib.ccg_matmat_c64.argtypes = [I64, I64, P, I64, P, I64, P, I64, P, S, P]
    lib.ccg_matmat_c64.restype = ctypes.c_int
    lib.ccg_bicgstab_block_mixed_ex.argtypes = [I64, I64, P, I64, P, I64, P, I64, P, I64,
                                                D, I32, D, I32, U32, P, S,
                                                ctypes.POINTER(_MixedResult), P, P]
    lib.ccg_bicgstab_block_mixed_ex.restype = ctypes.c_int
    lib.ccg_t3_op_bytes.argtypes = [I64]
    lib.ccg_t3_op_bytes.restype = S
    lib.ccg_t3_workspace_bytes.argtypes = [ctypes.c_int, I64]
    lib.ccg_t3_workspace_bytes.restype = S
    lib.ccg_t3_setup.argtypes = [I64, P, P, S, P]
    lib.ccg_t3_matvec.argtypes = [I64, P, P, P, P, S, P]
    for name in ("ccg_t3_bicgstab_ex", "ccg_t3_cocg_ex", "ccg_t3_cocr_ex"):
        getattr(lib, name).argtypes = [I64, P, P, P, D, I32, U32, P, S,
                                       ctypes.POINTER(_Result), P, P]
    for name in ("ccg_t3_setup", "ccg_t3_matvec", "ccg_t3_bicgstab_ex",
                 "ccg_t3_cocg_ex", "ccg_t3_cocr_ex"):
        getattr(lib, name).restype = ctypes.c_int
    lib.ccg_server_create.argtypes = [P, S, I32, P, ctypes.POINTER(P)]
    lib.ccg_server_destroy.argtypes = [P]
    lib.ccg_server_request_bytes.argtypes = [I64, I64]
    lib.ccg_server_request_bytes.restype = S
    lib.ccg_server_submit.argtypes = [P, I64, I64, P, I64, P, I64, P, I64, D, I32,
                                      ctypes.POINTER(I64)]
    lib.ccg_server_submit_mixed.argtypes = [P, I64, I64, P, I64, P, I64, P, I64, D, I32,
                                            D, I32, ctypes.POINTER(I64)]
    lib.ccg_server_request_bytes_mixed.argtypes = [I64, I64]
    lib.ccg_server_request_bytes_mixed.restype = S
    lib.ccg_server_step.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.ccg_server_poll.argtypes = [P, I64, ctypes.POINTER(I32),
                                    ctypes.POINTER(_Result)]
    lib.ccg_server_get_stats.argtypes = [P, ctypes.POINTER(_ServerStats)]
    lib.ccg_server_next_done.argtypes = [P, ctypes.POINTER(I64)]
    for name in ("ccg_server_create", "ccg_server_destroy", "ccg_server_submit",
                 "ccg_server_submit_mixed",
                 "ccg_server_step", "ccg_server_poll", "ccg_server_get_stats",
                 "ccg_server_next_done"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("ccg_matvec", "ccg_matvec_ex", "ccg_bicgstab", "ccg_cgnr",
                 "ccg_bicgstab_ex", "ccg_cgnr_ex", "ccg_matmat", "ccg_matmat_ex",
                 "ccg_bicgstab_block", "ccg_bicgstab_block_ex", "ccg_cocg",
                 "ccg_cocr", "ccg_cocg_ex", "ccg_cocr_ex", "ccg_bicgstab_mixed_ex",
                 "ccg_round_c64", "ccg_matvec_c64"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, name: str):
    if rc < 0:
        raise ValueError("%s: illegal argument %d" % (name, -rc))
    if rc > 0:
        raise CcgError("%s: HIP error %d" % (name, rc))


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _mat(A):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.dtype != torch.complex128 or \
            A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_cuda:
        raise TypeError("A must be a square complex128 CUDA tensor")
    n = A.shape[0]
    if n > 0 and A.stride(1) != 1:
        raise TypeError("A must be row-major (unit column stride)")
    lda = max(A.stride(0), 1) if n > 0 else 1
    return n, lda


def _vec(v, n, what):
    torch = _torch()
    if not isinstance(v, torch.Tensor) or v.dtype != torch.complex128 or \
            not v.is_cuda or v.numel() != n or (n > 0 and not v.is_contiguous()):
        raise TypeError("%s must be a contiguous complex128 CUDA tensor of %d "
                        "elements" % (what, n))
    return v


def ccg_workspace_bytes(method: int, n: int, nrhs: int = 1) -> int:
    return int(load().ccg_workspace_bytes(method, n, nrhs))


def ccg_matvec(op: int, A, x, y=None, stream=None):
    """y = A x (op = OP_N), A^H x (op = OP_C), or A x from the upper triangle
    of a complex symmetric A (op = OP_S); returns y."""
    n, lda = _mat(A)
    _vec(x, n, "x")
    if y is None:
        y = _torch().empty_like(x)
    _vec(y, n, "y")
    _check(load().ccg_matvec(op, n, A.data_ptr(), lda, x.data_ptr(),
                             y.data_ptr(), _stream(stream)), "ccg_matvec")
    return y


def ccg_matvec_ex(op: int, A, x, y, work, stream=None):
    n, lda = _mat(A)
    _vec(x, n, "x")
    _vec(y, n, "y")
    wp = work.data_ptr() if work is not None else None
    wb = work.numel() * work.element_size() if work is not None else 0
    _check(load().ccg_matvec_ex(op, n, A.data_ptr(), lda, x.data_ptr(),
                                y.data_ptr(), wp, wb, _stream(stream)),
           "ccg_matvec_ex")
    return y


def ccg_matvec_noalloc(op: int, A, x, y, stream=None):
    """ccg_matvec with its partial sums in the library's fixed device array
    (no allocation); returns y."""
    n, lda = _mat(A)
    _vec(x, n, "x")
    _vec(y, n, "y")
    _check(load().ccg_matvec_noalloc(op, n, A.data_ptr(), lda, x.data_ptr(),
                                     y.data_ptr(), _stream(stream)),
           "ccg_matvec_noalloc")
    return y


SMALL_MAX_N = 1024


def ccg_solve_small_batched(method: int, A, Y, X, tol=1e-10, maxit=1000, flags=0,
                            res=None, stream=None):
    """BiCGSTAB (method WS_BICGSTAB) or CGNR (WS_CGNR) on a batch of
    independent systems: A (batch, n, n), Y and X (batch, n) complex128
    device tensors (each system's matrix row-major).  res: an optional device
    buffer of batch result records (uint8 tensor of batch * 32 bytes).
    Asynchronous; returns res (read it with small_results)."""
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.dtype != torch.complex128 or A.dim() != 3 \
            or A.shape[1] != A.shape[2] or not A.is_cuda:
        raise TypeError("A must be a (batch, n, n) complex128 CUDA tensor")
    batch, n = A.shape[0], A.shape[1]
    for M, what in ((Y, "Y"), (X, "X")):
        if not isinstance(M, torch.Tensor) or M.dtype != torch.complex128 or \
                not M.is_cuda or tuple(M.shape) != (batch, n) or \
                (n > 0 and M.stride(1) != 1):
            raise TypeError("%s must be a (batch, n) complex128 CUDA tensor with "
                            "contiguous rows" % what)
    if n > 0 and A.stride(2) != 1:
        raise TypeError("A must be row-major within each system")
    lda = max(A.stride(1), 1) if n > 0 else 1
    if res is None:
        res = torch.empty(max(batch, 1) * ctypes.sizeof(_Result), dtype=torch.uint8,
                          device=A.device)
    _check(load().ccg_solve_small_batched(
        int(method), n, batch, A.data_ptr(), lda, A.stride(0), Y.data_ptr(), Y.stride(0),
        X.data_ptr(), X.stride(0), float(tol), int(maxit), int(flags), res.data_ptr(),
        _stream(stream)), "ccg_solve_small_batched")
    return res


def small_results(res, batch):
    """The result records of ccg_solve_small_batched as a list of Result."""
    raw = res[:batch * ctypes.sizeof(_Result)].cpu().numpy().tobytes()
    out = []
    for b in range(batch):
        r = _Result.from_buffer_copy(raw, b * ctypes.sizeof(_Result))
        out.append(Result(r.info, r.iters, r.matvecs, r.confirms, r.relres_rec,
                          r.relres_true))
    return out


READ_STREAM_SLAB = 262144


def ccg_read_stream(src, out=None, stream=None):
    """One read pass over the device tensor src (measurement aid); out: the
    per-slab sums (a complex128 tensor of at least ceil(bytes / slab)
    elements)."""
    torch = _torch()
    if not src.is_cuda or not src.is_contiguous():
        raise TypeError("src must be a contiguous CUDA tensor")
    nbytes = src.numel() * src.element_size()
    if out is None:
        out = torch.empty(max((nbytes + READ_STREAM_SLAB - 1) // READ_STREAM_SLAB, 1),
                          dtype=torch.complex128, device=src.device)
    _check(load().ccg_read_stream(src.data_ptr(), nbytes, out.data_ptr(),
                                  out.numel() * out.element_size(), _stream(stream)),
           "ccg_read_stream")
    return out


# hipEventDisableSystemFence: recording the event does no system-scope
# cache writeback and invalidation, which HIP recommends for events used only
# for timing (the fence would also delay the product the pair brackets).
_HIP_EVENT_DISABLE_SYSTEM_FENCE = 0x20000000


def _hip(lib, name, argtypes):
    """A HIP runtime function looked up through the library's handle, so it
    is the runtime the library (and torch) already use."""
    f = getattr(lib, name)
    f.argtypes = argtypes
    f.restype = ctypes.c_int
    return f


class EventLog:
    """Pairs of timing events recorded by the library around the dense
    complex128 products of the solves this host thread runs while attached
    (ccg_set_event_log); durations() gives each product's time in seconds.
    The events are HIP events created with hipEventDisableSystemFence."""

    def __init__(self, capacity: int, stride: int = 1, roles: int = 0):
        lib = load()
        create = _hip(lib, "hipEventCreateWithFlags",
                      [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint])
        self._elapsed = _hip(lib, "hipEventElapsedTime",
                             [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p])
        self._destroy = _hip(lib, "hipEventDestroy", [ctypes.c_void_p])
        self._events = []
        for _ in range(2 * max(int(capacity), 0)):
            e = ctypes.c_void_p()
            rc = create(ctypes.byref(e), _HIP_EVENT_DISABLE_SYSTEM_FENCE)
            if rc != 0:
                self.close()
                raise CcgError("hipEventCreateWithFlags failed (%d)" % rc)
            self._events.append(e.value)
        self._arr = (ctypes.c_void_p * len(self._events))(*self._events)
        self._log = _EventLog(ctypes.cast(self._arr, ctypes.POINTER(ctypes.c_void_p)),
                              capacity, 0, int(stride), 0, int(roles), 0)

    def close(self):
        """Destroy the events (after the recorded work has completed)."""
        for e in getattr(self, "_events", []):
            self._destroy(ctypes.c_void_p(e))
        self._events = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        self._log.count = 0
        self._log.seen = 0
        _check(load().ccg_set_event_log(ctypes.byref(self._log)), "ccg_set_event_log")
        return self

    def __exit__(self, *exc):
        load().ccg_set_event_log(None)

    @property
    def count(self) -> int:
        return int(self._log.count)

    @property
    def seen(self) -> int:
        return int(self._log.seen)

    def durations(self):
        _torch().cuda.synchronize()
        out = []
        for i in range(self.count):
            ms = ctypes.c_float()
            rc = self._elapsed(ctypes.byref(ms), ctypes.c_void_p(self._events[2 * i]),
                               ctypes.c_void_p(self._events[2 * i + 1]))
            if rc != 0:
                raise CcgError("hipEventElapsedTime failed (%d)" % rc)
            out.append(ms.value / 1e3)
        return out


def _short(name, A, y, x, tol, maxit, stream):
    n, lda = _mat(A)
    _vec(y, n, "y")
    _vec(x, n, "x")
    info = ctypes.c_int32(-1)
    _check(getattr(load(), name)(n, A.data_ptr(), lda, y.data_ptr(),
                                 x.data_ptr(), float(tol), int(maxit),
                                 ctypes.byref(info), _stream(stream)), name)
    return int(info.value)


def ccg_bicgstab(A, y, x, tol=1e-10, maxit=1000, stream=None) -> int:
    """BiCGSTAB on A x = y, x in/out; returns info."""
    return _short("ccg_bicgstab", A, y, x, tol, maxit, stream)


def ccg_cgnr(A, y, x, tol=1e-10, maxit=1000, stream=None) -> int:
    """CGNR on A x = y, x in/out; returns info."""
    return _short("ccg_cgnr", A, y, x, tol, maxit, stream)


def workspace(method: int, n: int, device=None):
    """Device workspace tensor (uint8) of the size the method needs."""
    torch = _torch()
    nbytes = max(ccg_workspace_bytes(method, n), 256)
    return torch.empty(nbytes, dtype=torch.uint8,
                       device=device or torch.device("cuda"))


def new_hist(maxit: int, device=None):
    """Per-iteration record (maxit x 8 float64 on the device, NaN-filled);
    columns alpha re/im, omega re/im, beta re/im, res_half, res_full."""
    torch = _torch()
    return torch.full((max(maxit, 1), 8), float("nan"), dtype=torch.float64,
                      device=device or torch.device("cuda"))


def _ex(name, method, A, y, x, tol, maxit, flags, work, hist, stream):
    n, lda = _mat(A)
    _vec(y, n, "y")
    _vec(x, n, "x")
    if work is None:
        work = workspace(method | (WS_SYM if flags & A_SYM_UPPER else 0), n,
                         A.device)
    res = _Result()
    _check(getattr(load(), name)(
        n, A.data_ptr(), lda, y.data_ptr(), x.data_ptr(), float(tol),
        int(maxit), int(flags), work.data_ptr(),
        work.numel() * work.element_size(), ctypes.byref(res),
        hist.data_ptr() if hist is not None else None, _stream(stream)), name)
    return Result(res.info, res.iters, res.matvecs, res.confirms,
                  res.relres_rec, res.relres_true)


def ccg_bicgstab_ex(A, y, x, tol=1e-10, maxit=1000, flags=0, work=None,
                    hist=None, stream=None) -> Result:
    return _ex("ccg_bicgstab_ex", WS_BICGSTAB, A, y, x, tol, maxit, flags,
               work, hist, stream)


def ccg_cgnr_ex(A, y, x, tol=1e-10, maxit=1000, flags=0, work=None,
                hist=None, stream=None) -> Result:
    return _ex("ccg_cgnr_ex", WS_CGNR, A, y, x, tol, maxit, flags, work, hist,
               stream)


def ccg_cocg(A, y, x, tol=1e-10, maxit=1000, stream=None) -> int:
    """COCG on complex symmetric A x = y, x in/out; returns info."""
    return _short("ccg_cocg", A, y, x, tol, maxit, stream)


def ccg_cocr(A, y, x, tol=1e-10, maxit=1000, stream=None) -> int:
    """COCR on complex symmetric A x = y, x in/out; returns info."""
    return _short("ccg_cocr", A, y, x, tol, maxit, stream)


def ccg_cocg_ex(A, y, x, tol=1e-10, maxit=1000, flags=0, work=None,
                hist=None, stream=None) -> Result:
    return _ex("ccg_cocg_ex", WS_COCG, A, y, x, tol, maxit, flags, work, hist,
               stream)


def ccg_cocr_ex(A, y, x, tol=1e-10, maxit=1000, flags=0, work=None,
                hist=None, stream=None) -> Result:
    return _ex("ccg_cocr_ex", WS_COCR, A, y, x, tol, maxit, flags, work, hist,
               stream)


def ccg_matvec_c64(A32, x, y=None, stream=None):
    """y = A32 x in complex64 (FP32 accumulation)."""
    torch = _torch()
    if not isinstance(A32, torch.Tensor) or A32.dtype != torch.complex64 or \
            A32.dim() != 2 or A32.shape[0] != A32.shape[1] or not A32.is_cuda:
        raise TypeError("A32 must be a square complex64 CUDA tensor")
    n = A32.shape[0]
    if n > 0 and A32.stride(1) != 1:
        raise TypeError("A32 must be row-major")
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex64 or \
            x.numel() != n or not x.is_cuda:
        raise TypeError("x must be a complex64 CUDA tensor of n elements")
    if y is None:
        y = torch.empty_like(x)
    _check(load().ccg_matvec_c64(n, A32.data_ptr(), max(A32.stride(0), 1) if n else 1,
                                 x.data_ptr(), y.data_ptr(), _stream(stream)),
           "ccg_matvec_c64")
    return y


def ccg_round_c64(src, dst=None, stream=None):
    """dst = complex64(src) for a 2-D row-major complex128 tensor."""
    torch = _torch()
    if not isinstance(src, torch.Tensor) or src.dtype != torch.complex128 or \
            not src.is_cuda or src.dim() != 2:
        raise TypeError("src must be a 2-D complex128 CUDA tensor")
    rows, cols = src.shape
    if dst is None:
        dst = torch.empty((rows, cols), dtype=torch.complex64, device=src.device)
    if dst.dtype != torch.complex64 or tuple(dst.shape) != (rows, cols):
        raise TypeError("dst must be a complex64 tensor of the same shape")
    lds = max(src.stride(0), cols, 1)
    ldd = max(dst.stride(0), cols, 1)
    _check(load().ccg_round_c64(rows, cols, src.data_ptr(), lds, dst.data_ptr(),
                                ldd, _stream(stream)), "ccg_round_c64")
    return dst


def ccg_bicgstab_mixed_ex(A, A32, y, x, tol=1e-10, maxit=10, tol_inner=1e-5,
                          maxit_inner=1000, flags=0, work=None,
                          stream=None) -> MixedResult:
    """FP64 refinement around an inner complex64 BiCGSTAB; x in/out."""
    torch = _torch()
    n, lda = _mat(A)
    if not isinstance(A32, torch.Tensor) or A32.dtype != torch.complex64 or \
            tuple(A32.shape) != (n, n) or not A32.is_cuda or \
            (n > 0 and A32.stride(1) != 1):
        raise TypeError("A32 must be an n x n row-major complex64 CUDA tensor")
    lda32 = max(A32.stride(0), 1) if n > 0 else 1
    _vec(y, n, "y")
    _vec(x, n, "x")
    if work is None:
        nbytes = max(ccg_workspace_bytes(WS_BICGSTAB_MIXED, n), 256)
        work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    res = _MixedResult()
    orr = np.full(max(int(maxit), 0) + 1, np.nan)
    _check(load().ccg_bicgstab_mixed_ex(
        n, A.data_ptr(), lda, A32.data_ptr(), lda32, y.data_ptr(), x.data_ptr(),
        float(tol), int(maxit), float(tol_inner), int(maxit_inner), int(flags),
        work.data_ptr(), work.numel() * work.element_size(), ctypes.byref(res),
        orr.ctypes.data if maxit >= 0 else None, _stream(stream)), "ccg_bicgstab_mixed_ex")
    return MixedResult(res.info, res.outer, res.inner_iters, res.matvecs64,
                       res.matvecs32, res.relres_true, orr)


def hist_numpy(hist) -> np.ndarray:
    return hist.detach().cpu().numpy()


def _rect(M, n, what):
    torch = _torch()
    if not isinstance(M, torch.Tensor) or M.dtype != torch.complex128 or \
            not M.is_cuda or M.dim() != 2 or M.shape[0] != n:
        raise TypeError("%s must be an n x k complex128 CUDA tensor" % what)
    if M.shape[1] > 0 and M.shape[0] > 0 and M.stride(1) != 1:
        raise TypeError("%s must be row-major (unit column stride)" % what)
    return M.shape[1], max(M.stride(0), M.shape[1], 1)


def ccg_matmat(A, B, Z=None, work=None, stream=None):
    """Z = A B for an n x k block B (FP64 matrix cores); returns Z."""
    n, lda = _mat(A)
    k, ldb = _rect(B, n, "B")
    if Z is None:
        Z = _torch().empty((n, k), dtype=B.dtype, device=B.device)
    kz, ldz = _rect(Z, n, "Z")
    if kz != k:
        raise TypeError("Z must have as many columns as B")
    if work is None:
        rc = load().ccg_matmat(n, k, A.data_ptr(), lda, B.data_ptr(), ldb,
                               Z.data_ptr(), ldz, _stream(stream))
    else:
        rc = load().ccg_matmat_ex(n, k, A.data_ptr(), lda, B.data_ptr(), ldb,
                                  Z.data_ptr(), ldz, work.data_ptr(),
                                  work.numel() * work.element_size(),
                                  _stream(stream))
    _check(rc, "ccg_matmat")
    return Z


def ccg_bicgstab_block(A, Y, X, tol=1e-10, maxit=1000, stream=None):
    """Block BiCGSTAB on A X = Y (n x k, k <= 64); X in/out; returns the k
    info codes."""
    n, lda = _mat(A)
    k, ldy = _rect(Y, n, "Y")
    kx, ldx = _rect(X, n, "X")
    if kx != k:
        raise TypeError("X must have as many columns as Y")
    info = (ctypes.c_int32 * max(k, 1))()
    _check(load().ccg_bicgstab_block(n, k, A.data_ptr(), lda, Y.data_ptr(), ldy,
                                     X.data_ptr(), ldx, float(tol), int(maxit),
                                     info, _stream(stream)),
           "ccg_bicgstab_block")
    return [int(info[j]) for j in range(k)]


def ccg_bicgstab_block_ex(A, Y, X, tol=1e-10, maxit=1000, flags=0, work=None,
                          stream=None):
    """Block BiCGSTAB with caller workspace and flags; returns k Results."""
    n, lda = _mat(A)
    k, ldy = _rect(Y, n, "Y")
    kx, ldx = _rect(X, n, "X")
    if kx != k:
        raise TypeError("X must have as many columns as Y")
    if work is None:
        torch = _torch()
        nbytes = max(ccg_workspace_bytes(WS_BICGSTAB_BLOCK, n, max(k, 1)), 256)
        work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    res = (_Result * max(k, 1))()
    _check(load().ccg_bicgstab_block_ex(
        n, k, A.data_ptr(), lda, Y.data_ptr(), ldy, X.data_ptr(), ldx,
        float(tol), int(maxit), int(flags), work.data_ptr(),
        work.numel() * work.element_size(), res, _stream(stream)),
        "ccg_bicgstab_block_ex")
    return [Result(r.info, r.iters, r.matvecs, r.confirms, r.relres_rec,
                   r.relres_true) for r in list(res)[:k]]


class Rejected(CcgError):
    """The request's footprint exceeds the server's whole pool."""


def ccg_server_request_bytes(n: int, k: int, mixed: bool = False) -> int:
    if mixed:
        return int(load().ccg_server_request_bytes_mixed(n, k))
    return int(load().ccg_server_request_bytes(n, k))


def _serve_mat(M, rows, what, square=False):
    torch = _torch()
    if not isinstance(M, torch.Tensor) or M.dtype != torch.complex128 or \
            M.dim() != 2 or M.shape[0] != rows or (square and M.shape[1] != rows):
        raise TypeError("%s must be a complex128 tensor with %d rows" % (what, rows))
    if M.numel() > 0 and M.stride(1) != 1:
        raise TypeError("%s must be row-major (unit column stride)" % what)
    return max(M.stride(0), M.shape[1], 1)


class Server:
    """Continuous-batching server of block BiCGSTAB requests (the
    ccg_server_* entry points).  ``pool`` is a device uint8 tensor or a byte
    count (then allocated here).  Tensors of a request may live on the device
    or in host memory; the server keeps references to them until the request
    is reported done."""

    def __init__(self, pool, max_active=64, stream=None):
        torch = _torch()
        if isinstance(pool, int):
            pool = torch.empty(pool, dtype=torch.uint8, device="cuda")
        self.pool = pool
        self._stream = _stream(stream)
        h = ctypes.c_void_p()
        _check(load().ccg_server_create(pool.data_ptr(), pool.numel(),
                                        int(max_active), self._stream,
                                        ctypes.byref(h)), "ccg_server_create")
        self._h = h
        self._keep = {}

    def submit(self, A, Y, X, tol=1e-10, maxit=1000, mixed=False, tol_inner=1e-5,
               maxit_inner=1000) -> int:
        """Queue a request; mixed: FP64 refinement around inner solves on the
        server's complex64 copy of A (maxit then counts outer steps)."""
        n = A.shape[0] if hasattr(A, "shape") else 0
        lda = _serve_mat(A, n, "A", square=True)
        ldy = _serve_mat(Y, n, "Y")
        ldx = _serve_mat(X, n, "X")
        k = Y.shape[1]
        if X.shape[1] != k:
            raise TypeError("X must have as many columns as Y")
        t = ctypes.c_int64(0)
        if mixed:
            rc = load().ccg_server_submit_mixed(self._h, n, k, A.data_ptr(), lda,
                                                Y.data_ptr(), ldy, X.data_ptr(), ldx,
                                                float(tol), int(maxit), float(tol_inner),
                                                int(maxit_inner), ctypes.byref(t))
        else:
            rc = load().ccg_server_submit(self._h, n, k, A.data_ptr(), lda,
                                          Y.data_ptr(), ldy, X.data_ptr(), ldx,
                                          float(tol), int(maxit), ctypes.byref(t))
        if rc == SERVER_REJECTED:
            raise Rejected("request of n=%d, k=%d does not fit the pool" % (n, k))
        _check(rc, "ccg_server_submit")
        self._keep[t.value] = (A, Y, X, k)
        return int(t.value)

    def step(self):
        a = ctypes.c_int32(0)
        q = ctypes.c_int32(0)
        _check(load().ccg_server_step(self._h, ctypes.byref(a), ctypes.byref(q)),
               "ccg_server_step")
        return int(a.value), int(q.value)

    def poll(self, ticket):
        """(state, results): results is the list of k Results once done."""
        k = self._keep[ticket][3]
        st = ctypes.c_int32(-1)
        res = (_Result * k)()
        _check(load().ccg_server_poll(self._h, ticket, ctypes.byref(st), res),
               "ccg_server_poll")
        if st.value != REQ_DONE:
            return int(st.value), None
        del self._keep[ticket]
        return REQ_DONE, [Result(r.info, r.iters, r.matvecs, r.confirms,
                                 r.relres_rec, r.relres_true) for r in res]

    def next_done(self) -> int:
        """Ticket of a finished request not handed out before, or 0."""
        t = ctypes.c_int64(0)
        _check(load().ccg_server_next_done(self._h, ctypes.byref(t)),
               "ccg_server_next_done")
        return int(t.value)

    def stats(self) -> dict:
        o = _ServerStats()
        _check(load().ccg_server_get_stats(self._h, ctypes.byref(o)),
               "ccg_server_get_stats")
        return {f: int(getattr(o, f)) for f, _ in o._fields_ if f != "pad"}

    def run_all(self, tickets):
        """Step until every ticket is done; returns {ticket: results}.
        Finished tickets outside ``tickets`` are handed out and dropped."""
        out = {}
        left = set(tickets)
        while left:
            self.step()
            while True:
                t = self.next_done()
                if not t:
                    break
                if t in left:
                    out[t] = self.poll(t)[1]
                    left.discard(t)
        return out

    def close(self):
        if self._h:
            _check(load().ccg_server_destroy(self._h), "ccg_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _rect64(M, n, what):
    torch = _torch()
    if not isinstance(M, torch.Tensor) or M.dtype != torch.complex64 or \
            not M.is_cuda or M.dim() != 2 or M.shape[0] != n:
        raise TypeError("%s must be an n x n complex64 CUDA tensor" % what)
    if M.numel() > 0 and M.stride(1) != 1:
        raise TypeError("%s must be row-major" % what)
    return max(M.stride(0), M.shape[1], 1)


def ccg_matmat_c64(A32, B, Z=None, work=None, stream=None):
    """Z = A32 B (A32 complex64, B rounded to complex64, FP32 accumulation on
    the matrix cores, FP64 slice sums); B and Z complex128."""
    torch = _torch()
    n = A32.shape[0]
    lda32 = _rect64(A32, n, "A32")
    k, ldb = _rect(B, n, "B")
    if Z is None:
        Z = torch.empty((n, k), dtype=torch.complex128, device=B.device)
    kz, ldz = _rect(Z, n, "Z")
    if kz != k:
        raise TypeError("Z must have as many columns as B")
    if work is None:
        work = torch.empty(max(ccg_workspace_bytes(WS_MATMAT_C64, n, max(k, 1)), 256),
                           dtype=torch.uint8, device=B.device)
    _check(load().ccg_matmat_c64(n, k, A32.data_ptr(), lda32, B.data_ptr(), ldb,
                                 Z.data_ptr(), ldz, work.data_ptr(),
                                 work.numel() * work.element_size(), _stream(stream)),
           "ccg_matmat_c64")
    return Z


def ccg_bicgstab_block_mixed_ex(A, A32, Y, X, tol=1e-10, maxit=10, tol_inner=1e-5,
                                maxit_inner=1000, flags=0, work=None, stream=None):
    """Mixed-precision block BiCGSTAB (k <= 64 columns); X in/out; returns k
    MixedResults."""
    torch = _torch()
    n, lda = _mat(A)
    lda32 = _rect64(A32, n, "A32")
    k, ldy = _rect(Y, n, "Y")
    kx, ldx = _rect(X, n, "X")
    if kx != k:
        raise TypeError("X must have as many columns as Y")
    if work is None:
        work = torch.empty(max(ccg_workspace_bytes(WS_BICGSTAB_BLOCK_MIXED, n, max(k, 1)), 256),
                           dtype=torch.uint8, device=A.device)
    res = (_MixedResult * max(k, 1))()
    orr = np.full((max(k, 1), max(int(maxit), 0) + 1), np.nan)
    _check(load().ccg_bicgstab_block_mixed_ex(
        n, k, A.data_ptr(), lda, A32.data_ptr(), lda32, Y.data_ptr(), ldy, X.data_ptr(), ldx,
        float(tol), int(maxit), float(tol_inner), int(maxit_inner), int(flags),
        work.data_ptr(), work.numel() * work.element_size(), res,
        orr.ctypes.data if maxit >= 0 else None, _stream(stream)),
        "ccg_bicgstab_block_mixed_ex")
    return [MixedResult(r.info, r.outer, r.inner_iters, r.matvecs64, r.matvecs32,
                        r.relres_true, orr[c]) for c, r in enumerate(list(res)[:k])]


# ------------------------------------------------ structured lattice operator

def ccg_t3_op_bytes(m: int) -> int:
    return int(load().ccg_t3_op_bytes(m))


def ccg_t3_workspace_bytes(method: int, m: int) -> int:
    return int(load().ccg_t3_workspace_bytes(method, m))


class T3Operator:
    """Three-level Toeplitz operator of an m^3 lattice (ccg_t3_setup): holds
    the transformed kernel on the device.  ``table`` is the (2m-1)^3 kernel
    (complex128, host array or device tensor) in the layout of
    ``inputs.lattice_table``."""

    def __init__(self, m: int, table, stream=None):
        torch = _torch()
        self.m = int(m)
        self.n = self.m ** 3
        w = 2 * self.m - 1
        if not isinstance(table, torch.Tensor):
            table = torch.from_numpy(np.ascontiguousarray(table))
        table = table.to("cuda").contiguous()
        if table.dtype != torch.complex128 or table.numel() != w ** 3:
            raise TypeError("table must hold (2m-1)^3 complex128 values")
        nb = ccg_t3_op_bytes(self.m)
        if nb == 0:
            raise ValueError("lattice edge m=%d out of range (1..128)" % self.m)
        self.op = torch.empty(nb, dtype=torch.uint8, device="cuda")
        _check(load().ccg_t3_setup(self.m, table.data_ptr(), self.op.data_ptr(), nb,
                                   _stream(stream)), "ccg_t3_setup")
        self._table = table  # kept until the set-up has run
        self._work = None

    def workspace(self, method: int):
        torch = _torch()
        return torch.empty(max(ccg_t3_workspace_bytes(method, self.m), 256),
                           dtype=torch.uint8, device="cuda")

    def matvec(self, x, y=None, work=None, stream=None):
        """y = A x (x, y complex128 device vectors of m^3 elements)."""
        _vec(x, self.n, "x")
        if y is None:
            y = _torch().empty_like(x)
        _vec(y, self.n, "y")
        if work is None:
            if self._work is None:
                self._work = self.workspace(WS_T3_MATVEC)
            work = self._work
        _check(load().ccg_t3_matvec(self.m, self.op.data_ptr(), x.data_ptr(),
                                    y.data_ptr(), work.data_ptr(),
                                    work.numel() * work.element_size(),
                                    _stream(stream)), "ccg_t3_matvec")
        return y

    def _solve(self, name, method, y, x, tol, maxit, flags, work, hist, stream):
        _vec(y, self.n, "y")
        _vec(x, self.n, "x")
        if work is None:
            work = self.workspace(method)
        res = _Result()
        _check(getattr(load(), name)(
            self.m, self.op.data_ptr(), y.data_ptr(), x.data_ptr(), float(tol),
            int(maxit), int(flags), work.data_ptr(),
            work.numel() * work.element_size(), ctypes.byref(res),
            hist.data_ptr() if hist is not None else None, _stream(stream)), name)
        return Result(res.info, res.iters, res.matvecs, res.confirms,
                      res.relres_rec, res.relres_true)

    def bicgstab(self, y, x, tol=1e-10, maxit=1000, flags=0, work=None, hist=None,
                 stream=None) -> Result:
        return self._solve("ccg_t3_bicgstab_ex", WS_BICGSTAB, y, x, tol, maxit, flags,
                           work, hist, stream)

    def cocg(self, y, x, tol=1e-10, maxit=1000, flags=0, work=None, hist=None,
             stream=None) -> Result:
        return self._solve("ccg_t3_cocg_ex", WS_COCG, y, x, tol, maxit, flags, work,
                           hist, stream)

    def cocr(self, y, x, tol=1e-10, maxit=1000, flags=0, work=None, hist=None,
             stream=None) -> Result:
        return self._solve("ccg_t3_cocr_ex", WS_COCR, y, x, tol, maxit, flags, work,
                           hist, stream)
