"""CPU oracle of the complex Krylov solvers -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never imports it,
and it never imports the product library.

It wraps ``ccg_oracle.c`` (plain sequential complex128 C, built with gcc and
``-ffp-contract=off``) through ctypes.  The C file documents what each routine
follows in the paper (Introduction: the problem A x = y; section 2.1: the
bicgstab and cgnr methods of the PIM90 set; section 3.4: COCR and COCG for
complex symmetric systems; Usage: matvec / cmatvec kept apart from the
iteration, tolerance epsilon_err and budget maxit).

Parity status: pinned for every routine (see tests/test_oracle_*.py: dense LU,
closed forms, finite termination, exact integer products, invariants, third
party cross-check, planted-mistake detection).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ccg_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "liboracle.so")

X0_ZERO = 1

LIB_OMP = os.path.join(BUILD_DIR, "liboracle_omp.so")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wno-unknown-pragmas",
          "-Werror=implicit-function-declaration",
          "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(src: str = SRC, out: str = LIB, openmp: bool = False) -> str:
    """Compile the oracle with gcc into ``out`` (always recompiles).  openmp:
    the timing-only build that shares the rows of the dense product among
    threads (same results bit for bit)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    extra = ["-fopenmp"] if openmp else []
    subprocess.run(["gcc", *CFLAGS, *extra, src, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build_all() -> None:
    """Both builds: the one-thread oracle and its OpenMP timing build."""
    build()
    build(out=LIB_OMP, openmp=True)


class _Stats(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("confirms", ctypes.c_int32),
                ("relres_rec", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


class _MixedStats(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("matvecs64", ctypes.c_int32),
                ("matvecs32", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("relres_true", ctypes.c_double)]


@dataclass
class MixedResult:
    x: np.ndarray
    info: int
    outer: int
    inner_iters: int
    matvecs64: int
    matvecs32: int
    relres_true: float
    outer_res: np.ndarray  # ||r|| / ||y|| at each outer check


HIST_FIELDS = ("alpha_re", "alpha_im", "omega_re", "omega_im", "beta_re",
               "beta_im", "res_half", "res_full")


@dataclass
class Result:
    x: np.ndarray
    info: int
    iters: int
    matvecs: int
    confirms: int
    relres_rec: float
    relres_true: float
    hist: np.ndarray  # (maxit, 8) float64, columns HIST_FIELDS

    def alpha(self):
        return self.hist[:, 0] + 1j * self.hist[:, 1]

    def omega(self):
        return self.hist[:, 2] + 1j * self.hist[:, 3]

    def beta(self):
        return self.hist[:, 4] + 1j * self.hist[:, 5]


class Oracle:
    """ctypes handle on one built copy of the oracle library."""

    def __init__(self, path: str | None = None):
        if path is None:
            path = LIB
            if not os.path.exists(path) or (
                    os.path.getmtime(path) < os.path.getmtime(SRC)):
                build()
        self.path = path
        self.lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        self.lib.oracle_threads.argtypes = [ctypes.c_int]
        self.lib.oracle_threads.restype = ctypes.c_int
        self.lib.oracle_matvec_c64.argtypes = [I64, P, I64, P, P]
        self.lib.oracle_matvec_c64.restype = None
        self.lib.oracle_bicgstab_mixed.argtypes = [
            I64, P, I64, P, I64, P, P, ctypes.c_double, ctypes.c_int32,
            ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
            ctypes.POINTER(_MixedStats), P]
        self.lib.oracle_bicgstab_mixed.restype = ctypes.c_int
        self.lib.oracle_bicgstab_mixed_wide.argtypes = \
            self.lib.oracle_bicgstab_mixed.argtypes
        self.lib.oracle_bicgstab_mixed_wide.restype = ctypes.c_int
        self.lib.oracle_matvec_c64_wide.argtypes = [I64, P, I64, P, P]
        self.lib.oracle_matvec_c64_wide.restype = None
        for name in ("oracle_matvec", "oracle_matvec_h", "oracle_matvec_sym_upper"):
            f = getattr(self.lib, name)
            f.argtypes = [I64, P, I64, P, P]
            f.restype = None
        for name in ("oracle_bicgstab", "oracle_cgnr", "oracle_cg",
                     "oracle_cocg", "oracle_cocr"):
            f = getattr(self.lib, name)
            f.argtypes = [I64, P, I64, P, P, ctypes.c_double, ctypes.c_int32,
                          ctypes.c_uint32, ctypes.POINTER(_Stats), P]
            f.restype = ctypes.c_int

    # -- products ---------------------------------------------------------
    @staticmethod
    def _mat(A):
        A = np.asarray(A)
        if A.dtype != np.complex128 or A.ndim != 2 or A.shape[0] != A.shape[1]:
            raise TypeError("A must be a square complex128 matrix")
        if A.shape[0] == 0:
            return A, 1
        if A.strides[1] != 16:
            raise TypeError("A must have unit column stride (row-major)")
        return A, A.strides[0] // 16

    def matvec(self, A, x):
        A, lda = self._mat(A)
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.empty(A.shape[0], dtype=np.complex128)
        self.lib.oracle_matvec(A.shape[0], A.ctypes.data, lda, x.ctypes.data,
                               y.ctypes.data)
        return y

    def matvec_sym_upper(self, A, x):
        """A x for complex symmetric A read from its upper triangle only."""
        A, lda = self._mat(A)
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.empty(A.shape[0], dtype=np.complex128)
        self.lib.oracle_matvec_sym_upper(A.shape[0], A.ctypes.data, lda,
                                         x.ctypes.data, y.ctypes.data)
        return y

    def matvec_h(self, A, x):
        A, lda = self._mat(A)
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.empty(A.shape[0], dtype=np.complex128)
        self.lib.oracle_matvec_h(A.shape[0], A.ctypes.data, lda, x.ctypes.data,
                                 y.ctypes.data)
        return y

    # -- solvers ----------------------------------------------------------
    def _solve(self, fn, A, y, x0, tol, maxit, flags):
        A, lda = self._mat(A)
        n = A.shape[0]
        y = np.ascontiguousarray(y, dtype=np.complex128)
        if x0 is None:
            x = np.zeros(n, dtype=np.complex128)
            flags |= X0_ZERO
        else:
            x = np.array(x0, dtype=np.complex128, copy=True)
        hist = np.full((max(maxit, 0), 8), np.nan)
        st = _Stats()
        rc = fn(n, A.ctypes.data, lda, y.ctypes.data, x.ctypes.data,
                float(tol), int(maxit), int(flags), ctypes.byref(st),
                hist.ctypes.data if maxit > 0 else None)
        if rc != 0:
            raise ValueError("oracle argument error %d" % rc)
        return Result(x, st.info, st.iters, st.matvecs, st.confirms,
                      st.relres_rec, st.relres_true, hist)

    def bicgstab(self, A, y, x0=None, tol=1e-10, maxit=1000, flags=0):
        return self._solve(self.lib.oracle_bicgstab, A, y, x0, tol, maxit,
                           flags)

    def cgnr(self, A, y, x0=None, tol=1e-10, maxit=1000, flags=0):
        return self._solve(self.lib.oracle_cgnr, A, y, x0, tol, maxit, flags)

    def cg(self, A, y, x0=None, tol=1e-10, maxit=1000, flags=0):
        return self._solve(self.lib.oracle_cg, A, y, x0, tol, maxit, flags)

    def cocg(self, A, y, x0=None, tol=1e-10, maxit=1000, flags=0):
        return self._solve(self.lib.oracle_cocg, A, y, x0, tol, maxit, flags)

    def cocr(self, A, y, x0=None, tol=1e-10, maxit=1000, flags=0):
        return self._solve(self.lib.oracle_cocr, A, y, x0, tol, maxit, flags)

    # -- mixed precision -----------------------------------------------------
    def matvec_c64(self, A32, x):
        A32 = np.asarray(A32)
        if A32.dtype != np.complex64 or A32.strides[1] != 8:
            raise TypeError("A32 must be a row-major complex64 matrix")
        x = np.ascontiguousarray(x, dtype=np.complex64)
        y = np.empty(A32.shape[0], dtype=np.complex64)
        self.lib.oracle_matvec_c64(A32.shape[0], A32.ctypes.data, A32.strides[0] // 8,
                                   x.ctypes.data, y.ctypes.data)
        return y

    def matvec_c64_wide(self, A32, x):
        """The complex64 product of a complex128 vector (x rounded to
        complex64, FP32 row sums widened to complex128)."""
        A32 = np.asarray(A32)
        if A32.dtype != np.complex64 or A32.strides[1] != 8:
            raise TypeError("A32 must be a row-major complex64 matrix")
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.empty(A32.shape[0], dtype=np.complex128)
        self.lib.oracle_matvec_c64_wide(A32.shape[0], A32.ctypes.data, A32.strides[0] // 8,
                                        x.ctypes.data, y.ctypes.data)
        return y

    def bicgstab_mixed(self, A, y, A32=None, x0=None, tol=1e-10, maxit=10,
                       tol_inner=1e-5, maxit_inner=1000):
        """FP64 refinement around an inner complex64 BiCGSTAB.  A32 defaults
        to A rounded to complex64."""
        return self._mixed(self.lib.oracle_bicgstab_mixed, A, y, A32, x0, tol, maxit,
                           tol_inner, maxit_inner)

    def bicgstab_mixed_wide(self, A, y, A32=None, x0=None, tol=1e-10, maxit=10,
                            tol_inner=1e-5, maxit_inner=1000):
        """FP64 refinement around an inner BiCGSTAB whose Krylov vectors stay
        complex128 and whose products are complex64 (the form of the solver
        for many right-hand sides)."""
        return self._mixed(self.lib.oracle_bicgstab_mixed_wide, A, y, A32, x0, tol, maxit,
                           tol_inner, maxit_inner)

    def bicgstab_block_mixed(self, A, Y, A32=None, X0=None, tol=1e-10, maxit=10,
                             tol_inner=1e-5, maxit_inner=1000, cols=None):
        """Each column of Y by its own bicgstab_mixed_wide (per-column
        refinement decisions); cols selects a subset."""
        Y = np.asarray(Y)
        cols = range(Y.shape[1]) if cols is None else cols
        if A32 is None:
            A32 = np.asarray(A).astype(np.complex64)
        return [self.bicgstab_mixed_wide(A, Y[:, c], A32, None if X0 is None else X0[:, c],
                                         tol, maxit, tol_inner, maxit_inner) for c in cols]

    def _mixed(self, fn, A, y, A32, x0, tol, maxit, tol_inner, maxit_inner):
        A, lda = self._mat(A)
        n = A.shape[0]
        if A32 is None:
            A32 = A.astype(np.complex64)
        A32 = np.ascontiguousarray(A32, dtype=np.complex64)
        y = np.ascontiguousarray(y, dtype=np.complex128)
        flags = 0
        if x0 is None:
            x = np.zeros(n, dtype=np.complex128)
            flags = X0_ZERO
        else:
            x = np.array(x0, dtype=np.complex128, copy=True)
        outer_res = np.full(max(maxit, 0) + 1, np.nan)
        st = _MixedStats()
        rc = fn(
            n, A.ctypes.data, lda, A32.ctypes.data, max(n, 1), y.ctypes.data,
            x.ctypes.data, float(tol), int(maxit), float(tol_inner),
            int(maxit_inner), flags, ctypes.byref(st), outer_res.ctypes.data)
        if rc != 0:
            raise ValueError("oracle argument error %d" % rc)
        return MixedResult(x, st.info, st.outer, st.inner_iters, st.matvecs64,
                           st.matvecs32, st.relres_true, outer_res)

    # -- many right-hand sides: the same routines, one column at a time ----
    def matmat(self, A, B, cols=None):
        """Z = A B, column by column through matvec (cols: a subset)."""
        B = np.asarray(B)
        cols = range(B.shape[1]) if cols is None else cols
        return np.stack([self.matvec(A, B[:, c]) for c in cols], axis=1)

    def bicgstab_block(self, A, Y, X0=None, tol=1e-10, maxit=1000, cols=None):
        """Each column of Y solved by its own BiCGSTAB (column-wise scalars
        and stop test); cols selects a subset.  Returns a list of Results."""
        Y = np.asarray(Y)
        cols = range(Y.shape[1]) if cols is None else cols
        return [self.bicgstab(A, Y[:, c], None if X0 is None else X0[:, c],
                              tol=tol, maxit=maxit) for c in cols]


    def threads(self, want: int = 0) -> int:
        """Set (want > 0) and return the thread count of the OpenMP build; 1
        for the one-thread build."""
        return int(self.lib.oracle_threads(int(want)))


_default: Oracle | None = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def get_omp() -> Oracle:
    """The OpenMP timing build (built on first use when missing)."""
    if not os.path.exists(LIB_OMP) or os.path.getmtime(LIB_OMP) < os.path.getmtime(SRC):
        build(out=LIB_OMP, openmp=True)
    return Oracle(LIB_OMP)
