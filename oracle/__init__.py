"""FP64 CPU oracle for BiCGStab on 7-point stencil systems and 2D 9-point systems.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
calls it and shares no code with it.

The arithmetic lives in ``s7_oracle.c`` (plain C, FP64, explicit CSR,
single-threaded left-to-right loops); this module only compiles it with gcc and
marshals numpy arrays.  What each function computes, and the readings of the
paper's Algorithm 1 it takes, are stated in the C file's header.

Pinned by ``tests/test_oracle_pins.py`` against: a dense matrix built from the
stencil definition (meshes up to 6^3), LAPACK dense solves, the closed-form
eigenpairs of separable constant-coefficient operators, SciPy's independent
BiCGStab, a hand-worked 2-unknown example (``tests/golden/``), the
recurrence-vs-true-residual invariant and the degenerate cases.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "s7_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
REASON_NONE, REASON_RHO_ZERO, REASON_RS_ZERO, REASON_YY_ZERO, REASON_NONFINITE = range(5)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-std=c99", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _State(C.Structure):
    _fields_ = [("rho", C.c_double), ("alpha", C.c_double), ("omega", C.c_double),
                ("beta", C.c_double), ("sigma", C.c_double), ("nb", C.c_double),
                ("tol", C.c_double), ("res_rec", C.c_double), ("iter", C.c_int64),
                ("max_iter", C.c_int64), ("status", C.c_int32), ("reason", C.c_int32),
                ("done", C.c_int32), ("half_exit", C.c_int32)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int64)
_fp = C.POINTER(C.c_float)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        lib.oracle_csr_nnz.restype = C.c_int64
        lib.oracle_csr_nnz.argtypes = [C.c_int32] * 3
        lib.oracle_build_csr.restype = C.c_int64
        lib.oracle_build_csr.argtypes = [C.c_int32] * 3 + [_fp] * 7 + [_ip, _ip, _dp]
        lib.oracle_csr_nnz_2d9.restype = C.c_int64
        lib.oracle_csr_nnz_2d9.argtypes = [C.c_int32] * 2
        lib.oracle_build_csr_2d9.restype = C.c_int64
        lib.oracle_build_csr_2d9.argtypes = [C.c_int32] * 2 + [_fp] * 9 + [_ip, _ip, _dp]
        lib.oracle_spmv.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, _dp]
        lib.oracle_set_threads.argtypes = [C.c_int32]
        lib.oracle_spmv_rows.argtypes = [C.c_int64, C.c_int64, _ip, _ip, _dp, _dp, _dp]
        lib.oracle_dot.restype = C.c_double
        lib.oracle_dot.argtypes = [C.c_int64, _dp, _dp]
        lib.oracle_jacobi_scale.restype = C.c_int
        lib.oracle_jacobi_scale.argtypes = [C.c_int64, _ip, _ip, _dp, _dp]
        lib.oracle_bicgstab_init.restype = C.c_int
        lib.oracle_bicgstab_init.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, _dp, _dp, _dp, _dp,
                                             C.c_double, C.c_int64, C.POINTER(_State)]
        lib.oracle_bicgstab_step.restype = C.c_int
        lib.oracle_bicgstab_step.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, _dp, _dp, _dp, _dp,
                                             _dp, _dp, C.POINTER(_State)]
        lib.oracle_bicgstab.restype = C.c_int
        lib.oracle_bicgstab.argtypes = [C.c_int64, _ip, _ip, _dp, _dp, _dp, C.c_double, C.c_int64,
                                        C.POINTER(_State), C.c_int64, _dp, _dp, _dp, _dp]
        lib.oracle_bicgstab_pipelined.restype = C.c_int
        lib.oracle_bicgstab_pipelined.argtypes = lib.oracle_bicgstab.argtypes
        _lib = lib
    return _lib


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    dims: tuple

    def copy(self):
        return CSR(self.n, self.rowptr, self.col, self.val.copy(), self.dims)


def build_csr(nx: int, ny: int, nz: int, coef) -> CSR:
    """CSR of the stencil operator from coef = (diag, xm, xp, ym, yp, zm, zp), float32 arrays."""
    lib = _load()
    n = nx * ny * nz
    cs = [np.ascontiguousarray(c, dtype=np.float32) for c in coef]
    assert len(cs) == 7 and all(c.size == n for c in cs)
    nnz = lib.oracle_csr_nnz(nx, ny, nz)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int64)
    val = np.zeros(nnz, dtype=np.float64)
    got = lib.oracle_build_csr(nx, ny, nz, *[c.ctypes.data_as(_fp) for c in cs],
                               _i(rowptr), _i(col), _d(val))
    assert got == nnz
    return CSR(n, rowptr, col, val, (nx, ny, nz))


def build_csr_2d9(nx: int, ny: int, coef) -> CSR:
    """CSR of the 2D 9-point operator from coef = (diag, w, e, s, n, sw, se, nw, ne), float32."""
    lib = _load()
    n = nx * ny
    cs = [np.ascontiguousarray(c, dtype=np.float32) for c in coef]
    assert len(cs) == 9 and all(c.size == n for c in cs)
    nnz = lib.oracle_csr_nnz_2d9(nx, ny)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int64)
    val = np.zeros(nnz, dtype=np.float64)
    got = lib.oracle_build_csr_2d9(nx, ny, *[c.ctypes.data_as(_fp) for c in cs], _i(rowptr), _i(col),
                                   _d(val))
    assert got == nnz
    return CSR(n, rowptr, col, val, (nx, ny, 1))


def spmv(A: CSR, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n, dtype=np.float64)
    _load().oracle_spmv(A.n, _i(A.rowptr), _i(A.col), _d(A.val), _d(x), _d(y))
    return y


def spmv_rows(A: CSR, x: np.ndarray, r0: int, r1: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(r1 - r0, dtype=np.float64)
    _load().oracle_spmv_rows(r0, r1, _i(A.rowptr), _i(A.col), _d(A.val), _d(x), _d(y))
    return y


def set_threads(t: int) -> None:
    """Threads of the SpMV row loop (timing only; results do not depend on it)."""
    _load().oracle_set_threads(int(t))


def dot(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return _load().oracle_dot(a.size, _d(a), _d(b))


def jacobi(A: CSR, b: np.ndarray):
    """(D^-1 A, D^-1 b) in FP64."""
    As = A.copy()
    bs = np.array(b, dtype=np.float64, copy=True)
    rc = _load().oracle_jacobi_scale(A.n, _i(As.rowptr), _i(As.col), _d(As.val), _d(bs))
    if rc != 0:
        raise ZeroDivisionError("zero diagonal entry")
    return As, bs


@dataclass
class Result:
    x: np.ndarray
    status: int
    reason: int
    iters: int
    res_rec: float
    rel_res_true: float
    half_exit: bool
    rho: np.ndarray
    alpha: np.ndarray
    omega: np.ndarray
    res_trace: np.ndarray


def true_rel_residual(A: CSR, b: np.ndarray, x: np.ndarray) -> float:
    r = np.asarray(b, dtype=np.float64) - spmv(A, x)
    nb = np.sqrt(dot(b, b))
    return float(np.sqrt(dot(r, r)) / nb) if nb > 0 else float(np.sqrt(dot(r, r)))


def bicgstab(A: CSR, b, x0=None, tol: float = 1e-8, max_iter: int = 500,
             jacobi_scaling: bool = True, ntrace: int = 0) -> Result:
    """Algorithm 1 in FP64.  With jacobi_scaling the iteration runs on (D^-1 A, D^-1 b);
    the true residual is reported for the unscaled system."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    As, bs = jacobi(A, b) if jacobi_scaling else (A, b)
    st = _State()
    nt = max(int(ntrace), 0)
    tr = [np.zeros(max(nt, 1)) for _ in range(4)]
    lib.oracle_bicgstab(A.n, _i(As.rowptr), _i(As.col), _d(As.val), _d(bs), _d(x), tol,
                        max_iter, C.byref(st), nt, *[_d(t) for t in tr])
    k = min(nt, int(st.iter))
    return Result(x, int(st.status), int(st.reason), int(st.iter), float(st.res_rec),
                  true_rel_residual(A, b, x), bool(st.half_exit),
                  tr[0][:k], tr[1][:k], tr[2][:k], tr[3][:k])


def bicgstab_pipelined(A: CSR, b, x0=None, tol: float = 1e-8, max_iter: int = 500,
                       jacobi_scaling: bool = True, ntrace: int = 0) -> Result:
    """Pipelined BiCGStab (Cools and Vanroose 2017) with one reduction per iteration, in
    FP64: the iterates of Algorithm 1 in exact arithmetic, with the matrix products
    carried by recurrences.  Same conventions as bicgstab()."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    As, bs = jacobi(A, b) if jacobi_scaling else (A, b)
    st = _State()
    nt = max(int(ntrace), 0)
    tr = [np.zeros(max(nt, 1)) for _ in range(4)]
    lib.oracle_bicgstab_pipelined(A.n, _i(As.rowptr), _i(As.col), _d(As.val), _d(bs), _d(x), tol,
                                  max_iter, C.byref(st), nt, *[_d(t) for t in tr])
    k = min(nt, int(st.iter))
    return Result(x, int(st.status), int(st.reason), int(st.iter), float(st.res_rec),
                  true_rel_residual(A, b, x), bool(st.half_exit),
                  tr[0][:k], tr[1][:k], tr[2][:k], tr[3][:k])


class Stepper:
    """Algorithm 1 one iteration at a time (for invariant checks)."""

    def __init__(self, A: CSR, b, x0=None, tol=1e-8, max_iter=500, jacobi_scaling=True):
        self.A, self.b = (jacobi(A, b) if jacobi_scaling else (A, np.asarray(b, np.float64)))
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)
        n = A.n
        self.x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        self.r, self.rhat, self.p, self.s, self.q, self.y = (np.zeros(n) for _ in range(6))
        self.st = _State()
        L = self.A
        _load().oracle_bicgstab_init(n, _i(L.rowptr), _i(L.col), _d(L.val), _d(self.b),
                                     _d(self.x), _d(self.r), _d(self.rhat), _d(self.p), tol,
                                     max_iter, C.byref(self.st))

    @property
    def done(self):
        return bool(self.st.done)

    def step(self):
        L = self.A
        return _load().oracle_bicgstab_step(L.n, _i(L.rowptr), _i(L.col), _d(L.val), _d(self.x),
                                            _d(self.r), _d(self.rhat), _d(self.p), _d(self.s),
                                            _d(self.q), _d(self.y), C.byref(self.st))
