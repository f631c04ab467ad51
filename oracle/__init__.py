"""FP64 CPU oracle for adaptive FSAI setup, application and PCG (ctypes front end of
``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the HIP product path, with which it shares no code.

Functions follow Sec. 2 of the paper (see ``oracle.c`` for the equation-by-equation notes):

* :func:`setup`      rows of G from the adaptive pattern procedure (eqs. DensSys, diagScal,
                     grapsi, exit_crit), either all rows or a listed subset;
* :func:`apply`      z = G^T (G r)  (eq. prec);
* :func:`pcg`        textbook preconditioned CG with M^-1 = G^T G (or M = I).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_INVALID_ARG, ERR_BAD_MATRIX, ERR_NOT_SPD, ERR_NO_MEMORY, ERR_NOT_CONVERGED = 0, 1, 2, 3, 4, 5
STOP_KMAX, STOP_EPS, STOP_NOCAND = 0, 1, 2
TIE_RTOL = 2.0 ** -26


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build() -> str:
    """Compile ``liboracle.so`` with gcc; -ffp-contract=off keeps products and sums rounded
    separately."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _bind(L):
    i32 = ctypes.c_int32
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    vp = ctypes.c_void_p
    L.oracle_check_csr.restype = ctypes.c_int
    L.oracle_check_csr.argtypes = [i32, i32p, i32p]
    L.oracle_afsai_rows.restype = ctypes.c_int
    L.oracle_afsai_rows.argtypes = [i32, i32p, i32p, f64p, i32, i32, ctypes.c_double, ctypes.c_double,
                                    i32, vp, i32, i32p, i32p, f64p, vp, vp, vp, i32]
    L.oracle_set_threads.restype = None
    L.oracle_set_threads.argtypes = [i32]
    L.oracle_spmv.restype = None
    L.oracle_spmv.argtypes = [i32, i32p, i32p, f64p, f64p, f64p]
    L.oracle_spmv_t.restype = None
    L.oracle_spmv_t.argtypes = [i32, i32p, i32p, f64p, f64p, f64p]
    L.oracle_apply.restype = None
    L.oracle_apply.argtypes = [i32, i32p, i32p, f64p, f64p, f64p, f64p]
    L.oracle_pcg.restype = ctypes.c_int
    L.oracle_pcg.argtypes = [i32, i32p, i32p, f64p, vp, vp, vp, f64p, f64p, ctypes.c_double, i32,
                             ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), vp]
    return L


def load_variant(path: str):
    """Bind a separately built copy of the oracle library (used by the tests that plant
    mistakes in a copy of oracle.c to show that the pins catch them)."""
    return _bind(ctypes.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr3(A):
    return (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
            np.ascontiguousarray(A.val, np.float64))


def check_csr(A) -> int:
    rp, ci, _ = _csr3(A)
    return lib().oracle_check_csr(A.n, rp, ci)


@dataclass
class Rows:
    """Per-row output of the setup for a list of rows."""

    rows: np.ndarray      # int32 [q]
    m: np.ndarray         # int32 [q]         pattern sizes
    cols: np.ndarray      # int32 [q, mmax]   pattern (ascending, i last), padded with -1
    vals: np.ndarray      # f64   [q, mmax]   scaled row of G, padded with 0
    psi: np.ndarray       # f64   [q, kmax+1] psi_{k,i}, NaN after the last step taken
    steps: np.ndarray     # int32 [q]
    reason: np.ndarray    # int32 [q]         STOP_KMAX / STOP_EPS / STOP_NOCAND


@dataclass
class Factor:
    """G as CSR (lower triangular, ascending columns, diagonal last in each row)."""

    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    rows: Rows

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def setup_rows(A, kmax: int, s: int, eps: float, rows=None, tau: float = TIE_RTOL,
               nthreads: int = 0) -> Rows:
    """Rows of G for the listed rows (all rows when ``rows`` is None)."""
    rp, ci, va = _csr3(A)
    n = A.n
    mmax = 1 + kmax * s
    if rows is None:
        q = n
        rows_arr = None
    else:
        rows_arr = np.ascontiguousarray(rows, np.int32)
        q = rows_arr.shape[0]
    m = np.zeros(q, np.int32)
    cols = np.full((q, mmax), -1, np.int32)
    vals = np.zeros((q, mmax), np.float64)
    psi = np.full((q, kmax + 1), np.nan)
    steps = np.zeros(q, np.int32)
    reason = np.zeros(q, np.int32)
    rc = lib().oracle_afsai_rows(n, rp, ci, va, kmax, s, float(eps), float(tau), q, _ptr(rows_arr), mmax,
                                 m, cols.reshape(-1), vals.reshape(-1), _ptr(psi), _ptr(steps), _ptr(reason),
                                 int(nthreads))
    if rc != OK:
        raise OracleError(rc, "oracle setup")
    # padded slots past m are not written by the C side; normalise them
    idx = np.arange(mmax)[None, :] >= m[:, None]
    cols[idx] = -1
    vals[idx] = 0.0
    return Rows(np.arange(n, dtype=np.int32) if rows_arr is None else rows_arr, m, cols, vals, psi, steps, reason)


def setup(A, kmax: int, s: int, eps: float, tau: float = TIE_RTOL, nthreads: int = 0) -> Factor:
    """The whole factor G as CSR."""
    R = setup_rows(A, kmax, s, eps, None, tau, nthreads)
    rp = np.zeros(A.n + 1, np.int64)
    np.cumsum(R.m, out=rp[1:])
    mask = np.arange(R.cols.shape[1])[None, :] < R.m[:, None]
    return Factor(rp.astype(np.int32), R.cols[mask].astype(np.int32), R.vals[mask].astype(np.float64), R)


def set_threads(nthreads: int) -> None:
    """Threads of the oracle's parallel loops started from the calling thread afterwards
    (results do not depend on it)."""
    lib().oracle_set_threads(int(nthreads))


def spmv(A, x: np.ndarray) -> np.ndarray:
    rp, ci, va = _csr3(A)
    y = np.empty(A.n, np.float64)
    lib().oracle_spmv(A.n, rp, ci, va, np.ascontiguousarray(x, np.float64), y)
    return y


def spmv_t(A, x: np.ndarray) -> np.ndarray:
    rp, ci, va = _csr3(A)
    y = np.empty(A.n, np.float64)
    lib().oracle_spmv_t(A.n, rp, ci, va, np.ascontiguousarray(x, np.float64), y)
    return y


def apply(G: Factor, r: np.ndarray) -> np.ndarray:
    z = np.empty(G.n, np.float64)
    t = np.empty(G.n, np.float64)
    lib().oracle_apply(G.n, np.ascontiguousarray(G.row_ptr, np.int32), np.ascontiguousarray(G.col, np.int32),
                       np.ascontiguousarray(G.val, np.float64), np.ascontiguousarray(r, np.float64), z, t)
    return z


@dataclass
class PCGResult:
    x: np.ndarray
    status: int
    iters: int
    relres: float
    true_relres: float
    history: np.ndarray


def pcg(A, G: Factor | None, b: np.ndarray, rtol: float = 1e-8, maxit: int | None = None,
        x0: np.ndarray | None = None) -> PCGResult:
    rp, ci, va = _csr3(A)
    n = A.n
    maxit = n if maxit is None else int(maxit)
    x = np.zeros(n, np.float64) if x0 is None else np.array(x0, np.float64, copy=True)
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0)
    tr = ctypes.c_double(0)
    hist = np.full(maxit + 1, np.nan)
    if G is None:
        g3 = (None, None, None)
    else:
        g3 = (np.ascontiguousarray(G.row_ptr, np.int32), np.ascontiguousarray(G.col, np.int32),
              np.ascontiguousarray(G.val, np.float64))
    rc = lib().oracle_pcg(n, rp, ci, va, _ptr(g3[0]), _ptr(g3[1]), _ptr(g3[2]),
                          np.ascontiguousarray(b, np.float64), x, float(rtol), maxit,
                          ctypes.byref(it), ctypes.byref(rr), ctypes.byref(tr), _ptr(hist))
    if rc not in (OK, ERR_NOT_CONVERGED):
        raise OracleError(rc, "oracle pcg")
    return PCGResult(x, rc, int(it.value), float(rr.value), float(tr.value), hist[: it.value + 1])
