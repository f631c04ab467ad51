"""Seeded synthetic SPD workloads shared by the oracle, the tests and the benchmark.

This module only constructs inputs (stencil matrices in CSR, right-hand sides); it holds
none of the adaptive-FSAI arithmetic.  The numeric work is in ``synth.c`` (plain C, built
with gcc by :func:`build`).

Workloads (stand-ins for the paper's benchmark matrices, which are not public):

* ``lap7``      7-point Poisson operator, the shape of the paper's ``pois198m`` matrix and of
                its weak-scaling problem (121^3 unknowns per GPU, Sec. 5.3).
* ``elast27``   27-point, 3 dof/node, log-normal cellwise coefficients: about 80 nonzeros
                per row like the paper's mechanics matrices (Table of benchmark matrices).

Every right-hand side is b = A x_true with x_true ~ U(-1, 1) drawn from SplitMix64.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

# stream ids of the counter-based generator
STREAM_XTRUE = 1
STREAM_BATCH = 11


def build() -> str:
    """Compile ``libsynth.so`` with gcc (host code only)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.synth_key.restype = ctypes.c_uint64
        L.synth_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.synth_uniform.restype = None
        L.synth_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_double, f64p]
        L.synth_normal.restype = None
        L.synth_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, f64p]
        L.synth_raw.restype = None
        L.synth_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, u64p]
        L.synth_matvec.restype = None
        L.synth_matvec.argtypes = [ctypes.c_int32, i32p, i32p, f64p, f64p, f64p]
        L.synth_lap7_nnz.restype = ctypes.c_int64
        L.synth_lap7_nnz.argtypes = [ctypes.c_int32] * 3
        L.synth_lap7.restype = None
        L.synth_lap7.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double] * 3 + [i32p, i32p, f64p]
        L.synth_lap7_lognormal.restype = None
        L.synth_lap7_lognormal.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.c_uint64, i32p, i32p, f64p]
        L.synth_elast27_nnz.restype = ctypes.c_int64
        L.synth_elast27_nnz.argtypes = [ctypes.c_int32]
        L.synth_elast27.restype = ctypes.c_int
        L.synth_elast27.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, i32p, i32p, f64p]
        _lib = L
    return _lib


@dataclass
class CSR:
    """Square sparse matrix, 0-based CSR, int32 indices, fp64 values, both triangles stored."""

    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    @staticmethod
    def from_dense(a: np.ndarray, keep_zeros_on_diag: bool = True) -> "CSR":
        a = np.asarray(a, dtype=np.float64)
        n = a.shape[0]
        rp = [0]
        cols, vals = [], []
        for i in range(n):
            for j in range(n):
                if a[i, j] != 0.0 or (keep_zeros_on_diag and i == j):
                    cols.append(j)
                    vals.append(a[i, j])
            rp.append(len(cols))
        return CSR(np.array(rp, np.int32), np.array(cols, np.int32), np.array(vals, np.float64))

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = m.tocsr()
        m.sort_indices()
        return CSR(m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))


def uniform(seed: int, stream: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    out = np.empty(n, np.float64)
    lib().synth_uniform(seed, stream, n, lo, hi, out)
    return out


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    lib().synth_normal(seed, stream, n, out)
    return out


def raw_u64(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.uint64)
    lib().synth_raw(seed, stream, n, out)
    return out


def matvec(A: CSR, x: np.ndarray) -> np.ndarray:
    y = np.empty(A.n, np.float64)
    lib().synth_matvec(A.n, A.row_ptr, A.col, A.val, np.ascontiguousarray(x, np.float64), y)
    return y


def lap7(nx: int, ny: int | None = None, nz: int | None = None, c=(1.0, 1.0, 1.0)) -> CSR:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    L = lib()
    n = nx * ny * nz
    nnz = L.synth_lap7_nnz(nx, ny, nz)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    va = np.empty(nnz, np.float64)
    L.synth_lap7(nx, ny, nz, float(c[0]), float(c[1]), float(c[2]), rp, ci, va)
    return CSR(rp, ci, va)


def lap7_lognormal(nx: int, ny: int, nz: int, sigma: float, seed: int) -> CSR:
    L = lib()
    n = nx * ny * nz
    nnz = L.synth_lap7_nnz(nx, ny, nz)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    va = np.empty(nnz, np.float64)
    L.synth_lap7_lognormal(nx, ny, nz, float(sigma), seed, rp, ci, va)
    return CSR(rp, ci, va)


def elast27(N: int, sigma: float, seed: int) -> CSR:
    L = lib()
    n = 3 * N ** 3
    nnz = L.synth_elast27_nnz(N)
    if nnz >= 2 ** 31:
        raise ValueError("nnz exceeds int32 indexing")
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    va = np.empty(nnz, np.float64)
    if L.synth_elast27(N, float(sigma), seed, rp, ci, va) != 0:
        raise MemoryError("synth_elast27: allocation failed")
    return CSR(rp, ci, va)


def random_spd_dense(n: int, seed: int, cond_scale: float = 1.0) -> np.ndarray:
    """Dense random SPD matrix B B^T + n I from seeded normals (tiny test cases)."""
    g = normal(seed, 99, n * n).reshape(n, n)
    a = g @ g.T * cond_scale + n * np.eye(n)
    return 0.5 * (a + a.T)


def random_sparse_spd(n: int, per_row: int, seed: int) -> CSR:
    """Symmetric matrix with about 2*per_row random off-diagonal entries per row, values
    U(-1, 1), made SPD by strict diagonal dominance (diagonal = 1 + sum of |off-diagonals|).
    Rows reach columns all over the matrix, so a pattern's candidate set is large."""
    import scipy.sparse as sp

    k = n * per_row
    u = raw_u64(seed, 21, 2 * k)
    rows = (u[:k] % np.uint64(n)).astype(np.int64)
    cols = (u[k:] % np.uint64(n)).astype(np.int64)
    vals = uniform(seed, 22, k)
    keep = rows != cols
    m = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m = (m + m.T).tocsr()
    m = m + sp.diags(1.0 + np.asarray(abs(m).sum(axis=1)).ravel())
    return CSR.from_scipy(m)


@dataclass
class Problem:
    """One linear system A x = b with its aFSAI parameters."""

    name: str
    A: CSR
    b: np.ndarray
    x_true: np.ndarray
    kmax: int
    s: int
    eps: float = 1e-2
    rtol: float = 1e-8
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.n


def _rhs(A: CSR, seed: int) -> tuple[np.ndarray, np.ndarray]:
    x = uniform(seed, STREAM_XTRUE, A.n)
    return matvec(A, x), x


def poisson7(N: int = 20, seed: int = 1, kmax: int = 5, s: int = 1) -> Problem:
    """3D 7-point Laplacian, Dirichlet, N^3 unknowns (N = 20: 8,000 unknowns)."""
    A = lap7(N)
    b, x = _rhs(A, seed)
    return Problem(f"poisson7_{N}", A, b, x, kmax, s, meta={"N": N, "seed": seed})


def elasticity27(N: int = 64, sigma: float = 1.0, seed: int = 2, kmax: int = 10, s: int = 2) -> Problem:
    """27-point 3-dof heterogeneous SPD operator on N^3 interior nodes (3 N^3 unknowns)."""
    A = elast27(N, sigma, seed)
    b, x = _rhs(A, seed)
    return Problem(f"elast27_{N}_s{sigma:g}", A, b, x, kmax, s, meta={"N": N, "sigma": sigma, "seed": seed})


def aniso_batch(nsys: int = 512, seed: int = 3, side_lo: int = 10, side_hi: int = 40,
                ratio_hi: float = 1e3, kmax: int = 5, s: int = 1) -> list[Problem]:
    """Independent anisotropic 7-point systems: sides ~ U{lo..hi}, coefficients (1, 1, a) with
    a ~ logU[1, ratio_hi] on a strong axis drawn uniformly from {x, y, z}."""
    u = uniform(seed, STREAM_BATCH, 5 * nsys, 0.0, 1.0).reshape(nsys, 5)
    probs = []
    span = side_hi - side_lo + 1
    for k in range(nsys):
        sides = [side_lo + min(span - 1, int(u[k, d] * span)) for d in range(3)]
        a = math.exp(u[k, 3] * math.log(ratio_hi))
        axis = min(2, int(u[k, 4] * 3))
        c = [1.0, 1.0, 1.0]
        c[axis] = a
        A = lap7(sides[0], sides[1], sides[2], c)
        b, x = _rhs(A, seed * 100003 + k)
        probs.append(Problem(f"aniso7_{k}", A, b, x, kmax, s,
                             meta={"sides": sides, "coef": c, "seed": seed, "index": k}))
    return probs


def block_diag(probs: list[Problem]) -> tuple[CSR, np.ndarray, np.ndarray, np.ndarray]:
    """The systems of a batch as one block-diagonal CSR matrix: (A, offsets, b, x_true), system
    k owning rows offsets[k] .. offsets[k+1]-1."""
    sizes = np.array([p.A.n for p in probs], dtype=np.int64)
    offsets = np.zeros(len(probs) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    nnzs = np.array([p.A.nnz for p in probs], dtype=np.int64)
    nnz_off = np.zeros(len(probs) + 1, dtype=np.int64)
    nnz_off[1:] = np.cumsum(nnzs)
    n, nnz = int(offsets[-1]), int(nnz_off[-1])
    if n >= 2**31 or nnz >= 2**31:
        raise ValueError("batch too large for int32 indices")
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    for k, p in enumerate(probs):
        o, e = int(offsets[k]), int(nnz_off[k])
        rp[o:o + p.A.n] = p.A.row_ptr[:-1] + e
        col[e:e + p.A.nnz] = p.A.col + o
        val[e:e + p.A.nnz] = p.A.val
    rp[n] = nnz
    b = np.concatenate([p.b for p in probs])
    x = np.concatenate([p.x_true for p in probs])
    return CSR(rp, col, val), offsets.astype(np.int32), b, x
