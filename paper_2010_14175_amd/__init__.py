"""Adaptive FSAI (aFSAI) preconditioner and PCG on AMD Instinct MI355X (gfx950).

Thin Python binding of the C ABI declared in ``include/afsai.h`` (``libafsai.so``, built from
``csrc/*.hip`` by :mod:`paper_2010_14175_amd.build`).  This module only marshals arguments:
PyTorch provides device memory and the stream, every step of the method runs in the HIP
kernels of the library.  There is no fallback: if the library is missing or fails to load,
every call raises.

Method: Isotton, Janna, Bernaschi, "A GPU-accelerated adaptive FSAI preconditioner for
massively parallel simulations", Sec. 2 (adaptive pattern, eqs. DensSys, diagScal, grapsi,
exit_crit) and Sec. 3 (GPU kernels).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafsai.so")
TIE_RTOL = 2.0 ** -26

OK, ERR_INVALID_ARG, ERR_BAD_MATRIX, ERR_NOT_SPD, ERR_NO_MEMORY, ERR_NOT_CONVERGED, ERR_TOO_LARGE, ERR_HIP = range(8)
F64, F32 = 0, 1
VALIDATE = 1
SETUP_F32 = 2
GRAD_F32 = 4
STOP_KMAX, STOP_EPS, STOP_NOCAND = 0, 1, 2

# every symbol the C header declares
EXPORTS = ("afsai_setup", "afsai_apply", "afsai_apply_noalloc", "pcg_solve", "afsai_setup_batched", "pcg_solve_batched",
           "afsai_server_create", "afsai_server_submit", "afsai_server_poll", "afsai_server_pending",
           "afsai_server_destroy", "afsai_spmv", "afsai_spmm", "pcg_solve_multi",
           "afsai_matrix_prepare", "afsai_matrix_destroy", "afsai_spmm_prepared", "pcg_solve_prepared",
           "afsai_get_setup_info", "afsai_export",
           "afsai_export_rows", "afsai_import", "afsai_destroy", "afsai_last_error", "afsai_set_option",
           "afsai_release_cache",
           "afsai_profile_enable", "afsai_profile_only", "afsai_profile_read")
(OPT_SETUP_GROUP, OPT_SETUP_TABLE, OPT_SPMV_GROUP, OPT_SPMV_UNROLL, OPT_PCG_CSR_A, OPT_PCG_FORM,
 OPT_SELL_WIDTH, OPT_PCG_GRAPH, OPT_SETUP_SLOTS, OPT_SELL_TAIL, OPT_SELL_UNEVEN, OPT_SETUP_FORM,
 OPT_SETUP_LANES, OPT_SETUP_CLAIM, OPT_SELL_RUNS) = range(1, 16)


class ServerConfigStruct(ctypes.Structure):
    pass


class RequestResultStruct(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("true_relres", ctypes.c_double), ("footprint", ctypes.c_int64),
                ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double), ("setup_done_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double)]


class CsrStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class ParamsStruct(ctypes.Structure):
    _fields_ = [("kmax", ctypes.c_int32), ("s", ctypes.c_int32), ("eps", ctypes.c_double),
                ("tie_rtol", ctypes.c_double), ("g_prec", ctypes.c_int32), ("flags", ctypes.c_uint32)]


ServerConfigStruct._fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                               ("setup_threads", ctypes.c_int32), ("params", ParamsStruct), ("rtol", ctypes.c_double),
                               ("maxit", ctypes.c_int32), ("max_heavy", ctypes.c_int32), ("heavy_nnz", ctypes.c_int64)]


class SetupInfoStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mmax", ctypes.c_int32), ("nnz_g", ctypes.c_int64), ("g_prec", ctypes.c_int32),
                ("rows_stop_kmax", ctypes.c_int32), ("rows_stop_eps", ctypes.c_int32),
                ("rows_stop_nocand", ctypes.c_int32), ("rows_retried", ctypes.c_int32),
                ("sum_log_psi", ctypes.c_double), ("ms", ctypes.c_double)]


class PcgInfoStruct(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("relres", ctypes.c_double),
                ("true_relres", ctypes.c_double), ("ms", ctypes.c_double)]


class KernelTimeStruct(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class AfsaiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[afsai status {code}] {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_14175_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        P = ctypes.POINTER
        L.afsai_setup.argtypes = [P(CsrStruct), P(ParamsStruct), vp, P(vp)]
        L.afsai_apply.argtypes = [vp, vp, vp, vp]
        L.afsai_apply_noalloc.argtypes = [vp, vp, vp, vp]
        L.pcg_solve.argtypes = [P(CsrStruct), vp, vp, vp, ctypes.c_double, i32, vp, P(PcgInfoStruct)]
        L.afsai_spmv.argtypes = [P(CsrStruct), vp, vp, vp]
        L.afsai_spmm.argtypes = [P(CsrStruct), ctypes.c_int32, vp, vp, vp]
        L.pcg_solve_multi.argtypes = [P(CsrStruct), vp, ctypes.c_int32, vp, vp, ctypes.c_double, i32, vp,
                                      P(PcgInfoStruct)]
        L.afsai_matrix_prepare.argtypes = [P(CsrStruct), vp, P(vp)]
        L.afsai_matrix_destroy.argtypes = [vp]
        L.afsai_matrix_destroy.restype = None
        L.afsai_spmm_prepared.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
        L.pcg_solve_prepared.argtypes = [vp, vp, vp, vp, ctypes.c_double, i32, vp, P(PcgInfoStruct)]
        L.afsai_server_create.argtypes = [P(ServerConfigStruct), P(vp)]
        L.afsai_server_submit.argtypes = [vp, P(CsrStruct), P(ParamsStruct), vp, vp, P(ctypes.c_int64)]
        L.afsai_server_poll.argtypes = [vp, P(RequestResultStruct), i32, P(i32), i32]
        L.afsai_server_pending.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64), P(i32)]
        L.afsai_server_destroy.argtypes = [vp]
        L.afsai_setup_batched.argtypes = [P(CsrStruct), i32, P(i32), P(ParamsStruct), vp, P(vp)]
        L.pcg_solve_batched.argtypes = [P(CsrStruct), vp, i32, P(i32), vp, vp, ctypes.c_double, i32, vp,
                                        P(PcgInfoStruct)]
        L.afsai_get_setup_info.argtypes = [vp, P(SetupInfoStruct)]
        L.afsai_export.argtypes = [vp, vp, vp, vp, vp]
        L.afsai_export_rows.argtypes = [vp, vp, vp, vp, vp]
        L.afsai_import.argtypes = [P(CsrStruct), i32, vp, P(vp)]
        L.afsai_destroy.argtypes = [vp]
        L.afsai_destroy.restype = None
        L.afsai_last_error.restype = ctypes.c_char_p
        L.afsai_set_option.argtypes = [i32, ctypes.c_int64]
        L.afsai_profile_enable.argtypes = [i32]
        L.afsai_profile_only.argtypes = [ctypes.c_char_p]
        L.afsai_profile_read.argtypes = [P(KernelTimeStruct), i32, P(i32), i32]
        for name in EXPORTS:
            if name not in ("afsai_destroy", "afsai_matrix_destroy", "afsai_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str, allow=(OK,)):
    if rc not in allow:
        raise AfsaiError(rc, f"{what}: {lib().afsai_last_error().decode(errors='replace')}")
    return rc


def _stream(stream=None):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_dev(t, shape, what: str):
    """Raises ValueError unless t is a contiguous float64 CUDA tensor of the given shape (the
    library reads and writes exactly that many elements through its pointer)."""
    import torch

    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
            or tuple(t.shape) != tuple(shape)):
        got = (f"{tuple(t.shape)} {t.dtype} on {t.device}{'' if t.is_contiguous() else ', not contiguous'}"
               if isinstance(t, torch.Tensor) else type(t).__name__)
        raise ValueError(f"{what}: expected a contiguous float64 CUDA tensor of shape {tuple(shape)}, got {got}")


class DeviceCSR:
    """A square CSR matrix resident on the GPU (int32 indices, fp64 values), held by torch
    tensors.  ``struct`` is the C view passed to the library."""

    def __init__(self, row_ptr, col, val):
        import torch

        self.row_ptr, self.col, self.val = row_ptr, col, val
        assert row_ptr.dtype == torch.int32 and col.dtype == torch.int32 and val.dtype == torch.float64
        assert row_ptr.is_contiguous() and col.is_contiguous() and val.is_contiguous()
        self.n = int(row_ptr.numel() - 1)
        self.nnz = int(col.numel())

    @property
    def struct(self) -> CsrStruct:
        return CsrStruct(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr())

    @staticmethod
    def from_host(A, device="cuda") -> "DeviceCSR":
        """From any object with numpy ``row_ptr``, ``col`` and ``val`` arrays."""
        import torch

        rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).to(device)
        va = torch.from_numpy(np.ascontiguousarray(A.val, np.float64)).to(device)
        return DeviceCSR(rp, ci, va)


@dataclass
class SetupInfo:
    n: int
    mmax: int
    nnz_g: int
    g_prec: int
    rows_stop_kmax: int
    rows_stop_eps: int
    rows_stop_nocand: int
    rows_retried: int
    sum_log_psi: float
    ms: float


@dataclass
class PcgInfo:
    status: int
    iters: int
    converged: bool
    relres: float
    true_relres: float
    ms: float


class Preconditioner:
    """Owns an ``afsai_precond`` handle (G and G^T on the device)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise RuntimeError("preconditioner already destroyed")
        return self._h

    def info(self) -> SetupInfo:
        s = SetupInfoStruct()
        _check(lib().afsai_get_setup_info(self.handle, ctypes.byref(s)), "afsai_get_setup_info")
        return SetupInfo(s.n, s.mmax, s.nnz_g, s.g_prec, s.rows_stop_kmax, s.rows_stop_eps, s.rows_stop_nocand,
                         s.rows_retried, s.sum_log_psi, s.ms)

    def export(self, stream=None):
        """G as (row_ptr int32, col int32, val f64) device tensors."""
        import torch

        inf = self.info()
        rp = torch.empty(inf.n + 1, dtype=torch.int32, device="cuda")
        ci = torch.empty(max(1, inf.nnz_g), dtype=torch.int32, device="cuda")
        va = torch.empty(max(1, inf.nnz_g), dtype=torch.float64, device="cuda")
        _check(lib().afsai_export(self.handle, _ptr(rp), _ptr(ci), _ptr(va), _stream(stream)), "afsai_export")
        return rp, ci[: inf.nnz_g], va[: inf.nnz_g]

    def export_rows(self, stream=None):
        """(psi, steps, reason) device tensors, one entry per row."""
        import torch

        n = self.info().n
        psi = torch.empty(n, dtype=torch.float64, device="cuda")
        steps = torch.empty(n, dtype=torch.int32, device="cuda")
        reason = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().afsai_export_rows(self.handle, _ptr(psi), _ptr(steps), _ptr(reason), _stream(stream)),
               "afsai_export_rows")
        return psi, steps, reason

    def apply(self, r, z=None, stream=None):
        """z = G^T (G r)."""
        import torch

        n = self.info().n
        _check_dev(r, (n,), "apply: r")
        if z is None:
            z = torch.empty_like(r)
        _check_dev(z, (n,), "apply: z")
        _check(lib().afsai_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)), "afsai_apply")
        return z

    def apply_noalloc(self, r, z, stream=None):
        """z = G^T (G r) through afsai_apply_noalloc (z must be given: the call allocates nothing)."""
        n = self.info().n
        _check_dev(r, (n,), "apply_noalloc: r")
        _check_dev(z, (n,), "apply_noalloc: z")
        _check(lib().afsai_apply_noalloc(self.handle, _ptr(r), _ptr(z), _stream(stream)), "afsai_apply_noalloc")
        return z

    def close(self):
        if self._h:
            lib().afsai_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def setup(A: DeviceCSR, kmax: int, s: int, eps: float, tie_rtol: float = TIE_RTOL, g_prec: int = F64,
          validate: bool = False, stream=None, setup_f32: bool = False, grad_f32: bool = False) -> Preconditioner:
    """Adaptive FSAI setup (``afsai_setup``); setup_f32: the per-row arithmetic in FP32;
    grad_f32: the gradient reads FP32 values of A (the factorisation stays FP64)."""
    p = ParamsStruct(int(kmax), int(s), float(eps), float(tie_rtol), int(g_prec),
                     (VALIDATE if validate else 0) | (SETUP_F32 if setup_f32 else 0) | (GRAD_F32 if grad_f32 else 0))
    h = ctypes.c_void_p()
    st = A.struct
    _check(lib().afsai_setup(ctypes.byref(st), ctypes.byref(p), _stream(stream), ctypes.byref(h)), "afsai_setup")
    return Preconditioner(h)


def import_factor(G: DeviceCSR, g_prec: int = F64, stream=None) -> Preconditioner:
    """A preconditioner from a given lower-triangular G (``afsai_import``)."""
    h = ctypes.c_void_p()
    st = G.struct
    _check(lib().afsai_import(ctypes.byref(st), int(g_prec), _stream(stream), ctypes.byref(h)), "afsai_import")
    return Preconditioner(h)


def pcg_solve(A: DeviceCSR, P: Preconditioner | None, b, x=None, rtol: float = 1e-8, maxit: int | None = None,
              stream=None, raise_on_error: bool = True):
    """Preconditioned CG (``pcg_solve``); x (device, fp64) holds x0 on entry when given.
    Returns (x, PcgInfo)."""
    import torch

    _check_dev(b, (A.n,), "pcg_solve: b")
    if x is None:
        x = torch.zeros_like(b)
    _check_dev(x, (A.n,), "pcg_solve: x")
    maxit = A.n if maxit is None else int(maxit)
    inf = PcgInfoStruct()
    st = A.struct
    rc = lib().pcg_solve(ctypes.byref(st), None if P is None else P.handle, _ptr(b), _ptr(x), float(rtol), maxit,
                         _stream(stream), ctypes.byref(inf))
    if raise_on_error:
        _check(rc, "pcg_solve", allow=(OK, ERR_NOT_CONVERGED))
    return x, PcgInfo(rc, inf.iters, bool(inf.converged), inf.relres, inf.true_relres, inf.ms)


class PreparedMatrix:
    """A's SELL-64 layout made once (``afsai_matrix_prepare``), for repeated products and
    solves with one matrix; ``spmm`` and ``pcg_solve`` give the unprepared calls' results bit
    for bit."""

    def __init__(self, A: DeviceCSR, stream=None):
        self.n = A.n
        h = ctypes.c_void_p()
        st = A.struct
        _check(lib().afsai_matrix_prepare(ctypes.byref(st), _stream(stream), ctypes.byref(h)), "afsai_matrix_prepare")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("PreparedMatrix: handle has been closed")
        return self._h

    def spmm(self, X, Y=None, stream=None):
        """Y = A X for an (n, k) row-major block of k = 1, 2, 4 or 8 vectors."""
        import torch

        if not isinstance(X, torch.Tensor) or X.dim() != 2:
            raise ValueError("PreparedMatrix.spmm: X must be an (n, k) tensor")
        _check_dev(X, (self.n, X.shape[1]), "PreparedMatrix.spmm: X")
        if Y is None:
            Y = torch.empty_like(X)
        _check_dev(Y, tuple(X.shape), "PreparedMatrix.spmm: Y")
        _check(lib().afsai_spmm_prepared(self.handle, int(X.shape[1]), _ptr(X), _ptr(Y), _stream(stream)),
               "afsai_spmm_prepared")
        return Y

    def pcg_solve(self, P: Preconditioner | None, b, x=None, rtol: float = 1e-8, maxit: int | None = None,
                  stream=None, raise_on_error: bool = True):
        """``pcg_solve_prepared``: returns (x, PcgInfo) as ``pcg_solve``."""
        import torch

        _check_dev(b, (self.n,), "PreparedMatrix.pcg_solve: b")
        if x is None:
            x = torch.zeros_like(b)
        _check_dev(x, (self.n,), "PreparedMatrix.pcg_solve: x")
        maxit = self.n if maxit is None else int(maxit)
        inf = PcgInfoStruct()
        rc = lib().pcg_solve_prepared(self.handle, None if P is None else P.handle, _ptr(b), _ptr(x), float(rtol),
                                      maxit, _stream(stream), ctypes.byref(inf))
        if raise_on_error:
            _check(rc, "pcg_solve_prepared", allow=(OK, ERR_NOT_CONVERGED))
        return x, PcgInfo(rc, inf.iters, bool(inf.converged), inf.relres, inf.true_relres, inf.ms)

    def close(self):
        if self._h:
            lib().afsai_matrix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_solve_multi(A: DeviceCSR, P: Preconditioner | None, B, rtol: float = 1e-8, maxit: int | None = None,
                    stream=None, raise_on_error: bool = True):
    """PCG for an (n, k) row-major block B of k = 1, 2, 4 or 8 right-hand sides, X0 = 0
    (``pcg_solve_multi``).  Returns (X, [PcgInfo per column])."""
    import torch

    if not isinstance(B, torch.Tensor) or B.dim() != 2:
        raise ValueError("pcg_solve_multi: B must be an (n, k) tensor")
    _check_dev(B, (A.n, B.shape[1]), "pcg_solve_multi: B")
    k = int(B.shape[1])
    X = torch.empty_like(B)
    maxit = A.n if maxit is None else int(maxit)
    infs = (PcgInfoStruct * max(1, k))()
    st = A.struct
    rc = lib().pcg_solve_multi(ctypes.byref(st), None if P is None else P.handle, k, _ptr(B), _ptr(X), float(rtol),
                               maxit, _stream(stream), infs)
    if raise_on_error:
        _check(rc, "pcg_solve_multi", allow=(OK, ERR_NOT_CONVERGED))
    return X, [PcgInfo(OK if infs[j].converged else rc, infs[j].iters, bool(infs[j].converged), infs[j].relres,
                       infs[j].true_relres, infs[j].ms) for j in range(k)]


def _offsets(offsets):
    import numpy as np

    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
    return off, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(off) - 1


def setup_batched(A: DeviceCSR, offsets, kmax: int, s: int, eps: float, tie_rtol: float = TIE_RTOL,
                  g_prec: int = F64, validate: bool = False, stream=None, setup_f32: bool = False) -> Preconditioner:
    """Setup of a batch of independent systems given as one block-diagonal matrix whose system
    k owns rows offsets[k] .. offsets[k+1]-1 (``afsai_setup_batched``)."""
    p = ParamsStruct(int(kmax), int(s), float(eps), float(tie_rtol), int(g_prec),
                     (VALIDATE if validate else 0) | (SETUP_F32 if setup_f32 else 0))
    off, optr, nsys = _offsets(offsets)
    h = ctypes.c_void_p()
    st = A.struct
    _check(lib().afsai_setup_batched(ctypes.byref(st), nsys, optr, ctypes.byref(p), _stream(stream), ctypes.byref(h)),
           "afsai_setup_batched")
    return Preconditioner(h)


def pcg_solve_batched(A: DeviceCSR, P: Preconditioner | None, offsets, b, x=None, rtol: float = 1e-8,
                      maxit: int | None = None, stream=None, raise_on_error: bool = True):
    """PCG on every system of a batch (``pcg_solve_batched``).  Returns (x, [PcgInfo per system])."""
    import torch

    off, optr, nsys = _offsets(offsets)
    _check_dev(b, (A.n,), "pcg_solve_batched: b")
    if x is None:
        x = torch.zeros_like(b)
    _check_dev(x, (A.n,), "pcg_solve_batched: x")
    maxit = int(max(off[1:] - off[:-1])) if maxit is None else int(maxit)
    infs = (PcgInfoStruct * nsys)()
    st = A.struct
    rc = lib().pcg_solve_batched(ctypes.byref(st), None if P is None else P.handle, nsys, optr, _ptr(b), _ptr(x),
                                 float(rtol), maxit, _stream(stream), infs)
    if raise_on_error:
        _check(rc, "pcg_solve_batched", allow=(OK, ERR_NOT_CONVERGED))
    return x, [PcgInfo(rc, f.iters, bool(f.converged), f.relres, f.true_relres, f.ms) for f in infs]


@dataclass
class RequestResult:
    ticket: int
    status: int
    iters: int
    converged: bool
    true_relres: float
    footprint: int
    submit_ms: float
    admit_ms: float
    setup_done_ms: float
    done_ms: float

    @property
    def latency_ms(self) -> float:
        return self.done_ms - self.submit_ms


class Server:
    """Serving loop (``afsai_server_*``): requests are admitted while slots and the device-memory
    budget allow, set up and solved concurrently; results come back through ``poll``."""

    def __init__(self, hbm_budget: int, max_slots: int, kmax: int, s: int, eps: float, rtol: float = 1e-8,
                 maxit: int = 100000, g_prec: int = F64, setup_threads: int = 2, tie_rtol: float = TIE_RTOL,
                 max_heavy: int = 0, heavy_nnz: int = 0):
        cfg = ServerConfigStruct(int(hbm_budget), int(max_slots), int(setup_threads),
                                 ParamsStruct(int(kmax), int(s), float(eps), float(tie_rtol), int(g_prec), 0),
                                 float(rtol), int(maxit), int(max_heavy), int(heavy_nnz))
        h = ctypes.c_void_p()
        _check(lib().afsai_server_create(ctypes.byref(cfg), ctypes.byref(h)), "afsai_server_create")
        self._h = h
        self._params = cfg.params
        self._keep = {}  # ticket -> (A, b, x) kept alive until the result is polled

    def submit(self, A: DeviceCSR, b, x, kmax: int | None = None, s: int | None = None, eps: float | None = None,
               g_prec: int | None = None) -> int:
        """Queues A x = b (device data; x is overwritten), with the server's setup parameters or the
        ones given here.  Returns the request's ticket."""
        _check_dev(b, (A.n,), "Server.submit: b")
        _check_dev(x, (A.n,), "Server.submit: x")
        t = ctypes.c_int64()
        st = A.struct
        p = None
        if kmax is not None or s is not None or eps is not None or g_prec is not None:
            d = self._params
            p = ctypes.byref(ParamsStruct(d.kmax if kmax is None else int(kmax), d.s if s is None else int(s),
                                          d.eps if eps is None else float(eps), d.tie_rtol,
                                          d.g_prec if g_prec is None else int(g_prec), 0))
        _check(lib().afsai_server_submit(self._h, ctypes.byref(st), p, _ptr(b), _ptr(x), ctypes.byref(t)),
               "afsai_server_submit")
        self._keep[t.value] = (A, b, x)
        return t.value

    def poll(self, wait_ms: int = 0, max_results: int = 256) -> list[RequestResult]:
        out = (RequestResultStruct * max_results)()
        cnt = ctypes.c_int32()
        _check(lib().afsai_server_poll(self._h, out, max_results, ctypes.byref(cnt), int(wait_ms)), "afsai_server_poll")
        res = []
        for r in out[: cnt.value]:
            self._keep.pop(r.ticket, None)
            res.append(RequestResult(r.ticket, r.status, r.iters, bool(r.converged), r.true_relres, r.footprint,
                                     r.submit_ms, r.admit_ms, r.setup_done_ms, r.done_ms))
        return res

    def pending(self) -> tuple[int, int, int]:
        """(requests not finished, device bytes admitted, slots admitted)."""
        o, b = ctypes.c_int64(), ctypes.c_int64()
        sl = ctypes.c_int32()
        _check(lib().afsai_server_pending(self._h, ctypes.byref(o), ctypes.byref(b), ctypes.byref(sl)),
               "afsai_server_pending")
        return o.value, b.value, sl.value

    def close(self):
        if self._h:
            lib().afsai_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmm(A: DeviceCSR, X, Y=None, stream=None):
    """Y = A X for an (n, k) row-major block of k = 1, 2, 4 or 8 vectors (``afsai_spmm``)."""
    import torch

    if not isinstance(X, torch.Tensor) or X.dim() != 2:
        raise ValueError("spmm: X must be an (n, k) tensor")
    _check_dev(X, (A.n, X.shape[1]), "spmm: X")
    if Y is None:
        Y = torch.empty_like(X)
    _check_dev(Y, tuple(X.shape), "spmm: Y")
    st = A.struct
    _check(lib().afsai_spmm(ctypes.byref(st), int(X.shape[1]), _ptr(X), _ptr(Y), _stream(stream)), "afsai_spmm")
    return Y


def spmv(A: DeviceCSR, x, y=None, stream=None):
    """y = A x (``afsai_spmv``)."""
    import torch

    _check_dev(x, (A.n,), "spmv: x")
    if y is None:
        y = torch.empty_like(x)
    _check_dev(y, (A.n,), "spmv: y")
    st = A.struct
    _check(lib().afsai_spmv(ctypes.byref(st), _ptr(x), _ptr(y), _stream(stream)), "afsai_spmv")
    return y


def release_cache():
    """Returns the library's cached device blocks to the HIP runtime."""
    _check(lib().afsai_release_cache(), "afsai_release_cache")


def set_option(option: int, value: int):
    """Process-wide tuning knob (``afsai_set_option``); 0 restores the automatic choice."""
    _check(lib().afsai_set_option(int(option), int(value)), "afsai_set_option")


def profile_enable(on: bool = True):
    _check(lib().afsai_profile_enable(1 if on else 0), "afsai_profile_enable")


def profile_only(names=None):
    """Times only the kernels named (``afsai_profile_only``); None times all of them."""
    arg = None if not names else ",".join(names).encode()
    _check(lib().afsai_profile_only(arg), "afsai_profile_only")


def profile_read(reset: bool = False) -> dict:
    """{kernel name: (launches, total_ms)} of the event timer."""
    cap = 64
    arr = (KernelTimeStruct * cap)()
    cnt = ctypes.c_int32(0)
    _check(lib().afsai_profile_read(arr, cap, ctypes.byref(cnt), 1 if reset else 0), "afsai_profile_read")
    return {arr[k].name.decode(): (int(arr[k].launches), float(arr[k].total_ms)) for k in range(cnt.value)}
