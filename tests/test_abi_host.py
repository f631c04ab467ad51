"""Host-side checks of the C ABI: the library loads, exports every symbol include/afsai.h
declares, and rejects bad arguments before touching the GPU (no compute call is made)."""
import ctypes
import os
import re

import pytest

import paper_2010_14175_amd as af

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afsai.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(af.LIB_PATH):
        from paper_2010_14175_amd import build as b

        b.build(verbose=False)
    return af.lib()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


def test_header_parses():
    fns = header_functions()
    assert "afsai_setup" in fns and "afsai_apply" in fns and "pcg_solve" in fns
    assert set(fns) == set(af.EXPORTS)


def test_exports_every_declared_symbol(L):
    for name in header_functions():
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    # sizes implied by the header's field lists on x86-64 (natural alignment)
    assert ctypes.sizeof(af.CsrStruct) == 4 + 4 + 3 * 8
    assert ctypes.sizeof(af.ParamsStruct) == 4 + 4 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(af.PcgInfoStruct) == 4 + 4 + 3 * 8
    assert ctypes.sizeof(af.SetupInfoStruct) == 8 + 8 + 4 * 6 + 8 + 8 + 8 - 8  # n,mmax | nnz | 6 ints | 2 doubles
    assert ctypes.sizeof(af.KernelTimeStruct) == 48 + 8 + 8


def _fake_csr(n=4, nnz=4):
    # non-null device-looking pointers; argument validation rejects before they are used
    return af.CsrStruct(n, nnz, 0x1000, 0x2000, 0x3000)


def test_invalid_arguments_rejected_on_host(L):
    h = ctypes.c_void_p()
    p = af.ParamsStruct(5, 1, 1e-2, af.TIE_RTOL, af.F64, 0)
    A = _fake_csr()
    assert L.afsai_setup(None, ctypes.byref(p), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert L.afsai_setup(ctypes.byref(A), None, None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    bad = af.ParamsStruct(-1, 1, 1e-2, af.TIE_RTOL, af.F64, 0)
    assert L.afsai_setup(ctypes.byref(A), ctypes.byref(bad), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    bad = af.ParamsStruct(3, 0, 1e-2, af.TIE_RTOL, af.F64, 0)
    assert L.afsai_setup(ctypes.byref(A), ctypes.byref(bad), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    bad = af.ParamsStruct(3, 1, -1.0, af.TIE_RTOL, af.F64, 0)
    assert L.afsai_setup(ctypes.byref(A), ctypes.byref(bad), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    bad = af.ParamsStruct(3, 1, 1e-2, 1.0, af.F64, 0)
    assert L.afsai_setup(ctypes.byref(A), ctypes.byref(bad), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    bad = af.ParamsStruct(3, 1, 1e-2, af.TIE_RTOL, 7, 0)
    assert L.afsai_setup(ctypes.byref(A), ctypes.byref(bad), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    big = af.ParamsStruct(16, 4, 1e-2, af.TIE_RTOL, af.F64, 0)  # 1 + 64 > 64
    assert L.afsai_setup(ctypes.byref(A), ctypes.byref(big), None, ctypes.byref(h)) == af.ERR_TOO_LARGE
    empty = af.CsrStruct(0, 0, 0x1000, 0x2000, 0x3000)
    assert L.afsai_setup(ctypes.byref(empty), ctypes.byref(p), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    nulls = af.CsrStruct(4, 4, 0, 0x2000, 0x3000)
    assert L.afsai_setup(ctypes.byref(nulls), ctypes.byref(p), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert h.value is None
    info = af.PcgInfoStruct()
    assert L.pcg_solve(ctypes.byref(A), None, None, None, 1e-8, 10, None, ctypes.byref(info)) == af.ERR_INVALID_ARG
    assert L.pcg_solve(ctypes.byref(A), None, ctypes.c_void_p(0x10), ctypes.c_void_p(0x20), 0.0, 10, None,
                       ctypes.byref(info)) == af.ERR_INVALID_ARG
    assert L.pcg_solve(ctypes.byref(A), None, ctypes.c_void_p(0x10), ctypes.c_void_p(0x20), 1e-8, -1, None,
                       ctypes.byref(info)) == af.ERR_INVALID_ARG
    assert L.afsai_apply(None, ctypes.c_void_p(0x10), ctypes.c_void_p(0x20), None) == af.ERR_INVALID_ARG
    assert L.afsai_get_setup_info(None, None) == af.ERR_INVALID_ARG
    assert L.afsai_export(None, None, None, None, None) == af.ERR_INVALID_ARG
    assert L.afsai_spmm(None, 3, None, None, None) == af.ERR_INVALID_ARG
    assert L.afsai_spmm(None, 4, None, None, None) == af.ERR_INVALID_ARG
    hm = ctypes.c_void_p(0x1)
    assert L.afsai_matrix_prepare(None, None, ctypes.byref(hm)) == af.ERR_INVALID_ARG
    assert hm.value is None
    assert L.afsai_matrix_prepare(ctypes.byref(A), None, None) == af.ERR_INVALID_ARG
    assert L.afsai_spmm_prepared(None, 4, None, None, None) == af.ERR_INVALID_ARG
    assert L.pcg_solve_prepared(None, None, None, None, 1e-8, 10, None, None) == af.ERR_INVALID_ARG
    L.afsai_matrix_destroy(None)
    assert L.pcg_solve_multi(None, None, 3, None, None, 1e-8, 10, None, None) == af.ERR_INVALID_ARG
    assert L.pcg_solve_multi(None, None, 2, None, None, 1e-8, 10, None, None) == af.ERR_INVALID_ARG
    assert L.afsai_import(None, 0, None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert b"null" in L.afsai_last_error() or len(L.afsai_last_error()) > 0
    L.afsai_destroy(None)


def test_options_validated_on_host(L):
    assert L.afsai_set_option(af.OPT_SPMV_GROUP, 3) == af.ERR_INVALID_ARG
    assert L.afsai_set_option(af.OPT_SETUP_TABLE, 4096) == af.ERR_INVALID_ARG
    assert L.afsai_set_option(99, 0) == af.ERR_INVALID_ARG
    assert L.afsai_set_option(af.OPT_SELL_RUNS, 2) == af.ERR_INVALID_ARG
    assert L.afsai_set_option(af.OPT_SELL_RUNS, 1) == af.OK
    assert L.afsai_set_option(af.OPT_SELL_RUNS, 0) == af.OK
    assert L.afsai_set_option(af.OPT_SPMV_GROUP, 16) == af.OK
    assert L.afsai_set_option(af.OPT_SPMV_GROUP, 0) == af.OK


def test_profile_toggle_without_gpu(L):
    assert L.afsai_profile_enable(0) == af.OK
    arr = (af.KernelTimeStruct * 4)()
    cnt = ctypes.c_int32(-1)
    assert L.afsai_profile_read(arr, 4, ctypes.byref(cnt), 1) == af.OK
    assert cnt.value == 0


def test_batched_arguments_rejected_on_host(L):
    h = ctypes.c_void_p()
    p = af.ParamsStruct(5, 1, 1e-2, af.TIE_RTOL, af.F64, 0)
    A = _fake_csr(n=10, nnz=10)
    I32 = ctypes.c_int32

    def offs(*v):
        return (I32 * len(v))(*v)

    assert L.afsai_setup_batched(ctypes.byref(A), 2, None, ctypes.byref(p), None, ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert L.afsai_setup_batched(ctypes.byref(A), 0, offs(0, 10), ctypes.byref(p), None,
                                 ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert L.afsai_setup_batched(ctypes.byref(A), 2, offs(1, 5, 10), ctypes.byref(p), None,
                                 ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert L.afsai_setup_batched(ctypes.byref(A), 2, offs(0, 5, 9), ctypes.byref(p), None,
                                 ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert L.afsai_setup_batched(ctypes.byref(A), 2, offs(0, 5, 5), ctypes.byref(p), None,
                                 ctypes.byref(h)) == af.ERR_INVALID_ARG
    assert h.value is None
    info = (af.PcgInfoStruct * 2)()
    x = ctypes.c_void_p(0x10)
    bb = ctypes.c_void_p(0x20)
    assert L.pcg_solve_batched(ctypes.byref(A), None, 2, offs(0, 7, 6), bb, x, 1e-8, 10, None, info) == af.ERR_INVALID_ARG
    assert L.pcg_solve_batched(ctypes.byref(A), None, 2, None, bb, x, 1e-8, 10, None, info) == af.ERR_INVALID_ARG
    assert L.pcg_solve_batched(ctypes.byref(A), None, 2, offs(0, 5, 10), bb, x, 0.0, 10, None, info) == af.ERR_INVALID_ARG


def test_binding_rejects_host_and_misshapen_blocks(L):
    """The binding checks every block it hands to the library (float64, contiguous, on the GPU,
    the right shape) before any call, so a host or short tensor never reaches a kernel."""
    import torch

    rp = torch.tensor([0, 1, 2], dtype=torch.int32)
    ci = torch.tensor([0, 1], dtype=torch.int32)
    va = torch.tensor([2.0, 3.0], dtype=torch.float64)
    A = af.DeviceCSR(rp, ci, va)
    with pytest.raises(ValueError, match="CUDA"):
        af.spmm(A, torch.zeros((2, 4), dtype=torch.float64))
    with pytest.raises(ValueError):
        af.spmm(A, torch.zeros(2, dtype=torch.float64))
    with pytest.raises(ValueError, match="CUDA"):
        af.pcg_solve_multi(A, None, torch.zeros((2, 2), dtype=torch.float64))
    with pytest.raises(ValueError, match="CUDA"):
        af.spmv(A, torch.zeros(2, dtype=torch.float64))
    with pytest.raises(ValueError, match="CUDA"):
        af.pcg_solve(A, None, torch.zeros(2, dtype=torch.float64))
