"""The C-ABI library loads and exports every entry point include/qb.h declares;
argument checks that need no GPU.  CPU only (no compute calls)."""
import ctypes
import os
import re

import pytest

import paper_1606_09402_amd as qb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "qb.h")).read()
    return re.findall(r"QB_API\s+[\w\s\*]+?\b(qb_\w+)\s*\(", txt)


def test_header_declares_the_boundary():
    names = set(_declared())
    for n in ("qb_fp_dense", "qb_ei_dense", "qb_fp_csr", "qb_ei_csr", "qb_workspace_bytes",
              "qb_gaussian_fill", "qb_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = qb.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_only_abi_symbols_exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", qb.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("nm not available")
    funcs = [l.split()[-1] for l in out.stdout.splitlines() if " T " in l]
    assert funcs and all(f.startswith("qb_") for f in funcs), funcs


def test_status_strings():
    assert qb.qb_status_string(0) == "QB_OK"
    assert qb.qb_status_string(-3) == "QB_ERR_WORKSPACE"
    assert qb.qb_status_string(2) == "QB_WARN_TOL_FLOOR"
    assert qb.qb_status_string(99) == "QB_UNKNOWN_STATUS"


def test_workspace_query_validates_arguments():
    ok = qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, 1e-2, 20, 800)
    assert ok > 8 * (800 * 800 + 1000 * 800)        # Omega, G, H chunks at l~ = 800
    assert qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, 1e-2, 0, 800) == 0     # b = 0
    assert qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, 1e-2, 129, 800) == 0   # b > 128
    assert qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, 1e-2, 20, 801) == 0    # l_max
    assert qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, -1.0, 20, 800) == 0    # tol
    assert qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, 1e-2, 20, 800, 30) == 0  # l~ % b
    small = qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, 1000, 800, 0, 1e-2, 20, 800, 100)
    assert 0 < small < ok
    ei = qb.qb_workspace_bytes(qb.QB_ALGO_EI, False, 1000, 800, 0, 1e-2, 20, 800)
    assert 0 < ei < ok


def test_entry_points_reject_bad_arguments_without_gpu():
    L = qb.lib()
    p = qb.QbParams(1e-2, 20, 0, 10, 0, 1, 1, 0)
    info = qb.QbInfo()
    # NULL matrix descriptor / NULL data pointer -> QB_ERR_ARG before any device work
    assert L.qb_fp_dense(None, ctypes.byref(p), None, 0, None, 0, None, 0, None, ctypes.byref(info)) == -1
    d = qb.QbDense(100, 50, 50, 0, 0, None)
    assert L.qb_ei_dense(ctypes.byref(d), ctypes.byref(p), None, 0, None, 0, None, 0, None, None) == -1
    d = qb.QbDense(100, 50, 40, 0, 0, 1 << 20)          # lda < n
    assert L.qb_fp_dense(ctypes.byref(d), ctypes.byref(p), None, 0, None, 0, None, 0, None, None) == -1
    d = qb.QbDense(100, 50, 50, 7, 0, 1 << 20)          # unknown element type
    assert L.qb_fp_dense(ctypes.byref(d), ctypes.byref(p), None, 0, None, 0, None, 0, None, None) == -5
    # the power scheme is randQB_FP's on binary64 A: EI and the bfloat16 form reject P > 0,
    # and P outside [0, 16] is a bad argument, all before any device work
    p_pow = qb.QbParams(1e-2, 20, 1, 10, 0, 1, 1, 0)
    d = qb.QbDense(100, 50, 50, 0, 0, 1 << 20)
    assert L.qb_ei_dense(ctypes.byref(d), ctypes.byref(p_pow), 1 << 20, 100, 1 << 20, 50, 1 << 20, 1 << 30,
                         None, None) == -5
    d16 = qb.QbDense(100, 50, 50, 1, 0, 1 << 20)
    assert L.qb_fp_dense(ctypes.byref(d16), ctypes.byref(p_pow), 1 << 20, 100, 1 << 20, 50, 1 << 20,
                         1 << 30, None, None) == -5
    for bad in (-1, 17):
        p_bad = qb.QbParams(1e-2, 20, bad, 10, 0, 1, 1, 0)
        assert L.qb_fp_dense(ctypes.byref(d), ctypes.byref(p_bad), 1 << 20, 100, 1 << 20, 50, 1 << 20,
                             1 << 30, None, None) == -1
        assert L.qb_workspace_bytes(0, 0, 100, 50, 0, ctypes.byref(p_bad)) == 0
    c = qb.QbCsr(100, 50, 10, None, None, None)
    assert L.qb_fp_csr(ctypes.byref(c), ctypes.byref(p), None, 0, None, 0, None, 0, None, None) == -1
    # COO: NULL descriptor, NULL arrays with nnz > 0, negative nnz
    assert L.qb_fp_coo(None, ctypes.byref(p), None, 0, None, 0, None, 0, None, None) == -1
    co = qb.QbCoo(100, 50, 10, None, None, None)
    assert L.qb_ei_coo(ctypes.byref(co), ctypes.byref(p), None, 0, None, 0, None, 0, None, None) == -1
    assert L.qb_coo_workspace_bytes(0, ctypes.byref(co), ctypes.byref(p)) == 0
    assert L.qb_coo_to_csr_bytes(ctypes.byref(qb.QbCoo(100, 50, -1, None, None, None))) == 0
    assert L.qb_coo_to_csr_bytes(ctypes.byref(qb.QbCoo(100, 50, 0, None, None, None))) > 0
    assert L.qb_gaussian_fill(1, 0, 0, 0, 0, 4, 4, None, 4, None) == -1


def test_trqrcp_argument_checks_without_gpu():
    L = qb.lib()
    ok = qb.qb_trqrcp_workspace_bytes(1000, 800, 1e-2, 32, 400, 8)
    assert ok > 8 * (800 * 40 + 1000 * 40)               # the sketch and its Gaussian
    assert qb.qb_trqrcp_workspace_bytes(1000, 800, 1e-2, 32, 400, -1) == 0
    assert qb.qb_trqrcp_workspace_bytes(1000, 800, 1e-2, 32, 400, 129) == 0
    assert qb.qb_trqrcp_workspace_bytes(1000, 800, 1e-2, 0, 400, 8) == 0
    assert qb.qb_trqrcp_workspace_bytes(1000, 800, 1e-2, 32, 801, 8) == 0
    p = qb.QbParams(1e-2, 20, 0, 10, 0, 1, 1, 0)
    d = qb.QbDense(100, 50, 50, 0, 0, 1 << 20)
    args = (1 << 20, 100, 1 << 20, 50, 1 << 20, 1 << 20, 1 << 30, None, None)
    assert L.qb_trqrcp_dense(None, ctypes.byref(p), 8, *args) == -1
    assert L.qb_trqrcp_dense(ctypes.byref(d), ctypes.byref(p), -1, *args) == -1
    assert L.qb_trqrcp_dense(ctypes.byref(d), ctypes.byref(p), 129, *args) == -1
    assert L.qb_trqrcp_dense(ctypes.byref(d), ctypes.byref(p), 8, 1 << 20, 100, 1 << 20, 50, None,
                             1 << 20, 1 << 30, None, None) == -1          # no pivot output
    p_pow = qb.QbParams(1e-2, 20, 1, 10, 0, 1, 1, 0)
    assert L.qb_trqrcp_dense(ctypes.byref(d), ctypes.byref(p_pow), 8, *args) == -5
    d16 = qb.QbDense(100, 50, 50, 1, 0, 1 << 20)
    assert L.qb_trqrcp_dense(ctypes.byref(d16), ctypes.byref(p), 8, *args) == -5


def test_noalloc_entry_rejects_before_device_work():
    """qb_fp_dense_noalloc checks its arguments and the scratch budget before any HIP call,
    so these run without a GPU (the pointers are never dereferenced)."""
    L = qb.lib()
    d = qb.QbDense(4096, 4096, 4096, qb.QB_F64, 0, 16, None)
    p = qb._params(1e-2, 64, 4096, 0, 1, True)
    info = qb.QbInfo()
    fake = ctypes.c_void_p(256)
    st = L.qb_fp_dense_noalloc(ctypes.byref(d), ctypes.byref(p), fake, 4096, fake, 4096, None,
                               ctypes.byref(info))
    assert st == qb.QB_ERR_WORKSPACE and info.status == st
    bad = qb._params(1e-2, 0, 4096, 0, 1, True)         # b = 0
    assert L.qb_fp_dense_noalloc(ctypes.byref(d), ctypes.byref(bad), fake, 4096, fake, 4096, None,
                                 None) == qb.QB_ERR_ARG
    assert L.qb_fp_dense_noalloc(None, ctypes.byref(p), fake, 4096, fake, 4096, None, None) == qb.QB_ERR_ARG
