"""Workspace layouts against the sizes their producers write (host only, no GPU).

A region of the caller's workspace that is shorter than what a kernel writes into it is
an out-of-bounds write on the device.  qb_layout_check recomputes, on the host, every
producer's extent with the same size functions the launchers use, for the problem given,
and compares it with the region make_layout carved."""
import ctypes
import itertools

import pytest

import paper_1606_09402_amd as qb


def _check(algo, sparse, dtype, m, n, nnz, b, l_max, l_tilde=0, power=0, oversample=0):
    L = qb.lib()
    L.qb_layout_check.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.POINTER(qb.QbParams), ctypes.c_int32]
    L.qb_layout_check.restype = ctypes.c_int
    p = qb._params(1e-2, b, l_max, l_tilde, 1, True, power)
    return L.qb_layout_check(algo, 1 if sparse else 0, dtype, m, n, nnz, ctypes.byref(p), oversample)


SHAPES = [(1, 1), (7, 5), (64, 64), (100, 37), (1000, 800), (600, 4100), (5000, 3000), (20000, 15000)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_dense_layouts(m, n):
    for algo, b, lt, power in itertools.product((qb.QB_ALGO_FP, qb.QB_ALGO_EI), (1, 16, 50, 64, 128),
                                                (0, -1), (0, 1)):
        if algo == qb.QB_ALGO_EI and power:
            continue
        lmax = min(m, n)
        assert _check(algo, False, qb.QB_F64, m, n, 0, b, lmax, lt, power) == qb.QB_OK, (algo, b, lt, power)


@pytest.mark.parametrize("m,n", SHAPES)
def test_lowp_layouts(m, n):
    for dt, b in itertools.product((qb.QB_BF16, qb.QB_FP8E4M3), (1, 20, 64, 128)):
        assert _check(qb.QB_ALGO_FP, False, dt, m, n, 0, b, min(m, n)) == qb.QB_OK, (dt, b)


@pytest.mark.parametrize("m,n,nnz", [(7, 5, 0), (100, 37, 300), (1000, 800, 20000), (50000, 20000, 500000),
                                     (500000, 200000, 5000000)])
def test_csr_layouts(m, n, nnz):
    for algo, b, power in itertools.product((qb.QB_ALGO_FP, qb.QB_ALGO_EI), (1, 50, 128), (0, 1)):
        if algo == qb.QB_ALGO_EI and power:
            continue
        lmax = min(m, n, 16384)
        assert _check(algo, True, qb.QB_F64, m, n, nnz, b, lmax, 0, power) == qb.QB_OK, (algo, b, power)


@pytest.mark.parametrize("m,n", SHAPES[1:])
def test_trqrcp_layouts(m, n):
    for b, over in itertools.product((1, 16, 64), (1, 8, 64)):
        assert _check(qb.QB_ALGO_EI, False, qb.QB_F64, m, n, 0, b, min(m, n), 0, 0, over) == qb.QB_OK


def test_layout_check_rejects_bad_arguments():
    assert _check(qb.QB_ALGO_FP, False, qb.QB_F64, 100, 50, 0, 0, 50) == qb.QB_ERR_ARG
    assert _check(7, False, qb.QB_F64, 100, 50, 0, 8, 50) == qb.QB_ERR_ARG
