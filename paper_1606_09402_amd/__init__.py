"""Python binding of the MI355X fixed-precision randomized QB library (libqb.so).

Thin ctypes marshalling over the C ABI declared in include/qb.h: the functions here
carry the same names as the C entry points, turn torch tensors into device pointers
and the current HIP stream, allocate the caller-owned outputs / workspace with torch,
and raise on error statuses.  Every step of the method runs in the library's HIP
kernels; there is no CPU fallback -- if libqb.so is missing the import of the library
fails loudly (build it with ``paper_1606_09402_amd.build.build()``).

Method: Yu, Gu, Li, "Efficient randomized algorithms for the fixed-precision low-rank
matrix approximation" (arXiv 1606.09402): randQB_FP (Algorithm 4, P = 0) and randQB_EI
(Algorithm 2) with the Frobenius error indicator of Theorem 1 / Algorithm 1.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch  # noqa: F401  (load torch's HIP runtime first: libqb.so then binds to it)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "libqb.so")

QB_OK, QB_NOT_CONVERGED, QB_WARN_TOL_FLOOR = 0, 1, 2
QB_ERR_ARG, QB_ERR_NONFINITE, QB_ERR_WORKSPACE, QB_ERR_HIP, QB_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
QB_ALGO_FP, QB_ALGO_EI = 0, 1
QB_F64, QB_BF16, QB_F32, QB_FP8E4M3 = 0, 1, 2, 3

_c_i64 = ctypes.c_int64
_c_i32 = ctypes.c_int32
_vp = ctypes.c_void_p


class QbDense(ctypes.Structure):
    _fields_ = [("m", _c_i64), ("n", _c_i64), ("lda", _c_i64), ("dtype", _c_i32),
                ("reserved", _c_i32), ("a", _vp), ("row_exp", _vp)]


class QbCsr(ctypes.Structure):
    _fields_ = [("m", _c_i64), ("n", _c_i64), ("nnz", _c_i64), ("rowptr", _vp), ("colind", _vp),
                ("val", _vp)]


class QbCoo(ctypes.Structure):
    _fields_ = [("m", _c_i64), ("n", _c_i64), ("nnz", _c_i64), ("row", _vp), ("col", _vp), ("val", _vp)]


class QbBatch(ctypes.Structure):
    _fields_ = [("batch", _c_i64), ("m", _c_i64), ("n", _c_i64), ("lda", _c_i64), ("stride_a", _c_i64),
                ("dtype", _c_i32), ("reserved", _c_i32), ("a", _vp)]


class QbParams(ctypes.Structure):
    _fields_ = [("tol_rel", ctypes.c_double), ("b", _c_i32), ("power", _c_i32), ("l_max", _c_i64),
                ("l_tilde", _c_i64), ("seed", ctypes.c_uint64), ("row_by_row", _c_i32),
                ("reserved", _c_i32)]


class QbInfo(ctypes.Structure):
    _fields_ = [("rank", _c_i64), ("E", ctypes.c_double), ("normA2", ctypes.c_double),
                ("status", _c_i32), ("passes", _c_i32), ("blocks", _c_i32), ("chunks", _c_i32),
                ("exhausted", _c_i32), ("fallbacks", _c_i32), ("ms", ctypes.c_double * 8),
                ("gemm_flops", ctypes.c_double * 2)]


class QBError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {qb_status_string(status)} ({status})")
        self.status = status


_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded libqb.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1606_09402_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.qb_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, _c_i64, _c_i64, _c_i64, P(QbParams)]
        L.qb_workspace_bytes.restype = ctypes.c_size_t
        L.qb_dense_workspace_bytes.argtypes = [ctypes.c_int, P(QbDense), P(QbParams)]
        L.qb_dense_workspace_bytes.restype = ctypes.c_size_t
        L.qb_sketch_lowp_bytes.argtypes = [P(QbDense), _c_i64]
        L.qb_sketch_lowp_bytes.restype = ctypes.c_size_t
        L.qb_sketch_lowp.argtypes = [P(QbDense), ctypes.c_uint64, _c_i64, _c_i64, _vp, _vp, _vp, _vp,
                                     ctypes.c_size_t, _vp]
        L.qb_sketch_lowp.restype = ctypes.c_int
        for nm in ("qb_fp_dense", "qb_ei_dense"):
            f = getattr(L, nm)
            f.argtypes = [P(QbDense), P(QbParams), _vp, _c_i64, _vp, _c_i64, _vp, ctypes.c_size_t, _vp,
                          P(QbInfo)]
            f.restype = ctypes.c_int
        L.qb_fp_dense_noalloc.argtypes = [P(QbDense), P(QbParams), _vp, _c_i64, _vp, _c_i64, _vp, P(QbInfo)]
        L.qb_fp_dense_noalloc.restype = ctypes.c_int
        for nm in ("qb_fp_csr", "qb_ei_csr"):
            f = getattr(L, nm)
            f.argtypes = [P(QbCsr), P(QbParams), _vp, _c_i64, _vp, _c_i64, _vp, ctypes.c_size_t, _vp,
                          P(QbInfo)]
            f.restype = ctypes.c_int
        L.qb_gaussian_fill.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _c_i64, _c_i64,
                                       _c_i64, _c_i64, _vp, _c_i64, _vp]
        L.qb_gaussian_fill.restype = ctypes.c_int
        L.qb_sumsq_workspace_bytes.argtypes = []
        L.qb_sumsq_workspace_bytes.restype = ctypes.c_size_t
        L.qb_sumsq_dense.argtypes = [P(QbDense), P(ctypes.c_double), _vp, _vp]
        L.qb_sumsq_dense.restype = ctypes.c_int
        L.qb_sketch_dense.argtypes = [P(QbDense), ctypes.c_uint64, _c_i64, _c_i64, _vp, _vp, _vp, _vp]
        L.qb_sketch_dense.restype = ctypes.c_int
        L.qb_csr_transpose_bytes.argtypes = [P(QbCsr)]
        L.qb_csr_transpose_bytes.restype = ctypes.c_size_t
        L.qb_sketch_csr.argtypes = [P(QbCsr), ctypes.c_uint64, _c_i64, _c_i64, _vp, _vp, _vp, _vp,
                                    P(ctypes.c_int), _vp]
        L.qb_sketch_csr.restype = ctypes.c_int
        L.qb_fixed_rank_workspace_bytes.argtypes = [P(QbBatch), _c_i64, _c_i32]
        L.qb_fixed_rank_workspace_bytes.restype = ctypes.c_size_t
        L.qb_fixed_rank_fwd.argtypes = [P(QbBatch), _c_i64, _c_i32, ctypes.c_uint64, _vp, _c_i64, _c_i64,
                                        _vp, _c_i64, _c_i64, _vp, ctypes.c_size_t, _vp, _vp]
        L.qb_fixed_rank_fwd.restype = ctypes.c_int
        L.qb_fixed_rank_bwd.argtypes = [P(QbBatch), _c_i64, _c_i32, ctypes.c_uint64, _vp, _c_i64, _c_i64,
                                        _vp, _c_i64, _c_i64, _vp, _c_i64, _c_i64, _vp, _c_i64, _c_i64,
                                        _vp, ctypes.c_size_t, _vp]
        L.qb_fixed_rank_bwd.restype = ctypes.c_int
        L.qb_coo_workspace_bytes.argtypes = [ctypes.c_int, P(QbCoo), P(QbParams)]
        L.qb_coo_workspace_bytes.restype = ctypes.c_size_t
        for nm in ("qb_fp_coo", "qb_ei_coo"):
            f = getattr(L, nm)
            f.argtypes = [P(QbCoo), P(QbParams), _vp, _c_i64, _vp, _c_i64, _vp, ctypes.c_size_t, _vp,
                          P(QbInfo)]
            f.restype = ctypes.c_int
        L.qb_coo_to_csr_bytes.argtypes = [P(QbCoo)]
        L.qb_coo_to_csr_bytes.restype = ctypes.c_size_t
        L.qb_coo_to_csr.argtypes = [P(QbCoo), _vp, _vp, _vp, P(_c_i64), _vp, ctypes.c_size_t, _vp]
        L.qb_coo_to_csr.restype = ctypes.c_int
        L.qb_sketch_onepass_bytes.argtypes = [P(QbDense), _c_i64, _c_i64]
        L.qb_sketch_onepass_bytes.restype = ctypes.c_size_t
        L.qb_sketch_onepass.argtypes = [P(QbDense), ctypes.c_uint64, _c_i64, _c_i64, _c_i64, _vp, _vp, _vp,
                                        _vp, ctypes.c_size_t, _vp]
        L.qb_sketch_onepass.restype = ctypes.c_int
        L.qb_trqrcp_workspace_bytes.argtypes = [_c_i64, _c_i64, P(QbParams), _c_i32]
        L.qb_trqrcp_workspace_bytes.restype = ctypes.c_size_t
        L.qb_trqrcp_dense.argtypes = [P(QbDense), P(QbParams), _c_i32, _vp, _c_i64, _vp, _c_i64, _vp, _vp,
                                      ctypes.c_size_t, _vp, P(QbInfo)]
        L.qb_trqrcp_dense.restype = ctypes.c_int
        L.qb_svd_workspace_bytes.argtypes = [_c_i64, _c_i64, _c_i64]
        L.qb_svd_workspace_bytes.restype = ctypes.c_size_t
        L.qb_svd_from_qb.argtypes = [_c_i64, _c_i64, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp,
                                     _vp, _c_i64, _vp, ctypes.c_size_t, _vp, P(_c_i32)]
        L.qb_svd_from_qb.restype = ctypes.c_int
        L.qb_status_string.argtypes = [ctypes.c_int]
        L.qb_status_string.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def qb_status_string(status: int) -> str:
    return lib().qb_status_string(int(status)).decode()


# ------------------------------------------------------------------ marshalling helpers


def _stream_ptr(dev: torch.device):
    return _vp(torch.cuda.current_stream(dev).cuda_stream)


def _check_dev(t: torch.Tensor, name: str, dtype=torch.float64):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")


_DTYPES = {torch.float64: QB_F64, torch.bfloat16: QB_BF16, torch.float8_e4m3fn: QB_FP8E4M3}


def _dense(A: torch.Tensor, row_exp: torch.Tensor | None = None) -> QbDense:
    """A: float64, bfloat16, or float8_e4m3fn with row_exp (int32, one per row): the
    matrix 2^row_exp[i] * A[i, j]."""
    if not A.is_cuda:
        raise ValueError("A must be a GPU tensor")
    if A.dtype not in _DTYPES:
        raise ValueError("A must be float64, bfloat16 or float8_e4m3fn")
    if A.dim() != 2 or A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise ValueError("A must be a row-major 2-D view (stride(1) == 1)")
    re_ptr = None
    if A.dtype == torch.float8_e4m3fn:
        if (row_exp is None or not row_exp.is_cuda or row_exp.dtype != torch.int32
                or row_exp.numel() != A.shape[0] or not row_exp.is_contiguous()):
            raise ValueError("an e4m3 A needs row_exp: a contiguous int32 GPU tensor with one entry per row")
        re_ptr = row_exp.data_ptr()
    return QbDense(A.shape[0], A.shape[1], A.stride(0), _DTYPES[A.dtype], 0, A.data_ptr(), re_ptr)


def _csr(m: int, n: int, rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor) -> QbCsr:
    _check_dev(rowptr, "rowptr", torch.int64)
    _check_dev(colind, "colind", torch.int32)
    _check_dev(val, "val")
    for t, nm in ((rowptr, "rowptr"), (colind, "colind"), (val, "val")):
        if not t.is_contiguous():
            raise ValueError(f"{nm} must be contiguous")
    if rowptr.numel() != m + 1 or colind.numel() != val.numel():
        raise ValueError("CSR arrays have inconsistent sizes")
    return QbCsr(m, n, val.numel(), rowptr.data_ptr(), colind.data_ptr(), val.data_ptr())


def _params(tol, b, l_max, l_tilde, seed, row_by_row, power=0) -> QbParams:
    return QbParams(float(tol), int(b), int(power), int(l_max), int(l_tilde), int(seed) & (2 ** 64 - 1),
                    1 if row_by_row else 0, 0)


@dataclass
class QBResult:
    Q: torch.Tensor          # m x rank view (column-major storage)
    B: torch.Tensor          # rank x n view
    rank: int
    E: float
    normA2: float
    status: int
    passes: int
    blocks: int
    chunks: int
    exhausted: int
    fallbacks: int
    ms: list = field(default_factory=list)
    gemm_flops: list = field(default_factory=list)
    Q_store: torch.Tensor | None = None   # l_max x m (row i = column i of Q)
    B_store: torch.Tensor | None = None   # l_max x n


def _run(kind: str, algo: int, sparse: bool, mat, m: int, n: int, dev, tol, b, l_max, l_tilde,
         seed, row_by_row, Q_store, B_store, ws, power=0) -> QBResult:
    L = lib()
    l_max = min(m, n) if l_max is None else int(l_max)
    p = _params(tol, b, l_max, l_tilde, seed, row_by_row, power)
    if kind.endswith("_coo"):
        need = L.qb_coo_workspace_bytes(algo, ctypes.byref(mat), ctypes.byref(p))
    elif sparse:
        need = L.qb_workspace_bytes(algo, 1, m, n, mat.nnz, ctypes.byref(p))
    else:
        need = L.qb_dense_workspace_bytes(algo, ctypes.byref(mat), ctypes.byref(p))
    fn = getattr(L, kind)
    if need == 0:   # invalid parameters: let the entry point report which status applies
        st = fn(ctypes.byref(mat), ctypes.byref(p), None, 0, None, 0, None, 0, _stream_ptr(dev), None)
        raise QBError(st if st < 0 else QB_ERR_ARG, kind)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    if Q_store is None:
        Q_store = torch.empty((l_max, m), dtype=torch.float64, device=dev)
    if B_store is None:
        B_store = torch.empty((l_max, n), dtype=torch.float64, device=dev)
    if Q_store.shape[0] < l_max or Q_store.stride(1) != 1 or Q_store.stride(0) < m:
        raise ValueError("Q_store must be at least l_max x m with unit column stride")
    if B_store.shape[0] < l_max or B_store.stride(1) != 1 or B_store.stride(0) < n:
        raise ValueError("B_store must be at least l_max x n with unit column stride")
    info = QbInfo()
    st = fn(ctypes.byref(mat), ctypes.byref(p), Q_store.data_ptr(), Q_store.stride(0),
            B_store.data_ptr(), B_store.stride(0), ws.data_ptr(), ws.numel(), _stream_ptr(dev),
            ctypes.byref(info))
    if st < 0:
        raise QBError(st, kind)
    r = int(info.rank)
    return QBResult(Q=Q_store[:r].T, B=B_store[:r], rank=r, E=info.E, normA2=info.normA2, status=st,
                    passes=info.passes, blocks=info.blocks, chunks=info.chunks,
                    exhausted=info.exhausted, fallbacks=info.fallbacks, ms=list(info.ms),
                    gemm_flops=list(info.gemm_flops), Q_store=Q_store, B_store=B_store)


# ------------------------------------------------------------------ public entry points


def qb_fp_dense(A: torch.Tensor, tol: float, b: int, seed: int, l_max=None, l_tilde: int = 0,
                row_by_row: bool = True, Q_store=None, B_store=None, ws=None, power: int = 0,
                row_exp: torch.Tensor | None = None) -> QBResult:
    """randQB_FP (Algorithm 4, P = 0) on dense A (GPU, row-major): float64, or for the
    precision form bfloat16 / float8_e4m3fn with row_exp (bfloat16 sketch products,
    binary64 block loop)."""
    d = _dense(A, row_exp)
    return _run("qb_fp_dense", QB_ALGO_FP, False, d, d.m, d.n, A.device, tol, b, l_max, l_tilde,
                seed, row_by_row, Q_store, B_store, ws, power)


def qb_fp_dense_noalloc(A: torch.Tensor, tol: float, b: int, seed: int, l_max=None, l_tilde: int = 0,
                        row_by_row: bool = True, Q_store=None, B_store=None, power: int = 0,
                        row_exp: torch.Tensor | None = None) -> QBResult:
    """qb_fp_dense without a workspace: the library works in its static device scratch array
    (QB_NOALLOC_SCRATCH_BYTES) and allocates nothing.  Pass Q_store / B_store to keep this
    wrapper from allocating them."""
    L = lib()
    d = _dense(A, row_exp)
    m, n, dev = d.m, d.n, A.device
    l_max = min(m, n) if l_max is None else int(l_max)
    p = _params(tol, b, l_max, l_tilde, seed, row_by_row, power)
    if Q_store is None:
        Q_store = torch.empty((l_max, m), dtype=torch.float64, device=dev)
    if B_store is None:
        B_store = torch.empty((l_max, n), dtype=torch.float64, device=dev)
    if Q_store.shape[0] < l_max or Q_store.stride(1) != 1 or Q_store.stride(0) < m:
        raise ValueError("Q_store must be at least l_max x m with unit column stride")
    if B_store.shape[0] < l_max or B_store.stride(1) != 1 or B_store.stride(0) < n:
        raise ValueError("B_store must be at least l_max x n with unit column stride")
    info = QbInfo()
    st = L.qb_fp_dense_noalloc(ctypes.byref(d), ctypes.byref(p), Q_store.data_ptr(), Q_store.stride(0),
                               B_store.data_ptr(), B_store.stride(0), _stream_ptr(dev), ctypes.byref(info))
    if st < 0:
        raise QBError(st, "qb_fp_dense_noalloc")
    r = int(info.rank)
    return QBResult(Q=Q_store[:r].T, B=B_store[:r], rank=r, E=info.E, normA2=info.normA2, status=st,
                    passes=info.passes, blocks=info.blocks, chunks=info.chunks,
                    exhausted=info.exhausted, fallbacks=info.fallbacks, ms=list(info.ms),
                    gemm_flops=list(info.gemm_flops), Q_store=Q_store, B_store=B_store)


def qb_ei_dense(A: torch.Tensor, tol: float, b: int, seed: int, l_max=None, row_by_row: bool = True,
                Q_store=None, B_store=None, ws=None, power: int = 0) -> QBResult:
    """randQB_EI (Algorithm 2) on dense float64 A (GPU, row-major)."""
    d = _dense(A)
    return _run("qb_ei_dense", QB_ALGO_EI, False, d, d.m, d.n, A.device, tol, b, l_max, 0, seed,
                row_by_row, Q_store, B_store, ws, power)


def qb_fp_csr(m: int, n: int, rowptr, colind, val, tol: float, b: int, seed: int, l_max=None,
              l_tilde: int = 0, row_by_row: bool = True, Q_store=None, B_store=None, ws=None,
              power: int = 0) -> QBResult:
    """randQB_FP on a CSR matrix (rowptr int64, colind int32, val float64; GPU tensors)."""
    c = _csr(m, n, rowptr, colind, val)
    return _run("qb_fp_csr", QB_ALGO_FP, True, c, m, n, val.device, tol, b, l_max, l_tilde, seed,
                row_by_row, Q_store, B_store, ws, power)


def qb_ei_csr(m: int, n: int, rowptr, colind, val, tol: float, b: int, seed: int, l_max=None,
              row_by_row: bool = True, Q_store=None, B_store=None, ws=None) -> QBResult:
    """randQB_EI on a CSR matrix."""
    c = _csr(m, n, rowptr, colind, val)
    return _run("qb_ei_csr", QB_ALGO_EI, True, c, m, n, val.device, tol, b, l_max, 0, seed,
                row_by_row, Q_store, B_store, ws)


@dataclass
class QRCPResult(QBResult):
    piv: torch.Tensor | None = None   # pivot columns in pivot order (rank entries, int32)


def qb_trqrcp_workspace_bytes(m: int, n: int, tol: float, b: int, l_max: int, oversample: int = 8,
                              seed: int = 0) -> int:
    p = _params(tol, b, l_max, 0, seed, True)
    return int(lib().qb_trqrcp_workspace_bytes(m, n, ctypes.byref(p), int(oversample)))


def qb_trqrcp_dense(A: torch.Tensor, tol: float, b: int, seed: int, oversample: int = 8, l_max=None,
                    row_by_row: bool = True, Q_store=None, B_store=None, piv_store=None,
                    ws=None) -> QRCPResult:
    """trQRCP driven by the indicator (Remark 3.2) on dense float64 A (GPU, row-major).
    B comes back in the original column order (B = R P^T); piv lists the pivot columns."""
    L = lib()
    d = _dense(A)
    m, n = d.m, d.n
    l_max = min(m, n) if l_max is None else int(l_max)
    p = _params(tol, b, l_max, 0, seed, row_by_row)
    dev = A.device
    need = L.qb_trqrcp_workspace_bytes(m, n, ctypes.byref(p), int(oversample))
    if need == 0:
        st = L.qb_trqrcp_dense(ctypes.byref(d), ctypes.byref(p), int(oversample), None, 0, None, 0, None,
                               None, 0, _stream_ptr(dev), None)
        raise QBError(st if st < 0 else QB_ERR_ARG, "qb_trqrcp_dense")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    if Q_store is None:
        Q_store = torch.empty((l_max, m), dtype=torch.float64, device=dev)
    if B_store is None:
        B_store = torch.empty((l_max, n), dtype=torch.float64, device=dev)
    if piv_store is None:
        piv_store = torch.empty(l_max, dtype=torch.int32, device=dev)
    if Q_store.shape[0] < l_max or Q_store.stride(1) != 1 or Q_store.stride(0) < m:
        raise ValueError("Q_store must be at least l_max x m with unit column stride")
    if B_store.shape[0] < l_max or B_store.stride(1) != 1 or B_store.stride(0) < n:
        raise ValueError("B_store must be at least l_max x n with unit column stride")
    if piv_store.numel() < l_max or piv_store.dtype != torch.int32 or not piv_store.is_contiguous():
        raise ValueError("piv_store must hold l_max contiguous int32")
    info = QbInfo()
    st = L.qb_trqrcp_dense(ctypes.byref(d), ctypes.byref(p), int(oversample), Q_store.data_ptr(),
                           Q_store.stride(0), B_store.data_ptr(), B_store.stride(0), piv_store.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream_ptr(dev), ctypes.byref(info))
    if st < 0:
        raise QBError(st, "qb_trqrcp_dense")
    r = int(info.rank)
    return QRCPResult(Q=Q_store[:r].T, B=B_store[:r], rank=r, E=info.E, normA2=info.normA2, status=st,
                      passes=info.passes, blocks=info.blocks, chunks=info.chunks,
                      exhausted=info.exhausted, fallbacks=info.fallbacks, ms=list(info.ms),
                      gemm_flops=list(info.gemm_flops), Q_store=Q_store, B_store=B_store,
                      piv=piv_store[:r])


def _coo(m: int, n: int, row: torch.Tensor, col: torch.Tensor, val: torch.Tensor) -> QbCoo:
    _check_dev(row, "row", torch.int32)
    _check_dev(col, "col", torch.int32)
    _check_dev(val, "val")
    for t, nm in ((row, "row"), (col, "col"), (val, "val")):
        if not t.is_contiguous():
            raise ValueError(f"{nm} must be contiguous")
    if not (row.numel() == col.numel() == val.numel()):
        raise ValueError("COO arrays have inconsistent sizes")
    return QbCoo(m, n, val.numel(), row.data_ptr(), col.data_ptr(), val.data_ptr())


def qb_fp_coo(m: int, n: int, row, col, val, tol: float, b: int, seed: int, l_max=None,
              l_tilde: int = 0, row_by_row: bool = True, Q_store=None, B_store=None, ws=None,
              power: int = 0) -> QBResult:
    """randQB_FP on COO triplets (row, col int32, val float64; GPU tensors; any order,
    duplicates summed).  ms[7] of the result is the conversion to CSR."""
    c = _coo(m, n, row, col, val)
    return _run("qb_fp_coo", QB_ALGO_FP, True, c, m, n, val.device, tol, b, l_max, l_tilde, seed,
                row_by_row, Q_store, B_store, ws, power)


def qb_ei_coo(m: int, n: int, row, col, val, tol: float, b: int, seed: int, l_max=None,
              row_by_row: bool = True, Q_store=None, B_store=None, ws=None) -> QBResult:
    """randQB_EI on COO triplets."""
    c = _coo(m, n, row, col, val)
    return _run("qb_ei_coo", QB_ALGO_EI, True, c, m, n, val.device, tol, b, l_max, 0, seed,
                row_by_row, Q_store, B_store, ws)


def coo_to_csr(m: int, n: int, row, col, val, ws=None):
    """The library's COO -> CSR conversion: (rowptr int64, colind int32, val float64)."""
    c = _coo(m, n, row, col, val)
    L = lib()
    need = L.qb_coo_to_csr_bytes(ctypes.byref(c))
    if need == 0:
        raise QBError(QB_ERR_ARG, "qb_coo_to_csr")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=val.device)
    nz = max(1, val.numel())
    rp = torch.empty(m + 1, dtype=torch.int64, device=val.device)
    ci = torch.empty(nz, dtype=torch.int32, device=val.device)
    va = torch.empty(nz, dtype=torch.float64, device=val.device)
    out = _c_i64(0)
    st = L.qb_coo_to_csr(ctypes.byref(c), rp.data_ptr(), ci.data_ptr(), va.data_ptr(), ctypes.byref(out),
                         ws.data_ptr(), ws.numel(), _stream_ptr(val.device))
    if st < 0:
        raise QBError(st, "qb_coo_to_csr")
    k = int(out.value)
    return rp, ci[:k], va[:k]


def qb_workspace_bytes(algo: int, sparse: bool, m: int, n: int, nnz: int, tol: float, b: int,
                       l_max: int, l_tilde: int = 0, power: int = 0) -> int:
    p = _params(tol, b, l_max, l_tilde, 0, True, power)
    return int(lib().qb_workspace_bytes(algo, 1 if sparse else 0, m, n, nnz, ctypes.byref(p)))


def qb_dense_workspace_bytes(algo: int, A: torch.Tensor, tol: float, b: int, l_max: int,
                             l_tilde: int = 0, row_exp: torch.Tensor | None = None,
                             power: int = 0) -> int:
    """Workspace bytes of qb_fp_dense / qb_ei_dense for this A (any supported dtype)."""
    p = _params(tol, b, l_max, l_tilde, 0, True, power)
    return int(lib().qb_dense_workspace_bytes(algo, ctypes.byref(_dense(A, row_exp)), ctypes.byref(p)))


def qb_gaussian_fill(seed: int, rows: int, cols: int, row0: int = 0, col0: int = 0,
                     stream_id: int = 0, batch: int = 0, out: torch.Tensor | None = None,
                     device="cuda") -> torch.Tensor:
    """Omega[row0:row0+rows, col0:col0+cols] (row-major float64 on the GPU)."""
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float64, device=device)
    _check_dev(out, "out")
    if out.dim() != 2 or out.shape[0] < rows or out.shape[1] < cols or out.stride(1) != 1:
        raise ValueError("out must be a row-major rows x cols view")
    st = lib().qb_gaussian_fill(int(seed) & (2 ** 64 - 1), stream_id, batch, row0, col0, rows, cols,
                                out.data_ptr(), out.stride(0), _stream_ptr(out.device))
    if st < 0:
        raise QBError(st, "qb_gaussian_fill")
    return out


def qb_sumsq_dense(A: torch.Tensor, row_exp: torch.Tensor | None = None) -> float:
    """||A||_F^2 of dense float64, bfloat16 or row-scaled e4m3 A as a deterministic GPU
    sum of squares."""
    L = lib()
    d = _dense(A, row_exp)
    ws = torch.empty(L.qb_sumsq_workspace_bytes(), dtype=torch.uint8, device=A.device)
    out = ctypes.c_double(0.0)
    st = L.qb_sumsq_dense(ctypes.byref(d), ctypes.byref(out), ws.data_ptr(), _stream_ptr(A.device))
    if st < 0:
        raise QBError(st, "qb_sumsq_dense")
    return out.value


def qb_sketch_dense(A: torch.Tensor, seed: int, col0: int, l: int):
    """(Omega, G = A Omega, H = A^T G) for Omega columns [col0, col0 + l)."""
    d = _dense(A)
    dev = A.device
    om = torch.empty((d.n, l), dtype=torch.float64, device=dev)
    g = torch.empty((d.m, l), dtype=torch.float64, device=dev)
    h = torch.empty((d.n, l), dtype=torch.float64, device=dev)
    st = lib().qb_sketch_dense(ctypes.byref(d), int(seed) & (2 ** 64 - 1), col0, l, om.data_ptr(),
                               g.data_ptr(), h.data_ptr(), _stream_ptr(dev))
    if st < 0:
        raise QBError(st, "qb_sketch_dense")
    return om, g, h


def qb_sketch_onepass_bytes_for(A: torch.Tensor, l: int, panel_rows: int = 0) -> int:
    d = _dense(A)
    return int(lib().qb_sketch_onepass_bytes(ctypes.byref(d), l, panel_rows))


def qb_sketch_onepass(A: torch.Tensor, seed: int, col0: int, l: int, panel_rows: int = 0, ws=None):
    """The single-pass sweep (Remark 4.2): (Omega, G, H) with A streamed once in row panels."""
    L = lib()
    d = _dense(A)
    dev = A.device
    need = L.qb_sketch_onepass_bytes(ctypes.byref(d), l, panel_rows)
    if need == 0:
        raise QBError(QB_ERR_ARG, "qb_sketch_onepass")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    om = torch.empty((d.n, l), dtype=torch.float64, device=dev)
    g = torch.empty((d.m, l), dtype=torch.float64, device=dev)
    h = torch.empty((d.n, l), dtype=torch.float64, device=dev)
    st = L.qb_sketch_onepass(ctypes.byref(d), int(seed) & (2 ** 64 - 1), col0, l, panel_rows, om.data_ptr(),
                             g.data_ptr(), h.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(dev))
    if st < 0:
        raise QBError(st, "qb_sketch_onepass")
    return om, g, h


def qb_sketch_lowp(A: torch.Tensor, seed: int, col0: int, l: int, row_exp: torch.Tensor | None = None):
    """Precision-form sweep on bfloat16 or row-scaled e4m3 A: (Omega_q, G_q, H = A_q^T G_q)
    as binary64."""
    L = lib()
    d = _dense(A, row_exp)
    if d.dtype not in (QB_BF16, QB_FP8E4M3):
        raise ValueError("qb_sketch_lowp takes a bfloat16 or float8_e4m3fn A")
    dev = A.device
    need = L.qb_sketch_lowp_bytes(ctypes.byref(d), l)
    if need == 0:
        raise QBError(QB_ERR_ARG, "qb_sketch_lowp")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    om = torch.empty((d.n, l), dtype=torch.float64, device=dev)
    g = torch.empty((d.m, l), dtype=torch.float64, device=dev)
    h = torch.empty((d.n, l), dtype=torch.float64, device=dev)
    st = L.qb_sketch_lowp(ctypes.byref(d), int(seed) & (2 ** 64 - 1), col0, l, om.data_ptr(),
                          g.data_ptr(), h.data_ptr(), ws.data_ptr(), need, _stream_ptr(dev))
    if st < 0:
        raise QBError(st, "qb_sketch_lowp")
    return om, g, h


def qb_sketch_csr(m: int, n: int, rowptr, colind, val, seed: int, col0: int, l: int, csc_ws=None):
    """(Omega, G = A Omega, H = A^T G) for CSR A; returns also the CSR(A^T) workspace."""
    L = lib()
    c = _csr(m, n, rowptr, colind, val)
    dev = val.device
    ready = ctypes.c_int(0)
    if csc_ws is None:
        csc_ws = torch.empty(L.qb_csr_transpose_bytes(ctypes.byref(c)), dtype=torch.uint8, device=dev)
    else:
        ready = ctypes.c_int(1)
    om = torch.empty((n, l), dtype=torch.float64, device=dev)
    g = torch.empty((m, l), dtype=torch.float64, device=dev)
    h = torch.empty((n, l), dtype=torch.float64, device=dev)
    st = L.qb_sketch_csr(ctypes.byref(c), int(seed) & (2 ** 64 - 1), col0, l, om.data_ptr(),
                         g.data_ptr(), h.data_ptr(), csc_ws.data_ptr(), ctypes.byref(ready),
                         _stream_ptr(dev))
    if st < 0:
        raise QBError(st, "qb_sketch_csr")
    return om, g, h, csc_ws


# ------------------------------------------------------------------ differentiation form

_BATCH_DTYPES = {torch.float32: QB_F32, torch.float64: QB_F64}


def _batch(A: torch.Tensor) -> QbBatch:
    """A (batch, m, n) GPU tensor, rows contiguous."""
    if not A.is_cuda or A.dtype not in _BATCH_DTYPES:
        raise ValueError("A must be a float32 or float64 GPU tensor")
    if A.dim() != 3 or A.stride(2) != 1 or A.stride(1) < A.shape[2]:
        raise ValueError("A must be (batch, m, n) with unit column stride")
    return QbBatch(A.shape[0], A.shape[1], A.shape[2], A.stride(1), A.stride(0), _BATCH_DTYPES[A.dtype], 0,
                   A.data_ptr())


def qb_fixed_rank_workspace_bytes(A: torch.Tensor, k: int, b: int) -> int:
    return int(lib().qb_fixed_rank_workspace_bytes(ctypes.byref(_batch(A)), int(k), int(b)))


def _ws_for(A, k, b, ws):
    need = qb_fixed_rank_workspace_bytes(A, k, b)
    if need == 0:
        raise QBError(QB_ERR_ARG, "qb_fixed_rank")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=A.device)
    return ws, need


def qb_fixed_rank_fwd(A: torch.Tensor, k: int, b: int, seed: int, ws=None, breakdown=None):
    """Fixed-rank randQB_FP of every matrix of A (batch, m, n): (Q (batch, m, k), B (batch, k, n)).

    breakdown: None (the call waits for the stream and raises on a CholeskyQR breakdown) or an
    int32 GPU tensor of one element that receives the breakdown flag in stream order (no wait;
    the caller checks it)."""
    d = _batch(A)
    ws, need = _ws_for(A, k, b, ws)
    bt, m, n = A.shape
    Q = torch.empty((bt, m, k), dtype=A.dtype, device=A.device)
    B = torch.empty((bt, k, n), dtype=A.dtype, device=A.device)
    flag = None
    if breakdown is not None:
        if breakdown.dtype != torch.int32 or not breakdown.is_cuda or breakdown.numel() < 1:
            raise ValueError("breakdown must be an int32 GPU tensor")
        flag = breakdown.data_ptr()
    st = lib().qb_fixed_rank_fwd(ctypes.byref(d), int(k), int(b), int(seed) & (2 ** 64 - 1), Q.data_ptr(),
                                 Q.stride(1), Q.stride(0), B.data_ptr(), B.stride(1), B.stride(0),
                                 ws.data_ptr(), ws.numel(), flag, _stream_ptr(A.device))
    if st < 0 or st == QB_NOT_CONVERGED:
        raise QBError(st, "qb_fixed_rank_fwd")
    return Q, B


def qb_fixed_rank_bwd(A: torch.Tensor, k: int, b: int, seed: int, Q: torch.Tensor, dQ=None, dB=None,
                      ws=None) -> torch.Tensor:
    """dL/dA of the fixed-rank map A -> (Q, B) given dL/dQ and dL/dB (either may be None)."""
    d = _batch(A)
    ws, need = _ws_for(A, k, b, ws)
    for t, nm in ((Q, "Q"), (dQ, "dQ"), (dB, "dB")):
        if t is not None and (t.dtype != A.dtype or not t.is_cuda or t.dim() != 3 or t.stride(2) != 1):
            raise ValueError(f"{nm} must be a (batch, rows, cols) GPU tensor of A's dtype, unit column stride")
    dA = torch.empty_like(A)
    nul = (None, 0, 0)
    q = (dQ.data_ptr(), dQ.stride(1), dQ.stride(0)) if dQ is not None else nul
    bb = (dB.data_ptr(), dB.stride(1), dB.stride(0)) if dB is not None else nul
    st = lib().qb_fixed_rank_bwd(ctypes.byref(d), int(k), int(b), int(seed) & (2 ** 64 - 1), Q.data_ptr(),
                                 Q.stride(1), Q.stride(0), *q, *bb, dA.data_ptr(), dA.stride(1),
                                 dA.stride(0), ws.data_ptr(), ws.numel(), _stream_ptr(A.device))
    if st < 0:
        raise QBError(st, "qb_fixed_rank_bwd")
    return dA


class FixedRankQB(torch.autograd.Function):
    """(Q, B) = fixed-rank randQB_FP(A) for a fixed Omega, with the library's hand-written
    backward (G = A Omega recomputed, not stored)."""

    @staticmethod
    def forward(ctx, A, k, b, seed):
        Q, B = qb_fixed_rank_fwd(A, k, b, seed)
        ctx.save_for_backward(A, Q)
        ctx.k, ctx.b, ctx.seed = k, b, seed
        return Q, B

    @staticmethod
    def backward(ctx, dQ, dB):
        A, Q = ctx.saved_tensors
        dQ = dQ.contiguous() if dQ is not None else None
        dB = dB.contiguous() if dB is not None else None
        dA = qb_fixed_rank_bwd(A, ctx.k, ctx.b, ctx.seed, Q, dQ, dB)
        return dA, None, None, None


def fixed_rank_qb(A: torch.Tensor, k: int, b: int, seed: int):
    """Differentiable fixed-rank QB of A ((batch, m, n) or (m, n), float32 or float64)."""
    if A.dim() == 2:
        Q, B = FixedRankQB.apply(A.unsqueeze(0).contiguous(), k, b, seed)
        return Q[0], B[0]
    return FixedRankQB.apply(A.contiguous(), k, b, seed)


def qb_svd_workspace_bytes(m: int, n: int, k: int) -> int:
    return int(lib().qb_svd_workspace_bytes(int(m), int(n), int(k)))


@dataclass
class SVDResult:
    U: torch.Tensor   # m x k view (column-major storage)
    s: torch.Tensor   # k, descending
    V: torch.Tensor   # n x k view (column-major storage)
    sweeps: int
    status: int


def svd_from_qb(Q: torch.Tensor, B: torch.Tensor, ws=None) -> SVDResult:
    """Eq. (3) on the GPU: A ~ QB = U diag(s) V^T.  Q is m x k with unit row stride
    (column-major, as QBResult.Q), B is k x n with unit column stride (as QBResult.B)."""
    m, k = Q.shape
    k2, n = B.shape
    if k2 != k or Q.dtype != torch.float64 or B.dtype != torch.float64 or not (Q.is_cuda and B.is_cuda):
        raise ValueError("Q (m x k) and B (k x n) must be float64 GPU tensors of matching k")
    if Q.stride(0) != 1 or B.stride(1) != 1:
        raise ValueError("Q must be column-major (unit row stride) and B row-major")
    need = qb_svd_workspace_bytes(m, n, k)
    if need == 0:
        raise QBError(QB_ERR_ARG, "qb_svd_from_qb")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=B.device)
    Ust = torch.empty((k, m), dtype=torch.float64, device=B.device)
    Vst = torch.empty((k, n), dtype=torch.float64, device=B.device)
    s = torch.empty(k, dtype=torch.float64, device=B.device)
    sweeps = _c_i32(0)
    st = lib().qb_svd_from_qb(m, n, k, Q.data_ptr(), Q.stride(1), B.data_ptr(), B.stride(0), Ust.data_ptr(),
                              m, s.data_ptr(), Vst.data_ptr(), n, ws.data_ptr(), ws.numel(),
                              _stream_ptr(B.device), ctypes.byref(sweeps))
    if st < 0:
        raise QBError(st, "qb_svd_from_qb")
    return SVDResult(U=Ust.T, s=s, V=Vst.T, sweeps=int(sweeps.value), status=st)
