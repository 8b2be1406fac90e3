"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only *makes* input matrices; it contains none of the QB method's
arithmetic and is imported by neither the GPU library nor the oracle.

Matrices follow the paper's test recipes:

* A = U diag(sigma) V^T with U, V having orthonormal columns drawn as the sign-fixed
  Q factor of a seeded Gaussian matrix (Haar / Stiefel, Mezzadri 2007); the sigma
  laws are those of Section 5.2 (Matrix 1: j^-2, Matrix 2: e^{-j/7}, Matrix 3:
  S-shape) and of Section 3.3 / Fig. 2 (e^{-j/20}, e^{-j/200}), plus the
  exponential and power laws of the benchmark workloads;
* a sparse CSR matrix with power-law column degrees, uniform row indices and
  log-normal values stands in for the paper's sparse experiments (Section 5.1,
  about 0.3% non-zeros, and the AMiner term-document matrix of Table 5, which is
  not available);
* exact-rank matrices X Y^T for reconstruction checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

# ------------------------------------------------------------------ sigma laws


def sigma_law(kind: str, count: int) -> np.ndarray:
    j = np.arange(1, count + 1, dtype=np.float64)
    if kind == "poly2":            # Matrix 1, slow decay (Section 5.2)
        return j ** -2.0
    if kind == "poly1.5":
        return j ** -1.5
    if kind == "exp7":             # Matrix 2, fast decay
        return np.exp(-j / 7.0)
    if kind == "sshape":           # Matrix 3, S-shape decay
        return 1e-4 + np.exp(-np.logaddexp(0.0, j - 30.0))
    if kind.startswith("exp"):     # e^{-j/d} for d = int(kind[3:])
        return np.exp(-j / float(kind[3:]))
    raise ValueError(kind)


# ------------------------------------------------------------------ dense


def _gen(seed: int, stream: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((seed * 1000003 + stream * 7919 + 12345) % (2 ** 63 - 1))
    return g


def haar_columns(rows: int, cols: int, seed: int, stream: int, device="cpu") -> torch.Tensor:
    """rows x cols matrix with orthonormal columns: sign-fixed QR of a Gaussian."""
    X = torch.randn(rows, cols, generator=_gen(seed, stream, device), dtype=torch.float64,
                    device=device)
    Q, R = torch.linalg.qr(X, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def lowrank_dense(m: int, n: int, sigma: np.ndarray, seed: int, noise_std: float = 0.0,
                  device="cpu") -> torch.Tensor:
    """Row-major float64 m x n matrix U diag(sigma) V^T (+ iid N(0, noise_std^2))."""
    r = len(sigma)
    U = haar_columns(m, r, seed, 1, device)
    V = haar_columns(n, r, seed, 2, device)
    s = torch.as_tensor(sigma, dtype=torch.float64, device=device)
    A = (U * s[None, :]) @ V.T
    del U, V
    if noise_std > 0:
        A += noise_std * torch.randn(m, n, generator=_gen(seed, 3, device), dtype=torch.float64,
                                     device=device)
    return A.contiguous()


def exact_rank(m: int, n: int, r: int, seed: int, device="cpu") -> torch.Tensor:
    """Gaussian X (m x r) times Gaussian Y^T (r x n): rank exactly r (a.s.)."""
    X = torch.randn(m, r, generator=_gen(seed, 1, device), dtype=torch.float64, device=device)
    Y = torch.randn(n, r, generator=_gen(seed, 2, device), dtype=torch.float64, device=device)
    return (X @ Y.T).contiguous()


def gaussian_dense(m: int, n: int, seed: int, device="cpu") -> torch.Tensor:
    return torch.randn(m, n, generator=_gen(seed, 4, device), dtype=torch.float64, device=device)


# ------------------------------------------------------------------ sparse


@dataclass
class CSR:
    m: int
    n: int
    rowptr: np.ndarray   # int64, m+1
    colind: np.ndarray   # int32, nnz, sorted within each row
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.val.size)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.m, self.n))


def powerlaw_degrees(m: int, n: int, nnz_target: int, tail: float, rng) -> np.ndarray:
    """Column degrees d_c = min(floor(d_min U^{-1/tail}), m), d_min fitted by bisection
    so that sum(d) is within 0.1% of nnz_target.  tail = 1.1 gives a degree density
    exponent of 2.1."""
    U = rng.random(n)
    U = np.maximum(U, 1e-300)
    base = U ** (-1.0 / tail)

    def total(dmin):
        return int(np.minimum(np.floor(dmin * base), m).sum())

    lo, hi = 1e-3, float(m)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < nnz_target:
            lo = mid
        else:
            hi = mid
        if abs(total(hi) - nnz_target) <= 0.001 * nnz_target:
            break
    d = np.minimum(np.floor(hi * base), m).astype(np.int64)
    return np.maximum(d, 1)


def powerlaw_csr(m: int, n: int, nnz_target: int, seed: int, tail: float = 1.1) -> CSR:
    """Sparse m x n CSR: power-law column degrees, rows uniform without replacement
    within each column, values exp(N(0,1)), column indices sorted within rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = powerlaw_degrees(m, n, nnz_target, tail, rng)
    cols = np.repeat(np.arange(n, dtype=np.int64), deg)
    rows = rng.integers(0, m, size=cols.size, dtype=np.int64)
    # redraw duplicates (row, col) until every column has distinct rows
    for _ in range(1000):
        key = cols * m + rows
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        idx = order[dup]
        full = deg[cols[idx]] >= m            # a full column keeps all rows exactly once
        if full.any():
            for c in np.unique(cols[idx[full]]):
                sel = np.nonzero(cols == c)[0]
                rows[sel] = rng.permutation(m)[:sel.size]
            continue
        rows[idx] = rng.integers(0, m, size=idx.size, dtype=np.int64)
    vals = np.exp(rng.standard_normal(cols.size))
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return CSR(m, n, rowptr, cols.astype(np.int32), vals.astype(np.float64))


# ------------------------------------------------------------------ named workloads

SEED_OMEGA = 0x1606094000000000
SEED_GEN = 0x16060940


@dataclass
class DenseWorkload:
    name: str
    m: int
    n: int
    sigma_kind: str
    rank_gen: int          # number of Stiefel columns used to build A
    noise_std: float
    b: int
    tol: float
    seed: int

    def make(self, device="cpu") -> torch.Tensor:
        sig = sigma_law(self.sigma_kind, self.rank_gen)
        return lowrank_dense(self.m, self.n, sig, self.seed, self.noise_std, device)

    def sigma(self) -> np.ndarray:
        return sigma_law(self.sigma_kind, self.rank_gen)


# Matrix 1 of Section 5.2 / Table 4 at 1000 x 800 (sigma_j = j^-2), b = 20, tol 1e-2
C1 = DenseWorkload("dense_1000x800_poly2_b20_tol1e-2", 1000, 800, "poly2", 800, 0.0, 20, 1e-2,
                   SEED_GEN + 1)
# Fig. 2(b) / Fig. 3 regime: 20000 x 15000, sigma_j = e^{-j/150}, noise std 1e-8, b=64, tol 1e-3
C2 = DenseWorkload("dense_20000x15000_exp150_noise1e-8_b64_tol1e-3", 20000, 15000, "exp150",
                   3000, 1e-8, 64, 1e-3, SEED_GEN + 2)
# same law at reduced size, used for oracle-size parity runs of the benchmark workload
C2_SMALL = DenseWorkload("dense_4000x3000_exp150_noise1e-8_b64_tol1e-3", 4000, 3000, "exp150",
                         1500, 1e-8, 64, 1e-3, SEED_GEN + 12)


# Precision form: 32768 x 32768, sigma_j = j^-1.5 on 4096 Stiefel columns (the dropped
# tail is 1.6e-4 of ||A||_F, far below tol), b = 128, tol 1e-2; A is stored in bfloat16
C4 = DenseWorkload("dense_32768x32768_poly1.5_b128_tol1e-2", 32768, 32768, "poly1.5", 4096, 0.0,
                   128, 1e-2, SEED_GEN + 4)
# the same law on a separate full-rank 4096 x 4096 instance for oracle-size parity runs
C4_SMALL = DenseWorkload("dense_4096x4096_poly1.5_b128_tol1e-2", 4096, 4096, "poly1.5", 4096, 0.0,
                         128, 1e-2, SEED_GEN + 14)


def to_bf16(A: torch.Tensor) -> torch.Tensor:
    """Storage of a float64 matrix in bfloat16 (input preparation of the precision form:
    the stored values are the matrix the method factorises)."""
    return A.to(torch.bfloat16).contiguous()


def to_e4m3_rows(A: torch.Tensor):
    """Storage of a float64 matrix in OCP e4m3fn with a power-of-two scale per row (input
    preparation of the precision form): row i is divided by 2^e_i, e_i the smallest
    exponent that brings its largest magnitude to at most 448, and converted by torch.
    Returns (A8 float8_e4m3fn, row_exp int32, A_q float64 = the stored values)."""
    amax = A.abs().amax(dim=1).clamp_min(1e-300)
    e = torch.ceil(torch.log2(amax / 448.0)).to(torch.int32)
    scale = torch.pow(2.0, -e.to(torch.float64))
    A8 = (A * scale[:, None]).to(torch.float8_e4m3fn).contiguous()
    Aq = A8.to(torch.float64) * torch.pow(2.0, e.to(torch.float64))[:, None]
    return A8, e.contiguous(), Aq


@dataclass
class SparseWorkload:
    name: str
    m: int
    n: int
    nnz: int
    b: int
    tol: float
    seed: int

    def make(self) -> CSR:
        return powerlaw_csr(self.m, self.n, self.nnz, self.seed)


C3 = SparseWorkload("csr_500000x200000_nnz5e6_powerlaw2.1_b50_tol0.6", 500000, 200000,
                    5_000_000, 50, 0.6, SEED_GEN + 3)
C3_SMALL = SparseWorkload("csr_20000x8000_nnz2e5_powerlaw2.1_b50_tol0.6", 20000, 8000, 200_000,
                          50, 0.6, SEED_GEN + 13)


@dataclass
class BatchWorkload:
    """A batch of dense matrices U_z diag(sigma) V_z^T with their own U_z, V_z per item."""
    name: str
    batch: int
    m: int
    n: int
    sigma_kind: str
    k: int
    b: int
    seed: int

    def make(self, device="cpu", dtype=torch.float32, items=None) -> torch.Tensor:
        items = list(range(self.batch)) if items is None else list(items)
        sig = sigma_law(self.sigma_kind, min(self.m, self.n))
        out = torch.empty((len(items), self.m, self.n), dtype=dtype, device=device)
        for z, it in enumerate(items):
            out[z] = lowrank_dense(self.m, self.n, sig, self.seed + 1009 * it, device=device).to(dtype)
        return out


# Differentiation form: 64 binary32 matrices 2048 x 1024, sigma_j = e^{-j/40}, rank 128, b = 32
C5 = BatchWorkload("batch64_2048x1024_exp40_k128_b32", 64, 2048, 1024, "exp40", 128, 32, SEED_GEN + 5)
