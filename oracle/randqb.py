"""Plain float64 oracle for randQB_EI and randQB_FP (test infrastructure only).

Written from Yu, Gu, Li, arXiv 1606.09402:

* Theorem 1 / eq. (5): for orthonormal Q and B = Q^T A,
  ||A - QB||_F^2 = ||A||_F^2 - ||B||_F^2, so E = ||A||^2 - sum ||B_i||^2 tracks the
  squared error without forming the residual (Algorithm 1, Theorem 2).
* Section 3.1, the row-by-row rule: the indicator may be decremented row by row; at the
  first row j where E < eps^2 the rows after j of B_i (columns of Q_i) are dropped.
* Algorithm 2 (randQB_EI): Q_i = orth(A Omega_i - Q (B Omega_i)), re-orthogonalise
  Q_i = orth(Q_i - Q (Q^T Q_i)), B_i = Q_i^T A.
* Algorithm 3 with the re-orthogonalisation of Algorithm 4, i.e. Algorithm 4 with power
  parameter P = 0 (randQB_FP): G = A Omega, H = A^T G once; per block
  Y_i = G_J - Q (B Omega_J); [Q_i, R_i] = qr(Y_i);
  [Q_i, R~_i] = qr(Q_i - Q (Q^T Q_i)); R_i = R~_i R_i;
  B_i = R_i^{-T} (H_J^T - Y_i^T Q B - Omega_J^T B^T B)   (eq. (23)).
* Section 5.4: the tolerance is relative, ||A - QB||_F < tol ||A||_F, and the
  SVD-optimal rank is the smallest k whose tail sum of sigma_j^2 meets it.

Readings where the paper is silent or inconsistent (each one is listed in the
design notes of the repository):

* stop test is E < eps^2 with eps^2 = tol*tol*||A||^2 (strict, as in Algorithms 1
  and 2; Algorithm 4 writes sqrt(E) < eps which is NaN for negative E);
* orth and qr both mean the Q factor of a thin QR with diag(R) >= 0;
* EI and FP draw Omega from one counter-indexed matrix: EI's Omega_i is FP's
  Omega(:, J) for the same global columns J;
* l~ (chunk width) defaults to min(50 b, l_max) (Section 5.4); when a chunk is
  used up without convergence the next l~ columns of Omega are drawn and G, H
  recomputed (the restart described after Algorithm 4), keeping Q, B and E;
* l_tilde = -1 selects an adaptive chunk schedule (the paper leaves the choice of l~
  open): the first chunk has 8 b columns; after a chunk of w columns (nb = ceil(w / b)
  blocks), the decay of the indicator per column over the chunk's second half (from the
  end of block floor(nb / 2) to the end of the chunk) is taken as geometric, and the next
  chunk is 1.1 times the columns needed to reach eps^2 plus b, rounded up to a multiple of
  b and kept in [b, 4 w]; no chunk exceeds min(50 b, l_max);
* exhaustion guard: before row j of a block is accepted, R_i(j,j) must exceed
  2^-40 ||G_J(:,j)||_2, otherwise the method stops before row j (the numerical
  rank of A has been reached and R_i^{-T} would divide by round-off);
* A = 0 returns rank 0; E < eps^2 before the first block (tol > 1) returns rank 0.
* power scheme (Algorithm 4, P >= 1): in the first chunk (Q empty) the P
  rounds G = orth(A Omega), Omega = orth(A^T G) run as written.  When a later chunk
  redraws Omega (the restart after Algorithm 4), the rounds act on the current residual
  A - Q B instead of A, i.e. G = orth(A Omega - Q (B Omega)) and
  Omega = orth(A^T G - B^T (Q^T G)); on A itself they would steer the new columns back
  into the range that Q already holds.  The sketch G = A Omega and H = A^T G then
  take the full A as written (the block loop deflates).  Each chunk costs 2 P + 2
  passes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import lowp, rng

# status codes (same meaning as the C ABI)
QB_OK = 0
QB_NOT_CONVERGED = 1
QB_WARN_TOL_FLOOR = 2
QB_ERR_ARG = -1
QB_ERR_NONFINITE = -2

EXHAUST_REL = 2.0 ** -40
UNIT_ROUNDOFF = 2.0 ** -53


# power-of-two scale of Omega before its e4m3 rounding (the "e4m3" precision form)
OMEGA_E4M3_SCALE = 2.0 ** 5


def tol_floor(u: float = UNIT_ROUNDOFF, delta: float = 0.01) -> float:
    """Theorem 3: E is accurate to relative delta only if eps > sqrt(4u/delta) ||A||_F."""
    return float(np.sqrt(4.0 * u / delta))


def sumsq(A) -> float:
    """||A||_F^2 as a sum of squares of the entries (not a norm squared), accumulated
    in x87 extended precision, then rounded to binary64 (Section 3.3)."""
    if sp.issparse(A):
        vals = np.asarray(A.data, dtype=np.float64).ravel()
        return float(np.sum(np.square(vals.astype(np.longdouble))))
    A = np.asarray(A)
    total = np.longdouble(0.0)
    rows_per = max(1, (1 << 22) // max(1, A.shape[1]))
    for r0 in range(0, A.shape[0], rows_per):
        blk = A[r0:r0 + rows_per].astype(np.longdouble)
        total += np.sum(blk * blk)
    return float(total)


def qr_pos(X: np.ndarray):
    """Thin Householder QR (LAPACK) with the signs fixed so that diag(R) >= 0."""
    Q, R = np.linalg.qr(X, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def omega(seed: int, n: int, col0: int, cols: int, batch: int = 0) -> np.ndarray:
    """Columns [col0, col0+cols) of the n-row Gaussian test matrix (stream 0)."""
    return rng.gaussian_matrix(seed, n, cols, 0, col0, stream=0, batch=batch)


def block_b(H_J, Y, Qk, Bk, W, R):
    """Eq. (23): B_i = R^{-T} (H_J^T - (Y^T Q) B - W^T B), W = B Omega_J."""
    S = H_J.T - (Y.T @ Qk) @ Bk - W.T @ Bk
    return scipy.linalg.solve_triangular(R, S, trans="T", lower=False)


def residual_sample(G_J, Om_J, Qk, Bk):
    """The residual's sample (A - Q B) Omega_J = G_J - Q (B Omega_J) for the next block,
    with G_J = A Omega_J; returns it and W = B Omega_J (B = Q^T A, so this samples
    (I - Q Q^T) A without forming Q B)."""
    W = Bk @ Om_J
    return G_J - Qk @ W, W


def orth_against(Y, Qk):
    """An orthonormal basis Q_i of range(Y) orthogonal to range(Q): the Q factor of Y,
    orthogonalised against Q once more and refactored (the re-orthogonalisation that
    Algorithm 4 adds to Algorithm 3), with the triangular factor R of Y = Q_i R + Q (...)
    (positive diagonal)."""
    Qi, R = qr_pos(Y)
    Qi, Rt = qr_pos(Qi - Qk @ (Qk.T @ Qi))
    return Qi, Rt @ R


def fp_block(G_J, Om_J, H_J, Qk, Bk):
    """One block of randQB_FP from the sketches G = A Omega and H = A^T G alone: the new
    basis block Q_i and B_i = Q_i^T A by eq. (23).  Returns (Q_i, B_i, R)."""
    Y, W = residual_sample(G_J, Om_J, Qk, Bk)
    Qi, R = orth_against(Y, Qk)
    return Qi, block_b(H_J, Y, Qk, Bk, W, R), R


def row_sumsq(Bi: np.ndarray) -> np.ndarray:
    return np.einsum("ij,ij->i", Bi, Bi)


class _Grow:
    """Growable column (Q) / row (B) storage."""

    def __init__(self, m, n):
        self.Q = np.empty((m, 0))
        self.B = np.empty((0, n))
        self.k = 0

    def append(self, Qi, Bi):
        self.Q = np.concatenate([self.Q, Qi], axis=1)
        self.B = np.concatenate([self.B, Bi], axis=0)
        self.k = self.Q.shape[1]


@dataclass
class QBResult:
    Q: np.ndarray
    B: np.ndarray
    rank: int
    E: float
    normA2: float
    status: int
    passes: int = 0
    blocks: int = 0
    chunks: int = 0
    exhausted: int = 0
    E_trace: list = field(default_factory=list)   # E after every block (Theorem 2)
    R_diag: list = field(default_factory=list)    # diag(R_i) per block
    omegas: list = field(default_factory=list)    # each chunk's Omega (keep_omega only)


def _check(A, tol_rel, b, l_max):
    m, n = A.shape
    if l_max is None:
        l_max = min(m, n)
    if not (1 <= b) or l_max < 0 or l_max > min(m, n) or not (tol_rel >= 0):
        raise ValueError("bad argument")
    return m, n, int(l_max)


def _scan_rows(Bi, R, gnorm, E, eps2, row_by_row):
    """The row-by-row stopping rule of Section 3.1 (or Algorithm 1's whole-block test when
    row_by_row is False) plus the exhaustion guard.  Returns (rows kept, new E, stop flag, exhausted flag)."""
    bw = Bi.shape[0]
    r = row_sumsq(Bi)
    if row_by_row:
        for j in range(bw):
            if not (R[j, j] > EXHAUST_REL * gnorm[j]):
                return j, E, True, True
            E = E - r[j]
            if E < eps2:
                return j + 1, E, True, False
        return bw, E, False, False
    for j in range(bw):
        if not (R[j, j] > EXHAUST_REL * gnorm[j]):
            return j, E - float(np.sum(r[:j])), True, True
    E = E - float(np.sum(r))
    return bw, E, E < eps2, False


def _finish(st, E, normA2, status_tol, exhausted, l_max, k, eps2, **kw):
    converged = E < eps2
    if converged:
        status = status_tol
    else:
        status = QB_NOT_CONVERGED
    return QBResult(Q=st.Q, B=st.B, rank=st.k, E=E, normA2=normA2, status=status,
                    exhausted=int(exhausted), **kw)


def _chunk_width(adaptive: bool, cap: int, b: int, left: int, w_prev: int, span: int,
                 e_prev: float, e_now: float, eps2: float) -> int:
    """Width of the next chunk of Omega columns (see the module notes): w_prev is the
    width of the chunk just used, and the indicator fell from e_prev to e_now over its
    last span columns."""
    if not adaptive:
        w = cap
    elif w_prev == 0:
        w = 8 * b
    elif span > 0 and e_now > 0.0 and e_prev > e_now and 0.0 < eps2 < e_now:
        rate = np.log(e_now / e_prev) / span
        need = np.log(eps2 / e_now) / rate
        want = 1.1 * need + b
        if want >= 4.0 * w_prev:
            w = 4 * w_prev
        else:
            w = max(b, -(-int(np.ceil(want)) // b) * b)
    else:
        w = 2 * w_prev
    return min(w, cap, left)


def power_omega(A, Om: np.ndarray, power: int, Q=None, B=None) -> np.ndarray:
    """The power scheme of Algorithm 4 on the residual A - Q B (Q, B empty in the first chunk):
    power times G = orth((A - QB) Omega), then Omega = orth((A - QB)^T G)."""
    deflate = Q is not None and Q.shape[1] > 0
    for _ in range(power):
        X = np.asarray(A @ Om)
        if deflate:
            X = X - Q @ (B @ Om)
        G, _ = qr_pos(X)
        X = np.asarray(A.T @ G)
        if deflate:
            X = X - B.T @ (Q.T @ G)
        Om, _ = qr_pos(X)
    return Om


def randqb_fp(A, tol_rel: float, b: int, seed: int, l_max=None, l_tilde: int = 0,
              row_by_row: bool = True, precision: str = "f64", power: int = 0,
              keep_omega: bool = False) -> QBResult:
    """randQB_FP for the fixed-precision problem (Algorithm 4; power scheme with P =
    power >= 0 rounds per chunk, binary64 only).  keep_omega stores each chunk's final
    Omega in the result (for tests).

    precision = "bf16" is the precision form: A must hold bfloat16 values (A_q); each
    chunk's Omega is rounded to bfloat16 (Omega_q), G = A_q Omega_q is rounded to
    bfloat16 (G_q), and H = A_q^T G_q is formed from that same G_q.  The block loop uses
    Omega_q, G_q and H in binary64, so eq. (23) still yields B_i = Q_i^T A_q and
    Theorem 1 holds for A_q with E starting from ||A_q||^2.

    precision = "e4m3" is the same form for a matrix stored in e4m3 with power-of-two row
    scales (its values are bfloat16 values), whose G product runs on 8-bit operands:
    Omega_q is the e4m3 rounding of 2^5 Omega, divided by 2^5 (|Omega| < 9 for the
    generator's Gaussians, so 2^5 Omega stays inside the format's range and the division
    is exact); G_q = bf16(A_q Omega_q), H = A_q^T G_q as above.  Any fixed Omega_q serves
    as the sketch: Theorem 1 and eq. (23) hold for whatever matrix the block loop uses."""
    m, n, l_max = _check(A, tol_rel, b, l_max)
    if precision not in ("f64", "bf16", "e4m3"):
        raise ValueError("precision must be 'f64', 'bf16' or 'e4m3'")
    if precision != "f64" and not lowp.is_bf16(A if not sp.issparse(A) else A.data):
        raise ValueError("the precision form takes A already stored in bfloat16 or e4m3")
    if power < 0 or (power > 0 and precision != "f64"):
        raise ValueError("the power scheme takes power >= 0 and binary64")
    adaptive = l_tilde == -1
    if l_tilde in (0, -1):
        l_tilde = min(50 * b, l_max)
    if l_tilde <= 0 or (l_tilde % b != 0 and l_tilde < l_max):
        raise ValueError("l_tilde must be a multiple of b")
    l_tilde = min(l_tilde, l_max)
    normA2 = sumsq(A)
    if not np.isfinite(normA2):
        return QBResult(np.empty((m, 0)), np.empty((0, n)), 0, normA2, normA2, QB_ERR_NONFINITE)
    eps2 = tol_rel * tol_rel * normA2
    status_tol = QB_WARN_TOL_FLOOR if tol_rel < tol_floor() else QB_OK
    st = _Grow(m, n)
    E = normA2
    if normA2 == 0.0 or E < eps2:
        return QBResult(st.Q, st.B, 0, E, normA2, status_tol)
    passes = blocks = chunks = 0
    exhausted = False
    trace, rdiag, omegas = [], [], []
    chunk_lo = chunk_hi = 0
    k_half = 0
    e_half = E
    Om = G = H = Gnorm = None
    while st.k < l_max:
        k = st.k
        if k == chunk_hi:                       # draw the next chunk of Omega
            w = _chunk_width(adaptive, l_tilde, b, l_max - k, chunk_hi - chunk_lo, chunk_hi - k_half,
                             e_half, E, eps2)
            chunk_lo = k
            chunk_hi = k + w
            # the decay over the second half of this chunk sizes the next one
            k_half = chunk_lo + b * ((-(-w // b)) // 2)
            e_half = E
            Om = omega(seed, n, chunk_lo, chunk_hi - chunk_lo)
            if power > 0:                           # the power scheme
                Om = power_omega(A, Om, power, st.Q, st.B)
                passes += 2 * power
            if keep_omega:
                omegas.append(Om.copy())
            if precision == "bf16":
                Om = lowp.round_bf16(Om)
                G = lowp.round_bf16(np.asarray(A @ Om))
            elif precision == "e4m3":
                Om = lowp.round_e4m3(Om * OMEGA_E4M3_SCALE) / OMEGA_E4M3_SCALE
                G = lowp.round_bf16(np.asarray(A @ Om))
            else:
                G = A @ Om
            H = A.T @ G
            G = np.asarray(G)
            H = np.asarray(H)
            Gnorm = np.sqrt(np.einsum("ij,ij->j", G, G))
            passes += 2
            chunks += 1
        bw = min(b, chunk_hi - k)
        J = slice(k - chunk_lo, k - chunk_lo + bw)
        Qi, Bi, R = fp_block(G[:, J], Om[:, J], H[:, J], st.Q, st.B)
        blocks += 1
        keep, E, stop, exh = _scan_rows(Bi, R, Gnorm[J], E, eps2, row_by_row)
        st.append(Qi[:, :keep], Bi[:keep])
        trace.append(E)
        rdiag.append(np.diag(R).copy())
        if st.k == k_half:
            e_half = E
        if stop:
            exhausted = exh
            break
    return _finish(st, E, normA2, status_tol, exhausted, l_max, st.k, eps2, passes=passes,
                   blocks=blocks, chunks=chunks, E_trace=trace, R_diag=rdiag, omegas=omegas)


def randqb_ei(A, tol_rel: float, b: int, seed: int, l_max=None,
              row_by_row: bool = True) -> QBResult:
    """randQB_EI (Algorithm 2) with the row-by-row indicator of Section 3.1."""
    m, n, l_max = _check(A, tol_rel, b, l_max)
    normA2 = sumsq(A)
    if not np.isfinite(normA2):
        return QBResult(np.empty((m, 0)), np.empty((0, n)), 0, normA2, normA2, QB_ERR_NONFINITE)
    eps2 = tol_rel * tol_rel * normA2
    status_tol = QB_WARN_TOL_FLOOR if tol_rel < tol_floor() else QB_OK
    st = _Grow(m, n)
    E = normA2
    if normA2 == 0.0 or E < eps2:
        return QBResult(st.Q, st.B, 0, E, normA2, status_tol)
    passes = blocks = 0
    exhausted = False
    trace, rdiag = [], []
    while st.k < l_max:
        k = st.k
        bw = min(b, l_max - k)
        Om_i = omega(seed, n, k, bw)
        G_i = np.asarray(A @ Om_i)                   # a pass over A
        gnorm = np.sqrt(np.einsum("ij,ij->j", G_i, G_i))
        Y, _ = residual_sample(G_i, Om_i, st.Q, st.B)
        Qi, R = orth_against(Y, st.Q)
        Bi = np.asarray((A.T @ Qi).T)                # B_i = Q_i^T A, a second pass over A
        passes += 2
        blocks += 1
        keep, E, stop, exh = _scan_rows(Bi, R, gnorm, E, eps2, row_by_row)
        st.append(Qi[:, :keep], Bi[:keep])
        trace.append(E)
        rdiag.append(np.diag(R).copy())
        if stop:
            exhausted = exh
            break
    return _finish(st, E, normA2, status_tol, exhausted, l_max, st.k, eps2, passes=passes,
                   blocks=blocks, chunks=0, E_trace=trace, R_diag=rdiag)


def randqb_fixed(A, Om: np.ndarray):
    """Basic randQB (Figure 1(a)) without oversampling: Q = qf(A Omega), B = Q^T A."""
    Q, _ = qr_pos(np.asarray(A @ Om))
    return Q, np.asarray((A.T @ Q).T)


def randqb_fp_fixed(A, Om: np.ndarray, b: int, reorth: bool = True):
    """Fixed-rank randQB_FP: Algorithm 3, with the re-orthogonalisation of Algorithm 4 when
    reorth is True.  The rank is Om.shape[1]; the last block may be narrower than b."""
    A = np.asarray(A)
    m, n = A.shape
    G = A @ Om
    H = A.T @ G
    Q = np.empty((m, 0))
    B = np.empty((0, n))
    l = Om.shape[1]
    for lo in range(0, l, b):
        J = slice(lo, min(l, lo + b))
        if reorth:
            Qi, Bi, _ = fp_block(G[:, J], Om[:, J], H[:, J], Q, B)
        else:   # Algorithm 3: B_i = R_i^{-T} (H_J^T - Omega_J^T B^T B), no re-orthogonalisation
            Y, W = residual_sample(G[:, J], Om[:, J], Q, B)
            Qi, R = qr_pos(Y)
            Bi = scipy.linalg.solve_triangular(R, H[:, J].T - W.T @ B, trans="T", lower=False)
        Q = np.concatenate([Q, Qi], axis=1)
        B = np.concatenate([B, Bi], axis=0)
    return Q, B


def jacobi_svd(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """One-sided Jacobi SVD (Hestenes): rotate column pairs of A until mutually
    orthogonal; singular values are the final column norms (descending)."""
    U = np.array(A, dtype=np.float64, copy=True)
    n = U.shape[1]
    for _ in range(max_sweeps):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                a = float(U[:, p] @ U[:, p])
                c_ = float(U[:, q] @ U[:, q])
                g = float(U[:, p] @ U[:, q])
                if abs(g) <= tol * np.sqrt(a * c_) or g == 0.0:
                    continue
                rotated = True
                zeta = (c_ - a) / (2.0 * g)
                t = np.copysign(1.0, zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta))
                cs = 1.0 / np.sqrt(1.0 + t * t)
                sn = cs * t
                up = U[:, p].copy()
                U[:, p] = cs * up - sn * U[:, q]
                U[:, q] = sn * up + cs * U[:, q]
        if not rotated:
            break
    s = np.sqrt(np.einsum("ij,ij->j", U, U))
    return np.sort(s)[::-1]


def svd_optimal_rank(sigma: np.ndarray, tol_rel: float) -> int:
    """Smallest k with sum_{j>k} sigma_j^2 < tol^2 sum_j sigma_j^2 (Section 5.4)."""
    s2 = np.sort(np.asarray(sigma, dtype=np.float64) ** 2)[::-1]
    total = float(np.sum(s2.astype(np.longdouble)))
    # tail[k] = sum_{j >= k} s2[j] (0-based), accumulated smallest first
    tail = np.cumsum(s2[::-1].astype(np.longdouble))[::-1]
    tail = np.append(tail, np.longdouble(0.0))
    thr = np.longdouble(tol_rel) ** 2 * np.longdouble(total)
    for k in range(len(s2) + 1):
        if tail[k] < thr:
            return k
    return len(s2)


def orth_loss_inf(Q: np.ndarray) -> float:
    """||Q^T Q - I||_inf (max absolute row sum), the loss-of-orthogonality measure of Fig. 2."""
    M = Q.T @ Q - np.eye(Q.shape[1])
    return float(np.max(np.sum(np.abs(M), axis=1))) if M.size else 0.0


def residual_sq(A, Q, B) -> float:
    """Directly computed ||A - QB||_F^2 (for checking E; never used by the method)."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    Rm = A - Q @ B
    return float(np.sum(Rm * Rm))
