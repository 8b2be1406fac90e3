"""Plain float64 oracle of trQRCP driven by the Frobenius error indicator (test
infrastructure only).

Remark 3.2 of Yu, Gu, Li (arXiv 1606.09402): the indicator of Algorithm 1 also serves
the truncated randomized QR with column pivoting (trQRCP, Duersch and Gu), because the
column permutation changes neither the Frobenius norm of B nor those of its rows.  With
B = R P^T (R in pivot order scattered back to the original columns) and orthonormal Q,
B = Q^T A, so Theorem 1 gives ||A - QB||_F^2 = ||A||^2 - ||B||^2 exactly as for randQB.

trQRCP as restated here (randomized QRCP of Duersch and Gu, blocked and truncated):

* one sketch S = Omega^T A of l = b + oversample rows, Omega the m x l Gaussian matrix of
  stream 1 of the counter generator (stream 0 is randQB's Omega);
* per block: QR with column pivoting of the current sketch (largest remaining column norm
  first, Businger-Golub; LAPACK's geqp3 here) gives the bw pivot columns J of the block and
  the sketch's triangular factor R~_11 in its rotated basis U^T S;
* the block is factored like a block of Algorithm 2 with A(:, J) in place of A Omega_i:
  Q_i = orth(A(:, J) - Q B(:, J)), re-orthogonalised Q_i = orth(Q_i - Q (Q^T Q_i)),
  R_i = R~ R, B_i = Q_i^T A (so B_i(:, J) = R_i up to rounding);
* the indicator is decremented row by row (Section 3.1), with the exhaustion guard of the
  randQB oracle (R_i(j, j) against ||A(:, J_j)||);
* sample update: the sketch of the new residual A - Q B - Q_i B_i is
  S - S(:, J) R_i^{-1} B_i (since Omega^T Q_i = S(:, J) R_i^{-1}); in the rotated basis
  only its first bw rows change, by R~_11 R_i^{-1} B_i, and the pivot columns drop out.

Readings (the paper gives only the remark): the oversampling defaults to 8 rows; ties in
the pivot choice go to the smallest column index; the sketch's Omega is drawn once.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from . import rng
from .randqb import (QB_NOT_CONVERGED, QB_OK, QB_WARN_TOL_FLOOR, QB_ERR_NONFINITE, _check,
                     _scan_rows, qr_pos, sumsq, tol_floor)

SKETCH_STREAM = 1
DEFAULT_OVERSAMPLE = 8


@dataclass
class QRCPResult:
    Q: np.ndarray
    B: np.ndarray          # R P^T: rows of R scattered back to the original columns
    piv: np.ndarray        # pivot columns in pivot order (rank entries)
    rank: int
    E: float
    normA2: float
    status: int
    passes: int = 0
    blocks: int = 0
    exhausted: int = 0
    E_trace: list = field(default_factory=list)


def sketch_omega(seed: int, m: int, l: int) -> np.ndarray:
    """The m x l Gaussian matrix of the sketch (stream 1 of the counter generator)."""
    return rng.gaussian_matrix(seed, m, l, 0, 0, stream=SKETCH_STREAM)


def trqrcp(A, tol_rel: float, b: int, seed: int, oversample: int = DEFAULT_OVERSAMPLE,
           l_max=None, row_by_row: bool = True, sketch=None, _update: bool = True) -> QRCPResult:
    """trQRCP with the row-by-row indicator.  `sketch` replaces Omega^T A (S = A gives the
    deterministic column-pivoted QR); `_update=False` drops the sample update (a planted
    mistake for the pins)."""
    m, n, l_max = _check(A, tol_rel, b, l_max)
    if oversample < 0:
        raise ValueError("bad argument")
    normA2 = sumsq(A)
    empty = (np.empty((m, 0)), np.empty((0, n)), np.empty(0, dtype=np.int64))
    if not np.isfinite(normA2):
        return QRCPResult(*empty, 0, normA2, normA2, QB_ERR_NONFINITE)
    eps2 = tol_rel * tol_rel * normA2
    status_tol = QB_WARN_TOL_FLOOR if tol_rel < tol_floor() else QB_OK
    E = normA2
    if normA2 == 0.0 or E < eps2:
        return QRCPResult(*empty, 0, E, normA2, status_tol)
    l = b + oversample
    if sketch is None:
        S = np.asarray(A.T @ sketch_omega(seed, m, l)).T    # the one sketch pass
        passes = 1
    else:
        S = np.array(sketch, dtype=np.float64)
        passes = 0
    active = np.arange(n)                 # original index of each sketch column
    Q = np.empty((m, 0))
    B = np.empty((0, n))
    piv = []
    blocks = 0
    exhausted = False
    trace = []
    while Q.shape[1] < l_max and active.size > 0:
        k = Q.shape[1]
        bw = min(b, l_max - k, active.size)
        _, Rs, P = scipy.linalg.qr(S, mode="economic", pivoting=True)
        J = active[P[:bw]]
        AJ = np.asarray(A[:, J].todense()) if hasattr(A, "todense") else np.asarray(A[:, J])
        gnorm = np.sqrt(np.einsum("ij,ij->j", AJ, AJ))
        Y = AJ - Q @ B[:, J]
        Qi, R = qr_pos(Y)
        Qi, Rt = qr_pos(Qi - Q @ (Q.T @ Qi))
        R = Rt @ R
        Bi = np.asarray((A.T @ Qi).T)                         # a pass over A
        passes += 1
        blocks += 1
        keep, E, stop, exh = _scan_rows(Bi, R, gnorm, E, eps2, row_by_row)
        Q = np.concatenate([Q, Qi[:, :keep]], axis=1)
        B = np.concatenate([B, Bi[:keep]], axis=0)
        piv.extend(int(j) for j in J[:keep])
        trace.append(E)
        if stop:
            exhausted = exh
            break
        rest = P[bw:]
        S_new = Rs[:, bw:].copy()
        if _update:
            M = scipy.linalg.solve_triangular(R, Rs[:bw, :bw].T, trans="T", lower=False).T
            S_new[:bw] -= M @ Bi[:, active[rest]]
        S = S_new
        active = active[rest]
    status = status_tol if E < eps2 else QB_NOT_CONVERGED
    return QRCPResult(Q, B, np.asarray(piv, dtype=np.int64), Q.shape[1], E, normA2, status,
                      passes=passes, blocks=blocks, exhausted=int(exhausted), E_trace=trace)
