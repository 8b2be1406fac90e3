"""Approximate truncated SVD from a QB factorisation (test infrastructure only).

Eq. (3): with an SVD of the small factor, B = U~ diag(s) V~^T, the product QB equals
(Q U~) diag(s) V~^T, and the leading k columns of Q U~ and V~ with the leading k values of s
approximate the rank-k SVD of A.  The SVD of B here is the library one (LAPACK through
NumPy), as in the paper's Matlab setting.

Singular vectors are fixed only up to a sign per pair (for distinct values).  The oracle
picks the sign that makes the entry of largest magnitude of each column of V positive (the
smallest row index among equal magnitudes); the GPU library uses the same rule, so the two
can be compared column by column.
"""
from __future__ import annotations

import numpy as np


def sign_rule(V: np.ndarray) -> np.ndarray:
    """+1 / -1 per column: the sign of the column's entry of largest magnitude."""
    if V.shape[1] == 0:
        return np.ones(0)
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return sgn


def svd_from_qb(Q: np.ndarray, B: np.ndarray):
    """Eq. (3): returns (U, s, V) with U = Q U~ (m x k), s descending (k), V (n x k) and
    Q B = U diag(s) V^T."""
    Ub, s, Vt = np.linalg.svd(np.asarray(B), full_matrices=False)
    V = Vt.T
    sgn = sign_rule(V)
    return (np.asarray(Q) @ Ub) * sgn, s, V * sgn
