"""Pins of the oracle's approximate SVD from QB (eq. (3)) against what the mathematics and
the paper fix.  CPU only.

* An exact-rank matrix U diag(sigma) V^T, factorised to its full rank, gives back sigma and
  the columns of U and V (up to the sign rule).
* Q B = U diag(s) V^T with orthonormal U and V.
* The values agree with the oracle's one-sided Jacobi SVD of B (another algorithm).
* Pythagoras: ||A - U_k diag(s_k) V_k^T||^2 = ||A - QB||^2 + sum_{j > k} s_j^2, because
  A - QB is orthogonal to the range of Q (Theorem 1's argument).
* Section 5.5 / Fig. 9: the top singular values from randQB_FP are indistinguishable from
  those of randQB with the same Omega.
"""
import numpy as np
import pytest

import workloads as W
from oracle import randqb as R
from oracle import svd as S


def test_exact_rank_recovers_the_generator():
    m, n, r = 300, 200, 30
    sig = np.exp(-np.arange(1, r + 1) / 6.0)
    U0 = W.haar_columns(m, r, 51, 1).numpy()
    V0 = W.haar_columns(n, r, 51, 2).numpy()
    A = (U0 * sig) @ V0.T
    res = R.randqb_fp(A, 1e-12, 8, 52, l_tilde=48)
    assert res.rank == r
    U, s, V = S.svd_from_qb(res.Q, res.B)
    assert np.max(np.abs(s - sig) / sig) < 1e-10
    sg = S.sign_rule(V0)
    assert np.max(np.abs(V - V0 * sg)) < 1e-9
    assert np.max(np.abs(U - U0 * sg)) < 1e-9


@pytest.mark.parametrize("kind,tol", [("poly2", 1e-3), ("exp20", 1e-6)])
def test_identity_orthogonality_and_jacobi(kind, tol):
    A = W.lowrank_dense(400, 250, W.sigma_law(kind, 250), 53).numpy()
    res = R.randqb_fp(A, tol, 10, 54)
    U, s, V = S.svd_from_qb(res.Q, res.B)
    k = res.rank
    assert U.shape == (400, k) and V.shape == (250, k) and s.shape == (k,)
    assert np.all(np.diff(s) <= 0)
    QB = res.Q @ res.B
    assert np.linalg.norm(QB - (U * s) @ V.T) <= 1e-13 * np.linalg.norm(QB)
    assert np.max(np.abs(U.T @ U - np.eye(k))) < 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(k))) < 1e-13
    sj = R.jacobi_svd(res.B.T.copy())
    assert np.max(np.abs(sj - s)) <= 1e-13 * s[0]


def test_truncation_pythagoras():
    A = W.lowrank_dense(300, 220, W.sigma_law("poly2", 220), 55).numpy()
    res = R.randqb_fp(A, 1e-3, 10, 56)
    U, s, V = S.svd_from_qb(res.Q, res.B)
    e_qb = R.residual_sq(A, res.Q, res.B)
    for k in (1, 5, res.rank // 2, res.rank):
        Ak = (U[:, :k] * s[:k]) @ V[:, :k].T
        lhs = float(np.sum((A - Ak) ** 2))
        rhs = e_qb + float(np.sum(s[k:] ** 2))
        assert abs(lhs - rhs) <= 1e-12 * np.sum(A * A)


def test_fig9_fp_equals_randqb_top_values():
    """Top 50 singular values with oversampling 10 (l = 60) on Matrix 1 and Matrix 2 laws."""
    for kind in ("poly2", "exp7"):
        A = W.lowrank_dense(500, 400, W.sigma_law(kind, 400), 57).numpy()
        Om = R.omega(58, 400, 0, 60)
        Qf, Bf = R.randqb_fp_fixed(A, Om, 10)
        Qr, Br = R.randqb_fixed(A, Om)
        _, sf, _ = S.svd_from_qb(Qf, Bf)
        _, sr, _ = S.svd_from_qb(Qr, Br)
        assert np.max(np.abs(sf[:50] - sr[:50]) / sr[:50]) < 1e-8, kind


def test_sign_rule():
    V = np.array([[0.1, -0.9], [-0.8, 0.2], [0.3, 0.9]])
    assert list(S.sign_rule(V)) == [-1.0, -1.0]
