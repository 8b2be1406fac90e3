"""Pins of the oracle's power scheme (Algorithm 4, P >= 1) against what the
paper and the mathematics fix.  CPU only.

* Closed form: orth(X) is the Q factor of a thin QR with diag(R) > 0, and that factor
  does not change when X is multiplied on the right by an upper-triangular matrix with
  positive diagonal.  P rounds of G = orth(A Omega), Omega = orth(A^T G) therefore give
  the Q factor of (A^T A)^P Omega_0; on the residual A~ = (I - Q Q^T) A of a restart they
  give the Q factor of (A~^T A~)^P Omega_0.
* With Omega replaced by the power iterate, the block loop is still Algorithm 4: the
  fixed-rank result is randQB on that Omega (Q = qf(A Omega_P), B = Q^T A).
* Theorem 1 (E equals ||A - QB||^2), Q^T Q = I, the Eckart-Young lower bound on the
  rank, and the pass count 2 P + 2 per chunk.
* Table 4: the ranks that randQB_FP with P = 1 reaches on the paper's three 8000 x 8000
  test matrices.
"""
import numpy as np
import pytest

import workloads as W
from conftest import read_golden
from oracle import randqb as R


def _lowrank(m, n, kind, seed, count=None):
    sig = W.sigma_law(kind, count or min(m, n))
    return W.lowrank_dense(m, n, sig, seed).numpy(), sig


@pytest.fixture(scope="module")
def mat():
    # sigma_j = e^{-j/20}: (A^T A)^2 keeps a condition number of about 1e5 over 40 columns
    return _lowrank(260, 200, "exp20", 31)


def _qf(X):
    return R.qr_pos(X)[0]


@pytest.mark.parametrize("P", [1, 2])
def test_power_omega_closed_form(mat, P):
    A, _ = mat
    Om0 = R.omega(41, A.shape[1], 0, 40)
    Om = R.power_omega(A, Om0, P)
    want = _qf(np.linalg.matrix_power(A.T @ A, P) @ Om0)
    assert np.max(np.abs(Om.T @ Om - np.eye(40))) < 1e-13
    assert np.max(np.abs(Om - want)) < 1e-8


def test_power_omega_deflated_closed_form(mat):
    """A restart: the rounds act on the residual A - Q B with B = Q^T A."""
    A, _ = mat
    Q = _qf(A @ R.omega(42, A.shape[1], 0, 24))
    B = Q.T @ A
    Om0 = R.omega(42, A.shape[1], 24, 32)
    At = A - Q @ (Q.T @ A)
    Om = R.power_omega(A, Om0, 1, Q, B)
    assert np.max(np.abs(Om - _qf(At.T @ At @ Om0))) < 1e-8
    # the undeflated rounds give a different basis (they return to range(Q))
    assert np.max(np.abs(R.power_omega(A, Om0, 1) - Om)) > 1e-2


def test_power_fixed_rank_is_randqb_on_the_iterate(mat):
    A, _ = mat
    l, b = 48, 16
    res = R.randqb_fp(A, 1e-14, b, 43, l_max=l, l_tilde=l, power=1, keep_omega=True)
    assert res.rank == l and res.chunks == 1 and res.passes == 4
    OmP = res.omegas[0]
    assert np.max(np.abs(OmP - _qf(A.T @ A @ R.omega(43, A.shape[1], 0, l)))) < 1e-8
    Qr, Br = R.randqb_fixed(A, OmP)
    assert np.max(np.abs(res.Q - Qr)) < 1e-9
    assert np.linalg.norm(res.B - Br) < 1e-10 * np.linalg.norm(A)


@pytest.mark.parametrize("P", [1, 2])
def test_power_indicator_and_rank(P):
    A, sig = _lowrank(400, 300, "poly2", 32)
    tol = 1e-3
    res = R.randqb_fp(A, tol, 10, 44, power=P)
    base = R.randqb_fp(A, tol, 10, 44)
    assert res.status == R.QB_OK
    assert abs(res.E - R.residual_sq(A, res.Q, res.B)) <= 1e-12 * res.normA2
    assert R.orth_loss_inf(res.Q) < 1e-12
    assert R.svd_optimal_rank(sig, tol) <= res.rank <= base.rank
    assert res.passes == (2 * P + 2) * res.chunks


def test_power_restart_deflates(mat):
    """Several chunks: chunk c's Omega is the closed form on the residual of the first
    k_c = c l~ columns (all blocks full before the last)."""
    A, _ = mat
    lt, b = 16, 8
    res = R.randqb_fp(A, 1e-4, b, 45, l_tilde=lt, power=1, keep_omega=True)
    assert res.chunks >= 3 and res.passes == 4 * res.chunks
    assert abs(res.E - R.residual_sq(A, res.Q, res.B)) <= 1e-12 * res.normA2
    for c in (1, 2):
        kc = c * lt
        Qc = res.Q[:, :kc]
        At = A - Qc @ (Qc.T @ A)
        Om0 = R.omega(45, A.shape[1], kc, lt)
        assert np.max(np.abs(res.omegas[c] - _qf(At.T @ At @ Om0))) < 1e-7, c


def test_power_sparse_equals_dense():
    import scipy.sparse as sp
    csr = W.powerlaw_csr(600, 300, 6000, 46)
    S = sp.csr_matrix((csr.val, csr.colind, csr.rowptr), shape=(csr.m, csr.n))
    D = S.toarray()
    a = R.randqb_fp(S, 0.5, 10, 47, power=1)
    d = R.randqb_fp(D, 0.5, 10, 47, power=1)
    assert a.rank == d.rank
    assert np.linalg.norm(a.B - d.B) < 1e-10 * np.sqrt(d.normA2)


def test_power_rejects_bad_arguments(mat):
    A, _ = mat
    with pytest.raises(ValueError):
        R.randqb_fp(A, 1e-2, 10, 1, power=-1)
    with pytest.raises(ValueError):
        R.randqb_fp(A.astype(np.float32).astype(np.float64), 1e-2, 10, 1, power=1,
                    precision="bf16")


@pytest.mark.parametrize("row", read_golden("table4_power_ranks.txt"),
                         ids=lambda r: f"{r[0]}-{r[1]}")
def test_table4_power_ranks(row):
    """Table 4, randQB_FP column (P = 1, b = 10) on 8000 x 8000 matrices of the three
    laws, generated from their leading singular triplets (2000 for the slow laws: the
    dropped tail is below 1% of eps^2).  The rank lies between the SVD rank and the
    printed one plus one (the printed value is one random instance)."""
    kind, tol, b, want, svd = row[0], float(row[1]), int(row[2]), int(row[3]), int(row[4])
    r = 300 if kind.startswith("exp") else 2000
    sig = W.sigma_law(kind, 8000)
    assert R.svd_optimal_rank(sig, tol) == svd
    A = W.lowrank_dense(8000, 8000, sig[:r], 77).numpy()
    res = R.randqb_fp(A, tol, b, 1234, power=1)
    assert res.status == R.QB_OK
    assert svd <= res.rank <= want + 1
    assert np.sqrt(max(res.E, 0.0) / res.normA2) < tol


# ---------------------------------------------------------------- planted mistakes


def _power_pins_pass(A):
    ok = True
    Om0 = R.omega(41, A.shape[1], 0, 40)
    ok &= np.max(np.abs(R.power_omega(A, Om0, 2) - _qf(np.linalg.matrix_power(A.T @ A, 2) @ Om0))) < 1e-8
    res = R.randqb_fp(A, 1e-4, 8, 45, l_tilde=16, power=1, keep_omega=True)
    Qc = res.Q[:, :16]
    At = A - Qc @ (Qc.T @ A)
    ok &= np.max(np.abs(res.omegas[1] - _qf(At.T @ At @ R.omega(45, A.shape[1], 16, 16)))) < 1e-7
    return bool(ok)


_real_power = R.power_omega


def _no_deflation(A, Om, power, Q=None, B=None):
    return _real_power(A, Om, power)


def _one_round(A, Om, power, Q=None, B=None):
    return _real_power(A, Om, min(power, 1), Q, B)


@pytest.mark.parametrize("mutant", [_no_deflation, _one_round])
def test_planted_power_mistakes_are_caught(monkeypatch, mat, mutant):
    A, _ = mat
    assert _power_pins_pass(A)
    monkeypatch.setattr(R, "power_omega", mutant)
    assert not _power_pins_pass(A)
