"""Pins of the FP64 oracle (randQB_FP / randQB_EI) against what the paper and the
mathematics fix: Theorems 1-3, Propositions 1-2, the randQB special case, Table 4,
the Eckart-Young bound, exact-rank reconstruction and a Jacobi SVD.  CPU only.

The last group plants plausible mistakes in the oracle (on the CPU) and checks that
these pins catch each of them."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from conftest import read_golden
from oracle import randqb as R


def _lowrank(m, n, kind, seed, count=None, noise=0.0):
    sig = W.sigma_law(kind, count or min(m, n))
    return W.lowrank_dense(m, n, sig, seed, noise).numpy(), sig


@pytest.fixture(scope="module")
def m1():
    return _lowrank(300, 200, "poly2", 11)


@pytest.fixture(scope="module")
def m2():
    return _lowrank(240, 260, "exp20", 12)


# ---------------------------------------------------------------- Table 4 / Theorem 3


def test_table4_svd_ranks():
    rows = read_golden("table4_svd_ranks.txt")
    assert len(rows) == 6
    for kind, n, tol, want in rows:
        sig = W.sigma_law(kind, int(n))
        assert R.svd_optimal_rank(sig, float(tol)) == int(want), (kind, tol)


def test_theorem3_floor_constants():
    # eps > sqrt(4 u / delta) ||A||_F with u ~ 1.11e-16 and delta = 1% gives 2.1e-7
    f = R.tol_floor()
    assert abs(f - 2.1e-7) < 0.01e-7
    assert abs(f * f - 4.4e-14) < 0.05e-14


def test_tol_floor_warning(m1):
    A, _ = m1
    res = R.randqb_fp(A, 1e-7, 10, 5, l_max=40)
    assert res.status in (R.QB_WARN_TOL_FLOOR, R.QB_NOT_CONVERGED)
    assert R.randqb_fp(A, 1e-2, 10, 5).status == R.QB_OK


# ---------------------------------------------------------------- Theorems 1 and 2


@pytest.mark.parametrize("algo", ["fp", "ei"])
@pytest.mark.parametrize("tol", [1e-1, 1e-2, 1e-3])
def test_theorem1_indicator_equals_residual(m1, algo, tol):
    A, _ = m1
    f = R.randqb_fp if algo == "fp" else R.randqb_ei
    res = f(A, tol, 10, 77)
    direct = R.residual_sq(A, res.Q, res.B)
    assert abs(res.E - direct) <= 1e-13 * res.normA2
    assert res.E < tol * tol * res.normA2
    assert res.status == R.QB_OK


def test_theorem2_trace_every_block(m2):
    A, _ = m2
    res = R.randqb_fp(A, 1e-6, 8, 3, row_by_row=False)
    assert len(res.E_trace) == res.blocks >= 5
    for i, E in enumerate(res.E_trace):
        k = min(8 * (i + 1), res.rank)
        direct = R.residual_sq(A, res.Q[:, :k], res.B[:k])
        assert abs(E - direct) <= 1e-13 * res.normA2


def test_orthonormal_q(m2):
    A, _ = m2
    for f in (R.randqb_fp, R.randqb_ei):
        res = f(A, 1e-5, 10, 4)
        assert R.orth_loss_inf(res.Q) < 1e-13


def test_normA2_is_sum_of_squares(m1):
    A, sig = m1
    assert abs(R.sumsq(A) - float(np.sum(sig ** 2))) < 1e-13 * float(np.sum(sig ** 2))
    Z = np.zeros((3, 4))
    Z[1, 2] = 3.0
    Z[2, 0] = -4.0
    assert R.sumsq(Z) == 25.0


# ---------------------------------------------------------------- Propositions 1-2


@pytest.mark.parametrize("b", [1, 7, 10, 16])
def test_fp_equals_ei(m2, b):
    A, _ = m2
    fp = R.randqb_fp(A, 1e-4, b, 21)
    ei = R.randqb_ei(A, 1e-4, b, 21)
    assert fp.rank == ei.rank
    nA = np.sqrt(fp.normA2)
    # Remark 4.1: FP's round-off in B_i grows with the number of blocks (215 at b = 1)
    assert np.linalg.norm(fp.B - ei.B) <= 1e-10 * nA
    assert np.max(np.abs(fp.Q - ei.Q)) <= 1e-10
    assert abs(fp.E - ei.E) <= 1e-12 * fp.normA2
    assert ei.passes == 2 * ei.blocks and fp.passes == 2 * fp.chunks


def test_fixed_rank_fp_equals_randqb(m1):
    A, _ = m1
    Om = R.omega(5, A.shape[1], 0, 60)
    Qf, Bf = R.randqb_fp_fixed(A, Om, 10)
    Qr, Br = R.randqb_fixed(A, Om)
    assert np.max(np.abs(Qf - Qr)) < 1e-9
    assert np.linalg.norm(Bf - Br) < 1e-10 * np.linalg.norm(A)
    # Algorithm 3 (no re-orthogonalisation) is the same map in exact arithmetic
    Q3, B3 = R.randqb_fp_fixed(A, Om[:, :30], 10, reorth=False)
    Qr3, Br3 = R.randqb_fixed(A, Om[:, :30])
    assert np.max(np.abs(Q3 - Qr3)) < 1e-8
    assert np.linalg.norm(B3 - Br3) < 1e-9 * np.linalg.norm(A)


def test_chunked_restart_matches_single_chunk(m2):
    A, _ = m2
    one = R.randqb_fp(A, 1e-3, 8, 9, l_tilde=200)
    many = R.randqb_fp(A, 1e-3, 8, 9, l_tilde=16)
    assert one.chunks == 1 and many.chunks > 2
    assert one.rank == many.rank
    assert many.passes == 2 * many.chunks
    assert np.linalg.norm(one.B - many.B) < 1e-11 * np.sqrt(one.normA2)


# ---------------------------------------------------------------- exact rank / SVD pins


def test_jacobi_svd_recovers_sigma():
    sig = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.25, 1e-3])
    A = W.lowrank_dense(20, 9, sig, 8).numpy()
    s = R.jacobi_svd(A)
    assert np.allclose(s[:7], sig, rtol=1e-13, atol=1e-15)
    assert np.all(s[7:] < 1e-14)


@pytest.mark.parametrize("algo", ["fp", "ei"])
def test_exact_rank_reconstruction(algo):
    r = 37
    A = W.exact_rank(120, 90, r, 14).numpy()
    f = R.randqb_fp if algo == "fp" else R.randqb_ei
    res = f(A, 1e-6, 10, 31)
    assert res.rank == r
    assert np.sqrt(R.residual_sq(A, res.Q, res.B)) <= 1e-13 * np.sqrt(res.normA2)
    # singular values of B are those of A when the rank is captured
    sa = R.jacobi_svd(A.T.copy())[:r]
    sb = R.jacobi_svd(res.B.T.copy())[:r]
    assert np.allclose(sa, sb, rtol=1e-10)


@pytest.mark.parametrize("algo", ["fp", "ei"])
def test_exhaustion_at_numerical_rank(algo):
    r = 23
    A = W.exact_rank(80, 70, r, 15).numpy()
    f = R.randqb_fp if algo == "fp" else R.randqb_ei
    res = f(A, 0.0, 10, 32)
    assert res.rank == r
    # with eps = 0 the run ends at the numerical rank either because the round-off
    # sized E turned negative (Section 3.3 notes E can go negative) or because the
    # exhaustion guard saw R_i(j,j) at round-off level
    if res.exhausted:
        assert res.status == R.QB_NOT_CONVERGED
    else:
        assert res.E < 0 and res.status == R.QB_WARN_TOL_FLOOR
    assert np.sqrt(R.residual_sq(A, res.Q, res.B)) <= 1e-13 * np.sqrt(res.normA2)


def test_scan_rows_guard_and_stop():
    Bi = np.array([[3.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    Rm = np.diag([1.0, 1e-13, 1.0])
    g = np.ones(3)
    # guard fires before row 1 (R(1,1) <= 2^-40 ||G_J(:,1)||)
    assert R._scan_rows(Bi, Rm, g, 100.0, 0.0, True) == (1, 91.0, True, True)
    # stop at the first row where E < eps^2, keeping that row
    Rm = np.eye(3)
    assert R._scan_rows(Bi, Rm, g, 14.0, 6.0, True) == (1, 5.0, True, False)
    assert R._scan_rows(Bi, Rm, g, 14.0, 3.0, True) == (2, 1.0, True, False)
    assert R._scan_rows(Bi, Rm, g, 14.0, 0.5, True) == (3, -1.0, True, False)
    assert R._scan_rows(Bi, Rm, g, 100.0, 0.5, True) == (3, 85.0, False, False)
    assert R._scan_rows(Bi, Rm, g, 100.0, 0.5, False) == (3, 85.0, False, False)
    # whole-block variant
    assert R._scan_rows(Bi, Rm, g, 14.0, 6.0, False) == (3, -1.0, True, False)


@pytest.mark.parametrize("tol", [3e-1, 1e-1, 3e-2, 1e-2, 1e-3])
def test_eckart_young_lower_bound(m1, tol):
    A, sig = m1
    opt = R.svd_optimal_rank(sig, tol)
    for f in (R.randqb_fp, R.randqb_ei):
        res = f(A, tol, 5, 41)
        assert res.rank >= opt


# ---------------------------------------------------------------- edge cases


def test_zero_matrix_and_large_tol(m1):
    A, _ = m1
    z = R.randqb_fp(np.zeros((30, 20)), 1e-2, 4, 1)
    assert z.rank == 0 and z.E == 0.0 and z.status == R.QB_OK
    big = R.randqb_fp(A, 1.5, 4, 1)
    assert big.rank == 0 and big.status == R.QB_OK


def test_lmax_reached_not_converged(m1):
    A, _ = m1
    res = R.randqb_fp(A, 1e-6, 10, 2, l_max=35)
    assert res.rank == 35 and res.status == R.QB_NOT_CONVERGED
    assert abs(res.E - R.residual_sq(A, res.Q, res.B)) <= 1e-13 * res.normA2


def test_whole_block_stopping(m1):
    A, _ = m1
    rb = R.randqb_fp(A, 1e-2, 10, 6, row_by_row=True)
    wb = R.randqb_fp(A, 1e-2, 10, 6, row_by_row=False)
    assert wb.rank % 10 == 0 and wb.rank >= rb.rank > wb.rank - 10


def test_wide_matrix_and_ragged_block():
    A = W.lowrank_dense(50, 130, W.sigma_law("exp7", 50), 17).numpy()
    fp = R.randqb_fp(A, 1e-12, 7, 3, l_max=50)
    ei = R.randqb_ei(A, 1e-12, 7, 3, l_max=50)
    assert fp.rank == ei.rank
    assert np.linalg.norm(fp.B - ei.B) < 1e-9 * np.sqrt(fp.normA2)


def test_nonfinite_input():
    A = np.ones((10, 8))
    A[3, 4] = np.nan
    assert R.randqb_fp(A, 1e-2, 2, 1).status == R.QB_ERR_NONFINITE
    A[3, 4] = np.inf
    assert R.randqb_ei(A, 1e-2, 2, 1).status == R.QB_ERR_NONFINITE


def test_sparse_equals_dense():
    csr = W.powerlaw_csr(400, 150, 3000, 5)
    S = csr.to_scipy()
    assert S.nnz == csr.nnz and np.all(np.diff(csr.rowptr) >= 0)
    D = S.toarray()
    for f in (R.randqb_fp, R.randqb_ei):
        a = f(S, 0.5, 10, 8)
        d = f(D, 0.5, 10, 8)
        assert a.rank == d.rank
        assert np.linalg.norm(a.B - d.B) < 1e-11 * np.sqrt(d.normA2)
        assert abs(a.E - R.residual_sq(D, a.Q, a.B)) < 1e-12 * a.normA2


def test_powerlaw_generator_shape():
    csr = W.powerlaw_csr(2000, 1000, 20000, 3)
    assert abs(csr.nnz - 20000) <= 0.002 * 20000 + 1000
    S = csr.to_scipy().tocsc()
    deg = np.diff(S.indptr)
    assert deg.max() > 10 * np.median(deg)           # heavy tail
    assert np.all(csr.val > 0)
    for i in range(0, 2000, 97):                    # sorted, distinct columns per row
        c = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


# ---------------------------------------------------------------- planted mistakes


def _pins_pass(A):
    """The cheap subset of the pins above, as a predicate."""
    fp = R.randqb_fp(A, 1e-3, 8, 19)
    ei = R.randqb_ei(A, 1e-3, 8, 19)
    ok = abs(fp.E - R.residual_sq(A, fp.Q, fp.B)) <= 1e-12 * fp.normA2
    ok &= fp.rank == ei.rank and np.linalg.norm(fp.B - ei.B) <= 1e-10 * np.sqrt(fp.normA2)
    ok &= abs(ei.E - R.residual_sq(A, ei.Q, ei.B)) <= 1e-12 * ei.normA2
    return bool(ok)


def _drop_wtb(H_J, Y, Qk, Bk, W_, Rm):
    import scipy.linalg
    S = H_J.T - (Y.T @ Qk) @ Bk
    return scipy.linalg.solve_triangular(Rm, S, trans="T", lower=False)


def _wrong_sign(H_J, Y, Qk, Bk, W_, Rm):
    import scipy.linalg
    S = H_J.T - (Y.T @ Qk) @ Bk + W_.T @ Bk
    return scipy.linalg.solve_triangular(Rm, S, trans="T", lower=False)


def _no_transpose(H_J, Y, Qk, Bk, W_, Rm):
    import scipy.linalg
    S = H_J.T - (Y.T @ Qk) @ Bk - W_.T @ Bk
    return scipy.linalg.solve_triangular(Rm, S, trans="N", lower=False)


def _row_sumsq_off(Bi):
    return np.einsum("ij,ij->i", Bi, Bi) * 0.5


@pytest.mark.parametrize("target,mutant", [
    ("block_b", _drop_wtb), ("block_b", _wrong_sign), ("block_b", _no_transpose),
    ("row_sumsq", _row_sumsq_off),
])
def test_planted_mistakes_are_caught(monkeypatch, m2, target, mutant):
    A, _ = m2
    assert _pins_pass(A)
    monkeypatch.setattr(R, target, mutant)
    assert not _pins_pass(A)


def test_planted_omega_misalignment_is_caught(monkeypatch, m2):
    A, _ = m2
    real = R.omega
    monkeypatch.setattr(R, "omega", lambda seed, n, col0, cols, batch=0: real(seed, n, col0 + 1, cols))
    fp = R.randqb_fp(A, 1e-3, 8, 19)
    monkeypatch.setattr(R, "omega", real)
    ei = R.randqb_ei(A, 1e-3, 8, 19)
    assert fp.rank != ei.rank or np.linalg.norm(fp.B - ei.B) > 1e-6 * np.sqrt(fp.normA2)


def test_adaptive_chunks_same_factorisation(m2):
    """The chunk schedule only regroups Omega's columns (the restart after Algorithm 4):
    Q, B, rank and E do not depend on it."""
    A, _ = m2
    fixed = R.randqb_fp(A, 1e-4, 8, 9)
    adapt = R.randqb_fp(A, 1e-4, 8, 9, l_tilde=-1)
    assert adapt.chunks >= 2 and adapt.passes == 2 * adapt.chunks
    assert adapt.rank == fixed.rank
    # chunk widths change the BLAS blocking of G and H; FP's B carries that round-off
    # amplified over the blocks (Remark 4.1)
    assert np.linalg.norm(adapt.B - fixed.B) < 1e-10 * np.sqrt(fixed.normA2)
    assert abs(adapt.E - fixed.E) < 1e-13 * fixed.normA2


def test_adaptive_chunk_width_rule():
    cw = R._chunk_width
    assert cw(True, 400, 8, 1000, 0, 0, 1.0, 1.0, 1e-6) == 64       # first chunk 8 b
    # E fell by e^-2 over the last 32 columns; eps^2 = e^-10 E needs 160 more -> 1.1*160+8
    w = cw(True, 4000, 8, 10000, 64, 32, 1.0, np.exp(-2.0), np.exp(-12.0))
    assert w == 184
    w = cw(True, 4000, 8, 10000, 64, 32, 1.0, np.exp(-1.0), np.exp(-12.0))
    assert w == 256                                                   # capped at 4 w
    assert cw(True, 50, 8, 1000, 64, 32, 1.0, 0.5, 1e-9) == 50       # never above the cap
    assert cw(True, 400, 8, 30, 64, 32, 1.0, 0.5, 1e-9) == 30        # nor past l_max
    assert cw(True, 400, 8, 1000, 64, 32, 1.0, -1e-3, 1e-9) == 128   # no decay info: double
    assert cw(False, 400, 8, 1000, 64, 32, 1.0, 0.5, 1e-9) == 400    # fixed schedule


def test_adaptive_schedule_measures_the_second_half(monkeypatch, m2):
    """The next chunk is sized from the indicator's decay over the previous chunk's second
    half: the rule sees span = w - b floor(nb / 2) and the E recorded at that block end."""
    A, _ = m2
    seen = []
    real = R._chunk_width

    def spy(adaptive, cap, b, left, w_prev, span, e_prev, e_now, eps2):
        seen.append((w_prev, span, e_prev, e_now))
        return real(adaptive, cap, b, left, w_prev, span, e_prev, e_now, eps2)

    monkeypatch.setattr(R, "_chunk_width", spy)
    res = R.randqb_fp(A, 1e-4, 8, 9, l_tilde=-1)
    assert len(seen) == res.chunks and seen[0][0] == 0
    w0, span, e_prev, e_now = seen[1]
    assert w0 == 64 and span == 32
    # E after 4 blocks (32 columns) and after 8 blocks of the first chunk
    assert e_prev == res.E_trace[3] and e_now == res.E_trace[7]
