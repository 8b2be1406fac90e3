"""Pins of the trQRCP oracle (Remark 3.2) against facts that do not come from the oracle:
brute-force greedy column pivoting on tiny matrices, LAPACK's column-pivoted QR when the
sketch is the matrix itself, Theorem 1's identity, the triangular shape of R, exact rank,
and the non-increasing diagonal of the deterministic pivoted QR.  Planted mistakes (no
sample update, a sign flip in it) must fail these pins."""
import numpy as np
import pytest
import scipy.linalg

from oracle import randqb as R
from oracle import trqrcp as T
import workloads as W


def _decaying(m, n, seed, decay=0.9):
    g = np.random.default_rng(seed)
    return g.standard_normal((m, n)) * (decay ** np.arange(n))[None, :] * \
        (1.0 + g.random(n))[None, :]


def _greedy_pivots(A, k):
    """Businger-Golub by brute force: at each step the column of largest residual norm
    (first index among equals), residuals by Gram-Schmidt against the chosen columns, done
    twice."""
    Rm = np.array(A, dtype=np.float64)
    n = Rm.shape[1]
    piv = []
    Qs = []
    for _ in range(k):
        norms = np.array([-1.0 if j in piv else float(np.dot(Rm[:, j], Rm[:, j])) for j in range(n)])
        p = int(np.argmax(norms))
        piv.append(p)
        q = Rm[:, p] / np.sqrt(norms[p])
        for qq in Qs:
            q = q - qq * np.dot(qq, q)
        q = q / np.linalg.norm(q)
        Qs.append(q)
        for _ in range(2):
            Rm = Rm - np.outer(q, q @ Rm)
    return piv


@pytest.mark.parametrize("m,n,b,seed", [(12, 9, 1, 1), (12, 9, 2, 2), (15, 11, 3, 3), (9, 14, 2, 4)])
def test_pivots_match_brute_force(m, n, b, seed):
    A = _decaying(m, n, seed)
    r = T.trqrcp(A, 1e-6, b, 0, sketch=A)
    assert r.rank >= 4
    assert list(r.piv) == _greedy_pivots(A, r.rank)


def test_planted_mistakes_fail_the_brute_force_pin():
    bad_stale, bad_sign = 0, 0
    for seed in range(1, 6):
        A = _decaying(14, 12, seed, decay=0.95)
        want = _greedy_pivots(A, 10)
        r = T.trqrcp(A, 1e-9, 2, 0, sketch=A, l_max=10, _update=False)
        bad_stale += list(r.piv) != want[:r.rank]
    assert bad_stale >= 3
    # a sign flip in the sample update: monkeypatch the solve to return -M
    orig = scipy.linalg.solve_triangular
    try:
        T.scipy.linalg.solve_triangular = lambda *a, **k: -orig(*a, **k)
        for seed in range(1, 6):
            A = _decaying(14, 12, seed, decay=0.95)
            want = _greedy_pivots(A, 10)
            r = T.trqrcp(A, 1e-9, 2, 0, sketch=A, l_max=10)
            bad_sign += list(r.piv) != want[:r.rank]
    finally:
        T.scipy.linalg.solve_triangular = orig
    assert bad_sign >= 3


def test_sketch_equal_to_a_is_lapack_qrcp():
    A = W.lowrank_dense(300, 200, W.sigma_law("poly1.5", 200), 11)
    A = A.numpy() if hasattr(A, "numpy") else A
    r = T.trqrcp(A, 1e-3, 16, 0, sketch=A)
    _, _, P = scipy.linalg.qr(A, pivoting=True)
    assert r.rank > 32
    assert np.array_equal(r.piv, P[:r.rank])


def test_deterministic_diag_nonincreasing():
    A = _decaying(80, 60, 7, decay=0.93)
    r = T.trqrcp(A, 1e-8, 8, 0, sketch=A)
    d = np.abs(np.diag(r.B[:, r.piv]))
    assert np.all(d[1:] <= d[:-1] * (1 + 1e-12))


@pytest.mark.parametrize("b,ovs", [(8, 8), (16, 0), (5, 3)])
def test_indicator_is_residual_and_r_triangular(b, ovs):
    A = W.lowrank_dense(400, 250, W.sigma_law("exp7", 250), 12)
    A = A.numpy() if hasattr(A, "numpy") else A
    r = T.trqrcp(A, 1e-4, b, 5, oversample=ovs)
    assert r.status == R.QB_OK
    res = R.residual_sq(A, r.Q, r.B)
    assert abs(r.E - res) <= 1e-12 * r.normA2
    assert res < 1e-8 * r.normA2
    assert R.orth_loss_inf(r.Q) < 1e-13
    Rp = r.B[:, r.piv]
    assert np.max(np.abs(np.tril(Rp, -1))) <= 1e-13 * np.sqrt(r.normA2)
    assert np.all(np.diff(r.E_trace) < 0)
    # the rank is the first row where the indicator drops below eps^2 (Section 3.1)
    k = r.rank
    assert R.residual_sq(A, r.Q[:, :k - 1], r.B[:k - 1]) >= 1e-8 * r.normA2
    assert r.passes == 1 + r.blocks
    assert len(set(r.piv.tolist())) == k


def test_exact_rank():
    g = np.random.default_rng(3)
    A = g.standard_normal((300, 37)) @ g.standard_normal((37, 200))
    r = T.trqrcp(A, 1e-10, 16, 9)
    assert r.rank == 37
    assert R.residual_sq(A, r.Q, r.B) <= 1e-24 * r.normA2 or r.E < 1e-20 * r.normA2


def test_rank_close_to_deterministic_and_above_optimal():
    A = W.lowrank_dense(600, 400, W.sigma_law("poly2", 400), 13)
    A = A.numpy() if hasattr(A, "numpy") else A
    sig = np.linalg.svd(A, compute_uv=False)
    for tol in (1e-2, 1e-3):
        kopt = R.svd_optimal_rank(sig, tol)
        det = T.trqrcp(A, tol, 16, 0, sketch=A).rank
        ran = T.trqrcp(A, tol, 16, 21).rank
        assert kopt <= ran <= int(1.3 * det) + 16
        assert kopt <= det


def test_degenerate_and_rejections():
    r = T.trqrcp(np.zeros((20, 10)), 1e-3, 4, 0)
    assert r.rank == 0 and r.status == R.QB_OK
    r = T.trqrcp(np.ones((20, 10)), 2.0, 4, 0)
    assert r.rank == 0
    r = T.trqrcp(np.ones((20, 10)), 1e-3, 4, 0)   # rank one
    assert r.rank == 1
    with pytest.raises(ValueError):
        T.trqrcp(np.ones((5, 5)), 1e-3, 0, 0)
    with pytest.raises(ValueError):
        T.trqrcp(np.ones((5, 5)), 1e-3, 2, 0, oversample=-1)
