"""GPU parity of the approximate SVD from QB (eq. (3)): the library's thin QR of B^T plus
one-sided Jacobi, through the C ABI, against the oracle (LAPACK SVD of B) on the same
seeded inputs, and against a known SVD.

Tolerances: singular values within 1e-12 sigma_1 (backward-stable factorisation of B: Weyl
gives |s_gpu - s_true| <= c u k ||B||_2); singular vectors of well-separated values within
1e-9 after the common sign rule (forward error u ||B||_2 / gap); Q B = U diag(s) V^T within
1e-12 ||B||_F; U^T U = I and V^T V = I within 1e-12 (columns of nonzero values).  The
end-to-end cases factorise A first (randQB_FP on GPU and in the oracle, each on its own)
and bound the top singular values by Weyl's inequality against those of A."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import randqb as R
from oracle import svd as S

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 7


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


def _known(m, n, k, sig, seed):
    """Q (m x k, orthonormal) and B = Ub diag(sig) Vb^T with known factors."""
    Q = W.haar_columns(m, k, seed, 1).numpy()
    Ub = W.haar_columns(k, k, seed, 2).numpy()
    Vb = W.haar_columns(n, k, seed, 3).numpy()
    return Q, (Ub * sig) @ Vb.T, Ub, Vb


def _gpu(qb, Q, B):
    Qd = torch.tensor(Q).cuda().T.contiguous().T     # column-major m x k
    Bd = torch.tensor(B).cuda().contiguous()
    r = qb.svd_from_qb(Qd, Bd)
    return r, r.U.cpu().numpy(), r.s.cpu().numpy(), r.V.cpu().numpy()


def _check_factor(Q, B, U, s, V, nz=None):
    k = len(s)
    nz = k if nz is None else nz
    QB = Q @ B
    assert np.all(np.diff(s) <= 0)
    assert np.linalg.norm(QB - (U * s) @ V.T) <= 1e-12 * np.linalg.norm(B)
    assert np.max(np.abs(U[:, :nz].T @ U[:, :nz] - np.eye(nz))) <= 1e-12
    assert np.max(np.abs(V.T @ V - np.eye(k))) <= 1e-12


@pytest.mark.parametrize("m,n,k", [(300, 200, 40), (1000, 800, 151), (200, 64, 64), (50, 40, 1),
                                   (5000, 3000, 300)])
def test_svd_known_factors(qb, m, n, k):
    _log(f"svd known {m}x{n} k={k}")
    sig = np.exp(-np.arange(k) / (0.2 * k + 1.0))
    Q, B, Ub, Vb = _known(m, n, k, sig, 61 + k)
    r, U, s, V = _gpu(qb, Q, B)
    _log(f"  sweeps {r.sweeps} status {r.status} max|ds| {np.max(np.abs(s - sig)):.2e}")
    assert r.status == qb.QB_OK
    assert np.max(np.abs(s - sig)) <= 1e-12 * sig[0]
    _check_factor(Q, B, U, s, V)
    sg = S.sign_rule(Vb)
    assert np.max(np.abs(V - Vb * sg)) <= 1e-9
    assert np.max(np.abs(U - (Q @ Ub) * sg)) <= 1e-9
    Uo, so, Vo = S.svd_from_qb(Q, B)
    assert np.max(np.abs(s - so)) <= 1e-12 * so[0]
    assert np.max(np.abs(V - Vo)) <= 1e-9 and np.max(np.abs(U - Uo)) <= 1e-9


def test_svd_rank_deficient_and_repeated(qb):
    """B of rank 45 < k = 50 (CholeskyQR of B^T breaks down: Householder fallback) with a
    repeated value: values, the product and orthogonality (vectors of a repeated value are
    not unique; those of the five round-off values are not checked)."""
    m, n, k = 400, 300, 50
    sig = np.exp(-np.arange(k) / 10.0)
    sig[3] = sig[4]
    sig[45:] = 0.0
    Q, B, _, _ = _known(m, n, k, sig, 71)
    r, U, s, V = _gpu(qb, Q, B)
    _log(f"rank-deficient: sweeps {r.sweeps} tail {s[44:]}")
    assert np.max(np.abs(s - sig)) <= 1e-12 * sig[0]
    _check_factor(Q, B, U, s, V, nz=45)


def test_svd_end_to_end(qb):
    """The 4000 x 3000 benchmark law: randQB_FP then eq. (3), on the GPU and in the oracle."""
    wl = W.C2_SMALL
    A = wl.make()
    An = A.numpy()
    res = qb.qb_fp_dense(A.cuda(), wl.tol, wl.b, SEED)
    r = qb.svd_from_qb(res.Q, res.B)
    s = r.s.cpu().numpy()
    ora = R.randqb_fp(An, wl.tol, wl.b, SEED)
    Uo, so, Vo = S.svd_from_qb(ora.Q, ora.B)
    assert res.rank == ora.rank and len(s) == len(so)
    nA = np.sqrt(ora.normA2)
    _log(f"end-to-end: rank {res.rank} sweeps {r.sweeps} max|s - s_oracle| {np.max(np.abs(s - so)):.2e}")
    assert np.max(np.abs(s - so)) <= 1e-10 * nA
    # Weyl: |s_j - sigma_j(A)| <= ||A - QB||_2 <= ||A - QB||_F < tol ||A||_F
    sA = np.linalg.svd(An, compute_uv=False)[: len(s)]
    assert np.max(np.abs(s - sA)) <= wl.tol * nA
    U, V = r.U.cpu().numpy(), r.V.cpu().numpy()
    top = 20   # well separated at the top of e^{-j/150}
    assert np.max(np.abs(V[:, :top] - Vo[:, :top])) <= 1e-6
    assert np.max(np.abs(U[:, :top] - Uo[:, :top])) <= 1e-6


def test_svd_full_size_properties(qb):
    """The 20000 x 15000 workload's factorisation (rank 1250) in the benchmark's launch
    configuration: product, orthogonality and Weyl's bound against the generator's law."""
    wl = W.C2
    seed = W.SEED_OMEGA | 2
    A = wl.make(device="cuda")
    res = qb.qb_fp_dense(A, wl.tol, wl.b, seed, l_max=min(wl.m, wl.n), l_tilde=-1)
    r = qb.svd_from_qb(res.Q, res.B)
    k = res.rank
    U, s, V = r.U, r.s, r.V
    QB = res.Q @ res.B
    prod = float(torch.linalg.matrix_norm(QB - (U * s) @ V.T) / torch.linalg.matrix_norm(res.B))
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    ou = float((U.T @ U - eye).abs().max())
    ov = float((V.T @ V - eye).abs().max())
    sn = s.cpu().numpy()
    nA = np.sqrt(res.normA2)
    sig = wl.sigma()[:k]
    _log(f"full size: k {k} sweeps {r.sweeps} product {prod:.2e} orth U {ou:.2e} V {ov:.2e} "
         f"max|s - sigma| {np.max(np.abs(sn - sig)):.2e}")
    assert r.status == qb.QB_OK
    # V = P W inherits the orthogonality of P, the CholeskyQR2 basis of the 15000 x 1250
    # panel B^T (about u k at its condition number); the bound is 64 k u
    bound = 64 * k * 2.0 ** -53
    assert prod <= bound and ou <= bound and ov <= bound
    # the generator's sigma_j plus noise of norm about 1e-8 (sqrt(m) + sqrt(n)) in the 2-norm
    assert np.max(np.abs(sn - sig)) <= wl.tol * nA + 1e-8 * (np.sqrt(wl.m) + np.sqrt(wl.n))
