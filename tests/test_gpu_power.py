"""GPU parity of the power scheme (Algorithm 4, P >= 1): the HIP path through
the C ABI against the binary64 oracle on the same seeded inputs, with the tolerances of
the P = 0 path (same rank, status, passes, blocks and chunks; E within 1e-10 ||A||^2; Q
and B within 1e-10 plus the method's forward-error scale; Q^T Q = I to 1e-12; E equal to
||A - QB||^2).  The power iterate is formed by block Gram-Schmidt with CholeskyQR on the
GPU and by Householder QR in the oracle; both are the Q factor of the same matrix, so the
cases keep the panels that the block loop reaches well conditioned.  Breakdown of
CholeskyQR (an exact-rank matrix) exercises the Householder fallback."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import randqb as R
from test_gpu_parity import _compare, _csr_dev

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 6


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


CASES = [
    # name, maker, tol, b, kwargs (power included)
    ("C1 Matrix-1 P=1", lambda: W.C1.make(), 1e-2, 20, {"power": 1}),
    ("poly2 400x300 P=2", lambda: W.lowrank_dense(400, 300, W.sigma_law("poly2", 300), 32), 1e-3, 10,
     {"power": 2}),
    ("restarts l~=16 P=1", lambda: W.lowrank_dense(260, 200, W.sigma_law("exp20", 200), 31), 1e-4, 8,
     {"power": 1, "l_tilde": 16}),
    ("ragged m<n b=7 P=1", lambda: W.lowrank_dense(150, 330, W.sigma_law("exp7", 150), 4), 1e-5, 7,
     {"power": 1, "l_tilde": 21}),
    ("adaptive P=1", lambda: W.lowrank_dense(900, 700, W.sigma_law("exp40", 700), 7), 1e-4, 16,
     {"power": 1, "l_tilde": -1}),
    ("exact rank 37 P=1", lambda: W.exact_rank(300, 200, 37, 14), 1e-6, 10, {"power": 1}),
    ("b=128 tall P=1", lambda: W.lowrank_dense(3000, 700, W.sigma_law("poly1.5", 700), 10), 1e-2, 128,
     {"power": 1}),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_power_parity_dense(qb, case):
    name, make, tol, b, kw = case
    _log(f"power parity {name}")
    A = make()
    An = A.numpy()
    res = qb.qb_fp_dense(A.cuda(), tol, b, SEED, **kw)
    ora = R.randqb_fp(An, tol, b, SEED, **kw)
    _log(f"  chunks {res.chunks}/{ora.chunks} passes {res.passes}/{ora.passes} "
         f"fallbacks {res.fallbacks} power ms {res.ms[6]:.2f}")
    _compare(res, ora, An, f"power {name}")
    assert res.chunks == ora.chunks


def test_power_lowers_rank(qb):
    """P = 1 against P = 0 on Matrix 1 at tol 1e-3: closer to the SVD rank (Table 4)."""
    A = W.lowrank_dense(2000, 1500, W.sigma_law("poly2", 1500), 33).cuda()
    r0 = qb.qb_fp_dense(A, 1e-3, 10, SEED)
    r1 = qb.qb_fp_dense(A, 1e-3, 10, SEED, power=1)
    opt = R.svd_optimal_rank(W.sigma_law("poly2", 1500), 1e-3)
    _log(f"poly2 2000x1500 tol 1e-3: svd {opt}, P=0 {r0.rank}, P=1 {r1.rank}")
    assert opt <= r1.rank < r0.rank
    assert r1.passes == 4 * r1.chunks


def test_power_parity_csr(qb):
    wl = W.C3_SMALL
    csr = wl.make()
    rp, ci, va = _csr_dev(csr)
    S = csr.to_scipy()
    _log(f"power csr {wl.name}")
    res = qb.qb_fp_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, SEED, power=1)
    ora = R.randqb_fp(S, wl.tol, wl.b, SEED, power=1)
    _compare(res, ora, S, "power csr")


def test_power_reproducible_and_rejections(qb):
    A = W.lowrank_dense(1200, 900, W.sigma_law("exp40", 900), 34).cuda()
    r1 = qb.qb_fp_dense(A, 1e-3, 32, SEED, power=1)
    r2 = qb.qb_fp_dense(A, 1e-3, 32, SEED, power=1)
    assert r1.rank == r2.rank and r1.E == r2.E
    assert torch.equal(r1.Q, r2.Q) and torch.equal(r1.B, r2.B)
    for kw, st in (({"power": -1}, qb.QB_ERR_ARG), ({"power": 17}, qb.QB_ERR_ARG)):
        with pytest.raises(qb.QBError) as e:
            qb.qb_fp_dense(A, 1e-3, 32, SEED, **kw)
        assert e.value.status == st
    with pytest.raises(qb.QBError) as e:
        qb.qb_fp_dense(W.to_bf16(A), 1e-2, 32, SEED, power=1)
    assert e.value.status == qb.QB_ERR_UNSUPPORTED


def test_power_full_size_properties(qb):
    """The 20000 x 15000 benchmark workload at P = 1 in the launch configuration the
    benchmark times (adaptive schedule, l_max = min(m, n)): E against the directly computed
    residual, orthogonality, rank between the SVD rank and the P = 0 rank, 2 P + 2 passes
    per chunk."""
    wl = W.C2
    seed = W.SEED_OMEGA | 2
    A = wl.make(device="cuda")
    r1 = qb.qb_fp_dense(A, wl.tol, wl.b, seed, l_max=min(wl.m, wl.n), l_tilde=-1, power=1)
    r0 = qb.qb_fp_dense(A, wl.tol, wl.b, seed, l_max=min(wl.m, wl.n), l_tilde=-1)
    res2 = float(torch.linalg.matrix_norm(A - r1.Q @ r1.B) ** 2)
    k = r1.rank
    orth = float((r1.Q.T @ r1.Q - torch.eye(k, dtype=torch.float64, device="cuda")).abs().sum(1).max())
    opt = R.svd_optimal_rank(wl.sigma(), wl.tol)
    _log(f"C2 P=1: rank {k} (P=0 {r0.rank}, svd {opt}) E/|A|^2 {r1.E / r1.normA2:.4e} "
         f"residual {res2 / r1.normA2:.4e} orth {orth:.2e} passes {r1.passes}")
    assert r1.status == qb.QB_OK
    assert abs(r1.E - res2) <= 1e-10 * r1.normA2
    assert orth <= 1e-12
    assert opt - 1 <= k < r0.rank
    assert r1.passes == 4 * r1.chunks


def test_power_csr_full_size_properties(qb):
    """The 500000 x 200000 CSR workload at P = 1 in the benchmark's launch configuration
    (l_max 16384, l~ = 50 b).  The residual cannot be formed densely, so: Q^T Q = I, and
    B = Q^T A on 64 sampled columns (with Q orthonormal this makes E = ||A||^2 - ||B||^2 the
    squared residual, Theorem 1), the indicator below eps^2, and 2 P + 2 passes per chunk."""
    wl = W.C3
    seed = W.SEED_OMEGA | 3
    csr = wl.make()
    rp, ci, va = _csr_dev(csr)
    res = qb.qb_fp_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, seed, l_max=16384, l_tilde=0, power=1)
    k = res.rank
    Q, B = res.Q, res.B
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    orth = float((Q.T @ Q - eye).abs().max())
    cols = np.random.default_rng(91).choice(csr.n, 64, replace=False)
    S = csr.to_scipy().tocsc()
    Acols = torch.tensor(S[:, cols].toarray(), device="cuda")
    dB = float(torch.linalg.matrix_norm(B[:, torch.tensor(cols, device="cuda")] - Q.T @ Acols))
    nB = float(torch.linalg.matrix_norm(B[:, torch.tensor(cols, device="cuda")]))
    _log(f"C3 P=1: rank {k} E_rel {np.sqrt(max(res.E, 0) / res.normA2):.4f} orth {orth:.2e} "
         f"|B - Q^T A|/|B| on sampled columns {dB / nB:.2e} passes {res.passes}")
    assert res.status == qb.QB_OK and res.E < (wl.tol ** 2) * res.normA2
    assert orth <= 1e-11
    assert dB <= 1e-9 * nB
    assert res.passes == 4 * res.chunks


@pytest.mark.parametrize("algo", ["fp_paper_rule", "ei"])
def test_csr_full_size_p0_properties(qb, algo):
    """The 500000 x 200000 CSR workload at P = 0 as the benchmark times it (l_max 16384;
    randQB_FP with the paper's l~ = 50 b, and randQB_EI), where the rank reaches about 14000
    and the drift of eq. (23) that Remark 4.1 describes is largest: Q^T Q = I, B = Q^T A on 64
    sampled columns (with Q orthonormal this makes E = ||A||^2 - ||B||^2 the squared
    residual, Theorem 1), E below eps^2, and the pass count (2 per chunk for randQB_FP, 2 per
    block for randQB_EI)."""
    wl = W.C3
    seed = W.SEED_OMEGA | 3
    csr = wl.make()
    rp, ci, va = _csr_dev(csr)
    _log(f"C3 P=0 {algo}")
    if algo == "ei":
        res = qb.qb_ei_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, seed, l_max=16384)
    else:
        res = qb.qb_fp_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, seed, l_max=16384, l_tilde=0)
    k = res.rank
    Q, B = res.Q, res.B
    orth = float((Q.T @ Q - torch.eye(k, dtype=torch.float64, device="cuda")).abs().max())
    cols = np.random.default_rng(92).choice(csr.n, 64, replace=False)
    S = csr.to_scipy().tocsc()
    Acols = torch.tensor(S[:, cols].toarray(), device="cuda")
    tc = torch.tensor(cols, device="cuda")
    dB = float(torch.linalg.matrix_norm(B[:, tc] - Q.T @ Acols))
    nB = float(torch.linalg.matrix_norm(B[:, tc]))
    _log(f"C3 P=0 {algo}: rank {k} E_rel {np.sqrt(max(res.E, 0) / res.normA2):.4f} orth {orth:.2e} "
         f"|B - Q^T A|/|B| on sampled columns {dB / nB:.2e} passes {res.passes} blocks {res.blocks}")
    assert res.status == qb.QB_OK and res.E < (wl.tol ** 2) * res.normA2
    assert 10000 <= k <= 16384
    assert orth <= 1e-11
    assert dB <= 1e-9 * nB
    if algo == "ei":
        assert res.passes == 2 * res.blocks
    else:
        assert res.passes == 2 * res.chunks
