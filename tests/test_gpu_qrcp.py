"""GPU parity of trQRCP driven by the indicator (Remark 3.2): the HIP path through the C ABI
against the oracle (oracle/trqrcp.py) on the same seeded inputs.

Bar: the pivots are index work decided in binary64 on both sides, and must be equal;
rank, status, passes and blocks equal; |E_gpu - E_oracle| <= 1e-10 ||A||^2; Q and B within
the bounds of the randQB_EI parity (B_i = Q_i^T A is formed directly, as in Algorithm 2):
||dB||_F <= 1e-10 ||A||_F + 1e3 u s1^2 / s_min, max |dQ| <= 1e-10 + 1e3 u s1 / s_min;
||Q^T Q - I||_inf <= 1e-12; E equal to ||A - QB||^2 within 1e-10 ||A||^2.  At the full
size of the 20000 x 15000 workload: properties that hold at any size."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import randqb as R
from oracle import trqrcp as T

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 3
U = 2.0 ** -53


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


def _compare(res, ora, A, label):
    nA2 = ora.normA2
    _log(f"{label}: gpu rank {res.rank} E {res.E:.6e} status {res.status} blocks {res.blocks} | "
         f"oracle rank {ora.rank} E {ora.E:.6e} status {ora.status} blocks {ora.blocks}")
    assert abs(res.normA2 - nA2) <= 1e-14 * max(nA2, 1e-300)
    piv = res.piv.cpu().numpy().astype(np.int64) if res.piv is not None else np.empty(0, np.int64)
    assert np.array_equal(piv, ora.piv)
    assert res.rank == ora.rank
    assert res.status == ora.status
    assert res.exhausted == ora.exhausted
    assert res.passes == ora.passes and res.blocks == ora.blocks
    assert abs(res.E - ora.E) <= 1e-10 * nA2
    if res.rank == 0:
        return
    Qg = res.Q.cpu().numpy()
    Bg = res.B.cpu().numpy()
    rows = np.sqrt(np.einsum("ij,ij->i", ora.B, ora.B))
    s1, smin = rows.max(), rows.min()
    b_bound = 1e-10 * np.sqrt(nA2) + 1e3 * U * s1 * s1 / smin
    q_bound = 1e-10 + 1e3 * U * s1 / smin
    db, dq = np.linalg.norm(Bg - ora.B), np.max(np.abs(Qg - ora.Q))
    _log(f"  |dB|_F {db:.3e} (bound {b_bound:.3e})  max|dQ| {dq:.3e} (bound {q_bound:.3e})")
    assert db <= b_bound
    assert dq <= q_bound
    assert R.orth_loss_inf(Qg) <= 1e-12
    assert abs(res.E - R.residual_sq(np.asarray(A), Qg, Bg)) <= 1e-10 * nA2


def _np(A):
    return A.numpy() if hasattr(A, "numpy") else np.asarray(A)


CASES = [
    # m, n, b, oversample, tol, spectrum, l_max
    (400, 250, 8, 8, 1e-4, "exp7", None),      # many blocks, ragged last block
    (700, 530, 20, 8, 1e-3, "poly2", None),    # ragged tiles, several blocks
    (300, 200, 16, 0, 1e-3, "poly1.5", None),  # no oversampling
    (1000, 800, 64, 8, 1e-2, "poly1.5", None),
    (60, 40, 1, 4, 1e-3, "exp7", None),        # b = 1: one pivot per block
    (500, 300, 16, 8, 1e-9, "poly2", 40),      # capped: not converged at l_max
    (256, 900, 32, 16, 1e-3, "sshape", None),  # wide
    (600, 400, 128, 128, 1e-3, "poly1.5", None),   # the tallest sketch: b + oversample = 256 rows
]


@pytest.mark.parametrize("m,n,b,ovs,tol,kind,l_max", CASES)
def test_trqrcp_vs_oracle(qb, m, n, b, ovs, tol, kind, l_max):
    label = f"trqrcp {m}x{n} b={b} ovs={ovs} tol={tol} {kind} l_max={l_max}"
    _log(label)
    A = _np(W.lowrank_dense(m, n, W.sigma_law(kind, min(m, n)), 17))
    ora = T.trqrcp(A, tol, b, SEED, oversample=ovs, l_max=l_max)
    res = qb.qb_trqrcp_dense(torch.from_numpy(A).cuda(), tol, b, SEED, oversample=ovs, l_max=l_max)
    _compare(res, ora, A, label)


def test_trqrcp_whole_block_stopping(qb):
    """Algorithm 1's whole-block test (row_by_row off): the rank is a multiple of b."""
    A = _np(W.lowrank_dense(600, 450, W.sigma_law("poly2", 450), 19))
    ora = T.trqrcp(A, 1e-3, 16, SEED, row_by_row=False)
    res = qb.qb_trqrcp_dense(torch.from_numpy(A).cuda(), 1e-3, 16, SEED, row_by_row=False)
    assert res.rank % 16 == 0
    _compare(res, ora, A, "trqrcp whole-block 600x450 b=16")


def test_trqrcp_strided_input(qb):
    """A row-major view with row stride 513 > n = 509 (misaligned rows)."""
    full = _np(W.lowrank_dense(420, 513, W.sigma_law("exp7", 420), 20))
    A = np.ascontiguousarray(full[:, :509])
    ora = T.trqrcp(A, 1e-4, 12, SEED, oversample=5)
    view = torch.from_numpy(full).cuda()[:, :509]
    assert view.stride(0) == 513
    res = qb.qb_trqrcp_dense(view, 1e-4, 12, SEED, oversample=5)
    _compare(res, ora, A, "trqrcp strided 420x509 ld=513 b=12")


def test_trqrcp_benchmark_law_small(qb):
    """The benchmark's spectrum law at 4000 x 3000 (b = 64, tol 1e-3)."""
    wl = W.C2_SMALL
    A = wl.make().numpy()
    ora = T.trqrcp(A, wl.tol, wl.b, SEED)
    res = qb.qb_trqrcp_dense(torch.from_numpy(A).cuda(), wl.tol, wl.b, SEED)
    _compare(res, ora, A, f"trqrcp {wl.name}")


def test_trqrcp_exact_rank(qb):
    g = np.random.default_rng(3)
    A = g.standard_normal((300, 37)) @ g.standard_normal((37, 200))
    ora = T.trqrcp(A, 1e-10, 16, SEED)
    res = qb.qb_trqrcp_dense(torch.from_numpy(A).cuda(), 1e-10, 16, SEED)
    _log(f"exact rank 37: gpu {res.rank} (E {res.E:.3e}) oracle {ora.rank}")
    assert res.rank == ora.rank == 37
    assert np.array_equal(res.piv.cpu().numpy(), ora.piv)


def test_trqrcp_degenerate(qb):
    Z = torch.zeros((40, 30), dtype=torch.float64, device="cuda")
    r = qb.qb_trqrcp_dense(Z, 1e-3, 8, SEED)
    assert r.rank == 0 and r.status == 0
    O = torch.ones((40, 30), dtype=torch.float64, device="cuda")
    assert qb.qb_trqrcp_dense(O, 2.0, 8, SEED).rank == 0        # tol > 1
    r = qb.qb_trqrcp_dense(O, 1e-3, 8, SEED)                      # rank one
    ora = T.trqrcp(np.ones((40, 30)), 1e-3, 8, SEED)
    assert r.rank == ora.rank == 1
    assert r.piv.cpu().numpy().tolist() == ora.piv.tolist()
    one = torch.full((1, 1), 3.0, dtype=torch.float64, device="cuda")
    r = qb.qb_trqrcp_dense(one, 1e-3, 4, SEED)
    assert r.rank == 1 and r.piv.cpu().tolist() == [0]


def test_trqrcp_reproducible_and_rejections(qb):
    A = W.lowrank_dense(700, 530, W.sigma_law("poly2", 530), 18).cuda()
    r1 = qb.qb_trqrcp_dense(A, 1e-3, 20, SEED)
    r2 = qb.qb_trqrcp_dense(A, 1e-3, 20, SEED)
    assert torch.equal(r1.piv, r2.piv)
    assert torch.equal(r1.Q, r2.Q) and torch.equal(r1.B, r2.B)
    with pytest.raises(qb.QBError):
        qb.qb_trqrcp_dense(A, 1e-3, 20, SEED, oversample=200)
    with pytest.raises(ValueError):                 # refused by the marshalling
        qb.qb_trqrcp_dense(A.float(), 1e-3, 20, SEED)
    with pytest.raises(qb.QBError) as e:            # binary64 only: the ABI's own refusal
        qb.qb_trqrcp_dense(A.to(torch.bfloat16), 1e-3, 20, SEED)
    assert e.value.status == -5


def test_trqrcp_full_size_properties(qb):
    """The 20000 x 15000 workload of the benchmark, b = 64, tol 1e-3."""
    wl = W.C2
    A = wl.make(device="cuda")
    m, n = A.shape
    _log(f"trqrcp full size {m}x{n}")
    r = qb.qb_trqrcp_dense(A, 1e-3, 64, SEED)
    _log(f"  rank {r.rank} E/|A|^2 {r.E / r.normA2:.3e} blocks {r.blocks} ms {r.ms[5]:.1f}")
    assert r.status == 0 and r.rank > 0
    assert r.passes == 1 + r.blocks
    Q, B = r.Q, r.B
    k = r.rank
    piv = r.piv.long()
    assert torch.unique(piv).numel() == k
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    assert (Q.T @ Q - eye).abs().max().item() <= 1e-11
    # Theorem 1: E equals the squared residual
    res = torch.linalg.matrix_norm(A - Q @ B).item() ** 2
    assert abs(res - r.E) <= 1e-9 * r.normA2
    assert r.E < 1e-6 * r.normA2
    # R = B(:, piv) is upper triangular up to rounding
    Rp = B[:, piv]
    assert torch.tril(Rp, -1).abs().max().item() <= 1e-12 * r.normA2 ** 0.5
    # B = Q^T A on sampled columns
    cols = torch.arange(0, n, max(1, n // 64), device="cuda")
    assert (B[:, cols] - Q.T @ A[:, cols]).abs().max().item() <= 1e-10 * r.normA2 ** 0.5
