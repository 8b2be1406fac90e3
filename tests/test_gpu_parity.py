"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs.

Tolerances (FP64 path): Omega bit-exact; same rank, status, passes and blocks;
|E_gpu - E_oracle| <= 1e-10 ||A||^2; ||Q^T Q - I||_inf <= 1e-12; E equal to the directly
computed ||A - QB||^2 within 1e-10 ||A||^2; and entrywise

    ||B_gpu - B_oracle||_F <= 1e-10 ||A||_F + 1e3 u sigma_1^2 / s_min
    max |Q_gpu - Q_oracle|  <= 1e-10          + 1e3 u sigma_1   / s_min

with u = 2^-53, sigma_1 ~ ||B(0,:)|| and s_min the smallest row norm of the oracle's B.
The second terms are the forward-error scale of the method itself: randQB_FP forms
B_i = R_i^{-T}(H_J^T - ...) from terms of size sigma_1^2 to get rows of size s_min
(Remark 4.1), and the trailing columns of Q are fixed only up to u ||A|| over the local
singular-value gap; for the tolerances of the benchmark workloads (1e-2, 1e-3) the
first terms dominate."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import randqb as R
from oracle import rng as ORNG

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 1


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------- Omega, ||A||^2, sketch


@pytest.mark.parametrize("rows,cols,row0,col0,seed", [
    (4096, 256, 0, 0, SEED), (513, 257, 3, 5, 7), (1, 1, 0, 9, 2 ** 63 + 5), (37, 2, 100000, 1, 0)])
def test_omega_bit_exact(qb, rows, cols, row0, col0, seed):
    _log(f"omega {rows}x{cols} @({row0},{col0}) seed {seed}")
    g = qb.qb_gaussian_fill(seed, rows, cols, row0=row0, col0=col0).cpu().numpy()
    o = ORNG.gaussian_matrix(seed, rows, cols, row0, col0)
    assert np.array_equal(g.view(np.int64), o.view(np.int64))


def test_omega_streams_and_batches_bit_exact(qb):
    g = qb.qb_gaussian_fill(11, 64, 33, stream_id=3, batch=7).cpu().numpy()
    o = ORNG.gaussian_matrix(11, 64, 33, stream=3, batch=7)
    assert np.array_equal(g.view(np.int64), o.view(np.int64))


@pytest.mark.parametrize("m,n", [(1000, 800), (1, 1), (3, 70001), (4097, 33)])
def test_sumsq(qb, m, n):
    _log(f"sumsq {m}x{n}")
    A = W.gaussian_dense(m, n, 5)
    got = qb.qb_sumsq_dense(A.cuda())
    want = R.sumsq(A.numpy())
    assert abs(got - want) <= 1e-14 * want


@pytest.mark.parametrize("m,n,l,col0,slice_cols", [
    (1000, 800, 200, 0, False),    # ragged tiles in every dimension
    (257, 129, 33, 5, True),       # odd ld (sliced view), odd Omega offset, misaligned rows
    (4096, 1024, 256, 64, False),  # aligned interior tiles
    (64, 4096, 16, 0, False),      # short and wide
])
def test_sketch_dense(qb, m, n, l, col0, slice_cols):
    _log(f"sketch {m}x{n} l={l} col0={col0} slice={slice_cols}")
    A = W.gaussian_dense(m, n + (1 if slice_cols else 0), 9)
    Ad = A.cuda()
    if slice_cols:
        A, Ad = A[:, :n], Ad[:, :n]
    om, g, h = qb.qb_sketch_dense(Ad, SEED, col0, l)
    An = A.numpy()
    Om = ORNG.gaussian_matrix(SEED, n, l, 0, col0)
    assert np.array_equal(om.cpu().numpy().view(np.int64), Om.view(np.int64))
    Gr = An @ Om
    Hr = An.T @ Gr
    gg, hh = g.cpu().numpy(), h.cpu().numpy()
    # error of an FP64 dot product of length K, relative to the magnitudes summed
    assert np.max(np.abs(gg - Gr)) <= 1e-13 * np.sqrt(n) * np.max(np.abs(An)) * np.max(np.abs(Om)) * 4
    assert np.linalg.norm(gg - Gr) <= 1e-14 * np.linalg.norm(Gr) * np.sqrt(n)
    assert np.linalg.norm(hh - Hr) <= 1e-14 * np.linalg.norm(Hr) * np.sqrt(m * n) + 1e-300


# ---------------------------------------------------------------- full method parity


U = 2.0 ** -53


def _compare(res, ora, A, label, q_tol=1e-10, b_tol=1e-10, e_tol=1e-10, orth_tol=1e-12):
    nA2 = ora.normA2
    _log(f"{label}: gpu rank {res.rank} E {res.E:.6e} status {res.status} | "
         f"oracle rank {ora.rank} E {ora.E:.6e} status {ora.status}")
    assert abs(res.normA2 - nA2) <= 1e-14 * max(nA2, 1e-300)
    assert res.rank == ora.rank
    assert res.status == ora.status
    assert res.exhausted == ora.exhausted
    assert res.passes == ora.passes and res.blocks == ora.blocks
    assert abs(res.E - ora.E) <= e_tol * nA2
    if res.rank == 0:
        return
    Qg = res.Q.cpu().numpy()
    Bg = res.B.cpu().numpy()
    rows = np.sqrt(np.einsum("ij,ij->i", ora.B, ora.B))
    s1, smin = rows[0], rows.min()
    b_bound = b_tol * np.sqrt(nA2) + 1e3 * U * s1 * s1 / smin
    q_bound = q_tol + 1e3 * U * s1 / smin
    db, dq = np.linalg.norm(Bg - ora.B), np.max(np.abs(Qg - ora.Q))
    _log(f"  |dB|_F {db:.3e} (bound {b_bound:.3e})  max|dQ| {dq:.3e} (bound {q_bound:.3e})")
    assert db <= b_bound
    assert dq <= q_bound
    assert R.orth_loss_inf(Qg) <= orth_tol
    An = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    assert abs(res.E - R.residual_sq(An, Qg, Bg)) <= 1e-10 * nA2


CASES = [
    # name, workload maker, tol, b, extra kwargs
    ("C1 Matrix-1 1000x800 b=20", lambda: W.C1.make(), 1e-2, 20, {}),
    ("exp20 600x500 b=16 tol1e-6", lambda: W.lowrank_dense(600, 500, W.sigma_law("exp20", 500), 3), 1e-6, 16, {}),
    ("ragged b=7 m<n", lambda: W.lowrank_dense(150, 330, W.sigma_law("exp7", 150), 4), 1e-5, 7, {}),
    ("b=1", lambda: W.lowrank_dense(90, 80, W.sigma_law("exp7", 80), 6), 1e-4, 1, {}),
    ("multi-chunk l~=32", lambda: W.lowrank_dense(700, 400, W.sigma_law("exp20", 400), 5), 1e-4, 16,
     {"l_tilde": 32}),
    ("adaptive chunks", lambda: W.lowrank_dense(900, 700, W.sigma_law("exp40", 700), 7), 1e-4, 16,
     {"l_tilde": -1}),
    ("whole-block stop", lambda: W.lowrank_dense(500, 300, W.sigma_law("poly2", 300), 8), 1e-3, 10,
     {"row_by_row": False}),
    ("l_max reached", lambda: W.lowrank_dense(400, 300, W.sigma_law("poly2", 300), 9), 1e-6, 10,
     {"l_max": 45}),
    ("exact rank 37", lambda: W.exact_rank(300, 200, 37, 14), 1e-6, 10, {}),
    ("b=128 tall", lambda: W.lowrank_dense(3000, 700, W.sigma_law("poly1.5", 700), 10), 1e-2, 128, {}),
]


@pytest.mark.parametrize("algo", ["fp", "ei"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_method_parity(qb, case, algo):
    name, make, tol, b, kw = case
    _log(f"parity {algo} {name}")
    A = make()
    An = A.numpy()
    Ad = A.cuda()
    if algo == "fp":
        res = qb.qb_fp_dense(Ad, tol, b, SEED, **kw)
        ora = R.randqb_fp(An, tol, b, SEED, **kw)
    else:
        kw = {k: v for k, v in kw.items() if k != "l_tilde"}
        res = qb.qb_ei_dense(Ad, tol, b, SEED, **kw)
        ora = R.randqb_ei(An, tol, b, SEED, **kw)
    _compare(res, ora, An, f"{algo} {name}")


def test_c2_small_parity(qb):
    """The benchmark workload's law at an oracle-friendly size (4000 x 3000)."""
    A = W.C2_SMALL.make()
    An = A.numpy()
    for algo, kw in (("fp", {}), ("fp", {"l_tilde": -1}), ("ei", {})):
        _log(f"C2-small {algo} {kw}")
        f = qb.qb_fp_dense if algo == "fp" else qb.qb_ei_dense
        g = R.randqb_fp if algo == "fp" else R.randqb_ei
        res = f(A.cuda(), W.C2_SMALL.tol, W.C2_SMALL.b, SEED, **kw)
        ora = g(An, W.C2_SMALL.tol, W.C2_SMALL.b, SEED, **kw)
        _compare(res, ora, An, f"C2-small {algo} {kw}")
        assert res.chunks == ora.chunks


def test_degenerate_inputs(qb):
    z = torch.zeros(40, 30, dtype=torch.float64, device="cuda")
    r = qb.qb_fp_dense(z, 1e-2, 4, SEED)
    assert r.rank == 0 and r.E == 0.0 and r.status == qb.QB_OK
    A = W.lowrank_dense(60, 50, W.sigma_law("poly2", 50), 2).cuda()
    r = qb.qb_ei_dense(A, 1.5, 4, SEED)
    assert r.rank == 0 and r.status == qb.QB_OK
    r = qb.qb_fp_dense(A, 1e-7, 4, SEED, l_max=20)
    assert r.status in (qb.QB_WARN_TOL_FLOOR, qb.QB_NOT_CONVERGED)
    bad = A.clone()
    bad[3, 7] = float("nan")
    with pytest.raises(qb.QBError) as e:
        qb.qb_fp_dense(bad, 1e-2, 4, SEED)
    assert e.value.status == qb.QB_ERR_NONFINITE
    with pytest.raises(qb.QBError) as e:
        qb.qb_ei_dense(A, 1e-2, 4, SEED, power=1)
    assert e.value.status == qb.QB_ERR_UNSUPPORTED


def test_below_theorem3_floor(qb):
    """tol below sqrt(4u/0.01) ~ 2.1e-7: E is only accurate to about 4u ||A||^2, so the
    rank is not comparable run to run; check the warning and E == ||A - QB||^2."""
    A = W.lowrank_dense(150, 330, W.sigma_law("exp7", 150), 4)
    for algo in ("fp", "ei"):
        f = qb.qb_fp_dense if algo == "fp" else qb.qb_ei_dense
        res = f(A.cuda(), 1e-9, 7, SEED)
        assert res.status in (qb.QB_WARN_TOL_FLOOR, qb.QB_NOT_CONVERGED)
        Qg, Bg = res.Q.cpu().numpy(), res.B.cpu().numpy()
        assert abs(res.E - R.residual_sq(A.numpy(), Qg, Bg)) <= 1e-13 * res.normA2
        assert R.orth_loss_inf(Qg) <= 1e-12


def test_exhaustion_guard_matches_oracle(qb):
    A = W.exact_rank(200, 150, 23, 15)
    for algo in ("fp", "ei"):
        f = qb.qb_fp_dense if algo == "fp" else qb.qb_ei_dense
        res = f(A.cuda(), 0.0, 10, SEED)
        _log(f"exhaust {algo}: rank {res.rank} E {res.E:.3e} exhausted {res.exhausted} "
             f"fallbacks {res.fallbacks}")
        assert res.rank == 23
        Qg, Bg = res.Q.cpu().numpy(), res.B.cpu().numpy()
        assert np.sqrt(R.residual_sq(A.numpy(), Qg, Bg)) <= 1e-12 * np.sqrt(res.normA2)


def test_bitwise_reproducible(qb):
    A = W.lowrank_dense(2000, 1500, W.sigma_law("exp150", 1500), 21).cuda()
    r1 = qb.qb_fp_dense(A, 1e-3, 64, SEED)
    r2 = qb.qb_fp_dense(A, 1e-3, 64, SEED)
    assert r1.rank == r2.rank and r1.E == r2.E
    assert torch.equal(r1.B, r2.B) and torch.equal(r1.Q, r2.Q)


# ---------------------------------------------------------------- sparse (CSR)


def _csr_dev(csr):
    return (torch.from_numpy(csr.rowptr).cuda(), torch.from_numpy(csr.colind).cuda(),
            torch.from_numpy(csr.val).cuda())


def test_sketch_csr(qb):
    csr = W.powerlaw_csr(3000, 1200, 30000, 4)
    rp, ci, va = _csr_dev(csr)
    om, g, h, _ = qb.qb_sketch_csr(csr.m, csr.n, rp, ci, va, SEED, 3, 300)
    S = csr.to_scipy()
    Om = ORNG.gaussian_matrix(SEED, csr.n, 300, 0, 3)
    Gr = S @ Om
    Hr = S.T @ Gr
    assert np.linalg.norm(g.cpu().numpy() - Gr) <= 1e-14 * np.linalg.norm(Gr)
    assert np.linalg.norm(h.cpu().numpy() - Hr) <= 1e-14 * np.linalg.norm(Hr)


@pytest.mark.parametrize("algo", ["fp", "ei"])
def test_csr_parity(qb, algo):
    wl = W.C3_SMALL
    csr = wl.make()
    rp, ci, va = _csr_dev(csr)
    S = csr.to_scipy()
    _log(f"csr {algo} {wl.name}")
    if algo == "fp":
        res = qb.qb_fp_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, SEED)
        ora = R.randqb_fp(S, wl.tol, wl.b, SEED)
    else:
        res = qb.qb_ei_csr(csr.m, csr.n, rp, ci, va, wl.tol, wl.b, SEED)
        ora = R.randqb_ei(S, wl.tol, wl.b, SEED)
    _compare(res, ora, S, f"csr {algo}")


# ---------------------------------------------------------------- full-size benchmark workload


def test_benchmark_workload_full_size(qb):
    """The 20000 x 15000 workload in the launch configuration bench.py times (same seed,
    l_max = min(m, n), l~ = 50 b), compared with the oracle on the same bits of A."""
    wl = W.C2
    seed = W.SEED_OMEGA | 2
    A = wl.make(device="cuda")
    torch.cuda.synchronize()
    An = A.cpu().numpy()
    for algo, kw in (("fp", {}), ("fp", {"l_tilde": -1}), ("ei", {})):
        _log(f"full-size {algo} {kw} {wl.name}")
        f = qb.qb_fp_dense if algo == "fp" else qb.qb_ei_dense
        g = R.randqb_fp if algo == "fp" else R.randqb_ei
        res = f(A, wl.tol, wl.b, seed, l_max=min(wl.m, wl.n), **kw)
        ora = g(An, wl.tol, wl.b, seed, **kw)
        _compare(res, ora, An, f"full-size {algo}")
        assert res.rank >= R.svd_optimal_rank(wl.sigma(), wl.tol) - 1
