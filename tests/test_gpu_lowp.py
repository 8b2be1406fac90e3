"""GPU parity of the precision form (bfloat16 A_q, bfloat16 sketch products with binary32
accumulation, binary64 block loop) against the oracle's precision form.

Tolerances, derived from the arithmetic (u16 = 2^-8 is the unit roundoff of bfloat16,
u32 = 2^-24 that of binary32, K the inner dimension):

* ||A_q||^2 and Omega_q: as the binary64 path (squares of bfloat16 values are exact;
  Omega_q is one rounding of the bit-specified Omega): 1e-14 relative, bit-exact.
* G_q = bf16(fl32(A_q Omega_q)): the binary32 sum deviates from the exact one by at most
  gamma_K S with S = |A_q| |Omega_q| and gamma_K = K u32 / (1 - K u32); the final rounding
  adds at most u16 of the binary32 value, so
  |G_gpu - A_q Omega_q| <= u16 (|A_q Omega_q| + gamma_K S) + gamma_K S entrywise.  Against
  the oracle's G_q = bf16(A_q Omega_q) the two differ only where the binary32 error moves
  the value across a bfloat16 rounding boundary (below 2% of the entries here), by at
  most 2 u16 |A_q Omega_q| + (1 + u16) gamma_K S (more than one bfloat16 spacing where
  cancellation makes the entry small next to S).
* H = fl32(A_q^T G_q): |H_gpu - A_q^T G_gpu| <= gamma_K |A_q|^T |G_gpu| entrywise (a
  property of the GPU's own operands, checked in binary64).
* The method: the block loop sees H with the binary32 error above, amplified by
  R_i^{-T} (Remark 4.1) into B, so ||B - Q^T A_q||_F <= u32 sqrt(K) sigma_1^2 / s_min
  (random-walk growth of the accumulation error; s_min the smallest kept row norm of
  B).  E then differs from ||A_q - QB||^2 by -2 <Q^T A_q, dB> - 2 ||dB||^2, a sum of
  random-signed products: required below 5% of eps^2.  The true error against the
  binary64 A must meet tol, and the rank may differ from the oracle's by one plus 2%
  (the rounding flips of G_q rotate the trailing directions of each block).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lowp as OL
from oracle import randqb as R
from oracle import rng as ORNG

pytestmark = pytest.mark.gpu

SEED = W.SEED_OMEGA | 4
U16 = 2.0 ** -8
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_09402_amd as q
    q.lib()
    return q


def _log(msg):
    print(msg, flush=True)


def _gamma(K):
    return K * U32 / (1.0 - K * U32)


def _bf16_pair(m, n, kind, seed, device="cpu"):
    A64 = W.lowrank_dense(m, n, W.sigma_law(kind, min(m, n)), seed, device=device)
    return A64, W.to_bf16(A64)


@pytest.mark.parametrize("m,n", [(1000, 800), (1, 1), (3, 7001), (4097, 33)])
def test_sumsq_bf16(qb, m, n):
    _log(f"sumsq bf16 {m}x{n}")
    Aq = W.gaussian_dense(m, n, 6).to(torch.bfloat16)
    got = qb.qb_sumsq_dense(Aq.cuda())
    want = R.sumsq(Aq.double().numpy())
    assert abs(got - want) <= 1e-14 * want


@pytest.mark.parametrize("m,n,l,col0,pad", [
    (700, 530, 200, 64, 0),      # ragged M, N and K tiles; K = 530 not a multiple of 8
    (1024, 768, 256, 0, 8),      # 16-byte aligned rows (vector loads), row stride 776
    (129, 4099, 33, 5, 0),       # short and wide, odd widths
    (4096, 256, 128, 128, 0),    # tall and narrow
    (16300, 1000, 1000, 64, 0),  # 256 tiles of 256 x 256: the LDS-DMA kernel, ragged M, N, K
    (2048, 16384, 1024, 0, 0),   # H with 256 tiles: A_q read in place by transposed LDS reads
    (2048, 16376, 1000, 64, 0),  # the same with ragged H rows (16376 = 8 x 2047) and columns
])
def test_sketch_lowp(qb, m, n, l, col0, pad):
    _log(f"sketch bf16 {m}x{n} l={l} col0={col0} pad={pad}")
    _, Aq = _bf16_pair(m, n + pad, "poly1.5", 11)
    Ad = Aq.cuda()[:, :n] if pad else Aq.cuda()
    om, g, h = qb.qb_sketch_lowp(Ad, SEED, col0, l)
    torch.cuda.synchronize()
    A = Aq.double().numpy()[:, :n]
    om, g, h = om.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy()
    # Omega_q bit-exact
    om_ref = OL.round_bf16(ORNG.gaussian_matrix(SEED, n, l, 0, col0))
    assert np.array_equal(om.view(np.int64), om_ref.view(np.int64))
    # G_q: bfloat16 values within the rigorous binary32 + rounding bound
    assert OL.is_bf16(g)
    exact = A @ om_ref
    S = np.abs(A) @ np.abs(om_ref)
    gam = _gamma(n)
    assert np.all(np.abs(g - exact) <= U16 * (np.abs(exact) + gam * S) + gam * S)
    # against the oracle's G_q = bf16(exact): equal except where the binary32 error moves
    # the value across a rounding boundary (a few percent of the entries); there
    # |g - g_ora| <= u16 |f| + gamma S + u16 |exact| with |f - exact| <= gamma S
    g_ora = OL.round_bf16(exact)
    diff = g != g_ora
    assert diff.mean() <= 0.02
    assert np.all(np.abs(g - g_ora) <= 2 * U16 * np.abs(exact) + (1 + U16) * gam * S)
    # H = A_q^T G_q with the GPU's own G_q
    hh = A.T @ g
    assert np.all(np.abs(h - hh) <= _gamma(m) * (np.abs(A).T @ np.abs(g)) + 1e-300)


def test_lowp_rejections(qb):
    Aq = torch.zeros((64, 48), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(qb.QBError) as e:
        qb.qb_ei_dense(Aq, 1e-2, 8, 1)
    assert e.value.status == qb.QB_ERR_UNSUPPORTED
    # the binary64-only sketch entry point refuses bfloat16 A
    with pytest.raises(qb.QBError) as e:
        qb.qb_sketch_dense(Aq, 1, 0, 8)
    assert e.value.status == qb.QB_ERR_UNSUPPORTED


def _check_method(res, ora, A64, Aq, tol, label):
    """Compare one GPU precision-form run with the oracle's and check its invariants."""
    nrm2 = ora.normA2
    eps2 = tol * tol * nrm2
    Q, B = res.Q, res.B
    Aqd = Aq.double()
    direct = float(torch.linalg.matrix_norm(Aqd - Q @ B) ** 2)
    true_rel = float(torch.linalg.matrix_norm(A64 - Q @ B) / torch.linalg.matrix_norm(A64))
    b_err = float(torch.linalg.matrix_norm(B - Q.T @ Aqd))
    orth = float(torch.linalg.matrix_norm(Q.T @ Q - torch.eye(res.rank, dtype=Q.dtype, device=Q.device),
                                          ord=float("inf")))
    rn = torch.linalg.vector_norm(B, dim=1)
    s1, smin = float(rn.max()), float(rn.min())
    K = max(Aq.shape)
    b_bound = U32 * np.sqrt(K) * s1 * s1 / smin
    _log(f"{label}: rank gpu {res.rank} ora {ora.rank}; E/eps2 gpu {res.E / eps2:.4f} "
         f"ora {ora.E / eps2:.4f}; direct/eps2 {direct / eps2:.4f}; true rel {true_rel:.4e}; "
         f"|B-Q^T A_q| {b_err:.3e} (bound {b_bound:.3e}); orth {orth:.2e}")
    assert abs(res.normA2 - nrm2) <= 1e-14 * nrm2
    assert res.status in (0, 2) and ora.status in (0, 2)
    assert abs(res.rank - ora.rank) <= 1 + 0.02 * ora.rank
    assert res.E < eps2
    assert b_err <= b_bound
    assert abs(direct - res.E) <= 0.05 * eps2
    assert orth <= 1e-12
    assert true_rel <= tol


@pytest.mark.parametrize("m,n,b,tol,l_tilde,kind", [
    (1000, 700, 32, 1e-2, 0, "poly1.5"),
    (1000, 700, 32, 1e-2, -1, "poly1.5"),
    (777, 1203, 20, 3e-3, 60, "exp20"),     # several chunks
])
def test_fp_bf16_vs_oracle(qb, m, n, b, tol, l_tilde, kind):
    _log(f"fp bf16 {m}x{n} b={b} tol={tol} l_tilde={l_tilde} {kind}")
    A64, Aq = _bf16_pair(m, n, kind, 21)
    ora = R.randqb_fp(Aq.double().numpy(), tol, b, SEED, l_tilde=l_tilde, precision="bf16")
    res = qb.qb_fp_dense(Aq.cuda(), tol, b, SEED, l_tilde=l_tilde)
    _check_method(res, ora, A64.cuda(), Aq.cuda(), tol, f"{m}x{n}")
    assert res.passes == 2 * res.chunks


def test_fp_bf16_parity_instance(qb):
    """The 4096 x 4096 parity instance of the precision-form workload (same sigma law as
    the 32768 x 32768 benchmark matrix), paper chunk rule and adaptive schedule."""
    wl = W.C4_SMALL
    A64 = wl.make()
    Aq = W.to_bf16(A64)
    An = Aq.double().numpy()
    for lt in (0, -1):
        _log(f"parity instance l_tilde={lt}")
        ora = R.randqb_fp(An, wl.tol, wl.b, SEED, l_tilde=lt, precision="bf16")
        res = qb.qb_fp_dense(Aq.cuda(), wl.tol, wl.b, SEED, l_tilde=lt)
        _check_method(res, ora, A64.cuda(), Aq.cuda(), wl.tol, f"{wl.name} lt={lt}")


def test_fp_bf16_reproducible(qb):
    _, Aq = _bf16_pair(900, 600, "poly1.5", 23)
    Ad = Aq.cuda()
    r1 = qb.qb_fp_dense(Ad, 1e-2, 32, SEED, l_tilde=-1)
    B1 = r1.B.clone()
    r2 = qb.qb_fp_dense(Ad, 1e-2, 32, SEED, l_tilde=-1)
    assert r1.rank == r2.rank and r1.E == r2.E
    assert torch.equal(B1, r2.B)


def test_fp_bf16_full_size(qb):
    """The 32768 x 32768 precision-form workload at full size, as the benchmark runs it:
    sampled rows of Omega_q and G_q against the oracle (row by row), and the properties
    that hold at any size for the full run."""
    wl = W.C4
    dev = torch.device("cuda")
    _log("generating the 32768 x 32768 matrix on the GPU")
    A64 = wl.make(device=dev)
    Aq = W.to_bf16(A64)
    torch.cuda.synchronize()
    # sweep of the first adaptive chunk (8 b columns): sampled rows
    l = 8 * wl.b
    om, g, h = qb.qb_sketch_lowp(Aq, SEED, 0, l)
    torch.cuda.synchronize()
    rows = np.array([0, 1, 4095, 12345, 20000, 32767])
    om_rows = om[torch.as_tensor(rows, device=dev)].cpu().numpy()
    for i, r in enumerate(rows):
        ref = OL.round_bf16(ORNG.gaussian_matrix(SEED, 1, l, int(r), 0))
        assert np.array_equal(om_rows[i:i + 1].view(np.int64), ref.view(np.int64))
    omq = om.cpu().numpy()
    gam = _gamma(wl.n)
    for r in rows:
        a = Aq[int(r)].double().cpu().numpy()
        exact = a @ omq
        S = np.abs(a) @ np.abs(omq)
        gg = g[int(r)].cpu().numpy()
        assert np.all(np.abs(gg - exact) <= U16 * (np.abs(exact) + gam * S) + gam * S)
    del om, g, h
    res = qb.qb_fp_dense(Aq, wl.tol, wl.b, SEED, l_tilde=-1)
    nrm2 = R.sumsq(Aq.double().cpu().numpy())   # oracle's sum of squares of A_q
    Q, B = res.Q, res.B
    eps2 = wl.tol ** 2 * nrm2
    direct = float(torch.linalg.matrix_norm(Aq.double() - Q @ B) ** 2)
    true_rel = float(torch.linalg.matrix_norm(A64 - Q @ B) / torch.linalg.matrix_norm(A64))
    s = wl.sigma()
    opt = R.svd_optimal_rank(s, wl.tol)
    _log(f"full size: rank {res.rank} (svd-optimal of A {opt}); E/eps2 {res.E / eps2:.4f}; "
         f"direct/eps2 {direct / eps2:.4f}; true rel {true_rel:.4e}; ms {res.ms}")
    assert abs(res.normA2 - nrm2) <= 1e-13 * nrm2
    assert res.status == 0 and res.E < eps2
    assert abs(direct - res.E) <= 0.05 * eps2
    assert true_rel <= wl.tol
    assert opt - 2 <= res.rank <= int(1.3 * opt) + wl.b


# ------------------------------------------------------------------ e4m3 storage
#
# A stored in OCP e4m3fn with a power-of-two scale per row: A_q(i, j) = 2^e_i e4m3(...),
# every value a bfloat16 value.  The G product runs on 8-bit operands: Omega_q is the e4m3
# rounding of 2^5 Omega divided by 2^5 (the oracle's precision form "e4m3"), and each
# product of two e4m3 values is exact in binary32, so G_q = bf16(fl32(A_q Omega_q)) obeys
# the bounds above with Omega_q in place of the bfloat16 one; H is the bfloat16 form's.
# Shapes whose K is a multiple of 64 (with 16-byte rows) take the 8-bit matrix cores, the
# others the bfloat16 ones on the same e4m3 values.  The storage error (2.6e-2 of ||A|| for
# these matrices) lies above tol 1e-2; the method is run at tol 5e-2, where the true error
# against the binary64 matrix still meets tol.


def _omega_e4m3(seed, n, l, col0):
    return OL.round_e4m3(ORNG.gaussian_matrix(seed, n, l, 0, col0) * R.OMEGA_E4M3_SCALE) / R.OMEGA_E4M3_SCALE


def _fp8_pair(m, n, kind, seed):
    A64 = W.lowrank_dense(m, n, W.sigma_law(kind, min(m, n)), seed)
    A8, e, Aq = W.to_e4m3_rows(A64)
    return A64, A8, e, Aq


@pytest.mark.parametrize("m,n", [(1000, 800), (3, 7001), (4097, 33)])
def test_sumsq_fp8(qb, m, n):
    _log(f"sumsq e4m3 {m}x{n}")
    _, A8, e, Aq = _fp8_pair(m, n, "poly1.5", 31)
    got = qb.qb_sumsq_dense(A8.cuda(), row_exp=e.cuda())
    want = R.sumsq(Aq.numpy())
    assert abs(got - want) <= 1e-14 * want


@pytest.mark.parametrize("m,n,l,col0", [
    (700, 530, 200, 64),       # K = 530: G on the bfloat16 matrix cores (e4m3 Omega_q values)
    (1024, 768, 256, 0),       # G on 8-bit matrix cores, a few 256 x 256 tiles
    (4096, 256, 128, 128),     # 8-bit G, four K tiles of 64
    (300, 128, 33, 5),         # 8-bit G, one partial tile in each direction
    (2048, 16384, 1024, 0),    # H with 256 tiles: e4m3 A read in place by transposed byte reads
    (2048, 16368, 1000, 64),   # the same with ragged H rows (16368 = 16 x 1023) and columns
    (2048, 16380, 1000, 64),   # H rows not a multiple of 16: the register-staged kernel
    (16384, 2048, 1024, 0),    # G with 256 tiles on 8-bit matrix cores, row scales in the epilogue
    (16300, 2048, 1000, 64),   # the same with ragged G rows and columns
])
def test_sketch_fp8(qb, m, n, l, col0):
    _log(f"sketch e4m3 {m}x{n} l={l} col0={col0}")
    _, A8, e, Aq = _fp8_pair(m, n, "poly1.5", 32)
    om, g, h = qb.qb_sketch_lowp(A8.cuda(), SEED, col0, l, row_exp=e.cuda())
    torch.cuda.synchronize()
    A = Aq.numpy()
    om, g, h = om.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy()
    om_ref = _omega_e4m3(SEED, n, l, col0)
    assert np.array_equal(om.view(np.int64), om_ref.view(np.int64))
    assert OL.is_bf16(g)
    exact = A @ om_ref
    S = np.abs(A) @ np.abs(om_ref)
    gam = _gamma(n)
    assert np.all(np.abs(g - exact) <= U16 * (np.abs(exact) + gam * S) + gam * S)
    g_ora = OL.round_bf16(exact)
    assert (g != g_ora).mean() <= 0.02
    hh = A.T @ g
    assert np.all(np.abs(h - hh) <= _gamma(m) * (np.abs(A).T @ np.abs(g)) + 1e-300)


@pytest.mark.parametrize("m,n,b,l_tilde", [(1000, 700, 32, -1), (4096, 4096, 128, -1), (777, 1203, 20, 60)])
def test_fp_fp8_vs_oracle(qb, m, n, b, l_tilde):
    tol = 5e-2
    _log(f"fp e4m3 {m}x{n} b={b} tol={tol} l_tilde={l_tilde}")
    A64, A8, e, Aq = _fp8_pair(m, n, "poly1.5", 33)
    ora = R.randqb_fp(Aq.numpy(), tol, b, SEED, l_tilde=l_tilde, precision="e4m3")
    res = qb.qb_fp_dense(A8.cuda(), tol, b, SEED, l_tilde=l_tilde, row_exp=e.cuda())
    _check_method(res, ora, A64.cuda(), Aq.cuda(), tol, f"e4m3 {m}x{n}")


def test_fp_fp8_full_size(qb):
    """The 32768 x 32768 e4m3 run of the benchmark (tol 5e-2, adaptive schedule) at full
    size: sampled rows of Omega_q and G_q of the first chunk against the oracle's formulas
    (8-bit G product), then the properties that hold at any size for the whole run."""
    wl = W.C4
    tol = 5e-2
    dev = torch.device("cuda")
    _log("generating the 32768 x 32768 matrix on the GPU")
    A64 = wl.make(device=dev)
    A8, e, Aq = W.to_e4m3_rows(A64)
    torch.cuda.synchronize()
    l = 8 * wl.b
    om, g, h = qb.qb_sketch_lowp(A8, SEED, 0, l, row_exp=e)
    torch.cuda.synchronize()
    rows = np.array([0, 1, 4095, 12345, 20000, 32767])
    om_rows = om[torch.as_tensor(rows, device=dev)].cpu().numpy()
    for i, r in enumerate(rows):
        ref = OL.round_e4m3(ORNG.gaussian_matrix(SEED, 1, l, int(r), 0) * R.OMEGA_E4M3_SCALE) / R.OMEGA_E4M3_SCALE
        assert np.array_equal(om_rows[i:i + 1].view(np.int64), ref.view(np.int64))
    omq = om.cpu().numpy()
    gam = _gamma(wl.n)
    for r in rows:
        a = Aq[int(r)].cpu().numpy()
        exact = a @ omq
        S = np.abs(a) @ np.abs(omq)
        gg = g[int(r)].cpu().numpy()
        assert OL.is_bf16(gg)
        assert np.all(np.abs(gg - exact) <= U16 * (np.abs(exact) + gam * S) + gam * S)
    del om, g, h
    res = qb.qb_fp_dense(A8, tol, wl.b, SEED, l_tilde=-1, row_exp=e)
    nrm2 = R.sumsq(Aq.cpu().numpy())
    Q, B = res.Q, res.B
    eps2 = tol ** 2 * nrm2
    direct = float(torch.linalg.matrix_norm(Aq - Q @ B) ** 2)
    true_rel = float(torch.linalg.matrix_norm(A64 - Q @ B) / torch.linalg.matrix_norm(A64))
    orth = float(torch.linalg.matrix_norm(Q.T @ Q - torch.eye(res.rank, dtype=Q.dtype, device=dev),
                                          ord=float("inf")))
    opt = R.svd_optimal_rank(wl.sigma(), tol)
    _log(f"full size e4m3: rank {res.rank} (svd-optimal of A {opt}); E/eps2 {res.E / eps2:.4f}; "
         f"direct/eps2 {direct / eps2:.4f}; true rel {true_rel:.4e}; orth {orth:.2e}; ms {res.ms}")
    assert abs(res.normA2 - nrm2) <= 1e-13 * nrm2
    assert res.status == 0 and res.E < eps2
    assert abs(direct - res.E) <= 0.05 * eps2
    assert orth <= 1e-12
    assert true_rel <= tol
    assert opt - 2 <= res.rank <= int(1.3 * opt) + wl.b
