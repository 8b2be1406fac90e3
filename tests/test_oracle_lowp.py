"""Pins of the oracle's precision form: the bfloat16 rounding and randQB_FP on a
bfloat16-stored matrix (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import lowp
from oracle import randqb as R
import workloads as W


# ------------------------------------------------------------------ rounding


def test_round_bf16_matches_binary32_to_bf16_conversion():
    # for binary32 inputs a single RNE step to bfloat16 is what torch's float32 ->
    # bfloat16 conversion does
    g = np.random.default_rng(7)
    x = np.concatenate([
        g.standard_normal(20000) * np.exp(g.uniform(-80, 80, 20000)),
        g.standard_normal(2000) * 1e-39,                   # binary32/bf16 subnormals
        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38]),
    ]).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    got = lowp.round_bf16(x)
    assert np.array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_round_bf16_ties_and_single_rounding():
    one = 1.0
    ulp = 2.0 ** -7                                   # spacing of bf16 in [1, 2)
    cases = {
        one + ulp / 2: one,                           # tie -> even (1.0)
        one + 3 * ulp / 2: one + 2 * ulp,             # tie -> even (1 + 2 ulp)
        one + ulp / 2 + 2.0 ** -40: one + ulp,        # just above the tie: up
        one + ulp / 2 - 2.0 ** -40: one,              # just below the tie: down
        -(one + ulp / 2 + 2.0 ** -40): -(one + ulp),
        2.0 - ulp / 4: 2.0,                           # carry into the exponent
        lowp.BF16_MAX: lowp.BF16_MAX,
        lowp.BF16_MAX + 2.0 ** 119: np.inf,           # midpoint to 2^128: tie to even = inf
        lowp.BF16_MAX + 2.0 ** 118: lowp.BF16_MAX,
        2.0 ** -133: 2.0 ** -133,                     # smallest subnormal
        2.0 ** -134: 0.0,                             # half of it: tie to even zero
        3 * 2.0 ** -134: 2.0 ** -132,                 # tie between 1 and 2 quanta -> 2
        2.0 ** -126 - 2.0 ** -140: 2.0 ** -126,       # rounds up into the normal range
    }
    for x, want in cases.items():
        got = float(lowp.round_bf16(np.array([x]))[0])
        assert got == want, (x, got, want)
    # a value that a rounding through binary32 first would send to 1.0
    x = one + ulp / 2 + 2.0 ** -40
    assert float(np.float32(x)) == one + ulp / 2     # binary32 rounds it onto the tie
    assert float(lowp.round_bf16(np.array([x]))[0]) == one + ulp


def test_round_bf16_is_nearest_by_enumeration():
    # enumerate every bf16 value in [2^-3, 2^3) and check that the rounding of random
    # points picks the nearest one (ties: even significand)
    vals = []
    for e in range(-3, 3):
        for mnt in range(128):
            vals.append((1.0 + mnt / 128.0) * 2.0 ** e)
    vals.append(8.0)
    vals = np.array(vals)
    g = np.random.default_rng(3)
    x = g.uniform(0.125, 7.99, 5000)
    got = lowp.round_bf16(x)
    idx = np.searchsorted(vals, x)
    lo, hi = vals[idx - 1], vals[idx]
    nearest = np.where(x - lo < hi - x, lo, hi)
    assert np.array_equal(got, nearest)
    assert lowp.is_bf16(got)
    assert not lowp.is_bf16(x)


def test_round_e4m3_matches_binary32_to_e4m3_conversion():
    # for binary32 inputs within the format's range a single RNE step to e4m3 is what
    # torch's float32 -> float8_e4m3fn conversion does
    g = np.random.default_rng(11)
    x = np.concatenate([
        g.standard_normal(50000) * np.exp(g.uniform(-14, 6, 50000)),
        g.uniform(-448.0, 448.0, 2000),
        g.uniform(-2.0 ** -6, 2.0 ** -6, 2000),                  # subnormals
        np.array([0.0, -0.0, 448.0, -448.0, 2.0 ** -9, -(2.0 ** -6)]),
    ]).astype(np.float32).astype(np.float64)
    x = x[np.abs(x) <= 448.0]
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).double().numpy()
    got = lowp.round_e4m3(x)
    assert np.array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_round_e4m3_ties_subnormals_and_range():
    cases = {
        1.0 + 1 / 16: 1.0,                     # tie between 1 and 1.125 -> even (1.0)
        1.0 + 3 / 16: 1.25,                    # tie between 1.125 and 1.25 -> even (1.25)
        1.0 + 1 / 16 + 2.0 ** -30: 1.125,      # just above the tie
        -(1.0 + 1 / 16 + 2.0 ** -30): -1.125,
        2.0 - 1 / 32: 2.0,                     # carry into the exponent
        2.0 ** -10: 0.0,                       # half the smallest subnormal: tie -> 0
        3 * 2.0 ** -10: 2.0 ** -8,             # tie between 1 and 2 quanta -> 2 quanta
        2.0 ** -6 - 2.0 ** -11: 2.0 ** -6,     # rounds up into the normal range
        7 * 2.0 ** -9: 7 * 2.0 ** -9,          # largest subnormal
        448.0: 448.0,
        456.0: 448.0,                          # below the midpoint 464 to the next binade step
        464.0: 448.0,                          # the midpoint: tie to the even 448 (m = 6)
    }
    for x, want in cases.items():
        got = float(lowp.round_e4m3(np.array([x]))[0])
        assert got == want, (x, got, want)
    assert np.isnan(lowp.round_e4m3(np.array([465.0]))[0])      # beyond the format
    assert np.isnan(lowp.round_e4m3(np.array([np.inf]))[0])


def test_round_e4m3_is_nearest_by_enumeration():
    # every positive e4m3 value, from the definition of the format
    vals = [m * 2.0 ** -9 for m in range(1, 8)]
    for e in range(1, 16):
        for m in range(8):
            if e == 15 and m == 7:
                continue                        # NaN encoding
            vals.append(2.0 ** (e - 7) * (1 + m / 8))
    vals = np.array(sorted(vals))
    assert vals[-1] == 448.0 and len(vals) == 126
    g = np.random.default_rng(5)
    x = np.exp(g.uniform(np.log(2.0 ** -9), np.log(447.0), 20000))
    got = lowp.round_e4m3(x)
    idx = np.searchsorted(vals, x)
    lo = vals[np.maximum(idx - 1, 0)]
    hi = vals[np.minimum(idx, len(vals) - 1)]
    nearest = np.where(x - lo < hi - x, lo, hi)
    assert np.array_equal(got, nearest)
    assert lowp.is_e4m3(got) and lowp.is_bf16(got)         # e4m3 values are bfloat16 values
    assert not lowp.is_e4m3(x)


# ------------------------------------------------------------------ precision form


def _bf16_matrix(m, n, kind, seed):
    A64 = W.lowrank_dense(m, n, W.sigma_law(kind, min(m, n)), seed)
    Aq = W.to_bf16(A64).double().numpy()
    return A64.numpy(), Aq


@pytest.mark.parametrize("l_tilde", [0, -1, 64])
def test_precision_form_indicator_is_exact_for_stored_matrix(l_tilde):
    """Theorem 1 for A_q: with H = A_q^T G_q built from the same rounded G_q the loop
    uses, eq. (23) gives B = Q^T A_q, so E equals ||A_q - QB||^2 in binary64."""
    A64, Aq = _bf16_matrix(600, 500, "poly1.5", 101)
    res = R.randqb_fp(Aq, 1e-2, 32, W.SEED_OMEGA | 7, l_tilde=l_tilde, precision="bf16")
    assert res.status == R.QB_OK
    nrm2 = R.sumsq(Aq)
    assert abs(res.normA2 - nrm2) <= 1e-15 * nrm2
    direct = R.residual_sq(Aq, res.Q, res.B)
    assert abs(direct - res.E) <= 1e-10 * nrm2
    assert res.E < (1e-2) ** 2 * nrm2
    assert np.linalg.norm(res.B - res.Q.T @ Aq) <= 1e-12 * np.sqrt(nrm2)
    assert R.orth_loss_inf(res.Q) <= 1e-12


def test_precision_form_rank_and_true_error_bounds():
    A64, Aq = _bf16_matrix(600, 500, "poly1.5", 102)
    tol = 1e-2
    res = R.randqb_fp(Aq, tol, 32, W.SEED_OMEGA | 8, precision="bf16")
    s = np.linalg.svd(Aq, compute_uv=False)
    # rank bracketed below by the SVD-optimal rank of the stored matrix
    assert res.rank >= R.svd_optimal_rank(s, tol)
    # ||A - QB|| <= ||A_q - QB|| + ||(I - QQ^T)(A - A_q)||  <= sqrt(E) + ||A - A_q||
    noise = np.linalg.norm(A64 - Aq)
    true = np.linalg.norm(A64 - res.Q @ res.B)
    assert true <= np.sqrt(max(res.E, 0.0)) + noise + 1e-12 * np.linalg.norm(A64)
    # bfloat16 storage error of this matrix is far below tol (2^-9 relative per entry)
    assert noise <= 2.0 ** -8 * np.linalg.norm(A64)


def test_precision_form_operands_are_rounded():
    """The sketch operands of the precision form are the bf16 roundings: with a
    bf16-valued A, one block of the precision form equals the binary64 method run on
    the rounded Omega (a fixed-rank check through randqb_fp_fixed)."""
    _, Aq = _bf16_matrix(300, 200, "exp7", 103)
    b = 16
    seed = W.SEED_OMEGA | 9
    res = R.randqb_fp(Aq, 1e-12, b, seed, l_max=b, l_tilde=b, precision="bf16")
    Om_q = lowp.round_bf16(R.omega(seed, 200, 0, b))
    G_q = lowp.round_bf16(Aq @ Om_q)
    Q, _ = R.qr_pos(G_q)
    assert res.rank == b
    assert np.allclose(np.abs(res.Q.T @ Q), np.eye(b), atol=1e-10)
    assert np.allclose(res.B, res.Q.T @ Aq, atol=1e-12)


def test_precision_form_rejects_unrounded_input():
    A64, _ = _bf16_matrix(100, 80, "poly2", 104)
    with pytest.raises(ValueError):
        R.randqb_fp(A64, 1e-2, 8, 1, precision="bf16")


# ------------------------------------------------------------------ e4m3 form (8-bit G product)


def _e4m3_matrix(m, n, kind, seed):
    A64 = W.lowrank_dense(m, n, W.sigma_law(kind, min(m, n)), seed)
    _, _, Aq = W.to_e4m3_rows(A64)
    return A64.numpy(), Aq.numpy()


def test_e4m3_form_indicator_is_exact_for_stored_matrix():
    """Theorem 1 for the e4m3-stored A_q with Omega_q rounded to e4m3: eq. (23) with
    H = A_q^T G_q still gives B = Q^T A_q, so E equals ||A_q - QB||^2."""
    _, Aq = _e4m3_matrix(500, 400, "poly1.5", 111)
    assert lowp.is_bf16(Aq)
    res = R.randqb_fp(Aq, 5e-2, 32, W.SEED_OMEGA | 17, precision="e4m3")
    assert res.status == R.QB_OK
    nrm2 = R.sumsq(Aq)
    assert abs(R.residual_sq(Aq, res.Q, res.B) - res.E) <= 1e-10 * nrm2
    assert res.E < (5e-2) ** 2 * nrm2
    assert np.linalg.norm(res.B - res.Q.T @ Aq) <= 1e-12 * np.sqrt(nrm2)
    assert R.orth_loss_inf(res.Q) <= 1e-12


def test_e4m3_form_omega_is_the_scaled_e4m3_rounding():
    """One block of the e4m3 form spans qf(bf16(A_q Omega_q)) with Omega_q =
    e4m3(2^5 Omega) / 2^5 -- and not the bfloat16 form's Omega_q."""
    _, Aq = _e4m3_matrix(300, 200, "exp7", 112)
    b, seed = 16, W.SEED_OMEGA | 18
    res = R.randqb_fp(Aq, 1e-12, b, seed, l_max=b, l_tilde=b, precision="e4m3")
    Om = R.omega(seed, 200, 0, b)
    Om_q = lowp.round_e4m3(Om * 32.0) / 32.0
    assert lowp.is_e4m3(Om_q * 32.0) and np.all(np.abs(Om * 32.0) < lowp.E4M3_MAX)
    Q, _ = R.qr_pos(lowp.round_bf16(Aq @ Om_q))
    assert np.allclose(np.abs(res.Q.T @ Q), np.eye(b), atol=1e-10)
    Q_bf, _ = R.qr_pos(lowp.round_bf16(Aq @ lowp.round_bf16(Om)))
    assert not np.allclose(np.abs(res.Q.T @ Q_bf), np.eye(b), atol=1e-6)


def test_e4m3_form_generator_range():
    """2^5 Omega fits the e4m3 range for every value the generator can produce: the
    Box-Muller radius sqrt(-2 ln u1) with u1 >= 2^-53 is below 8.6."""
    r_max = np.sqrt(-2.0 * np.log(2.0 ** -53))
    assert r_max < 8.6 and 32.0 * r_max < lowp.E4M3_MAX
    Om = R.omega(W.SEED_OMEGA | 19, 4096, 0, 64)
    assert np.abs(Om).max() < r_max
