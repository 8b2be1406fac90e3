"""Pins of the differentiation-form reference (CPU only): finite differences, the
equivalence of the reference map with the oracle's fixed-rank randQB_FP, and the closed
form of the surrogate's gradient."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import diff as D
from oracle import randqb as R

SEED = W.SEED_OMEGA | 5


def _matrix(m, n, kind, seed):
    return W.lowrank_dense(m, n, W.sigma_law(kind, min(m, n)), seed).numpy()


def _loss_np(A, Om, delta=D.DELTA):
    with torch.no_grad():
        At = torch.tensor(A)
        Q, B = D.qb_fixed_torch(At, torch.tensor(Om))
        return float(D.loss(At, Q, B, delta))


@pytest.mark.parametrize("kind", ["exp40", "poly1.5"])
def test_reference_gradient_matches_central_differences(kind):
    # 96 x 64, k = 32: central differences in binary64 with h = 1e-6
    A = _matrix(96, 64, kind, 301)
    Om = D.omega_fixed(SEED, 64, 32)
    L, g = D.grad_reference(A, Om)
    rs = np.random.default_rng(5)
    h = 1e-6
    for _ in range(4):
        E = rs.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (_loss_np(A + h * E, Om) - _loss_np(A - h * E, Om)) / (2 * h)
        an = float(np.sum(g * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.linalg.norm(g))


def test_reference_vjp_matches_central_differences():
    A = _matrix(96, 64, "exp40", 302)
    Om = D.omega_fixed(SEED, 64, 32)
    rs = np.random.default_rng(6)
    dQ = rs.standard_normal((96, 32))
    dB = rs.standard_normal((32, 64))
    g = D.vjp_reference(A, Om, dQ, dB)

    def f(X):
        with torch.no_grad():
            Q, B = D.qb_fixed_torch(torch.tensor(X), torch.tensor(Om))
            return float((Q * torch.tensor(dQ)).sum() + (B * torch.tensor(dB)).sum())

    h = 1e-6
    for _ in range(3):
        E = rs.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (f(A + h * E) - f(A - h * E)) / (2 * h)
        an = float(np.sum(g * E))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.linalg.norm(g))


@pytest.mark.parametrize("m,n,k,b", [(96, 64, 32, 16), (300, 200, 48, 16), (257, 190, 60, 20)])
def test_reference_map_is_fixed_rank_fp(m, n, k, b):
    """The remark after eq. (23): the blocked, re-orthogonalised FP recursion gives the same
    Q and B as qf(A Omega), Q^T A."""
    A = _matrix(m, n, "exp40", 303)
    Om = D.omega_fixed(SEED, n, k)
    Qf, Bf = R.randqb_fp_fixed(A, Om, b)
    with torch.no_grad():
        Qt, Bt = D.qb_fixed_torch(torch.tensor(A), torch.tensor(Om))
    assert np.allclose(Qf, Qt.numpy(), atol=1e-10)
    assert np.allclose(Bf, Bt.numpy(), atol=1e-10 * np.linalg.norm(A))


def test_surrogate_gradient_closed_form():
    rs = np.random.default_rng(8)
    B = rs.standard_normal((12, 40)) * np.exp(-np.arange(12) / 3.0)[:, None]
    Bt = torch.tensor(B, requires_grad=True)
    D.surrogate(Bt).backward()
    assert np.allclose(Bt.grad.numpy(), D.surrogate_grad_closed_form(B), atol=1e-10)
    # sum of sqrt(sigma^2 + delta^2) against an SVD
    s = np.linalg.svd(B, compute_uv=False)
    assert abs(float(D.surrogate(torch.tensor(B))) - np.sum(np.sqrt(s ** 2 + D.DELTA ** 2))) <= 1e-12


def test_omega_fixed_rounding():
    om64 = D.omega_fixed(SEED, 50, 8)
    om32 = D.omega_fixed(SEED, 50, 8, np.float32)
    assert np.array_equal(om32, om64.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(om32 - om64)) <= 2.0 ** -24 * np.max(np.abs(om64))
