"""Reference for the differentiation form (test infrastructure only).

The fixed-rank randQB_FP of Algorithm 3 with the re-orthogonalisation of Algorithm 4 (P = 0, no
stopping) computes, in exact arithmetic, Q = qf(A Omega) with diag(R) > 0 and B = Q^T A
for the fixed Gaussian Omega (the remark after eq. (23): all block variants give the same
Q and B).  This module writes that map in plain float64 torch on the CPU, so that
torch's own autograd (thin QR through torch.linalg.qr) gives the reference gradient of a
loss of (Q, B); it shares nothing with the GPU adjoint.

Loss used by the tests and the benchmark (not from the paper):
    L(A) = ||A - Q B||_F^2 + S_delta(B),   S_delta(B) = sum_j sqrt(sigma_j(B)^2 + delta^2),
a smoothed nuclear norm of B (delta = 1e-3); its gradient in B is
(B B^T + delta^2 I)^{-1/2} B.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rng

DELTA = 1e-3


def omega_fixed(seed: int, n: int, k: int, dtype=np.float64) -> np.ndarray:
    """The fixed Omega (n x k, stream 0, batch 0) rounded to the working precision."""
    om = rng.gaussian_matrix(seed, n, k, 0, 0, stream=0, batch=0)
    return om.astype(dtype).astype(np.float64)


def qb_fixed_torch(A: torch.Tensor, Om: torch.Tensor):
    """Q = qf(A Omega) with diag(R) > 0 and B = Q^T A (float64 torch, autograd-able)."""
    Q, R = torch.linalg.qr(A @ Om, mode="reduced")
    d = torch.sign(torch.diagonal(R, dim1=-2, dim2=-1))
    d = torch.where(d == 0, torch.ones_like(d), d)
    Q = Q * d.unsqueeze(-2)
    B = Q.transpose(-1, -2) @ A
    return Q, B


def surrogate(B: torch.Tensor, delta: float = DELTA) -> torch.Tensor:
    """S_delta(B) = sum_j sqrt(sigma_j^2 + delta^2), from the eigenvalues of B B^T."""
    lam = torch.linalg.eigvalsh(B @ B.transpose(-1, -2))
    return torch.sqrt(torch.clamp(lam, min=0.0) + delta * delta).sum()


def loss(A: torch.Tensor, Q: torch.Tensor, B: torch.Tensor, delta: float = DELTA) -> torch.Tensor:
    return ((A - Q @ B) ** 2).sum() + surrogate(B, delta)


def grad_reference(A: np.ndarray, Om: np.ndarray, delta: float = DELTA):
    """dL/dA by float64 autograd through qb_fixed_torch; returns (L, dL/dA)."""
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    Q, B = qb_fixed_torch(At, torch.tensor(Om, dtype=torch.float64))
    L = loss(At, Q, B, delta)
    L.backward()
    return L.item(), At.grad.numpy()


def vjp_reference(A: np.ndarray, Om: np.ndarray, dQ: np.ndarray, dB: np.ndarray) -> np.ndarray:
    """dL/dA for L = <dQ, Q> + <dB, B> (the adjoint of A -> (Q, B) applied to (dQ, dB))."""
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    Q, B = qb_fixed_torch(At, torch.tensor(Om, dtype=torch.float64))
    L = (Q * torch.tensor(dQ)).sum() + (B * torch.tensor(dB)).sum()
    L.backward()
    return At.grad.numpy()


def surrogate_grad_closed_form(B: np.ndarray, delta: float = DELTA) -> np.ndarray:
    """(B B^T + delta^2 I)^{-1/2} B from the eigendecomposition of B B^T."""
    lam, V = np.linalg.eigh(B @ B.T)
    s = 1.0 / np.sqrt(np.maximum(lam, 0.0) + delta * delta)
    return (V * s[None, :]) @ V.T @ B
