"""FP64 CPU reference gradient of SPOD outputs with respect to the raw data.

TEST INFRASTRUCTURE ONLY (same rule as the forward oracle).

The paper does not differentiate SPOD.  This module re-expresses the forward
definition of Sec. 2.3 (mean removal, blocks of eq. (blocks), DFT of eq.
(blocks-ft), the weighted inner product and eigenproblem of eq.
(spod-discrete-snapshots), and the modes Phi_k = Qhat_k Psi_k Lambda_k^{-1/2})
with plain PyTorch CPU float64 operations, and lets PyTorch's autograd produce
the gradient.  The eigenproblem uses torch.linalg.eigh (LAPACK) as a library
step; the readings R1-R10 of the forward oracle apply unchanged.

Complex gradients follow PyTorch's convention: for a real loss E and a
complex value z, the gradient is dE/dRe(z) + i dE/dIm(z).  The phase
convention R9 is applied with a detached pivot index, so a loss that does
not depend on eigenvector phases (every loss used here) gets the gradient
of the gauge-invariant problem.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .spod_oracle import block_count, dft_matrix, hann_periodic

__all__ = ["spod_torch", "reference_gradient"]


def spod_torch(q: torch.Tensor, nfft: int, noverlap: int, window=None, weights=None,
               n_modes: int = 5, eps: float = 1e-12, bins=None):
    """Differentiable FP64 SPOD on the CPU.  Returns (lam [K, L], phi [K, n, M])."""
    assert q.dtype == torch.float64 and q.device.type == "cpu"
    m_rows, nt = q.shape
    if window is None:
        window = hann_periodic(nfft)
    w = torch.as_tensor(np.asarray(window, np.float64))
    if weights is None:
        weights = np.full(m_rows, 1.0 / m_rows)
    W = torch.as_tensor(np.asarray(weights, np.float64))
    nb = block_count(nt, nfft, noverlap)
    s = nfft - noverlap
    kappa = 1.0 / math.sqrt((nb - 1) * float(torch.sum(w * w)))

    x = q - q.mean(dim=1, keepdim=True)                              # mean removal
    blk = x.unfold(1, nfft, s)[:, :nb, :] * w                          # [M, L, N_f]
    F = torch.as_tensor(dft_matrix(nfft, bins))                       # [N_f, K]
    qhat = kappa * torch.einsum("mln,nk->klm", blk.to(torch.complex128), F)
    G = torch.matmul(torch.conj(qhat) * W, qhat.transpose(1, 2))     # [K, L, L]
    G = 0.5 * (G + G.conj().transpose(1, 2))
    lam, V = torch.linalg.eigh(G)                                     # ascending
    lam = torch.flip(lam, dims=[-1])
    V = torch.flip(V, dims=[-1])
    piv = torch.argmax(V.detach().abs(), dim=1, keepdim=True)         # [K, 1, L]
    pv = torch.gather(V, 1, piv)
    V = V * (torch.conj(pv) / pv.abs())
    n_use = min(n_modes, nb)
    lam_n = lam[:, :n_use]
    valid = ((lam[:, :1] > 0) & (lam_n > eps * lam[:, :1])).detach()
    scale = torch.where(valid, torch.rsqrt(torch.where(valid, lam_n, torch.ones_like(lam_n))),
                        torch.zeros_like(lam_n))
    coef = V[:, :, :n_use] * scale[:, None, :].to(torch.complex128)
    phi = torch.matmul(coef.transpose(1, 2), qhat)                     # [K, n, M]
    return lam, phi


def reference_gradient(q_np: np.ndarray, nfft: int, noverlap: int, loss_fn, window=None,
                       weights=None, n_modes: int = 5, eps: float = 1e-12):
    """dE/dq for E = loss_fn(lam, phi), by autograd through spod_torch."""
    q = torch.tensor(np.asarray(q_np, dtype=np.float64), requires_grad=True)
    lam, phi = spod_torch(q, nfft, noverlap, window, weights, n_modes, eps)
    E = loss_fn(lam, phi)
    E.backward()
    return q.grad.numpy().copy(), float(E.detach())

