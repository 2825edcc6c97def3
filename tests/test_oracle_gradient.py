"""Pins of the FP64 reference gradient (CPU only): central finite differences
of the forward oracle, and the closed-form gradient of the total energy."""
import math

import numpy as np
import torch

import oracle as O
from oracle.gradient import reference_gradient, spod_torch


def _problem(seed=21, M=8, nt=96, nfft=16, nov=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.standard_normal((M, nt)) + np.cumsum(rng.standard_normal((M, nt)), axis=1) * 0.2
    W = rng.uniform(0.3, 1.2, M)
    return q, W, nfft, nov


def test_torch_forward_equals_numpy_oracle():
    q, W, nfft, nov = _problem()
    lam, phi = spod_torch(torch.tensor(q), nfft, nov, weights=W, n_modes=3)
    ref = O.spod(q, nfft, nov, weights=W, n_modes=3)
    np.testing.assert_allclose(lam.numpy(), ref["lam"], rtol=1e-10, atol=1e-13 * ref["lam"].max())
    for k in range(ref["phi"].shape[0]):
        for j in range(3):
            r = abs(np.vdot(ref["phi"][k, j], W * phi[k, j].numpy()))
            assert abs(r - 1) < 1e-8


def _loss_factory(W, bins, probes):
    Wt = torch.tensor(W)

    def loss(lam, phi):
        e = lam[bins, :3].sum()
        for i, k in enumerate(bins):
            e = e + torch.abs(torch.sum(torch.conj(probes[i]) * Wt * phi[k, 0])) ** 2
        return e
    return loss


def test_reference_gradient_matches_central_differences():
    q, W, nfft, nov = _problem()
    rng = np.random.Generator(np.random.PCG64(5))
    bins = [1, 2, 4, 6]
    probes = [torch.tensor(rng.standard_normal(q.shape[0]) + 1j * rng.standard_normal(q.shape[0]))
              for _ in bins]
    loss = _loss_factory(W, bins, probes)
    g, _ = reference_gradient(q, nfft, nov, loss, weights=W, n_modes=3)

    def f(x):
        with torch.no_grad():
            lam, phi = spod_torch(torch.tensor(x), nfft, nov, weights=W, n_modes=3)
            return float(loss(lam, phi))

    h = 1e-5
    idx = rng.choice(q.size, 64, replace=False)
    fd = np.empty(len(idx))
    for n, i in enumerate(idx):
        xp = q.copy().reshape(-1)
        xm = q.copy().reshape(-1)
        xp[i] += h
        xm[i] -= h
        fd[n] = (f(xp.reshape(q.shape)) - f(xm.reshape(q.shape))) / (2 * h)
    ga = g.reshape(-1)[idx]
    np.testing.assert_allclose(ga, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_energy_gradient_closed_form():
    """E = sum_k c_k tr(M_k) (c_k = 2 on interior bins) has
    dE/dq[m, t] = 2 kappa^2 N_f W_m (sum_{l: t in block l} w[t - l s]^2 x[m, t]
                                     - (1/N_t) sum_l sum_n w[n]^2 x[m, l s + n]),
    x = q - mean: no eigensolve is involved."""
    q, W, nfft, nov = _problem(seed=22, M=5, nt=130, nfft=16, nov=8)
    K = O.nfreq(nfft)
    c = torch.full((K,), 2.0, dtype=torch.float64)
    c[0] = 1.0
    c[-1] = 1.0

    def loss(lam, phi):
        return torch.sum(c[:, None] * lam)

    g, _ = reference_gradient(q, nfft, nov, loss, weights=W, n_modes=3)
    M, nt = q.shape
    L = O.block_count(nt, nfft, nov)
    s = nfft - nov
    w = O.hann_periodic(nfft)
    kappa2 = 1.0 / ((L - 1) * np.sum(w * w))
    x = q - q.mean(axis=1, keepdims=True)
    acc = np.zeros_like(q)
    tot = np.zeros(M)
    for ell in range(L):
        acc[:, ell * s: ell * s + nfft] += (w ** 2)[None, :] * x[:, ell * s: ell * s + nfft]
        tot += np.sum((w ** 2)[None, :] * x[:, ell * s: ell * s + nfft], axis=1)
    ref = 2 * kappa2 * nfft * W[:, None] * (acc - tot[:, None] / nt)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert math.isfinite(float(np.abs(g).sum()))
