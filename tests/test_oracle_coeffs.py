"""Pins of the expansion-coefficient and reconstruction oracle (CPU only).

Each pin is fixed by the mathematics of eq. (coeffs) and eq. (SPODrec), not by
re-typing them: data in the span of the basis give back their coefficients; the
residual of the projection is W-orthogonal to the basis; the long-time mean is
invisible to the coefficients; a complete basis reconstructs the data; and a
planted single-frequency field is rebuilt by its one SPOD mode.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import coeffs as C
from synth import fields


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _random_phi(rng, K, n, M):
    return rng.standard_normal((K, n, M)) + 1j * rng.standard_normal((K, n, M))


def test_gather_orders_columns_by_frequency_then_mode():
    phi = np.arange(4 * 3 * 2).reshape(4, 3, 2).astype(complex)
    P = C.gather_modes(phi, [1, 3], 2)
    assert P.shape == (2, 4)
    for col, (k, j) in enumerate([(1, 0), (1, 1), (3, 0), (3, 1)]):
        np.testing.assert_array_equal(P[:, col], phi[k, j])


def test_data_in_the_span_give_back_their_coefficients():
    rng = _rng(1)
    K, n, M, nt = 6, 4, 40, 25
    phi = _random_phi(rng, K, n, M)
    bins, n_r = [0, 2, 5], 3
    Phi = C.gather_modes(phi, bins, n_r)
    X = rng.standard_normal((9, nt)) + 1j * rng.standard_normal((9, nt))
    W = rng.uniform(0.2, 1.5, M)
    q = Phi @ X                                   # complex data exactly in the span
    A = C.expansion_coefficients(q, np.zeros(M), phi, W, bins, n_r)
    np.testing.assert_allclose(A, X, rtol=0, atol=1e-12 * np.abs(X).max())


def test_residual_is_w_orthogonal_to_the_basis():
    rng = _rng(2)
    p = fields.random_rows(48, 12 * 16 + 16, 32, 16, seed=3, offset=2.0, dtype=torch.float64)
    q = p.q.numpy()
    out = O.spod(q, 32, 16, weights=p.weights, n_modes=4)
    bins, n_r = [1, 4, 7, 10], 3
    A = C.expansion_coefficients(q, out["mean"], out["phi"], p.weights, bins, n_r)
    Phi = C.gather_modes(out["phi"], bins, n_r)
    res = (q - out["mean"][:, None]) - Phi @ A
    lhs = Phi.conj().T @ (p.weights[:, None] * res)
    ref = np.abs(C.projection_rhs(Phi, p.weights, q, out["mean"])).max()
    assert np.abs(lhs).max() <= 1e-12 * ref
    # without the weights the residual is not orthogonal: the pin sees W
    lhs_plain = Phi.conj().T @ res
    assert np.abs(lhs_plain).max() > 1e-6 * ref
    del rng


def test_mean_is_invisible_to_the_coefficients():
    rng = _rng(4)
    M, nt, K, n = 30, 50, 5, 3
    phi = _random_phi(rng, K, n, M)
    W = rng.uniform(0.1, 1.0, M)
    q = rng.standard_normal((M, nt))
    shift = 100.0 * rng.standard_normal(M)
    a1 = C.expansion_coefficients(q, q.mean(1), phi, W, [0, 3], 2)
    a2 = C.expansion_coefficients(q + shift[:, None], (q + shift[:, None]).mean(1), phi, W, [0, 3], 2)
    np.testing.assert_allclose(a2, a1, rtol=0, atol=1e-10 * np.abs(a1).max())
    # the mean is added back by the reconstruction
    r1 = C.reconstruct(phi, a1, q.mean(1), [0, 3], 2)
    r2 = C.reconstruct(phi, a2, (q + shift[:, None]).mean(1), [0, 3], 2)
    np.testing.assert_allclose(r2 - r1, np.repeat(shift[:, None], nt, 1), rtol=0, atol=1e-10 * 100)


def test_w_orthonormal_modes_of_one_frequency_project_directly():
    p = fields.random_rows(64, 10 * 16 + 16, 32, 16, seed=5, dtype=torch.float64)
    q = p.q.numpy()
    out = O.spod(q, 32, 16, weights=p.weights, n_modes=5)
    k = 6
    Phi = C.gather_modes(out["phi"], [k], 5)
    np.testing.assert_allclose(C.mode_gram(Phi, p.weights), np.eye(5), rtol=0, atol=1e-12)
    A = C.expansion_coefficients(q, out["mean"], out["phi"], p.weights, [k], 5)
    direct = (p.weights[:, None] * Phi).conj().T @ (q - out["mean"][:, None])
    np.testing.assert_allclose(A, direct, rtol=0, atol=1e-12 * np.abs(direct).max())


def test_complete_basis_reconstructs_the_data():
    rng = _rng(6)
    M, nt = 12, 40
    q = rng.standard_normal((M, nt)) + 3.0
    phi = _random_phi(rng, 4, 3, M)                # 4 frequencies x 3 modes = 12 = M columns
    W = rng.uniform(0.3, 2.0, M)
    mean = q.mean(1)
    A = C.expansion_coefficients(q, mean, phi, W, [0, 1, 2, 3], 3)
    rec = C.reconstruct(phi, A, mean, [0, 1, 2, 3], 3)
    np.testing.assert_allclose(rec, q, rtol=0, atol=1e-11)


def test_planted_single_frequency_field_is_rebuilt_by_its_mode():
    """q = a phi cos(2 pi b t / N_f + theta): the SPOD mode of bin b is phi times
    a unit phase (the phase convention fixes the eigenvectors Psi, and the mode
    carries the phase of the Fourier blocks), so one coefficient row rebuilds
    the field exactly and, undone by that phase, is the planted time signal."""
    p = fields.planted(nspace=200, nt=1024, nfft=128, noverlap=64, bins=(12,), amps=(2.0,),
                       sigma=0.0, seed=7, dtype=torch.float64)
    q = p.q.numpy()
    out = O.spod(q, 128, 64, weights=p.weights, n_modes=1)
    A = C.expansion_coefficients(q, out["mean"], out["phi"], p.weights, [12], 1)
    rec = C.reconstruct(out["phi"], A, out["mean"], [12], 1)
    np.testing.assert_allclose(rec, q, rtol=0, atol=1e-10 * np.abs(q).max())
    # the mode is e * phi with |e| = 1; e * A is the planted time signal
    # 2 cos(2 pi 12 t / 128 + theta) (theta read off its DFT: 96 whole periods)
    e = np.vdot(p.meta["phi"][:, 0], p.weights * out["phi"][12, 0])
    assert abs(abs(e) - 1.0) < 1e-12
    sig = e * A[0]
    np.testing.assert_allclose(np.imag(sig), 0.0, atol=1e-10)
    t = np.arange(1024)
    theta = np.angle(np.sum(np.real(sig) * np.exp(-2j * np.pi * 12 * t / 128)))
    np.testing.assert_allclose(np.real(sig), 2.0 * np.cos(2 * np.pi * 12 * t / 128 + theta),
                               rtol=0, atol=1e-9)


@pytest.mark.parametrize("bad", ["transposed_gram", "no_conjugate"])
def test_planted_mistakes_fail_the_span_pin(bad):
    """A transposed Phi^* W Phi or a missing conjugate in the right-hand side is
    caught by the span pin (checked on the CPU with a deliberately wrong copy)."""
    rng = _rng(8)
    K, n, M, nt = 5, 3, 30, 10
    phi = _random_phi(rng, K, n, M)
    W = rng.uniform(0.2, 1.5, M)
    Phi = C.gather_modes(phi, [1, 4], 3)
    X = rng.standard_normal((6, nt)) + 1j * rng.standard_normal((6, nt))
    q = Phi @ X
    B = C.mode_gram(Phi, W)
    rhs = C.projection_rhs(Phi, W, q, np.zeros(M))
    if bad == "transposed_gram":
        A = np.linalg.solve(B.T, rhs)
    else:
        A = np.linalg.solve(B, (W[:, None] * Phi).T @ q)
    assert np.abs(A - X).max() > 1e-3 * np.abs(X).max()
