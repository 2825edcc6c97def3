"""Pins of the FP64 oracle against facts fixed by the paper, by mathematics, and
by independent library routines (CPU only).

Each test is chosen so that a plausible slip in the oracle (a dropped factor,
a wrong sign or index, a transposed operand, a missing window or mean) makes
at least one of them fail.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.signal
import torch

import oracle as O
from synth import fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- block count
def test_block_count_matches_paper_printed_values():
    with open(os.path.join(GOLDEN, "paper_block_counts.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        assert O.block_count(c["nt"], c["nfft"], c["noverlap"]) == c["L"], c["cite"]


def test_block_count_workloads():
    assert O.block_count(1024, 128, 64) == 15
    assert O.block_count(4096, 256, 128) == 31
    assert O.block_count(8192, 512, 256) == 31


def test_one_sided_count_both_parities():
    # K = floor(N/2)+1 is the number of distinct non-negative frequencies of a
    # real length-N DFT: exactly numpy's rfft length, for even and odd N.
    for n in (7, 8, 63, 64, 255, 256):
        assert O.nfreq(n) == np.fft.rfft(np.zeros(n)).shape[0]


# ---------------------------------------------------------------- window, DFT
def test_hann_is_scipy_periodic_hann_and_has_three_tap_spectrum():
    for n in (16, 128, 512):
        w = O.hann_periodic(n)
        np.testing.assert_allclose(w, scipy.signal.get_window("hann", n), atol=1e-15)
        W = np.fft.fft(w)
        ref = np.zeros(n, complex)
        ref[0], ref[1], ref[-1] = n / 2, -n / 4, -n / 4
        np.testing.assert_allclose(W, ref, atol=1e-12 * n)


def test_dft_matrix_is_numpy_rfft():
    rng = _rng(3)
    for n in (8, 15, 64, 73, 360):
        x = rng.standard_normal((5, n))
        np.testing.assert_allclose(x @ O.dft_matrix(n), np.fft.rfft(x, axis=1), atol=1e-12)


def test_fourier_blocks_against_numpy_rfft_of_each_block():
    rng = _rng(4)
    M, nt, nfft, nov = 7, 200, 32, 12
    q = rng.standard_normal((M, nt)) + 3.0
    w = rng.uniform(0.2, 1.0, nfft)
    L = O.block_count(nt, nfft, nov)
    s = nfft - nov
    mean = q.mean(axis=1)
    qh = O.fourier_blocks(q, nfft, nov, w)
    kappa = 1 / math.sqrt((L - 1) * np.sum(w * w))
    for ell in range(L):
        blk = (q[:, ell * s: ell * s + nfft] - mean[:, None]) * w
        np.testing.assert_allclose(qh[:, ell, :], kappa * np.fft.rfft(blk, axis=1).T, atol=1e-12)


# ---------------------------------------------------------------- mean
def test_mean_is_exact_sum():
    rng = _rng(5)
    q = rng.standard_normal((9, 777)) * 10.0 ** rng.integers(-3, 4, (9, 1)) + 1e3
    m = O.temporal_mean(q)
    ref = np.array([math.fsum(r) / q.shape[1] for r in q])
    np.testing.assert_allclose(m, ref, rtol=1e-15, atol=0)


# ---------------------------------------------------------------- Welch (M = 1)
@pytest.mark.parametrize("nfft,nov,nt", [(64, 32, 1000), (128, 64, 1024), (63, 21, 700)])
def test_single_dof_is_welch_psd(nfft, nov, nt):
    """With one degree of freedom, lambda_1(k) = W * L/(L-1) * P_welch(k) / c_k,
    c_k = 2 on interior bins (1 at DC and at Nyquist), where P_welch is scipy's
    one-sided density estimate with the same Hann segments and no detrending."""
    rng = _rng(6)
    x = np.cumsum(rng.standard_normal(nt)) * 0.1 + rng.standard_normal(nt) + 5.0
    Wm = 0.37
    L = O.block_count(nt, nfft, nov)
    out = O.spod(x[None, :], nfft, nov, weights=np.array([Wm]), n_modes=1)
    lam = out["lam"][:, 0]
    f, P = scipy.signal.welch(x - x.mean(), fs=1.0, window="hann", nperseg=nfft, noverlap=nov,
                              detrend=False, scaling="density", return_onesided=True)
    c = np.full(P.shape, 2.0)
    c[0] = 1.0
    if nfft % 2 == 0:
        c[-1] = 1.0
    np.testing.assert_allclose(lam, Wm * L / (L - 1) * P / c, rtol=1e-12, atol=1e-15 * lam.max())


# ---------------------------------------------------------------- Parseval / trace
@pytest.mark.parametrize("nfft,nov", [(32, 16), (33, 11)])
def test_parseval_energy(nfft, nov):
    """sum_k c_k tr(M_k) = kappa^2 N_f sum_l sum_m W_m sum_n w[n]^2 (q - mean)^2."""
    rng = _rng(7)
    M, nt = 11, 300
    q = rng.standard_normal((M, nt)) + rng.standard_normal((M, 1))
    W = rng.uniform(0.1, 2.0, M)
    w = O.hann_periodic(nfft)
    out = O.spod(q, nfft, nov, w, W)
    c = np.full(O.nfreq(nfft), 2.0)
    c[0] = 1.0
    if nfft % 2 == 0:
        c[-1] = 1.0
    lhs = np.sum(c * np.real(np.trace(out["gram"], axis1=1, axis2=2)))
    L = O.block_count(nt, nfft, nov)
    s = nfft - nov
    kappa2 = 1.0 / ((L - 1) * np.sum(w * w))
    x = q - q.mean(axis=1, keepdims=True)
    e = sum(np.sum(W[:, None] * (w[None, :] ** 2) * x[:, l * s: l * s + nfft] ** 2) for l in range(L))
    np.testing.assert_allclose(lhs, kappa2 * nfft * e, rtol=1e-13)


def test_trace_identity_and_gram_hermitian():
    p = fields.random_rows(40, 600, 64, 32, seed=8)
    out = O.spod(p.q.numpy(), 64, 32, weights=p.weights)
    G = out["gram"]
    np.testing.assert_allclose(G, np.conj(np.transpose(G, (0, 2, 1))), atol=1e-15 * np.abs(G).max())
    tr = np.real(np.trace(G, axis1=1, axis2=2))
    np.testing.assert_allclose(out["lam"].sum(axis=1), tr, rtol=1e-12)
    # diagonal of M_k is the weighted energy of each block at bin k
    d = np.einsum("klm,m->kl", np.abs(out["qhat"]) ** 2, p.weights)
    np.testing.assert_allclose(np.real(np.diagonal(G, axis1=1, axis2=2)), d, rtol=1e-13)


# ---------------------------------------------------------------- snapshots vs CSD
def test_method_of_snapshots_equals_direct_csd_eigenproblem():
    """eq. (spod-discrete) with Chat_k = Qhat_k Qhat_k^*/(L-1) (eq. (csd-discrete))
    and the snapshot form give the same eigenvalues, and the modes agree up
    to a phase.  Qhat is built here from numpy's rfft, not from the oracle."""
    rng = _rng(9)
    M, nfft, nov = 6, 16, 8
    nt = nfft + 29 * (nfft - nov)           # L = 30 > M
    q = rng.standard_normal((M, nt))
    W = rng.uniform(0.3, 1.5, M)
    w = O.hann_periodic(nfft)
    L = O.block_count(nt, nfft, nov)
    assert L == 30
    s = nfft - nov
    x = q - q.mean(axis=1, keepdims=True)
    X = np.stack([np.fft.rfft(x[:, l * s: l * s + nfft] * w, axis=1) for l in range(L)], axis=2)
    X /= math.sqrt(np.sum(w * w))              # [M, K, L], unit window energy
    out = O.spod(q, nfft, nov, w, W, n_modes=M)
    sw = np.sqrt(W)
    for k in range(O.nfreq(nfft)):
        Qk = X[:, k, :]
        C = Qk @ Qk.conj().T / (L - 1)
        lam_d, V = np.linalg.eigh(sw[:, None] * C * sw[None, :])
        lam_d, V = lam_d[::-1], V[:, ::-1]
        np.testing.assert_allclose(out["lam"][k, :M], lam_d, rtol=1e-10, atol=1e-13 * lam_d[0])
        Phi_d = V / sw[:, None]
        for j in range(M):
            if lam_d[j] < 1e-9 * lam_d[0]:
                continue
            inner = abs(np.vdot(Phi_d[:, j], W * out["phi"][k, j]))
            assert abs(inner - 1.0) < 1e-9
        resid = C @ (W[:, None] * out["phi"][k].T) - out["phi"][k].T * out["lam"][k, :M]
        assert np.abs(resid).max() < 1e-12 * lam_d[0]


# ---------------------------------------------------------------- Jacobi
def _hermitian_cases():
    rng = _rng(10)
    out = []
    for n in (2, 5, 31, 32, 63):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        out.append(A + A.conj().T)                                   # indefinite
        B = rng.standard_normal((n, max(1, n // 3))) + 1j * rng.standard_normal((n, max(1, n // 3)))
        out.append(B @ B.conj().T)                                   # PSD, rank deficient
        D = np.diag(10.0 ** np.linspace(0, -12, n))
        U, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        out.append(U @ D @ U.conj().T)                               # graded spectrum
    E = np.diag([3.0, 3.0, 1.0, 1.0, 1.0, 0.5])
    U, _ = np.linalg.qr(rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)))
    out.append(U @ E @ U.conj().T)                                   # degenerate
    return out


@pytest.mark.parametrize("A", _hermitian_cases(), ids=lambda a: f"n{a.shape[0]}")
def test_jacobi_matches_lapack_eigh(A):
    A = 0.5 * (A + A.conj().T)
    lam, V, sweeps = O.jacobi_eigh(A)
    assert sweeps[0] > 0
    lam, V = O.sort_and_phase(lam, V)
    ref = np.linalg.eigvalsh(A)[::-1]
    nrm = np.linalg.norm(A)
    np.testing.assert_allclose(lam[0], ref, atol=1e-13 * nrm, rtol=0)
    n = A.shape[0]
    assert np.abs(A @ V[0] - V[0] * lam[0]).max() < 1e-13 * nrm
    assert np.abs(V[0].conj().T @ V[0] - np.eye(n)).max() < 1e-13


def test_sort_and_phase_conventions():
    lam = np.array([[1.0, 3.0, 2.0, 3.0]])
    V = np.eye(4, dtype=complex)[None] * np.exp(1j * np.array([0.3, 1.1, -2.0, 2.5]))[None, None, :]
    V[0, 2, 0] = 0.5j                                      # column 0: largest modulus is row 0
    ls, Vs = O.sort_and_phase(lam, V)
    assert ls.tolist() == [[3.0, 3.0, 2.0, 1.0]]
    assert np.allclose(np.abs(Vs[0, :, 0]), np.abs(V[0, :, 1]))   # stable on the tie
    for j in range(4):
        piv = np.argmax(np.abs(Vs[0, :, j]))
        assert abs(Vs[0, piv, j].imag) < 1e-15 and Vs[0, piv, j].real > 0


# ---------------------------------------------------------------- modes
def test_modes_are_w_orthonormal():
    p = fields.random_rows(50, 900, 64, 32, seed=11)
    out = O.spod(p.q.numpy(), 64, 32, weights=p.weights, n_modes=8)
    W = p.weights
    for k in range(out["phi"].shape[0]):
        P = out["phi"][k]                                  # [n, M]
        G = np.conj(P) @ (W[:, None] * P.T)
        np.testing.assert_allclose(G, np.eye(P.shape[0]), atol=1e-11)


@pytest.mark.parametrize("dft", ["matrix", "fft"])
def test_planted_modes_closed_form(dft):
    """Noise-free planted field: with the periodic Hann, sum w = N/2 and
    sum w^2 = 3N/8, so a cosine of amplitude a on a W-unit mode at bin b gives
    lambda_1(b) = L/(L-1) * a^2 * N_f / 6, and the Hann leakage (-N/4 at +-1)
    gives lambda_1(b +- 1) = lambda_1(b) / 4; everything else is zero.  Both
    forms of the block transform (the DFT sum with the twiddle table, and the
    library FFT step) are held to it."""
    p = fields.planted(sigma=0.0, seed=1)
    q = p.q.numpy()
    nfft, nov = 128, 64
    L = O.block_count(q.shape[1], nfft, nov)
    if dft == "matrix":
        out = O.spod(q, nfft, nov, weights=p.weights, n_modes=3)
    else:
        out = O.spod_chunked(q, nfft, nov, weights=p.weights, n_modes=3, chunk=300, dft="fft")
    lam = out["lam"]
    top = lam.max()
    seen = set()
    for b, a, i in zip(p.meta["bins"], p.meta["amps"], range(3)):
        ref = L / (L - 1) * a * a * nfft / 6.0
        np.testing.assert_allclose(lam[b, 0], ref, rtol=1e-13)
        np.testing.assert_allclose(lam[b - 1, 0], ref / 4, rtol=1e-13)
        np.testing.assert_allclose(lam[b + 1, 0], ref / 4, rtol=1e-13)
        assert lam[b, 1] < 1e-12 * ref
        phi_i = p.meta["phi"][:, i]
        inner = abs(np.vdot(phi_i, p.weights * out["phi"][b, 0]))
        assert abs(inner - 1.0) < 1e-12
        seen |= {b - 1, b, b + 1}
    others = [k for k in range(lam.shape[0]) if k not in seen]
    assert np.abs(lam[others]).max() < 1e-12 * top
    # with the parity workload's noise the leading values move only slightly
    pn = fields.planted(sigma=0.1, seed=1)
    outn = O.spod(pn.q.numpy(), nfft, nov, weights=pn.weights, n_modes=3)
    for b, a in zip(pn.meta["bins"], pn.meta["amps"]):
        ref = L / (L - 1) * a * a * nfft / 6.0
        assert abs(outn["lam"][b, 0] / ref - 1) < 2e-3


def test_rank_deficient_modes_are_zero_and_not_counted():
    p = fields.planted(nspace=4, nt=1024, sigma=0.0, seed=2, bins=(5, 12, 30))
    out = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=5)
    assert out["n_valid"].max() <= 4
    for k in range(out["phi"].shape[0]):
        nv = out["n_valid"][k]
        assert np.all(out["phi"][k, nv:] == 0)


# ---------------------------------------------------------------- invariances
def test_invariances():
    p = fields.random_rows(30, 700, 64, 32, seed=12)
    q = p.q.numpy()
    W = p.weights
    base = O.spod(q, 64, 32, weights=W, n_modes=4)
    # a constant field added to every snapshot changes nothing
    shifted = O.spod(q + 50.0 * _rng(1).standard_normal((q.shape[0], 1)), 64, 32, weights=W, n_modes=4)
    np.testing.assert_allclose(shifted["qhat"], base["qhat"], atol=1e-11 * np.abs(base["qhat"]).max())
    np.testing.assert_allclose(shifted["lam"], base["lam"], rtol=1e-9, atol=1e-12 * base["lam"].max())
    # W -> a W scales lambda by a and Phi by a^-1/2
    a = 3.7
    scaled = O.spod(q, 64, 32, weights=a * W, n_modes=4)
    np.testing.assert_allclose(scaled["lam"], a * base["lam"], rtol=1e-11, atol=1e-14 * base["lam"].max())
    for k in range(0, 33, 8):
        for j in range(2):
            r = abs(np.vdot(scaled["phi"][k, j], W * base["phi"][k, j])) * math.sqrt(a)
            assert abs(r - 1) < 1e-9
    # permuting degrees of freedom permutes the rows of Phi
    perm = _rng(2).permutation(q.shape[0])
    pm = O.spod(q[perm], 64, 32, weights=W[perm], n_modes=4)
    np.testing.assert_allclose(pm["lam"], base["lam"], rtol=1e-11, atol=1e-14 * base["lam"].max())
    for k in range(0, 33, 8):
        r = abs(np.vdot(pm["phi"][k, 0], W[perm] * base["phi"][k, 0][perm]))
        assert abs(r - 1) < 1e-9


def test_chunked_equals_whole():
    p = fields.random_rows(70, 500, 32, 16, seed=13)
    q = p.q.numpy()
    a = O.spod(q, 32, 16, weights=p.weights, n_modes=3)
    b = O.spod_chunked(q, 32, 16, weights=p.weights, n_modes=3, chunk=16)
    np.testing.assert_allclose(b["gram"], a["gram"], atol=1e-13 * np.abs(a["gram"]).max())
    np.testing.assert_allclose(b["lam"], a["lam"], rtol=1e-12, atol=1e-15 * a["lam"].max())
    np.testing.assert_allclose(b["phi"], a["phi"], atol=1e-10 * np.abs(a["phi"]).max())
    sel = [0, 3, 7]
    c = O.spod_chunked(q, 32, 16, weights=p.weights, n_modes=3, chunk=16, bins=sel, mode_rows=[5, 1])
    np.testing.assert_allclose(c["lam"], a["lam"][sel], rtol=1e-12, atol=1e-15 * a["lam"].max())
    np.testing.assert_allclose(c["phi"], a["phi"][sel][:, :, [5, 1]], atol=1e-10 * np.abs(a["phi"]).max())
    # the library FFT form of the block transform gives the same path
    done = []
    d = O.spod_chunked(q, 32, 16, weights=p.weights, n_modes=3, chunk=16, dft="fft",
                       progress=done.append)
    assert done == list(range(16, 70, 16)) + [70]
    np.testing.assert_allclose(d["gram"], a["gram"], atol=1e-13 * np.abs(a["gram"]).max())
    np.testing.assert_allclose(d["lam"], a["lam"], rtol=1e-12, atol=1e-15 * a["lam"].max())
    np.testing.assert_allclose(d["phi"], a["phi"], atol=1e-10 * np.abs(a["phi"]).max())
    e = O.spod_chunked(q, 32, 16, weights=p.weights, n_modes=3, chunk=16, bins=sel, dft="fft")
    np.testing.assert_allclose(e["lam"], a["lam"][sel], rtol=1e-12, atol=1e-15 * a["lam"].max())
    for odd in (33, 35):       # odd block length: the one-sided set has no Nyquist bin
        qo = q[:, :400]
        np.testing.assert_allclose(O.fourier_blocks(qo, odd, 11, dft="fft"),
                                   O.fourier_blocks(qo, odd, 11), atol=1e-12)


def test_generator_is_seeded():
    a = fields.jet_like(seed=2, nx=16, ny=8, nt=64, nfft=16, noverlap=8)
    b = fields.jet_like(seed=2, nx=16, ny=8, nt=64, nfft=16, noverlap=8)
    c = fields.jet_like(seed=3, nx=16, ny=8, nt=64, nfft=16, noverlap=8)
    assert torch.equal(a.q, b.q) and not torch.equal(a.q, c.q)
    e = fields.era_like(nlon=16, nlat=8, nt=64, nfft=16, noverlap=8)
    assert e.q.shape == (256, 64) and np.isfinite(e.q.numpy()).all()
    # cos(lat) midpoint quadrature integrates the sphere to 4 pi per variable,
    # up to the midpoint-rule factor (h/2)/sin(h/2) of the latitude step h
    h = math.pi / 8
    np.testing.assert_allclose(e.weights.sum(), 2 * 4 * math.pi * (h / 2) / math.sin(h / 2), rtol=1e-12)
