"""Plain FP64 CPU SPOD: the oracle the HIP path is checked against.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path (the HIP
library and its Python binding) never calls it, and it shares no code, tables or
helpers with that path.

Every function follows the discrete SPOD of the paper, Sec. 2.3 ("Practical
implementation"), step by step and in its notation:

  * Q in R^{M x N_t}, M = M_space * M_vars                     eq. (data-matrix)
  * temporal mean removed                          Sec. 2.1, Sec. 2.3 (first par.)
  * L (possibly overlapping) blocks Q^(l) of N_f snapshots     eq. (blocks)
  * DFT in time of every block                                  eq. (blocks-ft)
  * regroup per frequency: Qhat_k = [qhat_k^(1) .. qhat_k^(L)]  eq. (blocks-k)
  * Chat_k = Qhat_k Qhat_k^* / (L-1)                            eq. (csd-discrete)
  * method of snapshots: Qhat_k^* W Qhat_k Psi_k = Psi_k Lambda_k,
    Phi_k = Qhat_k Psi_k Lambda_k^{-1/2}                        eq. (spod-discrete-snapshots)
  * one-sided frequency set for real data                      eq. (discrete_modes)

Readings where the paper is silent or inconsistent (each one is listed in the
design notes of the repository):

  R1  The Bessel factor 1/(L-1) of eq. (csd-discrete) is folded into Qhat as
      1/sqrt(L-1), so that the snapshot eigenvalues equal those of Chat_k W and
      Phi_k^* W Phi_k = I holds (the orthonormality stated after eq.
      (spod-discrete-snapshots)).
  R2  Window: the paper only cites Welch's method; the default is the periodic
      (DFT-even) Hann window w[n] = 1/2 - 1/2 cos(2 pi n / N_f).
  R3  DFT scale: kappa = 1 / sqrt((L-1) * sum_n w[n]^2), sampling step 1.
  R4  DFT sign e^{-2 pi i k n / N_f}, as in the kernel of eq. (csd).
  R5  One-sided count K = floor(N_f/2) + 1 (the printed ceil(N_f/2)+1 is one
      too many for odd N_f); interior bins are not doubled.
  R6  The mean is the long-time sample mean over all N_t snapshots.
  R7  Block l covers snapshots [l*s, l*s + N_f), s = N_f - N_overlap, starting
      at t = 0; snapshots past the last block are dropped from the blocks (but
      they do enter the mean).
  R8  Eigenvalues sorted descending (stable by index on exact ties).
  R9  Eigenvector phase: the entry of largest modulus (lowest index on ties)
      is made real and positive.
  R10 Modes with lambda_j <= eps * lambda_1(k) (or lambda_1(k) <= 0) are set to
      zero and not counted as valid.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "block_count", "nfreq", "hann_periodic", "dft_scale", "temporal_mean",
    "dft_matrix", "fourier_blocks", "gram", "jacobi_eigh", "sort_and_phase",
    "modes", "spod", "spod_chunked",
]


# --------------------------------------------------------------------------
# Shapes: eq. (blocks) and eq. (discrete_modes)
# --------------------------------------------------------------------------
def block_count(nt: int, nfft: int, noverlap: int) -> int:
    """Number of Welch blocks L (eq. (blocks), reading R7).

    Block l starts at l*s with s = N_f - N_overlap; the last block must end at
    or before N_t, so L = floor((N_t - N_overlap) / s).
    """
    s = nfft - noverlap
    if s <= 0:
        raise ValueError("noverlap must be smaller than nfft")
    return (nt - noverlap) // s


def nfreq(nfft: int) -> int:
    """One-sided frequency count for real data (eq. (discrete_modes), R5)."""
    return nfft // 2 + 1


def hann_periodic(nfft: int) -> np.ndarray:
    """Periodic (DFT-even) Hann window, reading R2."""
    n = np.arange(nfft, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / nfft)


def dft_scale(window: np.ndarray, nblocks: int) -> float:
    """kappa = 1/sqrt((L-1) sum w^2): readings R1 and R3 (eq. (csd-discrete))."""
    return 1.0 / math.sqrt((nblocks - 1) * float(np.sum(np.asarray(window, np.float64) ** 2)))


# --------------------------------------------------------------------------
# Step 0: temporal mean (Sec. 2.1 zero-average process; Sec. 2.3)
# --------------------------------------------------------------------------
def temporal_mean(q: np.ndarray) -> np.ndarray:
    """Long-time mean of every degree of freedom (row of Q), in float64 (R6)."""
    q = np.asarray(q)
    return np.sum(q, axis=1, dtype=np.float64) / q.shape[1]


# --------------------------------------------------------------------------
# Step 2: DFT of every block, eq. (blocks-ft), regrouped as eq. (blocks-k)
# --------------------------------------------------------------------------
def dft_matrix(nfft: int, bins=None) -> np.ndarray:
    """Exact twiddle matrix F[n, k] = exp(-2 pi i (k n mod N_f) / N_f)  (R4).

    The product k*n is reduced modulo N_f in integers before the angle is
    formed, so every entry is one of the N_f correctly rounded roots of unity.
    """
    if bins is None:
        bins = np.arange(nfreq(nfft))
    bins = np.asarray(bins, dtype=np.int64)
    n = np.arange(nfft, dtype=np.int64)
    idx = np.mod(np.outer(n, bins), nfft)
    ang = 2.0 * np.pi * np.arange(nfft, dtype=np.float64) / nfft
    table = np.cos(ang) - 1j * np.sin(ang)
    return table[idx]


def fourier_blocks(q: np.ndarray, nfft: int, noverlap: int, window=None,
                   mean=None, bins=None, dft: str = "matrix") -> np.ndarray:
    """Qhat[k, l, m] for the rows of q (eqs. (blocks), (blocks-ft), (blocks-k)).

    q        : [M, N_t] real snapshot rows (any float dtype; upcast to float64).
    mean     : [M] temporal mean to subtract; computed from q when None.
    bins     : frequency indices to return (default: all K one-sided bins).
    dft      : "matrix" - the DFT sum of eq. (blocks-ft) as a product with the
               exact twiddle table (the definition written out);
               "fft"    - the same sum by numpy's FFT of the windowed block (a
               library step; the two agree to rounding, which a pin checks).
               Used where the full sum over every bin is too slow.
    Returns complex128 [len(bins), L, M], already scaled by kappa (R1, R3).
    """
    q = np.asarray(q)
    m_rows, nt = q.shape
    if window is None:
        window = hann_periodic(nfft)
    window = np.asarray(window, dtype=np.float64)
    nb = block_count(nt, nfft, noverlap)
    s = nfft - noverlap
    if mean is None:
        mean = temporal_mean(q)
    kappa = dft_scale(window, nb)
    if dft == "fft":
        sel = np.arange(nfreq(nfft)) if bins is None else np.asarray(bins, dtype=np.int64)
        out = np.empty((len(sel), nb, m_rows), dtype=np.complex128)
        for ell in range(nb):
            seg = q[:, ell * s: ell * s + nfft].astype(np.float64) - mean[:, None]
            seg *= window[None, :]
            out[:, ell, :] = np.fft.rfft(seg, axis=1)[:, sel].T * kappa
        return out
    if dft != "matrix":
        raise ValueError("dft must be 'matrix' or 'fft'")
    F = dft_matrix(nfft, bins)                      # [N_f, nbins]
    out = np.empty((F.shape[1], nb, m_rows), dtype=np.complex128)
    for ell in range(nb):
        seg = q[:, ell * s: ell * s + nfft].astype(np.float64) - mean[:, None]
        seg *= window[None, :]
        out[:, ell, :] = (seg @ F).T * kappa
    return out


# --------------------------------------------------------------------------
# Steps 3-4: weighted inner product, eq. (spod-discrete-snapshots)
# --------------------------------------------------------------------------
def gram(qhat: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """M_k = Qhat_k^* W Qhat_k for every k: entry (i, j) is
    sum_m conj(qhat[k, i, m]) W_m qhat[k, j, m]."""
    w = np.asarray(weights, dtype=np.float64)
    return np.matmul(np.conj(qhat) * w[None, None, :], np.transpose(qhat, (0, 2, 1)))


# --------------------------------------------------------------------------
# Step 5: eigendecomposition of each Hermitian M_k, by cyclic Jacobi
# --------------------------------------------------------------------------
def jacobi_eigh(a: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic (row-by-row) complex Jacobi for a batch of Hermitian matrices.

    a : [B, n, n] Hermitian.  Returns (lam [B, n] unsorted, V [B, n, n] with
    eigenvector j in column j, sweeps [B]).  The pair (p, q) is rotated when
    |a_pq| > tol * sqrt(|a_pp a_qq|) and |a_pq| > 1e-300; a matrix has
    converged after a sweep without rotations.  Each plane rotation reduces
    the Hermitian 2x2 block [[a, c], [conj(c), b]] by the unitary
      J = [[cs, sn e^{i phi}], [-sn e^{-i phi}, cs]],  c = |c| e^{i phi},
    whose real angle comes from the symmetric Schur decomposition of
    [[a, |c|], [|c|, b]] (Golub & Van Loan, "Matrix Computations", sec. 8.5).
    """
    A = np.array(a, dtype=np.complex128, copy=True)
    if A.ndim == 2:
        A = A[None]
    nb, n, _ = A.shape
    V = np.tile(np.eye(n, dtype=np.complex128), (nb, 1, 1))
    sweeps = np.zeros(nb, dtype=np.int64)
    active = np.ones(nb, dtype=bool)
    for sweep in range(1, max_sweeps + 1):
        rotated = np.zeros(nb, dtype=bool)
        for p in range(n - 1):
            for q in range(p + 1, n):
                app = A[:, p, p].real.copy()
                aqq = A[:, q, q].real.copy()
                apq = A[:, p, q].copy()
                r = np.abs(apq)
                need = active & (r > 1e-300) & (r > tol * np.sqrt(np.abs(app * aqq)))
                if not need.any():
                    continue
                rotated |= need
                idx = np.nonzero(need)[0]
                r_i = r[idx]
                e = apq[idx] / r_i                       # e^{i phi}
                tau = (aqq[idx] - app[idx]) / (2.0 * r_i)
                t = np.where(tau >= 0, 1.0, -1.0) / (np.abs(tau) + np.sqrt(1.0 + tau * tau))
                cs = 1.0 / np.sqrt(1.0 + t * t)
                sn = t * cs
                # columns: A <- A J
                Ap = A[idx, :, p].copy()
                Aq = A[idx, :, q].copy()
                A[idx, :, p] = Ap * cs[:, None] - Aq * (sn * np.conj(e))[:, None]
                A[idx, :, q] = Ap * (sn * e)[:, None] + Aq * cs[:, None]
                # rows: A <- J^H A
                Ap = A[idx, p, :].copy()
                Aq = A[idx, q, :].copy()
                A[idx, p, :] = Ap * cs[:, None] - Aq * (sn * e)[:, None]
                A[idx, q, :] = Ap * (sn * np.conj(e))[:, None] + Aq * cs[:, None]
                A[idx, p, q] = 0.0
                A[idx, q, p] = 0.0
                A[idx, p, p] = app[idx] - t * r_i
                A[idx, q, q] = aqq[idx] + t * r_i
                # eigenvectors: V <- V J
                Vp = V[idx, :, p].copy()
                Vq = V[idx, :, q].copy()
                V[idx, :, p] = Vp * cs[:, None] - Vq * (sn * np.conj(e))[:, None]
                V[idx, :, q] = Vp * (sn * e)[:, None] + Vq * cs[:, None]
        sweeps[active] = sweep
        active &= rotated
        if not active.any():
            break
    sweeps[active] = -max_sweeps          # did not converge
    lam = np.real(np.diagonal(A, axis1=1, axis2=2)).copy()
    return lam, V, sweeps


def sort_and_phase(lam: np.ndarray, V: np.ndarray):
    """Descending order, stable on ties (R8); phase convention R9."""
    lam = np.asarray(lam)
    order = np.argsort(-lam, axis=-1, kind="stable")
    lam_s = np.take_along_axis(lam, order, axis=-1)
    V_s = np.take_along_axis(V, order[:, None, :], axis=-1)
    piv = np.argmax(np.abs(V_s), axis=1)                    # first max per column
    pv = np.take_along_axis(V_s, piv[:, None, :], axis=1)[:, 0, :]
    mag = np.abs(pv)
    ph = np.where(mag > 0, np.conj(pv) / np.where(mag > 0, mag, 1.0), 1.0)
    V_s = V_s * ph[:, None, :]
    return lam_s, V_s


# --------------------------------------------------------------------------
# Step 5b: modes, Phi_k = Qhat_k Psi_k Lambda_k^{-1/2}
# --------------------------------------------------------------------------
def modes(qhat: np.ndarray, lam: np.ndarray, psi: np.ndarray, n_modes: int,
          eps: float = 1e-12):
    """phi[k, j, m] = sum_l qhat[k, l, m] psi[k, l, j] / sqrt(lam[k, j]) for the
    leading n_modes; invalid modes (R10) are zero.  Returns (phi, n_valid)."""
    nk, nb, _ = qhat.shape
    n_modes = min(n_modes, nb)
    lam_n = lam[:, :n_modes]
    valid = (lam[:, :1] > 0) & (lam_n > eps * lam[:, :1])
    scale = np.where(valid, 1.0 / np.sqrt(np.where(valid, lam_n, 1.0)), 0.0)
    coef = psi[:, :, :n_modes] * scale[:, None, :]            # [K, L, n]
    phi = np.matmul(np.transpose(coef, (0, 2, 1)), qhat)      # [K, n, M]
    return phi, valid.sum(axis=1).astype(np.int32)


# --------------------------------------------------------------------------
# The whole path
# --------------------------------------------------------------------------
def spod(q, nfft: int, noverlap: int, window=None, weights=None, n_modes: int = 5,
         eps: float = 1e-12):
    """End-to-end SPOD of one snapshot matrix (all of it in memory)."""
    q = np.asarray(q)
    m_rows, nt = q.shape
    if window is None:
        window = hann_periodic(nfft)
    if weights is None:
        weights = np.full(m_rows, 1.0 / m_rows)
    mean = temporal_mean(q)
    qhat = fourier_blocks(q, nfft, noverlap, window, mean)
    M = gram(qhat, weights)
    lam, V, sweeps = jacobi_eigh(M)
    lam, psi = sort_and_phase(lam, V)
    phi, n_valid = modes(qhat, lam, psi, n_modes, eps)
    return {"mean": mean, "qhat": qhat, "gram": M, "lam": lam, "psi": psi,
            "phi": phi, "n_valid": n_valid, "sweeps": sweeps}


def spod_chunked(q, nfft: int, noverlap: int, window=None, weights=None,
                 n_modes: int = 5, eps: float = 1e-12, chunk: int = 8192,
                 bins=None, want_modes: bool = True, mode_rows=None, dft: str = "matrix",
                 progress=None):
    """The same path streamed over chunks of degrees of freedom.

    This is the spatial split of Sec. 3.1 done sequentially: the Gram of every
    frequency is accumulated chunk by chunk in a first pass, the eigenproblems
    are solved, and the modes come from a second pass that recomputes Qhat.
    `bins` restricts the work to selected frequencies; `mode_rows` restricts
    the second pass to selected degrees of freedom (the rest of phi is not
    formed).  `dft` is passed to fourier_blocks; `progress(rows_done)` is
    called after every chunk of the first pass (for long runs).
    """
    q = np.asarray(q)
    m_rows, nt = q.shape
    if window is None:
        window = hann_periodic(nfft)
    if weights is None:
        weights = np.full(m_rows, 1.0 / m_rows)
    weights = np.asarray(weights, dtype=np.float64)
    nk = nfreq(nfft) if bins is None else len(bins)
    nb = block_count(nt, nfft, noverlap)
    mean = np.empty(m_rows, dtype=np.float64)
    G = np.zeros((nk, nb, nb), dtype=np.complex128)
    for c0 in range(0, m_rows, chunk):
        c1 = min(m_rows, c0 + chunk)
        qc = q[c0:c1]
        mean[c0:c1] = temporal_mean(qc)
        qh = fourier_blocks(qc, nfft, noverlap, window, mean[c0:c1], bins, dft=dft)
        G += gram(qh, weights[c0:c1])
        if progress is not None:
            progress(c1)
    lam, V, sweeps = jacobi_eigh(G)
    lam, psi = sort_and_phase(lam, V)
    out = {"mean": mean, "gram": G, "lam": lam, "psi": psi, "sweeps": sweeps}
    if want_modes:
        rows = np.arange(m_rows) if mode_rows is None else np.asarray(mode_rows)
        n_use = min(n_modes, nb)
        phi = np.empty((nk, n_use, len(rows)), dtype=np.complex128)
        n_valid = None
        for c0 in range(0, len(rows), chunk):
            r = rows[c0:c0 + chunk]
            qh = fourier_blocks(q[r], nfft, noverlap, window, mean[r], bins, dft=dft)
            phi[:, :, c0:c0 + len(r)], n_valid = modes(qh, lam, psi, n_modes, eps)
        out["phi"] = phi
        out["n_valid"] = n_valid
        out["mode_rows"] = rows
    return out
