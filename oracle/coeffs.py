"""Plain FP64 CPU expansion coefficients and reconstruction (SPOD for data
compression): the oracle the HIP path is checked against.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP path.

Following the paper's section on SPOD for data compression:

  * Phi gathers the retained modes arranged by frequency as in
    eq. (discrete_modes): for every retained frequency (in increasing order)
    its leading L_r modes, so column r = i * L_r + j is mode j of the i-th
    retained frequency;
  * the coefficients are the weighted oblique projection of the data onto
    that basis, A = (Phi^* W Phi)^{-1} Phi^* W Q                   eq. (coeffs)
  * the data are approximated by Q~ = Phi_r A_r                   eq. (SPODrec)

Readings where the paper is silent (listed in the design notes too):

  R15 Q in eq. (coeffs) is the data with the long-time mean removed (R6): the
      modes describe the fluctuations, and the mean carries no SPOD content.
  R16 Only the one-sided frequency set of eq. (discrete_modes) is retained, so
      Phi_r A_r is complex for real data.  The reconstruction of real data is
      its real part plus the mean: Q~ = Re(Phi_r A_r) + qbar 1^T.  Its error is
      never larger (elementwise in modulus) than that of the complex
      projection, and it is exact whenever the data lie in the span of Phi_r.
  R17 (Phi^* W Phi) must be invertible: every retained mode must be valid
      (R10).  The oracle solves with a library LU; the HIP path factors the
      Hermitian positive definite matrix by Cholesky.
"""
from __future__ import annotations

import numpy as np

__all__ = ["gather_modes", "mode_gram", "projection_rhs", "expansion_coefficients",
           "reconstruct"]


def gather_modes(phi, bins, n_r: int):
    """Phi_r as an M x R matrix (columns ordered by frequency, then mode).

    phi: [K, n_modes, M] modes of every frequency (as returned by spod);
    bins: retained frequencies (increasing); n_r: modes kept per frequency."""
    phi = np.asarray(phi)
    cols = [phi[k, j] for k in bins for j in range(n_r)]
    return np.stack(cols, axis=1).astype(np.complex128)


def mode_gram(Phi, weights):
    """Phi^* W Phi, the matrix inverted in eq. (coeffs)."""
    W = np.asarray(weights, dtype=np.float64)
    return Phi.conj().T @ (W[:, None] * Phi)


def projection_rhs(Phi, weights, q, mean):
    """Phi^* W Q' with Q' = Q - qbar 1^T (R15): the right-hand side of eq. (coeffs)."""
    W = np.asarray(weights, dtype=np.float64)
    qp = np.asarray(q) - np.asarray(mean)[:, None]
    return (W[:, None] * Phi).conj().T @ qp


def expansion_coefficients(q, mean, phi, weights, bins, n_r: int):
    """A = (Phi^* W Phi)^{-1} Phi^* W Q'  (eq. (coeffs)), an R x N_t complex
    matrix with R = len(bins) * n_r."""
    Phi = gather_modes(phi, bins, n_r)
    B = mode_gram(Phi, weights)
    C = projection_rhs(Phi, weights, q, mean)
    return np.linalg.solve(B, C)


def reconstruct(phi, A, mean, bins, n_r: int):
    """Q~ = Re(Phi_r A_r) + qbar 1^T  (eq. (SPODrec) with R16)."""
    Phi = gather_modes(phi, bins, n_r)
    return np.real(Phi @ np.asarray(A)) + np.asarray(mean, dtype=np.float64)[:, None]
