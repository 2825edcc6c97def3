"""Element-wise comparison rules between the HIP path and the FP64 oracle.

Each rule scales the tolerance the way the stage's rounding error scales:
  * Fourier blocks: the error of a length-N transform is proportional to the
    norm of the whole block, so element [k, l, m] is compared against
    ||qhat[:, l, m]|| (Parseval), not against its own magnitude;
  * Gram: entry (i, j) against sqrt(M_ii M_jj) (Cauchy-Schwarz);
  * eigenvalues: relative to themselves plus a floor relative to the largest
    eigenvalue of the frequency (an FP64 Gram resolves lambda_j only to about
    eps * lambda_1);
  * modes: only where the eigenvalue is separated from its neighbours (else
    the mode is not unique); phase-aligned under W, then element-wise, and as
    the sine of the W-angle computed without cancellation.
"""
from __future__ import annotations

import numpy as np


def as_np(t):
    try:
        import torch
        if isinstance(t, torch.Tensor):
            return t.detach().cpu().numpy()
    except ImportError:
        pass
    return np.asarray(t)


def check_qhat(gpu, ora, rtol, what="qhat"):
    gpu, ora = as_np(gpu), as_np(ora)
    assert gpu.shape == ora.shape, (gpu.shape, ora.shape)
    scale = np.sqrt(np.sum(np.abs(ora) ** 2, axis=0, keepdims=True))       # [1, L, M]
    floor = 1e-300 + 1e-6 * scale.max()
    err = np.abs(gpu - ora) / np.maximum(scale, floor)
    worst = float(err.max()) if err.size else 0.0
    assert worst <= rtol, f"{what}: max scaled error {worst:.3e} > {rtol:.1e} at {np.unravel_index(err.argmax(), err.shape)}"
    return worst


def check_gram(gpu, ora, rtol):
    gpu, ora = as_np(gpu), as_np(ora)
    d = np.sqrt(np.abs(np.real(np.diagonal(ora, axis1=1, axis2=2))))      # [K, L]
    scale = d[:, :, None] * d[:, None, :]
    floor = 1e-300 + 1e-12 * scale.max()
    err = np.abs(gpu - ora) / np.maximum(scale, floor)
    worst = float(err.max())
    assert worst <= rtol, f"gram: max scaled error {worst:.3e} > {rtol:.1e} at {np.unravel_index(err.argmax(), err.shape)}"
    return worst


def eig_errors(lam_gpu, lam_ora, n=None):
    """Relative eigenvalue errors |dl_j| / |l_j| for the leading n per frequency."""
    g, o = as_np(lam_gpu), as_np(lam_ora)
    if n is not None:
        g, o = g[:, :n], o[:, :n]
    return np.abs(g - o) / np.maximum(np.abs(o), 1e-300)


def check_eig(lam_gpu, lam_ora, rtol, floor_rel=1e-13, n=None):
    g, o = as_np(lam_gpu), as_np(lam_ora)
    if n is not None:
        g, o = g[:, :n], o[:, :n]
    top = np.abs(o[:, :1])
    tol = rtol * np.abs(o) + floor_rel * top + 1e-15 * np.abs(o).max()
    bad = np.abs(g - o) > tol
    if bad.any():
        k, j = np.argwhere(bad)[0]
        raise AssertionError(f"eigenvalue k={k} j={j}: gpu {g[k, j]!r} oracle {o[k, j]!r} "
                             f"(rel {abs(g[k, j] - o[k, j]) / max(abs(o[k, j]), 1e-300):.2e})")
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-300)))


def check_eig_mixed(lam_gpu, lam_ora, M, n=5, rtol=1e-4):
    """Mixed-precision eigenvalue bar: |dl_j| <= rtol * l_j + 2^-24 sqrt(32/M) l_1(k).

    The second term is the floor set by FP32 rounding of the 32-product MFMA
    partial sums: each rounding is about 2^-24 of a partial sum, the M/32 of
    them average out, and their projection onto an eigenvalue far below
    l_1(k) is a fixed fraction of l_1(k).  At M ~ 1e6 it is ~3e-10 l_1.
    Returns the plain maximum relative error for reporting."""
    g, o = as_np(lam_gpu)[:, :n], as_np(lam_ora)[:, :n]
    floor = 2.0 ** -24 * np.sqrt(32.0 / M) * np.abs(o[:, :1])
    bad = np.abs(g - o) > rtol * np.abs(o) + floor
    if bad.any():
        k, j = np.argwhere(bad)[0]
        raise AssertionError(f"mixed eigenvalue k={k} j={j}: gpu {g[k, j]!r} oracle {o[k, j]!r} "
                             f"l1 {o[k, 0]!r}")
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-300)))


def separated(lam, j, rel_gap):
    """True when lam[j] is separated from every other eigenvalue by rel_gap * lam[0]."""
    lam = np.asarray(lam)
    others = np.delete(lam, j)
    return lam[0] > 0 and np.min(np.abs(others - lam[j])) > rel_gap * abs(lam[0])


def mode_sine(phi_g, phi_o, W):
    """sin of the W-angle between two vectors, as ||(I - P_o) phi_g||_W / ||phi_g||_W."""
    no = np.sqrt(np.real(np.vdot(phi_o, W * phi_o)))
    u = phi_o / no
    c = np.vdot(u, W * phi_g)
    r = phi_g - u * c
    ng = np.sqrt(np.real(np.vdot(phi_g, W * phi_g)))
    return float(np.sqrt(np.real(np.vdot(r, W * r))) / max(ng, 1e-300))


def check_modes(phi_gpu, phi_ora, lam_ora, W, n_valid, sin_tol, elem_tol, rel_gap):
    """Compare valid, separated modes.  Returns (max sine, number compared)."""
    pg, po, lo = as_np(phi_gpu), as_np(phi_ora), as_np(lam_ora)
    W = np.asarray(W)
    worst, count = 0.0, 0
    K, n, _ = po.shape
    for k in range(K):
        for j in range(min(n, int(n_valid[k]))):
            if not separated(lo[k], j, rel_gap):
                continue
            s = mode_sine(pg[k, j], po[k, j], W)
            assert s <= sin_tol, f"mode k={k} j={j}: sine {s:.2e} > {sin_tol:.1e}"
            c = np.vdot(pg[k, j], W * po[k, j])
            ph = c / abs(c) if abs(c) > 0 else 1.0
            e = np.max(np.abs(pg[k, j] * ph - po[k, j])) / max(np.max(np.abs(po[k, j])), 1e-300)
            assert e <= elem_tol, f"mode k={k} j={j}: element error {e:.2e} > {elem_tol:.1e}"
            worst = max(worst, s)
            count += 1
    return worst, count


def check_invalid_modes_zero(phi_gpu, n_valid):
    pg = as_np(phi_gpu)
    for k in range(pg.shape[0]):
        assert np.all(pg[k, int(n_valid[k]):] == 0), f"invalid modes at k={k} are not zero"
