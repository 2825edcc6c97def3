"""Element-wise comparison rules between the HIP path and the FP64 oracle.

Each rule scales the tolerance the way the stage's rounding error scales:
  * Fourier blocks: the error of a length-N transform is proportional to the
    norm of the whole block, so element [k, l, m] is compared against
    ||qhat[:, l, m]|| (Parseval), not against its own magnitude;
  * Gram: entry (i, j) against sqrt(M_ii M_jj) (Cauchy-Schwarz);
  * eigenvalues: relative to themselves for every eigenvalue at or above a
    stated fraction theta of the largest one of the frequency (see the bars
    below); below it the bar is taken at theta * lambda_1;
  * modes: a mode separated from its neighbours is unique (phase convention):
    phase-aligned under W, then element-wise, and as the sine of the W-angle
    computed without cancellation; the modes of a cluster of close eigenvalues
    are compared as a subspace (largest principal angle under W).
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


# Eigenvalue bars.  The relative bar applies to every eigenvalue at or above
# theta * lambda_1(k); below that (eigenvalues the precision cannot resolve
# relatively: near-null ones, and the ones whose modes are not valid on the
# mixed path) the same bar is taken at theta * lambda_1(k), i.e. an absolute
# error of rtol * theta * lambda_1(k).
#   FP64 path : rtol 1e-10, theta 1e-5  (absolute floor 1e-15 lambda_1)
#   mixed path: rtol 1e-4,  theta 1e-6  (the mixed path's valid-mode threshold)
THETA_FP64 = 1e-5
THETA_MIXED = 1e-6


def _eig_bar(g, o, rtol, theta, what):
    top = np.abs(o[:, :1])
    scale = np.maximum(np.abs(o), theta * top)
    excess = np.abs(g - o) / np.maximum(rtol * scale, 1e-300)
    if excess.size and excess.max() > 1.0:
        k, j = np.unravel_index(excess.argmax(), excess.shape)
        raise AssertionError(
            f"{what} eigenvalue k={k} j={j}: gpu {g[k, j]!r} oracle {o[k, j]!r} "
            f"(rel {abs(g[k, j] - o[k, j]) / max(abs(o[k, j]), 1e-300):.2e}, "
            f"lambda_1 {o[k, 0]!r}, bar {rtol:.0e} x max(|l_j|, {theta:.0e} l_1))")


def worst_eig(lam_gpu, lam_ora, theta, n=None):
    """(k, j, plain relative error) of the worst eigenvalue at or above
    theta * lambda_1(k) among the leading n."""
    g, o = as_np(lam_gpu), as_np(lam_ora)
    if n is not None:
        g, o = g[:, :n], o[:, :n]
    rel = np.abs(g - o) / np.maximum(np.abs(o), 1e-300)
    rel = np.where(np.abs(o) >= theta * np.abs(o[:, :1]), rel, 0.0)
    k, j = np.unravel_index(rel.argmax(), rel.shape)
    return int(k), int(j), float(rel[k, j])


def check_eig(lam_gpu, lam_ora, rtol=1e-10, theta=THETA_FP64, n=None):
    """FP64 bar (see above).  Returns the plain maximum relative error over the
    eigenvalues the relative bar covers."""
    g, o = as_np(lam_gpu), as_np(lam_ora)
    if n is not None:
        g, o = g[:, :n], o[:, :n]
    _eig_bar(g, o, rtol, theta, "FP64")
    return worst_eig(g, o, theta)[2]


def check_eig_mixed(lam_gpu, lam_ora, M=None, n=5, rtol=1e-4, theta=THETA_MIXED):
    """Mixed-precision bar: 1e-4 relative on the leading n eigenvalues of every
    frequency at or above theta * lambda_1(k) (M is accepted for old callers and
    not used).  Returns the plain maximum relative error over those."""
    g, o = as_np(lam_gpu)[:, :n], as_np(lam_ora)[:, :n]
    _eig_bar(g, o, rtol, theta, "mixed")
    return worst_eig(g, o, theta)[2]


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


def clusters(lam, rel_gap):
    """Index ranges [a, b) of eigenvalues whose neighbours are closer than
    rel_gap * lambda_1 (lam sorted descending)."""
    lam = np.asarray(lam)
    out, a = [], 0
    for j in range(1, len(lam) + 1):
        if j == len(lam) or abs(lam[j - 1] - lam[j]) > rel_gap * abs(lam[0]):
            out.append((a, j))
            a = j
    return out


def subspace_sine(G, O, W):
    """Sine of the largest principal angle under W between span(G) and span(O)
    (columns), as the 2-norm of (I - P_O) Q_G for W-orthonormal bases."""
    sw = np.sqrt(np.asarray(W, dtype=np.float64))[:, None]
    qg, _ = np.linalg.qr(sw * G)
    qo, _ = np.linalg.qr(sw * O)
    r = qg - qo @ (qo.conj().T @ qg)
    return float(np.linalg.norm(r, 2))


def check_modes(phi_gpu, phi_ora, lam_ora, W, n_valid, sin_tol, elem_tol, rel_gap):
    """Compare valid modes.  A mode whose eigenvalue is separated from every
    other one by rel_gap * lambda_1 is unique (phase convention): it is compared
    as the sine of its W-angle and element-wise after phase alignment.  The
    modes of a cluster of closer eigenvalues are compared as a subspace: the
    largest principal angle under W between the GPU's and the oracle's span.
    A cluster that crosses the n_modes cut has no complete oracle basis and is
    not compared.  Returns (max sine, number of modes compared)."""
    pg, po, lo = as_np(phi_gpu), as_np(phi_ora), as_np(lam_ora)
    W = np.asarray(W)
    worst, count = 0.0, 0
    K, n, _ = po.shape
    for k in range(K):
        nv = min(n, int(n_valid[k]))
        for a, b in clusters(lo[k], rel_gap):
            if a >= nv:
                break
            if b > nv:
                continue
            if b - a == 1:
                j = a
                s = mode_sine(pg[k, j], po[k, j], W)
                assert s <= sin_tol, f"mode k={k} j={j}: sine {s:.2e} > {sin_tol:.1e}"
                c = np.vdot(pg[k, j], W * po[k, j])
                ph = c / abs(c) if abs(c) > 0 else 1.0
                e = np.max(np.abs(pg[k, j] * ph - po[k, j])) / max(np.max(np.abs(po[k, j])), 1e-300)
                assert e <= elem_tol, f"mode k={k} j={j}: element error {e:.2e} > {elem_tol:.1e}"
            else:
                s = subspace_sine(pg[k, a:b].T, po[k, a:b].T, W)
                assert s <= sin_tol, f"modes k={k} j={a}..{b - 1}: subspace sine {s:.2e} > {sin_tol:.1e}"
            worst = max(worst, s)
            count += b - a
    return worst, count


def check_invalid_modes_zero(phi_gpu, n_valid):
    pg = as_np(phi_gpu)
    for k in range(pg.shape[0]):
        assert np.all(pg[k, int(n_valid[k]):] == 0), f"invalid modes at k={k} are not zero"


# ---------------------------------------------------------------------------
# packed Fourier blocks (SPOD_QHAT_BFP20), written here from the layout that
# include/spod.h documents, independently of the library's kernels
# ---------------------------------------------------------------------------
PK_SB_DOFS, PK_SB_BYTES = 128, 656


def pk_row_bytes(M):
    return -(-M // PK_SB_DOFS) * PK_SB_BYTES


def unpack_qhat(buf, K, L, M):
    """Decode a packed qhat (bytes or uint8 array) to complex128 [K, L, M]."""
    b = np.frombuffer(as_np(buf).tobytes(), dtype=np.uint8)
    nsb = -(-M // PK_SB_DOFS)
    assert b.size == K * L * nsb * PK_SB_BYTES, (b.size, K, L, M)
    sb = b.reshape(K * L, nsb, PK_SB_BYTES)
    e = sb[:, :, :8].view(np.int8).astype(np.int64)                    # [rows, nsb, 8]
    grp = sb[:, :, 16:].reshape(K * L, nsb, 8, 80)
    h = grp[:, :, :, :64].copy().view("<i2").astype(np.int64)           # [rows, nsb, 8, 32]
    nib16 = grp[:, :, :, 64:].copy().view("<u2").astype(np.int64)       # [rows, nsb, 8, 8]
    nib = np.stack([(nib16 >> (4 * i)) & 15 for i in range(4)], axis=-1).reshape(h.shape)
    mant = h * 16 + nib
    scale = np.where(e == 127, np.nan, np.ldexp(1.0, np.clip(e, -1074, 1023)))
    v = mant * scale[..., None]                                          # [rows, nsb, 8, 32]
    v = v.reshape(K * L, nsb * 128, 2)
    out = (v[:, :, 0] + 1j * v[:, :, 1]).reshape(K, L, nsb * 128)
    return out[:, :, :M], out[:, :, M:], sb


def pack_qhat(qh):
    """Encode complex [K, L, M] values into the packed layout (round to nearest,
    exponent E with |v| 2^-E < 2^19 per group of 16 degrees of freedom)."""
    K, L, M = qh.shape
    nsb = -(-M // PK_SB_DOFS)
    pad = nsb * 128 - M
    z = np.pad(np.asarray(qh, np.complex128), ((0, 0), (0, 0), (0, pad))).reshape(K * L, nsb, 8, 16)
    v = np.stack([z.real, z.imag], axis=-1).reshape(K * L, nsb, 8, 32)
    mx = np.abs(v).max(axis=-1)
    ex = np.frexp(mx)[1]
    e = np.where(mx > 0, np.maximum(ex - 19, -128), -128).astype(np.int64)
    mant = np.clip(np.rint(np.ldexp(v, -e[..., None])), -524288, 524287).astype(np.int64)
    h = (mant >> 4).astype("<i2")
    nib = (mant & 15).reshape(K * L, nsb, 8, 8, 4)
    nib16 = (nib[..., 0] | (nib[..., 1] << 4) | (nib[..., 2] << 8) | (nib[..., 3] << 12)).astype("<u2")
    out = np.zeros((K * L, nsb, PK_SB_BYTES), dtype=np.uint8)
    out[:, :, :8] = e.astype(np.int8).view(np.uint8)
    grp = np.concatenate([h.view(np.uint8).reshape(K * L, nsb, 8, 64),
                          nib16.view(np.uint8).reshape(K * L, nsb, 8, 16)], axis=-1)
    out[:, :, 16:] = grp.reshape(K * L, nsb, 640)
    return out.reshape(-1)


def check_packed_format(sb, M):
    """Layout invariants of a packed qhat (the sb view from unpack_qhat):
    header bytes 8..15 zero, mantissas of every non-zero group normalised
    (largest magnitude in [2^18, 2^19]), degrees of freedom past M zero."""
    rows, nsb, _ = sb.shape
    assert not sb[:, :, 8:16].any(), "header bytes 8..15 must be zero"
    e = sb[:, :, :8].view(np.int8).astype(np.int64)
    grp = sb[:, :, 16:].reshape(rows, nsb, 8, 80)
    h = grp[:, :, :, :64].copy().view("<i2").astype(np.int64)
    nib16 = grp[:, :, :, 64:].copy().view("<u2").astype(np.int64)
    nib = np.stack([(nib16 >> (4 * i)) & 15 for i in range(4)], axis=-1).reshape(h.shape)
    mant = h * 16 + nib
    amax = np.abs(mant).max(axis=-1)
    live = (amax > 0) & (e != 127)
    assert np.all(amax[live] >= 2 ** 18) and np.all(amax[live] <= 2 ** 19), "mantissas not normalised"
    assert np.all(e[amax == 0] == -128), "zero groups must carry exponent -128"
    dofs = mant.reshape(rows, nsb * 128, 2)
    assert not dofs[:, M:].any(), "degrees of freedom past M must be zero"
