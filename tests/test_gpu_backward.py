"""Gradient of the SPOD path through spod_backward (MI355X only).

Compared against the FP64 CPU reference gradient (PyTorch autograd through
the oracle's definition of Sec. 2.3, tests/test_oracle_gradient.py pins it),
against the closed-form gradient of the total energy, and against central
differences of the GPU's own FP64 forward at full size.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.gradient import reference_gradient
from synth import fields

pytestmark = pytest.mark.gpu

# FP64 path: the eigenvector derivative divides by eigenvalue gaps, so the
# bound is relative to the largest gradient entry; the CPU reference uses
# LAPACK's eigh, the GPU its own Jacobi solver.
TOL_FP64 = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_11808_amd  # noqa: F401  (fails loudly when libspod.so is missing)
    yield


def _plan(p, precision="fp64", window=None):
    from paper_2309_11808_amd import Plan
    return Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, window=window, weights=p.weights,
                precision=precision)


def _separated_bins(lam, count, top=4, gap=1e-3, prefer=()):
    """Frequencies whose leading `top` eigenvalues are pairwise separated,
    |l_i - l_j| >= gap * max(l_i, l_j), so that the sum of the leading
    eigenvalues and the leading mode are differentiable there.  Bins in
    `prefer` come first; the rest are spread over the band."""
    good = []
    for k in range(lam.shape[0]):
        l = lam[k, :top]
        if l[-1] <= 0:
            continue
        d = np.abs(l[:, None] - l[None, :]) - gap * np.maximum(l[:, None], l[None, :])
        d[np.diag_indices(len(l))] = 1.0
        if d.min() >= 0:
            good.append(k)
    assert len(good) >= 1
    first = [k for k in prefer if k in good][:count]
    rest = [k for k in good if k not in first]
    n = min(count - len(first), len(rest))
    pick = np.unique(np.linspace(0, len(rest) - 1, n).round().astype(int)) if n > 0 else []
    return sorted(first + [rest[i] for i in pick])


def _probes(nb, M, W, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal((nb, M)) + 1j * rng.standard_normal((nb, M))
    p /= np.sqrt(np.sum(W * np.abs(p) ** 2, axis=1, keepdims=True))     # W-unit
    return torch.as_tensor(p)


def _make_loss(W, probes, n_lam=3, phase=False):
    """E = sum_k sum_{j<n_lam} lambda_j(k) + sum_k |<p_k, phi_1(k)>_W|^2
    (+ sum of Re(phi_1(k))[:4]^2, which depends on the phase convention)."""
    def loss(lam_s, phi_s):
        dev = phi_s.device
        Wt = torch.as_tensor(W, device=dev, dtype=torch.float64)
        pr = probes.to(dev)
        f1 = phi_s[:, 0].to(torch.complex128)
        e = lam_s[:, :n_lam].sum() + (torch.abs((torch.conj(pr) * Wt * f1).sum(-1)) ** 2).sum()
        if phase:
            e = e + (f1[:, :4].real ** 2).sum()
        return e
    return loss


def _reference(p, loss, bins, window, n_modes):
    def full(lam, phi):
        if bins is None:
            return loss(lam, phi)
        idx = torch.as_tensor(bins)
        return loss(lam[idx], phi[idx])
    q64 = p.q.cpu().numpy().astype(np.float64)
    g, _ = reference_gradient(q64, p.nfft, p.noverlap, full, window=window, weights=p.weights,
                              n_modes=n_modes)
    return g


def _gpu_grad(p, loss, bins, window, n_modes, precision="fp64", keep_qhat=False):
    from paper_2309_11808_amd import spod
    plan = _plan(p, precision, window)
    q = p.q.cuda().requires_grad_(True)
    lam_s, phi_s = spod(q, plan, n_modes=n_modes, bins=bins, keep_qhat=keep_qhat)
    E = loss(lam_s, phi_s)
    E.backward()
    torch.cuda.synchronize()
    g = q.grad.detach().cpu().numpy().astype(np.float64)
    plan.close()
    return g


def _rel(g, ref):
    return float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))


def _planted_case():
    p = fields.planted(sigma=0.1, seed=1)
    ref = O.spod(p.q.numpy(), p.nfft, p.noverlap, weights=p.weights, n_modes=1)
    return p, ref["lam"]


# ---------------------------------------------------------------------------
# 32 x 32 planted workload (N_t = 1024, N_f = 128, 15 blocks, 65 bins)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("selected,keep_qhat,phase", [
    (True, False, False),      # the loss's 8 bins; blocks recomputed at those bins
    (True, True, False),       # 8 bins, forward's blocks kept
    (False, False, False),     # every bin, recomputed
    (False, True, True),       # every bin, kept and overwritten in place; phase-dependent loss
])
def test_gradient_planted_fp64(selected, keep_qhat, phase):
    p, lam = _planted_case()
    F8 = _separated_bins(lam, 8, prefer=p.meta["bins"])
    W = p.weights
    probes = _probes(len(F8), p.M, W, seed=7)
    if selected:
        bins, loss = F8, _make_loss(W, probes, phase=phase)
    else:
        # the same loss written on full-size outputs
        inner = _make_loss(W, probes, phase=phase)
        idx = torch.as_tensor(F8)

        def loss(lam_a, phi_a):
            i = idx.to(lam_a.device)
            return inner(lam_a.index_select(0, i), phi_a.index_select(0, i))
        bins = None
    ref = _reference(p, loss, bins, None, 5)
    g = _gpu_grad(p, loss, bins, None, 5, keep_qhat=keep_qhat)
    err = _rel(g, ref)
    print(f"planted fp64 selected={selected} keep={keep_qhat} phase={phase}: {err:.2e}")
    assert err <= TOL_FP64, f"gradient error {err:.2e}"


# ragged tiles, overlaps of 0, 1/2 and 3/4, windows with 2, 3 and N non-zero
# DFT bins, float32 and float64 inputs
BWD_CASES = [
    # nfft, noverlap, M, extra samples, input dtype, window
    (16, 8, 37, 3, torch.float64, "hann"),
    (32, 0, 45, 7, torch.float64, "hamming"),
    (64, 48, 33, 5, torch.float64, "hann"),
    (128, 64, 70, 0, torch.float64, "random"),
    (256, 128, 41, 13, torch.float32, "hann"),
    (512, 256, 21, 100, torch.float64, "hann"),
    (1024, 512, 19, 17, torch.float64, "hamming"),
]


def _window(kind, nfft, seed):
    if kind == "hann":
        return None
    if kind == "hamming":
        return 0.54 - 0.46 * np.cos(2 * np.pi * np.arange(nfft) / nfft)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.1, 1.0, nfft)


@pytest.mark.parametrize("nfft,nov,M,extra,dtype,wkind", BWD_CASES)
def test_gradient_variants_fp64(nfft, nov, M, extra, dtype, wkind):
    L = 6 + (nfft % 5)
    nt = (L - 1) * (nfft - nov) + nfft + extra
    p = fields.random_rows(M, nt, nfft, nov, seed=nfft + M, dtype=dtype, offset=2.0)
    window = _window(wkind, nfft, nfft)
    q64 = p.q.numpy().astype(np.float64)
    lam = O.spod(q64, nfft, nov, window=window, weights=p.weights, n_modes=1)["lam"]
    bins = _separated_bins(lam, 4)
    n_modes = 3
    loss = _make_loss(p.weights, _probes(len(bins), M, p.weights, seed=3), n_lam=3)
    ref = _reference(p, loss, bins, window, n_modes)
    g = _gpu_grad(p, loss, bins, window, n_modes)
    # float32 inputs: g_q is returned in float32
    tol = TOL_FP64 if dtype == torch.float64 else 2e-7
    err = _rel(g, ref)
    print(f"variant nfft={nfft} nov={nov} M={M} {wkind}: {err:.2e}")
    assert err <= tol, f"gradient error {err:.2e}"


# block lengths other than a power of two up to 1024 (the mixed-radix
# transform and its adjoint; the forward's blocks are kept): radices 2, 3, 5
# and the paper's 73, a power of two above 1024, hops of 1/2, 1/4 and 2/3 of N_f
GEN_CASES = [
    # nfft, noverlap, M, extra samples, input dtype, window, all bins
    (24, 12, 37, 5, torch.float64, "hann", False),
    (100, 25, 29, 3, torch.float64, "random", True),
    (146, 73, 41, 0, torch.float32, "hann", False),
    (150, 50, 23, 9, torch.float64, "hamming", True),
    (1536, 768, 13, 11, torch.float64, "hann", False),
    (2190, 1095, 9, 4, torch.float64, "hamming", False),
    (8760, 4380, 6, 7, torch.float64, "hann", False),       # the paper's one-year hourly block
]


@pytest.mark.parametrize("nfft,nov,M,extra,dtype,wkind,all_bins", GEN_CASES)
def test_gradient_general_lengths_fp64(nfft, nov, M, extra, dtype, wkind, all_bins):
    L = 4 + (nfft % 3)
    nt = (L - 1) * (nfft - nov) + nfft + extra
    p = fields.random_rows(M, nt, nfft, nov, seed=nfft + M, dtype=dtype, offset=2.0)
    window = _window(wkind, nfft, nfft)
    q64 = p.q.numpy().astype(np.float64)
    lam = O.spod(q64, nfft, nov, window=window, weights=p.weights, n_modes=1)["lam"]
    bins = None if all_bins else _separated_bins(lam, 4)
    n_modes = 2
    nb = lam.shape[0] if all_bins else len(bins)
    loss = _make_loss(p.weights, _probes(nb, M, p.weights, seed=5), n_lam=2)
    ref = _reference(p, loss, bins, window, n_modes)
    g = _gpu_grad(p, loss, bins, window, n_modes)
    tol = TOL_FP64 if dtype == torch.float64 else 2e-7
    err = _rel(g, ref)
    print(f"general nfft={nfft} nov={nov} M={M} {wkind} all_bins={all_bins}: {err:.2e}")
    assert err <= tol, f"gradient error {err:.2e}"


def test_backward_general_length_needs_blocks_and_a_selection():
    from paper_2309_11808_amd import SpodError
    p = fields.random_rows(12, 3 * 1536 + 5, 1536, 768, seed=2)   # K = 769 > 513
    plan = _plan(p)
    q = p.q.cuda()
    out = _forward(plan, q, 1)
    g_lam = torch.ones(2, plan.nblocks, dtype=torch.float64, device="cuda")
    # no stored blocks: the mixed-radix transform has no bin selection to recompute from
    with pytest.raises(SpodError) as ei:
        plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, bins=[3, 9])
    assert ei.value.status == -2
    # every bin (769 > 513)
    with pytest.raises(SpodError) as ei:
        plan.backward(q, out["lam"], out["psi"], g_lam=torch.ones_like(out["lam"]),
                      qhat=out["qhat"])
    assert ei.value.status == -2
    # a selection with the stored blocks works
    g = plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, bins=[3, 9], qhat=out["qhat"])
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    plan.close()


# ---------------------------------------------------------------------------
# mixed-precision plans (complex64 blocks, FP32 transforms)
# ---------------------------------------------------------------------------
# the mixed plans' eigenvector error (about 1e-6 relative to lambda_1 from the
# split Gram) is amplified by lambda_1 / gap <= 100 at the loss's bins (gap
# 1e-2); measured 3e-6 to 1e-5
MIXED_TOL = {"fp32": 1e-4, "bf16x4": 1e-4, "fp16x4": 1e-4}


@pytest.mark.parametrize("precision", ["fp32", "bf16x4", "fp16x4"])
def test_gradient_planted_mixed(precision):
    p, lam = _planted_case()
    p32 = fields.Problem(q=p.q.to(torch.float32), weights=p.weights, nspace=p.nspace,
                         nvar=p.nvar, nfft=p.nfft, noverlap=p.noverlap)
    F8 = _separated_bins(lam, 8, gap=1e-2, prefer=p.meta["bins"])
    loss = _make_loss(p.weights, _probes(len(F8), p.M, p.weights, seed=7))
    ref = _reference(p32, loss, F8, None, 5)
    g = _gpu_grad(p32, loss, F8, None, 5, precision=precision)
    err = _rel(g, ref)
    print(f"planted {precision}: {err:.2e}")
    assert err <= MIXED_TOL[precision], f"{precision} gradient error {err:.2e}"


# ---------------------------------------------------------------------------
# the raw entry point: partial gradients, stored vs recomputed blocks, errors
# ---------------------------------------------------------------------------
def _forward(plan, q, n_modes):
    out = plan.forward(q, n_modes)
    torch.cuda.synchronize()
    return out


def test_backward_lam_only_and_phi_only_add_up():
    p, lam = _planted_case()
    plan = _plan(p)
    q = p.q.cuda()
    out = _forward(plan, q, 5)
    bins = _separated_bins(lam, 6, prefer=p.meta["bins"])
    nb, L, K = len(bins), plan.nblocks, plan.nfreq
    rng = np.random.Generator(np.random.PCG64(11))
    g_lam = torch.as_tensor(rng.standard_normal((nb, L))).cuda()
    g_phi = torch.as_tensor(rng.standard_normal((nb, 5, p.M)) +
                            1j * rng.standard_normal((nb, 5, p.M))).cuda()
    a = plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, n_modes=5, bins=bins)
    b = plan.backward(q, out["lam"], out["psi"], g_phi=g_phi, n_modes=5, bins=bins)
    c = plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, g_phi=g_phi, n_modes=5, bins=bins)
    # the same with the forward's blocks instead of recomputing them
    d = plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, g_phi=g_phi, n_modes=5, bins=bins,
                      qhat=out["qhat"])
    torch.cuda.synchronize()
    a, b, c, d = (x.cpu().numpy() for x in (a, b, c, d))
    assert _rel(a + b, c) <= 1e-13
    # recomputed blocks come from the same transform kernel: identical results
    assert np.array_equal(c, d)

    # dense call with zero rows outside the selection gives the same gradient
    g_lam_f = torch.zeros(K, L, dtype=torch.float64, device="cuda")
    g_phi_f = torch.zeros(K, 5, p.M, dtype=torch.complex128, device="cuda")
    idx = torch.as_tensor(bins, device="cuda")
    g_lam_f[idx] = g_lam
    g_phi_f[idx] = g_phi
    e = plan.backward(q, out["lam"], out["psi"], g_lam=g_lam_f, g_phi=g_phi_f, n_modes=5)
    torch.cuda.synchronize()
    assert _rel(e.cpu().numpy(), c) <= 1e-12
    plan.close()


def test_backward_rejects_bad_arguments():
    from paper_2309_11808_amd import SpodError
    p, _ = _planted_case()
    plan = _plan(p)
    q = p.q.cuda()
    out = _forward(plan, q, 5)
    g_lam = torch.ones(2, plan.nblocks, dtype=torch.float64, device="cuda")
    for bad in ([3, 3], [5, 2], [-1, 4], [4, plan.nfreq]):
        with pytest.raises(SpodError) as ei:
            plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, bins=bad)
        assert ei.value.status == -1
    # g_qhat may alias qhat only without a selection
    with pytest.raises(SpodError) as ei:
        plan.backward(q, out["lam"], out["psi"], g_lam=g_lam, bins=[1, 2], qhat=out["qhat"],
                      g_qhat=out["qhat"][:2])
    assert ei.value.status == -1
    plan.close()
    # a hop of 7/8 nfft has no in-register overlap-add
    p2 = fields.random_rows(16, 64 * 7 + 8, 64, 8, seed=1)
    plan2 = _plan(p2)
    q2 = p2.q.cuda()
    out2 = _forward(plan2, q2, 1)
    with pytest.raises(SpodError) as ei:
        plan2.backward(q2, out2["lam"], out2["psi"],
                       g_lam=torch.ones_like(out2["lam"]))
    assert ei.value.status == -2
    plan2.close()


# ---------------------------------------------------------------------------
# the differentiation workload at full size: the 256 x 128 x 3 jet-like field,
# N_t = 4096, N_f = 256, 31 blocks, 129 bins (FP64 path)
# ---------------------------------------------------------------------------
def _energy_gradient_rows(q_rows, W_rows, nfft, nov, window):
    """dE/dq for E = sum_k c_k tr(M_k) (c_k = 2 on interior bins), per row:
    2 kappa^2 N_f W_m (sum_{l: t in block l} w[t - l s]^2 x[t] - mean_t(...))."""
    M, nt = q_rows.shape
    L = O.block_count(nt, nfft, nov)
    s = nfft - nov
    kappa2 = 1.0 / ((L - 1) * np.sum(window ** 2))
    x = q_rows - q_rows.mean(axis=1, keepdims=True)
    acc = np.zeros_like(x)
    for ell in range(L):
        acc[:, ell * s: ell * s + nfft] += (window ** 2)[None, :] * x[:, ell * s: ell * s + nfft]
    acc -= acc.sum(axis=1, keepdims=True) / nt
    return 2 * kappa2 * nfft * W_rows[:, None] * acc


@pytest.fixture(scope="module")
def jet64():
    p = fields.jet_like(seed=2, device="cuda", dtype=torch.float32)
    p.q = p.q.double()
    torch.cuda.empty_cache()
    return p, p.q


def test_energy_gradient_full_size(jet64):
    p, q = jet64
    plan = _plan(p)
    out = _forward(plan, q, 1)
    K, L = plan.nfreq, plan.nblocks
    c = torch.full((K, L), 2.0, dtype=torch.float64, device="cuda")
    c[0] = 1.0
    c[-1] = 1.0
    g = plan.backward(q, out["lam"], out["psi"], g_lam=c)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(5))
    rows = np.sort(rng.choice(p.M, 64, replace=False))
    rows = np.concatenate([rows, [0, p.M - 1]])
    ref = _energy_gradient_rows(q[rows].cpu().numpy(), p.weights[rows], p.nfft, p.noverlap,
                                O.hann_periodic(p.nfft))
    err = _rel(g[rows].cpu().numpy(), ref)
    print(f"energy gradient full size: {err:.2e}")
    assert err <= 1e-12, f"energy gradient error {err:.2e}"
    plan.close()


def test_directional_derivative_full_size(jet64):
    """<g, v> against (E(q + h v) - E(q - h v)) / 2h with the FP64 GPU forward,
    for the loss on 8 separated bins (3 eigenvalues + probe of the leading mode)."""
    from paper_2309_11808_amd import spod
    p, q = jet64
    plan = _plan(p)
    out = _forward(plan, q, 5)
    lam = out["lam"].cpu().numpy()
    del out
    F8 = _separated_bins(lam, 8)
    loss = _make_loss(p.weights, _probes(len(F8), p.M, p.weights, seed=9))
    qg = q.clone().requires_grad_(True)
    lam_s, phi_s = spod(qg, plan, n_modes=5, bins=F8)
    E = loss(lam_s, phi_s)
    E.backward()
    g = qg.grad
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    v = torch.randn(q.shape, generator=gen, dtype=torch.float64, device="cuda")
    dd = float((g * v).sum())
    h = 1e-5
    with torch.no_grad():
        ep = float(loss(*spod(q + h * v, plan, n_modes=5, bins=F8)))
        em = float(loss(*spod(q - h * v, plan, n_modes=5, bins=F8)))
    fd = (ep - em) / (2 * h)
    print(f"directional derivative: fd {fd!r} adjoint {dd!r} rel {abs(fd - dd) / abs(dd):.2e}")
    assert abs(fd - dd) <= 1e-5 * abs(dd), (fd, dd)
    plan.close()


def test_central_differences_64_entries_full_size(jet64):
    """dE/dq at 64 seeded entries against (E(q + h e) - E(q - h e)) / 2h,
    h = 1e-4, with the FP64 GPU forward, for the 8-bin loss."""
    from paper_2309_11808_amd import spod
    p, q = jet64
    plan = _plan(p)
    out = _forward(plan, q, 5)
    lam = out["lam"].cpu().numpy()
    del out
    F8 = _separated_bins(lam, 8)
    loss = _make_loss(p.weights, _probes(len(F8), p.M, p.weights, seed=9))
    qg = q.clone().requires_grad_(True)
    lam_s, phi_s = spod(qg, plan, n_modes=5, bins=F8)
    loss(lam_s, phi_s).backward()
    g = qg.grad.detach()
    rng = np.random.Generator(np.random.PCG64(64))
    ent = rng.choice(q.numel(), 64, replace=False)
    h = 1e-4
    qp = q.clone()
    flat = qp.view(-1)
    fd = np.empty(64)
    with torch.no_grad():
        for n, e in enumerate(ent):
            x0 = float(flat[e])
            flat[e] = x0 + h
            ep = float(loss(*spod(qp, plan, n_modes=5, bins=F8)))
            flat[e] = x0 - h
            em = float(loss(*spod(qp, plan, n_modes=5, bins=F8)))
            flat[e] = x0
            fd[n] = (ep - em) / (2 * h)
    with torch.no_grad():
        E0 = float(loss(*spod(q, plan, n_modes=5, bins=F8)))
    ga = g.view(-1)[torch.as_tensor(ent, device="cuda")].cpu().numpy()
    err = np.abs(fd - ga)
    # a central difference resolves dE only to the rounding of E itself,
    # about eps |E| / h, besides its O(h^2) truncation
    noise = 10.0 * np.finfo(np.float64).eps * abs(E0) / h
    agg = float(np.linalg.norm(fd - ga) / np.linalg.norm(ga))
    print(f"central differences: E {E0:.4e}, rounding floor {noise:.1e}, max |fd - g| "
          f"{err.max():.2e}, max |g| {np.abs(ga).max():.2e}, aggregate rel {agg:.2e}")
    assert np.all(err <= 1e-4 * np.abs(ga) + noise)
    assert agg <= 1e-4
    plan.close()
