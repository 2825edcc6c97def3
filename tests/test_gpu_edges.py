"""Edge cases of the whole path (MI355X only): tiny M, the fewest blocks,
a one-bin backward with every mode in the loss, a one-problem batch."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.gradient import reference_gradient
from synth import fields
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_11808_amd  # noqa: F401
    yield


def _plan(p, precision="fp64", window=None):
    from paper_2309_11808_amd import Plan
    return Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, window=window, weights=p.weights,
                precision=precision)


@pytest.mark.parametrize("M,nfft,nov,L", [(1, 16, 8, 5), (2, 32, 16, 2), (3, 64, 0, 3),
                                          (17, 128, 64, 2)])
def test_tiny_problems_end_to_end(M, nfft, nov, L):
    nt = (L - 1) * (nfft - nov) + nfft + 3
    p = fields.random_rows(M, nt, nfft, nov, seed=M + nfft, dtype=torch.float64, offset=1.0)
    ref = O.spod(p.q.numpy(), nfft, nov, weights=p.weights, n_modes=min(5, L))
    plan = _plan(p)
    assert plan.nblocks == L
    out = plan.forward(p.q.cuda(), n_modes=min(5, L))
    torch.cuda.synchronize()
    PT.check_eig(out["lam"], ref["lam"], rtol=1e-10)
    np.testing.assert_array_equal(out["n_valid"].cpu().numpy(), ref["n_valid"])
    PT.check_invalid_modes_zero(out["phi"], out["n_valid"].cpu().numpy())
    PT.check_modes(out["phi"], ref["phi"], ref["lam"], p.weights, ref["n_valid"], sin_tol=1e-8,
                   elem_tol=1e-6, rel_gap=1e-6)
    plan.close()


def _best_separated_bin(lam):
    """The bin whose whole spectrum is best separated (relative to lambda_1)."""
    best, k_best = -1.0, 1
    for k in range(1, lam.shape[0] - 1):
        l = np.sort(lam[k])[::-1]
        if l[-1] <= 0:
            continue
        g = np.min(-np.diff(l)) / l[0]
        if g > best:
            best, k_best = g, k
    return k_best, best


def test_backward_one_bin_every_mode():
    """Loss on all L eigenvalues and all L modes of one frequency."""
    from paper_2309_11808_amd import spod
    M, nfft, nov, L = 64, 32, 16, 7
    nt = (L - 1) * (nfft - nov) + nfft
    p = fields.random_rows(M, nt, nfft, nov, seed=71, dtype=torch.float64)
    lam = O.spod(p.q.numpy(), nfft, nov, weights=p.weights, n_modes=1)["lam"]
    k, gap = _best_separated_bin(lam)
    assert gap > 1e-3
    rng = np.random.Generator(np.random.PCG64(72))
    probes = torch.as_tensor(rng.standard_normal((L, M)) + 1j * rng.standard_normal((L, M)))
    W = p.weights

    def loss(lam_s, phi_s):
        Wt = torch.as_tensor(W, device=phi_s.device)
        inner = (torch.conj(probes.to(phi_s.device)) * Wt * phi_s[0]).sum(-1)
        return (lam_s[0] * torch.arange(1, L + 1, device=lam_s.device)).sum() + (inner.abs() ** 2).sum()

    g_ref, _ = reference_gradient(p.q.numpy(), nfft, nov, lambda a, b: loss(a[[k]], b[[k]]),
                                  weights=W, n_modes=L)
    plan = _plan(p)
    q = p.q.cuda().requires_grad_(True)
    lam_s, phi_s = spod(q, plan, n_modes=L, bins=[k])
    loss(lam_s, phi_s).backward()
    torch.cuda.synchronize()
    g = q.grad.cpu().numpy()
    err = float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref)))
    print(f"one bin (k={k}, gap {gap:.1e}), all modes: {err:.2e}")
    # eigenvector sensitivity ~ eps / gap
    assert err <= max(1e-10, 1e-13 / gap)
    plan.close()


def test_batch_of_one_with_clamped_modes():
    from paper_2309_11808_amd import Batch, Plan
    p = fields.random_rows(301, 40 * 16 + 16, 32, 16, seed=5, dtype=torch.float32)
    q = p.q.cuda()
    b = Batch([{"nspace": p.nspace, "nvar": 1, "nt": p.nt, "nfft": 32, "noverlap": 16,
                "weights": p.weights}], precision="fp32", n_modes=80)
    assert b.items[0].n_modes == b.items[0].nblocks
    res = b.forward([q])[0]
    plan = Plan(p.nspace, 1, p.nt, 32, 16, weights=p.weights, precision="fp32")
    out = plan.forward(q, n_modes=plan.nblocks)
    torch.cuda.synchronize()
    for key in ("lam", "psi", "phi", "mean", "n_valid"):
        assert torch.equal(res[key], out[key]), key
    plan.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x4", "fp16x4+bfp20"])
@pytest.mark.parametrize("bad", ["nan", "inf"])
def test_non_finite_data_is_reported(precision, bad):
    """One NaN row or one infinite sample: every frequency's Gram is then not
    finite.  The eigensolver must say so (info = SPOD_INFO_NONFINITE) instead of
    reporting convergence, write every eigenvalue and eigenvector entry (as NaN:
    the outputs are pre-filled with a finite sentinel), count no valid mode, and
    store zero modes.  The out-of-core call returns SPOD_ERR_NUMERIC."""
    from paper_2309_11808_amd import OutOfCore, SpodError, _native as N
    p = fields.random_rows(40, 600, 64, 32, seed=5, dtype=torch.float64)
    q = p.q.clone()
    if bad == "nan":
        q[7, :] = float("nan")
    else:
        q[11, 100] = float("inf")
    from paper_2309_11808_amd import Plan
    packed = precision.endswith("+bfp20")
    precision = precision.split("+")[0]
    plan = Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, weights=p.weights, precision=precision,
                options={"qhat_format": "bfp20"} if packed else None)
    qdev = q.to(torch.float64 if precision == "fp64" else torch.float32).cuda()
    K, L = plan.nfreq, plan.nblocks
    qhat, mean = plan.blocks_fft(qdev)
    gram = plan.csd(qhat)
    lam = torch.full((K, L), 12345.0, dtype=torch.float64, device="cuda")
    psi = torch.full((K, L, L), 777.0 + 1j, dtype=torch.complex128, device="cuda")
    info = torch.full((K,), 99, dtype=torch.int32, device="cuda")
    plan.eig(gram, lam=lam, psi=psi, info=info)
    phi = torch.full((K, 5, plan.M), 3.0, dtype=plan.cdtype, device="cuda")
    n_valid = torch.full((K,), 99, dtype=torch.int32, device="cuda")
    plan.modes(qhat, lam, psi, 5, phi=phi, n_valid=n_valid)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == N.SPOD_INFO_NONFINITE).all(), info
    assert torch.isnan(lam).all() and torch.isnan(psi.real).all() and torch.isnan(psi.imag).all()
    assert (n_valid.cpu().numpy() == 0).all()
    assert (phi == 0).all()
    # the synchronous out-of-core call reports it as a status
    o = OutOfCore(plan, dtype=qdev.dtype, chunk_rows=256, n_modes=3, resident=0)
    with pytest.raises(SpodError) as ei:
        o.forward(q=qdev.cpu())
    assert ei.value.status == N.SPOD_ERR_NUMERIC
    o.close()
    plan.close()


def test_finite_data_next_to_non_finite_plan_is_unaffected():
    """A plan that saw non-finite data keeps working on finite data."""
    p = fields.random_rows(40, 600, 64, 32, seed=6, dtype=torch.float64)
    plan = _plan(p)
    q = p.q.clone()
    q[3, 5] = float("nan")
    plan.forward(q.cuda(), n_modes=3)
    out = plan.forward(p.q.cuda(), n_modes=3)
    torch.cuda.synchronize()
    ref = O.spod(p.q.numpy(), p.nfft, p.noverlap, weights=p.weights, n_modes=3)
    assert int(out["info"].min()) > 0
    PT.check_eig(out["lam"], ref["lam"], rtol=1e-10)
    plan.close()
