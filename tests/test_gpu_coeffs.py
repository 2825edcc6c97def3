"""Expansion coefficients and reconstruction (spod_coeffs, spod_reconstruct),
MI355X only.

Two kinds of checks against the FP64 oracle (oracle/coeffs.py):
  * the kernels alone: the GPU step is fed the oracle's own modes and mean (or
    the oracle's coefficients), so its error is the kernels' rounding only;
  * end to end: the GPU forward pass and coefficients against the oracle's
    forward pass and coefficients.
Shapes span several 64-wide tiles with ragged edges in M, N_t and R.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import coeffs as OC
from synth import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_11808_amd  # noqa: F401
    yield


def _plan(p, precision):
    from paper_2309_11808_amd import Plan
    return Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, weights=p.weights, precision=precision)


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x) - ref)) / np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def rows_case():
    # M = 1500 (23 tiles + 28), N_t = 712 (11 tiles + 8), 21 blocks, 33 bins
    p = fields.random_rows(1500, 21 * 32 + 40, 64, 32, seed=31, offset=0.7, dtype=torch.float64)
    ref = O.spod(p.q.numpy(), 64, 32, weights=p.weights, n_modes=5)
    return p, ref


# R = 24 (one tile), 100 (two tiles, ragged), 165 (three tiles)
SELECTIONS = [([1, 3, 4, 8, 15, 20], 4), ([0, 2, 5, 6, 9, 11, 12, 14, 17, 19, 21, 22, 24, 26, 27, 28,
                                          29, 30, 31, 32], 5), (list(range(33)), 5)]


@pytest.mark.parametrize("sel", range(len(SELECTIONS)))
def test_kernels_on_oracle_modes_fp64(rows_case, sel):
    p, ref = rows_case
    bins, n_r = SELECTIONS[sel]
    plan = _plan(p, "fp64")
    q = p.q.cuda()
    phi = torch.as_tensor(ref["phi"]).cuda()
    mean = torch.as_tensor(ref["mean"]).cuda()
    a, info = plan.coeffs(q, mean, phi, bins, n_r)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    a_ref = OC.expansion_coefficients(p.q.numpy(), ref["mean"], ref["phi"], p.weights, bins, n_r)
    err = _rel(a.cpu().numpy(), a_ref)
    cond = np.linalg.cond(OC.mode_gram(OC.gather_modes(ref["phi"], bins, n_r), p.weights))
    print(f"R={len(bins) * n_r}: coefficient rel err {err:.2e} (cond {cond:.1e})")
    assert err <= 1e-13 * cond
    # reconstruction from the oracle's coefficients
    rec = plan.reconstruct(phi, bins, n_r, torch.as_tensor(a_ref).cuda(), mean, dtype=torch.float64)
    rec_ref = OC.reconstruct(ref["phi"], a_ref, ref["mean"], bins, n_r)
    torch.cuda.synchronize()
    rerr = _rel(rec.cpu().numpy(), rec_ref)
    print(f"R={len(bins) * n_r}: reconstruction rel err {rerr:.2e}")
    assert rerr <= 1e-13
    plan.close()


def test_end_to_end_fp64(rows_case):
    p, ref = rows_case
    bins, n_r = SELECTIONS[1]
    plan = _plan(p, "fp64")
    out = plan.forward(p.q.cuda(), n_modes=5)
    a, info = plan.coeffs(p.q.cuda(), out["mean"], out["phi"], bins, n_r)
    rec = plan.reconstruct(out["phi"], bins, n_r, a, out["mean"], dtype=torch.float64)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    a_ref = OC.expansion_coefficients(p.q.numpy(), ref["mean"], ref["phi"], p.weights, bins, n_r)
    rec_ref = OC.reconstruct(ref["phi"], a_ref, ref["mean"], bins, n_r)
    ea, er = _rel(a.cpu().numpy(), a_ref), _rel(rec.cpu().numpy(), rec_ref)
    print(f"end to end fp64: coefficients {ea:.2e}, reconstruction {er:.2e}")
    assert ea <= 1e-8 and er <= 1e-10
    plan.close()


@pytest.mark.parametrize("precision", ["bf16x4", "fp32"])
def test_complex64_modes(rows_case, precision):
    """Mixed plans keep complex64 modes and coefficients: the kernels widen them
    to FP64, so against the oracle on the same (rounded) modes the error is the
    complex64 rounding of A."""
    p, ref = rows_case
    bins, n_r = SELECTIONS[1]
    plan = _plan(p, precision)
    phi64 = ref["phi"].astype(np.complex64)
    q32 = p.q.float()
    a, info = plan.coeffs(q32.cuda(), torch.as_tensor(ref["mean"]).cuda(),
                          torch.as_tensor(phi64).cuda(), bins, n_r)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and a.dtype == torch.complex64
    a_ref = OC.expansion_coefficients(q32.double().numpy(), ref["mean"], phi64.astype(np.complex128),
                                      p.weights, bins, n_r)
    err = _rel(a.cpu().numpy(), a_ref)
    print(f"{precision}: coefficient rel err {err:.2e}")
    assert err <= 1e-6
    rec = plan.reconstruct(torch.as_tensor(phi64).cuda(), bins, n_r,
                           torch.as_tensor(a_ref.astype(np.complex64)).cuda(),
                           torch.as_tensor(ref["mean"]).cuda(), dtype=torch.float32)
    rec_ref = OC.reconstruct(phi64.astype(np.complex128), a_ref.astype(np.complex64).astype(np.complex128),
                             ref["mean"], bins, n_r)
    torch.cuda.synchronize()
    assert _rel(rec.cpu().numpy(), rec_ref) <= 1e-6
    plan.close()


def test_planted_field_reconstructed_by_its_mode():
    p = fields.planted(nspace=1000, nt=1024, nfft=128, noverlap=64, bins=(12,), amps=(2.0,),
                       sigma=0.0, seed=7, dtype=torch.float64)
    plan = _plan(p, "fp64")
    q = p.q.cuda()
    out = plan.forward(q, n_modes=1)
    a, info = plan.coeffs(q, out["mean"], out["phi"], [12], 1)
    rec = plan.reconstruct(out["phi"], [12], 1, a, out["mean"], dtype=torch.float64)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    err = _rel(rec.cpu().numpy(), p.q.numpy())
    print(f"planted single mode: reconstruction rel err {err:.2e}")
    assert err <= 1e-11
    plan.close()


def test_dependent_modes_report_the_pivot():
    p = fields.random_rows(300, 8 * 32 + 32, 64, 32, seed=33, dtype=torch.float64)
    plan = _plan(p, "fp64")
    out = plan.forward(p.q.cuda(), n_modes=3)
    phi = out["phi"].clone()
    phi[4, 1] = 0                                      # column 4 of bins [2, 4] x 3 modes
    a, info = plan.coeffs(p.q.cuda(), out["mean"], phi, [2, 4], 3)
    torch.cuda.synchronize()
    assert int(info.item()) == 5
    assert torch.count_nonzero(a) == 0
    plan.close()


def test_bad_arguments():
    from paper_2309_11808_amd import SpodError
    p = fields.random_rows(200, 8 * 32 + 32, 64, 32, seed=34, dtype=torch.float64)
    plan = _plan(p, "fp64")
    out = plan.forward(p.q.cuda(), n_modes=3)
    q, mean, phi = p.q.cuda(), out["mean"], out["phi"]
    for bins, n_r in (([3, 2], 1), ([0, 33], 1), ([1], 4), ([1], 0), ([], 1)):
        with pytest.raises(SpodError) as ei:
            plan.coeffs(q, mean, phi, bins, n_r)
        assert ei.value.status == -1, (bins, n_r)
    plan.close()
