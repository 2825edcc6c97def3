"""The transform for block lengths that are not powers of two (or above 1024),
MI355X only: mixed-radix stages in LDS with a direct sum per output, against
the FP64 oracle (whose DFT is pinned to numpy's rfft for any length).

Lengths cover small primes, a large prime factor (73, as in the paper's
8760 = 2^3 3 5 73 hourly blocks), odd N_f (K = (N_f + 1) / 2), powers of two
above 1024, ragged M (odd: a last unpaired row) and several overlaps.  The
plan merges a 3 with a 5 into one radix-15 stage and two 3s into a radix-9
stage, and runs the odd stages first: 60 = 15 4, 360 = 15 3 8, 504 = 9 7 8
and 675 = 15 15 3 take those paths.  Odd
radices take 1 to 6 output pairs per work item, with W_r^{jk} from the plan's
per-stage table (1001 = 7 11 13, 527 = 17 31 and the prime 1019 reach several
counts, with table rows beyond (r + 1) / 2 pairs that store nothing)."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import fields
from tests import parity as PT

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


CASES = [  # nfft, noverlap, M, L
    (12, 6, 37, 6), (24, 12, 64, 5), (60, 30, 101, 4), (73, 0, 50, 3), (100, 50, 33, 4),
    (146, 73, 20, 3), (360, 180, 17, 3), (2048, 1024, 9, 3), (730, 365, 12, 3),
    (1001, 500, 15, 3), (527, 263, 19, 3), (1019, 509, 11, 3),
    (504, 252, 23, 3), (675, 300, 10, 3),
]
C64_CASES = CASES[:5] + CASES[-5:] + [(8760, 4380, 7, 2)]


@pytest.mark.parametrize("nfft,nov,M,L", CASES, ids=[f"N{c[0]}" for c in CASES])
def test_fourier_blocks_match_oracle_fp64(nfft, nov, M, L):
    nt = (L - 1) * (nfft - nov) + nfft + 5
    p = fields.random_rows(M, nt, nfft, nov, seed=nfft, offset=1.5, dtype=torch.float64)
    plan = _plan(p, "fp64")
    assert plan.nblocks == L and plan.nfreq == nfft // 2 + 1
    qhat, mean = plan.blocks_fft(p.q.cuda())
    torch.cuda.synchronize()
    ref_mean = O.temporal_mean(p.q.numpy())
    ref = O.fourier_blocks(p.q.numpy(), nfft, nov, O.hann_periodic(nfft), ref_mean, None)
    np.testing.assert_allclose(mean.cpu().numpy(), ref_mean, rtol=0, atol=1e-14 * 3)
    err = PT.check_qhat(qhat.cpu().numpy(), ref, 1e-12)
    print(f"N={nfft}: fp64 qhat rel err {err:.2e}")
    plan.close()


@pytest.mark.parametrize("nfft,nov,M,L", C64_CASES, ids=[f"N{c[0]}" for c in C64_CASES])
def test_fourier_blocks_match_oracle_complex64(nfft, nov, M, L):
    nt = (L - 1) * (nfft - nov) + nfft + 5
    p = fields.random_rows(M, nt, nfft, nov, seed=nfft + 1, offset=1.5, dtype=torch.float32)
    plan = _plan(p, "bf16x4")
    qhat, _ = plan.blocks_fft(p.q.cuda())
    torch.cuda.synchronize()
    q64 = p.q.double().numpy()
    ref = O.fourier_blocks(q64, nfft, nov, O.hann_periodic(nfft), O.temporal_mean(q64), None)
    err = PT.check_qhat(qhat.cpu().numpy(), ref, 2e-6)
    print(f"N={nfft}: complex64 qhat rel err {err:.2e}")
    plan.close()


def test_hourly_year_blocks_end_to_end():
    """N_f = 8760 (one year of hours), 50% overlap, 4 blocks: the whole path
    against the oracle."""
    nfft, nov, M, L = 8760, 4380, 256, 4
    nt = (L - 1) * (nfft - nov) + nfft
    p = fields.random_rows(M, nt, nfft, nov, seed=8760, offset=0.5, dtype=torch.float64)
    ref = O.spod(p.q.numpy(), nfft, nov, weights=p.weights, n_modes=3)
    plan = _plan(p, "fp64")
    out = plan.forward(p.q.cuda(), n_modes=3)
    torch.cuda.synchronize()
    PT.check_eig(out["lam"], ref["lam"], rtol=1e-10)
    s, n = PT.check_modes(out["phi"], ref["phi"], ref["lam"], p.weights, ref["n_valid"],
                          sin_tol=1e-8, elem_tol=1e-6, rel_gap=1e-6)
    print(f"N=8760 end to end: modes compared {n}, worst sine {s:.2e}")
    assert n > 1000
    plan.close()


def test_general_transform_limits():
    from paper_2309_11808_amd import Plan, SpodError
    p = fields.random_rows(4, 3 * 12000, 12000, 0, seed=1, dtype=torch.float64)
    plan = _plan(p, "fp64")                     # complex128 above 10240: the two-pass transform
    qhat, _ = plan.blocks_fft(p.q.cuda())
    torch.cuda.synchronize()
    ref = O.fourier_blocks(p.q.numpy(), 12000, 0, O.hann_periodic(12000),
                           O.temporal_mean(p.q.numpy()), None, dft="fft")
    err = PT.check_qhat(qhat.cpu().numpy(), ref, 1e-12)
    print(f"N=12000 (two passes, 100 x 120): complex128 qhat rel err {err:.2e}")
    plan.close()
    # above 20480 the length must split into two factors <= 4096 (a prime cannot)
    with pytest.raises(SpodError) as ei:
        Plan(4, 1, 3 * 20483, 20483, 0)
    assert ei.value.status == -2
    plan = _plan(p, "fp32")                     # complex64 blocks: one LDS buffer above ~10080
    q32 = p.q.float()
    qhat, _ = plan.blocks_fft(q32.cuda())
    torch.cuda.synchronize()
    q64 = q32.double().numpy()
    ref = O.fourier_blocks(q64, 12000, 0, O.hann_periodic(12000), O.temporal_mean(q64), None)
    err = PT.check_qhat(qhat.cpu().numpy(), ref, 2e-6)
    print(f"N=12000 (single LDS buffer): complex64 qhat rel err {err:.2e}")
    plan.close()


def test_backward_general_length_without_blocks_is_refused():
    """Any block length other than a power of two up to 1024 needs the
    forward's blocks: the mixed-radix transform has no bin selection to
    recompute them from (the gradients themselves: test_gpu_backward.py)."""
    from paper_2309_11808_amd import SpodError
    p = fields.random_rows(16, 4 * 30 + 60, 60, 30, seed=2, dtype=torch.float64)
    plan = _plan(p, "fp64")
    out = plan.forward(p.q.cuda(), n_modes=2)
    with pytest.raises(SpodError) as ei:
        plan.backward(p.q.cuda(), out["lam"], out["psi"], g_lam=torch.ones_like(out["lam"]))
    assert ei.value.status == -2
    plan.close()


# ---------------------------------------------------------------------------
# blocks beyond one workgroup's LDS: the two-pass transform N = A B (A the
# largest divisor <= sqrt(N)); the oracle's library-FFT form of the transform
# ---------------------------------------------------------------------------
LONG_CASES = [  # nfft, noverlap, M, L
    (30030, 15015, 5, 2),      # 2 3 5 7 11 13: A = 165, B = 182
    (40960, 20480, 4, 2),      # 2^13 5: A = 160, B = 256
    (65536, 0, 3, 2),          # 2^16: A = B = 256
    (87600, 43800, 6, 3),      # the paper's ten-year hourly blocks: A = 292, B = 300
]


@pytest.mark.parametrize("precision", ["fp64", "bf16x4"])
@pytest.mark.parametrize("nfft,nov,M,L", LONG_CASES, ids=[f"N{c[0]}" for c in LONG_CASES])
def test_long_blocks_match_oracle(nfft, nov, M, L, precision):
    nt = (L - 1) * (nfft - nov) + nfft + 5
    dt = torch.float64 if precision == "fp64" else torch.float32
    p = fields.random_rows(M, nt, nfft, nov, seed=nfft % 1000, offset=1.5, dtype=dt)
    plan = _plan(p, precision)
    assert plan.nblocks == L
    qhat, mean = plan.blocks_fft(p.q.cuda())
    torch.cuda.synchronize()
    q64 = p.q.double().numpy()
    ref_mean = O.temporal_mean(q64)
    ref = O.fourier_blocks(q64, nfft, nov, O.hann_periodic(nfft), ref_mean, None, dft="fft")
    np.testing.assert_allclose(mean.cpu().numpy(), ref_mean, rtol=0, atol=1e-13 * 3)
    err = PT.check_qhat(qhat.cpu().numpy(), ref, 1e-12 if precision == "fp64" else 2e-6)
    print(f"N={nfft} two passes: {precision} qhat rel err {err:.2e}")
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x4"])
def test_ten_year_blocks_end_to_end(precision):
    """N_f = 87,600 hourly samples (ten years), 50% overlap, L = 8 blocks as in
    the paper's ERA5 analysis: eigenvalues at 8 frequencies against the
    oracle (library-FFT form of the transform)."""
    nfft, nov, M, L = 87600, 43800, 96, 8
    nt = (L - 1) * (nfft - nov) + nfft
    dt = torch.float64 if precision == "fp64" else torch.float32
    p = fields.random_rows(M, nt, nfft, nov, seed=876, offset=0.5, dtype=dt)
    bins = [0, 1, 2, 10, 365, 1000, 20000, nfft // 2]
    ref = O.spod_chunked(p.q.double().numpy(), nfft, nov, weights=p.weights, n_modes=3,
                         chunk=32, bins=bins, want_modes=False, dft="fft")
    plan = _plan(p, precision)
    out = plan.forward(p.q.cuda(), n_modes=3)
    torch.cuda.synchronize()
    lam = out["lam"].index_select(0, torch.as_tensor(bins, device="cuda")).cpu().numpy()
    if precision == "fp64":
        err = PT.check_eig(lam, ref["lam"], rtol=1e-10, n=3)
    else:
        err = PT.check_eig_mixed(lam, ref["lam"], n=3)
    assert int(out["info"].min()) > 0
    print(f"N=87600, L=8 end to end ({precision}): leading eigenvalue rel err {err:.2e}")
    plan.close()
