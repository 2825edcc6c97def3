"""Parity of the HIP path (through the C ABI) with the FP64 oracle, stage by
stage and end to end, on seeded inputs (MI355X only)."""
import math

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
    import paper_2309_11808_amd  # noqa: F401  (fails loudly when libspod.so is missing)
    yield


def _plan(prob, precision="fp64", window=None, **opt):
    from paper_2309_11808_amd import Plan
    return Plan(prob.nspace, prob.nvar, prob.nt, prob.nfft, prob.noverlap, window=window,
                weights=prob.weights, precision=precision, options=opt or None)


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _rand_problem(M, nt, nfft, nov, seed, dtype=torch.float64, offset=0.0):
    p = fields.random_rows(M, nt, nfft, nov, seed=seed, offset=offset, dtype=dtype)
    return p


# ---------------------------------------------------------------------------
# stage 1-2: mean and Fourier blocks
# ---------------------------------------------------------------------------
FFT_CASES = [
    # nfft, noverlap, M, extra samples, input dtype, offset, window
    (8, 4, 37, 3, torch.float64, 0.0, "hann"),
    (16, 8, 65, 0, torch.float64, 5.0, "random"),
    (32, 0, 33, 7, torch.float64, 0.0, "hamming"),
    (64, 32, 129, 11, torch.float64, 100.0, "hann"),
    (64, 48, 31, 5, torch.float64, 0.0, "hann"),
    (128, 64, 70, 0, torch.float32, 3.0, "random"),
    (128, 96, 17, 9, torch.float64, 0.0, "hamming"),
    (256, 128, 97, 13, torch.float32, 0.0, "hann"),
    (256, 0, 40, 1, torch.float64, 0.0, "hann"),
    (512, 256, 67, 100, torch.float32, 10.0, "hann"),
    (512, 256, 45, 3, torch.float32, 0.0, "random"),
    (512, 128, 33, 0, torch.float64, 0.0, "hann"),
    (1024, 512, 35, 17, torch.float64, 1.0, "hamming"),
    (1024, 512, 19, 0, torch.float32, 0.0, "hann"),
]


def _window(kind, nfft, seed):
    if kind == "hann":
        return None
    if kind == "hamming":                      # two non-zero DFT bins: single-pass mean
        return 0.54 - 0.46 * np.cos(2 * np.pi * np.arange(nfft) / nfft)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.1, 1.0, nfft)         # every bin non-zero: separate mean pass


@pytest.mark.parametrize("prec", ["fp64", "bf16x4"])
@pytest.mark.parametrize("nfft,nov,M,extra,dtype,offset,wkind", FFT_CASES)
def test_blocks_fft_matches_oracle(prec, nfft, nov, M, extra, dtype, offset, wkind):
    L = 3 + (nfft % 5)
    nt = (L - 1) * (nfft - nov) + nfft + extra
    p = _rand_problem(M, nt, nfft, nov, seed=nfft + M, dtype=dtype, offset=offset)
    window = _window(wkind, nfft, nfft)
    plan = _plan(p, prec, window=window)
    qhat, mean = plan.blocks_fft(p.q.cuda())
    torch.cuda.synchronize()
    q64 = p.q.numpy().astype(np.float64)
    ora = O.fourier_blocks(q64, nfft, nov, window)
    np.testing.assert_allclose(mean.cpu().numpy(), O.temporal_mean(q64), rtol=1e-14,
                               atol=1e-15 * (1 + abs(offset)))
    rtol = 2e-13 if prec == "fp64" else 4e-6
    PT.check_qhat(qhat, ora, rtol)


def test_blocks_fft_without_mean_buffer_uses_workspace():
    p = _rand_problem(50, 600, 64, 32, seed=3)
    plan = _plan(p)
    qhat, _ = plan.blocks_fft(p.q.cuda(), want_mean=False)
    torch.cuda.synchronize()
    PT.check_qhat(qhat, O.fourier_blocks(p.q.numpy(), 64, 32), 2e-13)


# ---------------------------------------------------------------------------
# stages 3-4: weighted Gram (fed with the oracle's qhat)
# ---------------------------------------------------------------------------
GRAM_TOL = {"fp64": 1e-13, "fp32": 3e-6, "bf16x4": 3e-5, "fp16x4": 2e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x4", "fp16x4"])
@pytest.mark.parametrize("L,M", [(2, 1), (7, 300), (15, 1024), (16, 77), (31, 5000), (32, 2049),
                                 (33, 130), (47, 700), (63, 257), (64, 64), (65, 500), (80, 3001),
                                 (100, 257), (155, 2000), (160, 64)])
def test_csd_matches_oracle(prec, L, M):
    if L > 64 and prec == "fp32":
        pytest.skip("the FP32 form is limited to 64 blocks (test_large_nblocks_fp32_is_refused)")
    nfft, nov = 16, 8
    nt = (L - 1) * 8 + 16
    p = _rand_problem(M, nt, nfft, nov, seed=L * 7 + M)
    plan = _plan(p, prec, gram_split=3 if M > 1000 else 0)
    qh = O.fourier_blocks(p.q.numpy(), nfft, nov)
    if prec != "fp64":
        qh = qh.astype(np.complex64)
    gram = plan.csd(_dev(np.ascontiguousarray(qh)))
    torch.cuda.synchronize()
    ora = O.gram(qh.astype(np.complex128), p.weights)
    PT.check_gram(gram, ora, GRAM_TOL[prec])


# ---------------------------------------------------------------------------
# stage 5: eigendecomposition (fed with the oracle's Gram)
# ---------------------------------------------------------------------------
def _herm_batch(L, K, seed, kind):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(K):
        if kind == "psd":
            B = rng.standard_normal((L, 2 * L)) + 1j * rng.standard_normal((L, 2 * L))
            out.append(B @ B.conj().T)
        elif kind == "lowrank":
            r = max(1, L // 4)
            B = rng.standard_normal((L, r)) + 1j * rng.standard_normal((L, r))
            out.append(B @ B.conj().T)
        elif kind == "graded":
            U, _ = np.linalg.qr(rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L)))
            out.append(U @ np.diag(10.0 ** np.linspace(0, -10, L)) @ U.conj().T)
        elif kind == "degenerate":
            U, _ = np.linalg.qr(rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L)))
            d = np.repeat(np.arange(L // 2 + 1, 0, -1), 2)[:L].astype(float)
            out.append(U @ np.diag(d) @ U.conj().T)
        elif kind == "diagonal":
            out.append(np.diag(rng.uniform(0, 1, L)).astype(complex))
        elif kind == "zero":
            out.append(np.zeros((L, L), complex))
    A = np.stack(out)
    return 0.5 * (A + np.conj(np.transpose(A, (0, 2, 1))))


@pytest.mark.parametrize("L", [2, 3, 8, 15, 31, 32, 33, 63, 64, 65, 96, 155, 160])
@pytest.mark.parametrize("kind", ["psd", "lowrank", "graded", "degenerate", "diagonal", "zero"])
def test_eig_matches_oracle(L, kind):
    """Up to 64 blocks against the oracle's Jacobi; above (A and V in the
    workspace) against LAPACK's eigh with the oracle's ordering and phase
    convention (the oracle's Python Jacobi takes about 20 s per batch at
    L = 160; test_many_blocks_end_to_end runs it at L = 155)."""
    nfft = 16
    nt = (L - 1) * 8 + 16
    p = _rand_problem(4, nt, nfft, 8, seed=1)
    plan = _plan(p)
    assert plan.nblocks == L
    K = plan.nfreq
    A = _herm_batch(L, K, seed=L, kind=kind)
    lam, psi, info = plan.eig(_dev(A))
    torch.cuda.synchronize()
    if L <= 64:
        lo, Vo, sw = O.jacobi_eigh(A)
    else:
        lo, Vo = np.linalg.eigh(A)
    lo, psio = O.sort_and_phase(lo, Vo)
    info = info.cpu().numpy()
    assert (info > 0).all(), info
    PT.check_eig(lam, lo, rtol=1e-12, theta=1e-2)
    lg, pg = lam.cpu().numpy(), psi.cpu().numpy()
    nrm = np.linalg.norm(A, axis=(1, 2))
    for k in range(K):
        # residual and orthonormality of the GPU eigenvectors
        assert np.abs(A[k] @ pg[k] - pg[k] * lg[k]).max() <= 1e-13 * max(nrm[k], 1e-300) + 1e-300
        assert np.abs(pg[k].conj().T @ pg[k] - np.eye(L)).max() < 1e-13
        for j in range(L):
            if kind in ("zero",) or not PT.separated(lo[k], j, 1e-6):
                continue
            np.testing.assert_allclose(pg[k][:, j], psio[k][:, j], atol=1e-10)
            piv = np.argmax(np.abs(pg[k][:, j]))
            assert pg[k][piv, j].imag == 0 and pg[k][piv, j].real > 0


def test_eig_sweep_cap_reports_non_convergence():
    L = 15
    p = _rand_problem(4, (L - 1) * 8 + 16, 16, 8, seed=1)
    A = _herm_batch(L, 9, seed=2, kind="psd")
    plan0 = _plan(p, max_sweeps=0)
    _, _, info0 = plan0.eig(_dev(A))
    plan1 = _plan(p, max_sweeps=1)
    _, _, info1 = plan1.eig(_dev(A))
    torch.cuda.synchronize()
    assert (info0.cpu().numpy() == 0).all()
    assert (info1.cpu().numpy() == -1).all()


# ---------------------------------------------------------------------------
# modes (fed with the oracle's qhat, lambda, psi)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "bf16x4"])
@pytest.mark.parametrize("n_modes", [1, 5, 15])
def test_modes_match_oracle(prec, n_modes):
    p = _rand_problem(301, 1024, 128, 64, seed=5)
    out = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=n_modes,
                 eps=1e-12 if prec == "fp64" else 1e-6)
    plan = _plan(p, prec)
    qh = out["qhat"] if prec == "fp64" else out["qhat"].astype(np.complex64)
    phi, nv = plan.modes(_dev(np.ascontiguousarray(qh)), _dev(out["lam"]), _dev(out["psi"]), n_modes)
    torch.cuda.synchronize()
    assert (nv.cpu().numpy() == out["n_valid"]).all()
    ora = O.modes(qh.astype(np.complex128), out["lam"], out["psi"], n_modes,
                  eps=1e-12 if prec == "fp64" else 1e-6)[0]
    tol = 1e-13 if prec == "fp64" else 2e-6
    g = phi.cpu().numpy()
    scale = np.abs(ora).max(axis=2, keepdims=True) + 1e-300
    err = (np.abs(g - ora) / scale).max()
    assert err <= tol, err


def test_modes_rank_deficient_are_zero():
    p = fields.planted(nspace=4, nt=1024, sigma=0.0, seed=2)
    out = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=6)
    plan = _plan(p)
    phi, nv = plan.modes(_dev(out["qhat"]), _dev(out["lam"]), _dev(out["psi"]), 6)
    torch.cuda.synchronize()
    nv = nv.cpu().numpy()
    assert (nv == out["n_valid"]).all() and nv.max() <= 4
    PT.check_invalid_modes_zero(phi, nv)


# ---------------------------------------------------------------------------
# end to end
# ---------------------------------------------------------------------------
def _end_to_end(p, prec, n_modes=5):
    plan = _plan(p, prec)
    out = plan.forward(p.q.cuda(), n_modes=n_modes)
    torch.cuda.synchronize()
    return plan, {k: v.cpu().numpy() for k, v in out.items()}


def test_planted_field_fp64_end_to_end():
    p = fields.planted(seed=1, sigma=0.1)
    _, g = _end_to_end(p, "fp64")
    o = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=5)
    np.testing.assert_allclose(g["mean"], o["mean"], rtol=1e-13,
                               atol=1e-15 * np.abs(p.q.numpy()).max())
    PT.check_qhat(g["qhat"], o["qhat"], 2e-13)
    PT.check_gram(g["gram"], o["gram"], 1e-12)
    assert (g["info"] > 0).all()
    PT.check_eig(g["lam"], o["lam"], rtol=1e-10)
    assert (g["n_valid"] == o["n_valid"]).all()
    s, n = PT.check_modes(g["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], sin_tol=1e-9,
                          elem_tol=1e-8, rel_gap=1e-6)
    assert n > 100


def test_planted_field_closed_form_on_gpu():
    """sigma = 0: lambda_1(b) = L/(L-1) a^2 N_f / 6 at the planted bins."""
    p = fields.planted(seed=1, sigma=0.0)
    _, g = _end_to_end(p, "fp64", n_modes=3)
    L = 15
    for b, a, i in zip(p.meta["bins"], p.meta["amps"], range(3)):
        ref = L / (L - 1) * a * a * 128 / 6.0
        assert abs(g["lam"][b, 0] / ref - 1) < 1e-12
        assert abs(g["lam"][b + 1, 0] / (ref / 4) - 1) < 1e-12
        phi_i = p.meta["phi"][:, i]
        assert abs(abs(np.vdot(phi_i, p.weights * g["phi"][b, 0])) - 1) < 1e-11


@pytest.mark.parametrize("prec", ["fp32", "bf16x4", "fp16x4"])
def test_planted_field_mixed_end_to_end(prec):
    p = fields.planted(seed=1, sigma=0.1, dtype=torch.float32)
    _, g = _end_to_end(p, prec)
    o = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=5, eps=1e-6)
    # The FP32 form rounds every 8-product MFMA partial to FP32 before it
    # reaches FP64 (24-bit operands have no exact-integer form on the FP32
    # matrix cores): about 2^-24 sqrt(8/M) lambda_1 per Gram entry, which at
    # M = 1024 reaches 1e-4 of an eigenvalue ~2e5 below lambda_1 (this field's
    # noise eigenvalues).  It is held to the relative bar from 1e-4 lambda_1 up;
    # the split forms meet it from 1e-6 lambda_1 up.
    PT.check_eig_mixed(g["lam"], o["lam"], n=5, theta=1e-4 if prec == "fp32" else PT.THETA_MIXED)
    s, n = PT.check_modes(g["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], sin_tol=1e-3,
                          elem_tol=1e-2, rel_gap=1e-3)
    assert n > 100


@pytest.mark.parametrize("prec", ["fp64", "bf16x4"])
def test_random_rows_with_offsets_end_to_end(prec):
    p = _rand_problem(1031, 2 * 256 + 77, 64, 32, seed=9, offset=50.0,
                      dtype=torch.float64 if prec == "fp64" else torch.float32)
    _, g = _end_to_end(p, prec, n_modes=4)
    o = O.spod(p.q.numpy(), 64, 32, weights=p.weights, n_modes=4, eps=1e-12 if prec == "fp64" else 1e-6)
    if prec == "fp64":
        PT.check_eig(g["lam"], o["lam"], rtol=1e-10)
        PT.check_modes(g["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], 1e-8, 1e-7, 1e-6)
    else:
        PT.check_eig_mixed(g["lam"], o["lam"], p.M, n=4)
        PT.check_modes(g["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], 1e-3, 1e-2, 1e-3)


# ---------------------------------------------------------------------------
# boundary behaviour on the device
# ---------------------------------------------------------------------------
def test_stage_errors_on_device():
    import ctypes as C
    from paper_2309_11808_amd import _native as N
    from paper_2309_11808_amd.spod import lib
    p = _rand_problem(100, 512, 64, 32, seed=4)
    plan = _plan(p)
    qh = torch.zeros(plan.nfreq, plan.nblocks, plan.M, dtype=torch.complex128, device="cuda")
    g = torch.zeros(plan.nfreq, plan.nblocks, plan.nblocks, dtype=torch.complex128, device="cuda")
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    st = lib().spod_csd(plan._h, C.c_void_p(qh.data_ptr()), C.c_void_p(g.data_ptr()),
                        C.c_void_p(small.data_ptr()), 8, None)
    assert st == N.SPOD_ERR_WORKSPACE
    st = lib().spod_modes(plan._h, C.c_void_p(qh.data_ptr()), C.c_void_p(qh.data_ptr()),
                          C.c_void_p(g.data_ptr()), plan.nblocks + 1, C.c_void_p(qh.data_ptr()),
                          None, None, 0, None)
    assert st == N.SPOD_ERR_INVALID_ARG
    # precision and options are frozen after the first stage call
    assert lib().spod_plan_set_precision(plan._h, N.SPOD_PREC_FP32) == N.SPOD_ERR_INVALID_ARG
    assert math.isfinite(plan.workspace_bytes)


@pytest.mark.parametrize("nfft", [64, 256, 512])
@pytest.mark.parametrize("precision", ["fp64", "bf16x4"])
def test_fft_tile_option(nfft, precision):
    """The transform tile (16 or 32 DOFs per workgroup) only regroups DOFs:
    every tile gives the same blocks bit for bit, and other values are
    rejected."""
    from paper_2309_11808_amd import SpodError
    dt = torch.float64 if precision == "fp64" else torch.float32
    p = _rand_problem(333, 5 * nfft // 2 + 7, nfft, nfft // 2, seed=nfft + 7)
    q = _dev(p.q.to(dt))
    ref = None
    for tile in (0, 16, 32):
        plan = _plan(p, precision, fft_tile=tile)
        qhat, mean = plan.blocks_fft(q)
        torch.cuda.synchronize()
        if ref is None:
            ref = (qhat.clone(), mean.clone())
        else:
            assert torch.equal(qhat, ref[0]) and torch.equal(mean, ref[1]), tile
        plan.close()
    for bad in (8, 64, -1):
        with pytest.raises(SpodError) as ei:
            _plan(p, precision, fft_tile=bad)
        assert ei.value.status == -1


# ---------------------------------------------------------------------------
# packed Fourier blocks (20-bit block floating point, SPOD_QHAT_BFP20)
# ---------------------------------------------------------------------------
PACKED_FFT_CASES = [
    (8, 4, 37, 3, torch.float64, 0.0, "hann"),
    (16, 8, 65, 0, torch.float64, 5.0, "random"),
    (64, 32, 129, 11, torch.float64, 100.0, "hann"),
    (128, 64, 70, 0, torch.float32, 3.0, "random"),
    (256, 128, 97, 13, torch.float32, 0.0, "hann"),
    (256, 0, 40, 1, torch.float64, 0.0, "hann"),
    (512, 256, 300, 3, torch.float32, 10.0, "hann"),
    (512, 128, 33, 0, torch.float64, 0.0, "hann"),
    (1024, 512, 35, 17, torch.float64, 1.0, "hamming"),
]


def _packed_plan(p, prec="fp16x4", window=None, **opt):
    return _plan(p, prec, window=window, qhat_format="bfp20", **opt)


@pytest.mark.parametrize("nfft,nov,M,extra,dtype,offset,wkind", PACKED_FFT_CASES)
def test_blocks_fft_packed_matches_oracle(nfft, nov, M, extra, dtype, offset, wkind):
    """Packed blocks decode to the oracle's within the FP32 transform's error
    (4e-6 of the block norm) plus the 20-bit rounding (2^-19 of the largest
    real or imaginary part in the group of 16 degrees of freedom), and keep the
    layout's invariants (normalised mantissas, zero padding)."""
    L = 3 + (nfft % 5)
    nt = (L - 1) * (nfft - nov) + nfft + extra
    p = _rand_problem(M, nt, nfft, nov, seed=nfft + M, dtype=dtype, offset=offset)
    window = _window(wkind, nfft, nfft)
    plan = _packed_plan(p, window=window)
    q = p.q.to(torch.float32).cuda()
    qhat, mean = plan.blocks_fft(q)
    torch.cuda.synchronize()
    K = plan.nfreq
    dec, _, sb = PT.unpack_qhat(qhat.cpu().numpy(), K, L, M)
    PT.check_packed_format(sb, M)
    q64 = q.cpu().numpy().astype(np.float64)
    ora = O.fourier_blocks(q64, nfft, nov, window)
    np.testing.assert_allclose(mean.cpu().numpy(), O.temporal_mean(q64), rtol=1e-14,
                               atol=1e-15 * (1 + abs(offset)))
    norm = np.sqrt(np.sum(np.abs(ora) ** 2, axis=0, keepdims=True))
    pad = (-M) % 16
    parts = np.stack([ora.real, ora.imag], axis=-1)
    gmax = np.abs(np.pad(parts, ((0, 0), (0, 0), (0, pad), (0, 0)))).reshape(K, L, -1, 32).max(-1)
    gmax = np.repeat(gmax, 16, axis=2)[:, :, :M]
    err = np.abs(dec - ora) - (4e-6 * norm + 2.0 ** -19 * np.sqrt(2.0) * gmax)
    assert err.max() <= 0.0, f"packed blocks beyond the bound by {err.max():.3e}"
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x4", "fp16x4"])
@pytest.mark.parametrize("L,M", [(2, 1), (7, 300), (15, 1024), (16, 77), (31, 5000), (33, 130),
                                 (47, 700), (64, 200)])
def test_csd_packed_matches_oracle(prec, L, M):
    """The Gram of packed blocks (encoded on the host from the layout's
    definition) against the oracle's Gram of the same decoded values."""
    nfft, nov = 16, 8
    nt = (L - 1) * 8 + 16
    p = _rand_problem(M, nt, nfft, nov, seed=L * 7 + M)
    plan = _packed_plan(p, prec, gram_split=3 if M > 1000 else 0)
    qh = O.fourier_blocks(p.q.numpy(), nfft, nov)
    buf = PT.pack_qhat(qh)
    dec, _, _ = PT.unpack_qhat(buf, plan.nfreq, L, M)
    assert buf.size == plan.qhat_bytes
    gram = plan.csd(torch.as_tensor(buf).cuda())
    torch.cuda.synchronize()
    PT.check_gram(gram, O.gram(dec, p.weights), GRAM_TOL[prec])
    plan.close()


def test_modes_packed_matches_oracle():
    L, M, nfft, nov = 15, 1031, 32, 16
    nt = (L - 1) * 16 + 32
    p = _rand_problem(M, nt, nfft, nov, seed=77)
    plan = _packed_plan(p, "fp16x4")
    qh = O.fourier_blocks(p.q.numpy(), nfft, nov)
    buf = PT.pack_qhat(qh)
    dec, _, _ = PT.unpack_qhat(buf, plan.nfreq, L, M)
    lam, V, _ = O.jacobi_eigh(O.gram(dec, p.weights))
    lam, psi = O.sort_and_phase(lam, V)
    phi, n_valid = plan.modes(torch.as_tensor(buf).cuda(), _dev(lam), _dev(psi), 5)
    torch.cuda.synchronize()
    ref, nv = O.modes(dec, lam, psi, 5, eps=1e-6)
    np.testing.assert_array_equal(n_valid.cpu().numpy(), nv)
    g = phi.cpu().numpy()
    scale = np.abs(ref).max(axis=2, keepdims=True) + 1e-300
    assert (np.abs(g - ref) / scale).max() < 2e-6
    plan.close()


@pytest.mark.parametrize("prec", ["fp16x4", "bf16x4"])
def test_planted_field_packed_end_to_end(prec):
    """The planted field (lambda_1 / lambda_5 ~ 2e5 at the planted bins) through
    packed blocks meets the mixed-path bars; the backward of a packed plan
    recomputes complex blocks and gives the complex plan's gradient."""
    p = fields.planted(seed=1, sigma=0.1, dtype=torch.float32)
    plan = _packed_plan(p, prec)
    out = plan.forward(p.q.cuda(), n_modes=5)
    torch.cuda.synchronize()
    o = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=5, eps=1e-6)
    err = PT.check_eig_mixed(out["lam"], o["lam"], n=5)
    s, n = PT.check_modes(out["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], sin_tol=1e-3,
                          elem_tol=1e-2, rel_gap=1e-3)
    assert n > 100 and int(out["info"].min()) > 0
    print(f"packed {prec}: eigenvalue rel err {err:.2e}, mode sine {s:.2e}")
    bins = list(p.meta["bins"])
    g_lam = torch.zeros(len(bins), plan.nblocks, dtype=torch.float64, device="cuda")
    g_lam[:, :3] = 1.0
    lam_b, psi_b = out["lam"][bins].contiguous(), out["psi"]
    g1 = plan.backward(p.q.cuda(), out["lam"], psi_b, g_lam=g_lam, bins=bins)
    cplan = _plan(p, prec)
    g2 = cplan.backward(p.q.cuda(), out["lam"], psi_b, g_lam=g_lam, bins=bins)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    cplan.close()
    plan.close()


@pytest.mark.parametrize("L,M,n_modes", [(15, 1031, 5), (31, 4096, 5), (40, 777, 20), (64, 300, 17),
                                         (3, 50, 3)])
def test_modes_mfma_matches_oracle(L, M, n_modes):
    """The matrix-core modes kernel (FP32 products and sums on
    v_mfma_f32_16x16x4f32) against the oracle's modes of the same complex64
    blocks, and against the vector-ALU kernel, with more than 16 modes (two
    mode groups), odd M, and a near-null eigenvalue (a zero mode)."""
    nfft, nov = 16, 8
    nt = (L - 1) * 8 + 16
    p = _rand_problem(M, nt, nfft, nov, seed=L + M)
    plan = _plan(p, "fp16x4", modes_kernel="mfma")
    vplan = _plan(p, "fp16x4")
    qh = O.fourier_blocks(p.q.numpy(), nfft, nov).astype(np.complex64)
    lam, V, _ = O.jacobi_eigh(O.gram(qh.astype(np.complex128), p.weights))
    lam, psi = O.sort_and_phase(lam, V)
    lam[:, n_modes - 1] = 1e-9 * lam[:, :1].ravel()          # below the valid-mode threshold
    qd = _dev(qh)
    phi, n_valid = plan.modes(qd, _dev(lam), _dev(psi), n_modes)
    phv, nvv = vplan.modes(qd, _dev(lam), _dev(psi), n_modes)
    torch.cuda.synchronize()
    ref, nv = O.modes(qh.astype(np.complex128), lam, psi, n_modes, eps=1e-6)
    np.testing.assert_array_equal(n_valid.cpu().numpy(), nv)
    np.testing.assert_array_equal(nvv.cpu().numpy(), nv)
    g = phi.cpu().numpy()
    assert np.all(g[:, n_modes - 1] == 0)
    scale = np.abs(ref).max(axis=2, keepdims=True) + 1e-300
    assert (np.abs(g - ref) / scale).max() < 2e-6
    assert (np.abs(g - phv.cpu().numpy()) / scale).max() < 2e-6
    plan.close()
    vplan.close()


def test_large_nblocks_fp32_is_refused():
    from paper_2309_11808_amd import SpodError, _native as N
    p = _rand_problem(100, 64 * 8 + 16, 16, 8, seed=3)
    plan = _plan(p, "fp32")
    assert plan.nblocks == 65
    qh = torch.zeros(plan.nfreq, 65, 100, dtype=torch.complex64, device="cuda")
    with pytest.raises(SpodError) as ei:
        plan.csd(qh)
    assert ei.value.status == N.SPOD_ERR_UNSUPPORTED
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp16x4", "bf16x4"])
def test_many_blocks_end_to_end(prec):
    """155 blocks (the paper's jet analysis uses N_f = 256 at 50% overlap and
    L = 155), here with N_f = 32 so the oracle's Jacobi stays fast: the
    L > 64 Gram, eigensolver (A and V in the workspace) and modes."""
    nfft, nov, L = 32, 16, 155
    nt = (L - 1) * 16 + 32 + 5
    p = _rand_problem(1500, nt, nfft, nov, seed=155,
                      dtype=torch.float64 if prec == "fp64" else torch.float32, offset=2.0)
    plan = _plan(p, prec)
    assert plan.nblocks == L
    out = plan.forward(p.q.cuda(), n_modes=8)
    torch.cuda.synchronize()
    eps = 1e-12 if prec == "fp64" else 1e-6
    o = O.spod(p.q.numpy(), nfft, nov, weights=p.weights, n_modes=8, eps=eps)
    assert int(out["info"].min()) > 0
    if prec == "fp64":
        err = PT.check_eig(out["lam"], o["lam"], rtol=1e-10)
        PT.check_modes(out["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], 1e-8, 1e-6, 1e-6)
    else:
        err = PT.check_eig_mixed(out["lam"], o["lam"], n=8)
        PT.check_modes(out["phi"], o["phi"], o["lam"], p.weights, o["n_valid"], 1e-3, 1e-2, 1e-3)
    print(f"L = 155 {prec}: eigenvalue rel err {err:.2e}")
    plan.close()
