"""Parity at the workloads' full sizes (MI355X only).

The HIP path runs the whole problem in the same configuration the benchmark
times; the FP64 oracle (streamed over chunks of degrees of freedom, the
paper's spatial split done sequentially) computes the outputs it can afford:
the eigenvalues and modes of selected frequencies, the modes at sampled
degrees of freedom, the means, and sampled Fourier blocks.
"""
import time

import numpy as np
import pytest
import torch

import oracle as O
from synth import fields
from tests import parity as PT

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_11808_amd  # noqa: F401
    yield


def _plan(p, precision):
    """precision: a form name, with "+bfp20" for packed Fourier blocks."""
    from paper_2309_11808_amd import Plan
    packed = precision.endswith("+bfp20")
    return Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, weights=p.weights,
                precision=precision.split("+")[0],
                options={"qhat_format": "bfp20"} if packed else None)


def _modes_rows_error(phi_gpu, phi_ora, n_valid, lam, rel_gap):
    """Largest relative error of the sampled rows of every valid, separated
    mode (the phase convention makes the modes unique)."""
    worst = 0.0
    for k in range(phi_ora.shape[0]):
        for j in range(min(phi_ora.shape[1], int(n_valid[k]))):
            if not PT.separated(lam[k], j, rel_gap):
                continue
            o = phi_ora[k, j]
            e = np.linalg.norm(phi_gpu[k, j] - o) / np.linalg.norm(o)
            worst = max(worst, float(e))
    return worst


# ---------------------------------------------------------------------------
# jet-like field: 256 x 128 x 3, N_t = 4096 float32, N_f = 256, 31 blocks, 129 bins
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def jet():
    p = fields.jet_like(seed=2, device="cuda", dtype=torch.float32)
    q_host = p.q.cpu().numpy()
    bins = [0, 10, 20, 35, 50, 77, 100, 128]          # the 4 packet bins and 4 others
    rng = np.random.Generator(np.random.PCG64(12))
    rows = np.sort(rng.choice(p.M, 512, replace=False))
    ref = O.spod_chunked(q_host, p.nfft, p.noverlap, weights=p.weights, n_modes=5,
                         chunk=16384, bins=bins, mode_rows=rows)
    # eigenvalues at every one of the 129 bins (library-FFT form of the transform)
    ref["lam_all"] = O.spod_chunked(q_host, p.nfft, p.noverlap, weights=p.weights, n_modes=5,
                                    chunk=16384, want_modes=False, dft="fft")["lam"]
    print("[jet fixture] oracle done", flush=True)
    return p, bins, rows, ref


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x4", "fp16x4", "fp16x4+bfp20"])
def test_jet_field_full_size(jet, precision):
    p, bins, rows, ref = jet
    plan = _plan(p, precision)
    out = plan.forward(p.q, n_modes=5)
    torch.cuda.synchronize()
    idx = torch.as_tensor(bins, device="cuda")
    lam = out["lam"].cpu().numpy()
    np.testing.assert_allclose(out["mean"].cpu().numpy(), ref["mean"], rtol=0,
                               atol=1e-13 * float(np.abs(ref["mean"]).max()) + 1e-12)
    np.testing.assert_allclose(ref["lam_all"][bins], ref["lam"], rtol=1e-12,
                               atol=1e-15 * float(ref["lam"].max()))
    if precision == "fp64":
        err = PT.check_eig(lam, ref["lam_all"], rtol=1e-10, n=5)
        k, j, _ = PT.worst_eig(lam, ref["lam_all"], PT.THETA_FP64, n=5)
        tol_modes, gap = 1e-7, 1e-6
    else:
        err = PT.check_eig_mixed(lam, ref["lam_all"], n=5, rtol=1e-4)
        k, j, _ = PT.worst_eig(lam, ref["lam_all"], PT.THETA_MIXED, n=5)
        tol_modes, gap = 1e-3, 1e-3
    phi = out["phi"].index_select(0, idx)[:, :, torch.as_tensor(rows, device="cuda")].cpu().numpy()
    merr = _modes_rows_error(phi, ref["phi"], out["n_valid"].index_select(0, idx).cpu().numpy(),
                             ref["lam"], gap)
    print(f"jet {precision}: leading-5 eigenvalue rel err {err:.2e} (worst k={k} j={j}) over "
          f"{lam.shape[0]} bins, sampled mode rows {merr:.2e}", flush=True)
    assert merr <= tol_modes
    assert int(out["info"].min()) > 0
    plan.close()


# ---------------------------------------------------------------------------
# ERA-like field: 1024 x 512 x 2, N_t = 8192 float32, N_f = 512, 31 blocks,
# 257 bins, in the benchmark's launch configuration: the leading eigenvalues
# at every bin, the full modes at 8 bins, sampled Fourier blocks and mode rows
# ---------------------------------------------------------------------------
ERA_MODE_BINS = [3, 8, 17, 40, 90, 200, 100, 256]    # the 6 planted bins and 2 noise bins


@pytest.fixture(scope="module")
def era():
    p = fields.era_like(seed=3, device="cuda", dtype=torch.float32)
    rng = np.random.Generator(np.random.PCG64(13))
    rows = np.sort(rng.choice(p.M, 256, replace=False))
    q_host = p.q.cpu().numpy()
    t = time.perf_counter()

    def progress(done):
        if done % (1 << 17) == 0 or done == p.M:
            print(f"[era fixture] oracle Gram pass, all 257 bins: {done} of {p.M} rows, "
                  f"{time.perf_counter() - t:.0f} s", flush=True)
    # every bin: the library-FFT form of the block transform (pinned against
    # the twiddle-table form), Gram accumulated chunk by chunk
    ref = O.spod_chunked(q_host, p.nfft, p.noverlap, weights=p.weights, n_modes=5,
                         chunk=16384, want_modes=False, dft="fft", progress=progress)
    # Fourier blocks of the sampled rows at every frequency
    ref["qhat_rows"] = O.fourier_blocks(q_host[rows], p.nfft, p.noverlap, O.hann_periodic(p.nfft),
                                        ref["mean"][rows], None)
    # the second pass: full modes at ERA_MODE_BINS (twiddle-table DFT at those bins)
    window = O.hann_periodic(p.nfft)
    sel = ERA_MODE_BINS
    phi = np.empty((len(sel), 5, p.M), dtype=np.complex128)
    for c0 in range(0, p.M, 1 << 16):
        r = slice(c0, min(p.M, c0 + (1 << 16)))
        qh = O.fourier_blocks(q_host[r], p.nfft, p.noverlap, window, ref["mean"][r], sel)
        phi[:, :, r], nv = O.modes(qh, ref["lam"][sel], ref["psi"][sel], 5, 1e-12)
        if r.stop % (1 << 18) == 0 or r.stop == p.M:
            print(f"[era fixture] oracle modes pass to row {r.stop}: {time.perf_counter() - t:.0f} s",
                  flush=True)
    ref["phi_sel"] = phi
    ref["n_valid_sel"] = nv
    del q_host
    return p, rows, ref


@pytest.mark.parametrize("precision", ["fp16x4+bfp20", "fp16x4", "bf16x4", "fp64"])
def test_era_field_full_size(era, precision):
    p, rows, ref = era
    plan = _plan(p, precision)
    out = plan.forward(p.q, n_modes=5)
    torch.cuda.synchronize()
    rows_d = torch.as_tensor(rows, device="cuda")
    mean = out["mean"].index_select(0, rows_d).cpu().numpy()
    np.testing.assert_allclose(mean, ref["mean"][rows], rtol=0,
                               atol=1e-13 * float(np.abs(ref["mean"]).max()) + 1e-12)
    if precision.endswith("+bfp20"):
        qerr = float("nan")          # packed blocks: checked element-wise in test_gpu_parity
    else:
        qh = out["qhat"][:, :, rows_d].cpu().numpy()
        qtol = 1e-12 if precision == "fp64" else 2e-6
        qerr = PT.check_qhat(qh, ref["qhat_rows"], qtol)
    # leading 5 eigenvalues at every one of the 257 bins
    lam = out["lam"].cpu().numpy()
    if precision == "fp64":
        err = PT.check_eig(lam, ref["lam"], rtol=1e-10, n=5)
        k, j, _ = PT.worst_eig(lam, ref["lam"], PT.THETA_FP64, n=5)
        sin_tol, elem_tol, gap = 1e-8, 1e-6, 1e-6
    else:
        err = PT.check_eig_mixed(lam, ref["lam"], n=5, rtol=1e-4)
        k, j, _ = PT.worst_eig(lam, ref["lam"], PT.THETA_MIXED, n=5)
        sin_tol, elem_tol, gap = 1e-3, 1e-2, 1e-3
    assert int(out["info"].min()) > 0
    # full modes at 8 bins: sine of the W-angle (subspace angles in clusters)
    sel = torch.as_tensor(ERA_MODE_BINS, device="cuda")
    phi = out["phi"].index_select(0, sel).cpu().numpy()
    n_valid = out["n_valid"].index_select(0, sel).cpu().numpy()
    eps = 1e-12 if precision == "fp64" else 1e-6          # the valid-mode thresholds
    lsel = ref["lam"][ERA_MODE_BINS, :5]
    np.testing.assert_array_equal(n_valid, (lsel > eps * lsel[:, :1]).sum(axis=1))
    msin, count = PT.check_modes(phi, ref["phi_sel"], ref["lam"][ERA_MODE_BINS], p.weights,
                                 n_valid, sin_tol=sin_tol, elem_tol=elem_tol, rel_gap=gap)
    print(f"era {precision}: qhat {qerr:.2e}; leading-5 eigenvalue rel err {err:.2e} "
          f"(worst k={k} j={j}) over 257 bins; mode sine {msin:.2e} over {count} modes "
          f"at {len(ERA_MODE_BINS)} bins", flush=True)
    del out
    plan.close()
    torch.cuda.empty_cache()


def test_era_field_out_of_core(era):
    """The same workload streamed from pinned host memory in 32 chunks of
    32768 rows with nothing kept resident: both passes read all of Q."""
    from paper_2309_11808_amd import OutOfCore
    p, rows, ref = era
    plan = _plan(p, "fp16x4")
    q_host = torch.empty(tuple(p.q.shape), dtype=torch.float32, pin_memory=True)
    q_host.copy_(p.q)
    o = OutOfCore(plan, dtype=torch.float32, chunk_rows=32768, n_modes=5, resident=0)
    assert o.n_chunks == 32
    out = o.forward(q=q_host)
    mean = out["mean"].numpy()[rows]
    np.testing.assert_allclose(mean, ref["mean"][rows], rtol=0,
                               atol=1e-13 * float(np.abs(ref["mean"]).max()) + 1e-12)
    lam = out["lam"].cpu().numpy()
    err = PT.check_eig_mixed(lam, ref["lam"], n=5, rtol=1e-4)
    phi = out["phi"][ERA_MODE_BINS].numpy()
    n_valid = out["n_valid"].cpu().numpy()[ERA_MODE_BINS]
    msin, count = PT.check_modes(phi, ref["phi_sel"], ref["lam"][ERA_MODE_BINS], p.weights,
                                 n_valid, sin_tol=1e-3, elem_tol=1e-2, rel_gap=1e-3)
    print(f"era out-of-core fp16x4: eigenvalue rel err {err:.2e} over 257 bins, mode sine "
          f"{msin:.2e} over {count} modes", flush=True)
    assert int(out["info"].min()) > 0
    del out, q_host
    o.close()
    plan.close()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def era_modes(era):
    """The oracle's full modes of three frequencies of the ERA-like field (from
    the era fixture's second pass)."""
    ref = era[2]
    bins = [3, 8, 17]
    idx = [ERA_MODE_BINS.index(b) for b in bins]
    return bins, {"phi": ref["phi_sel"][idx], "mean": ref["mean"]}


def test_era_field_coefficients_and_reconstruction(era, era_modes):
    """Coefficients over 15 modes (5 of 3 frequencies) of the full field, and a
    reconstruction, by the kernels on the oracle's modes: coefficients compared
    at 16 time columns, the reconstruction at 256 rows."""
    from oracle import coeffs as OC
    p, rows, _ = era
    bins, ref = era_modes
    plan = _plan(p, "fp64")
    K, M, nt = plan.nfreq, plan.M, plan.nt
    phi = torch.zeros((K, 5, M), dtype=torch.complex128, device="cuda")
    phi[bins] = torch.as_tensor(ref["phi"]).cuda()
    mean = torch.as_tensor(ref["mean"]).cuda()
    a, info = plan.coeffs(p.q, mean, phi, bins, 5)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    cols = np.arange(0, nt, nt // 16)
    Phi = OC.gather_modes(ref["phi"], [0, 1, 2], 5)
    B = OC.mode_gram(Phi, p.weights)
    rhs = OC.projection_rhs(Phi, p.weights, p.q[:, cols].cpu().double().numpy(), ref["mean"])
    a_ref = np.linalg.solve(B, rhs)
    err = float(np.abs(a[:, cols].cpu().numpy() - a_ref).max() / np.abs(a_ref).max())
    print(f"era coefficients (R = 15, FP64): rel err {err:.2e} at 16 columns")
    assert err <= 1e-12
    # reconstruction from seeded coefficients
    rng = np.random.Generator(np.random.PCG64(21))
    a_in = rng.standard_normal((15, nt)) + 1j * rng.standard_normal((15, nt))
    rec = plan.reconstruct(phi, bins, 5, torch.as_tensor(a_in).cuda(), mean, dtype=torch.float32)
    rec_rows = rec[torch.as_tensor(rows, device="cuda")].cpu().double().numpy()
    rec_ref = np.real(Phi[rows] @ a_in) + ref["mean"][rows, None]
    rerr = float(np.abs(rec_rows - rec_ref).max() / np.abs(rec_ref).max())
    print(f"era reconstruction (float32 output): rel err {rerr:.2e} at 256 rows")
    assert rerr <= 1e-6
    del a, rec, phi
    plan.close()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# the paper's jet analysis block structure: N_f = 256, 50% overlap, L = 155
# blocks, on the jet-like field (256 x 128 x 3, N_t = 19,968 float32)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def jet155():
    p = fields.jet_like(seed=2, nt=19968, device="cuda", dtype=torch.float32)
    assert fields.block_count_of(p.nt, p.nfft, p.noverlap) == 155
    q_host = p.q.cpu().numpy()
    bins = [0, 10, 20, 35, 50, 77, 100, 128]
    t = time.perf_counter()
    ref = O.spod_chunked(q_host, p.nfft, p.noverlap, weights=p.weights, n_modes=5,
                         chunk=8192, bins=bins, want_modes=False)
    print(f"[jet155 fixture] oracle Gram and Jacobi at 8 bins: {time.perf_counter() - t:.0f} s",
          flush=True)
    del q_host
    return p, bins, ref


@pytest.mark.parametrize("precision", ["fp64", "fp16x4"])
def test_jet_155_blocks_full_size(jet155, precision):
    p, bins, ref = jet155
    plan = _plan(p, precision)
    assert plan.nblocks == 155
    out = plan.forward(p.q, n_modes=5)
    torch.cuda.synchronize()
    lam = out["lam"].index_select(0, torch.as_tensor(bins, device="cuda")).cpu().numpy()
    if precision == "fp64":
        err = PT.check_eig(lam, ref["lam"], rtol=1e-10, n=5)
    else:
        err = PT.check_eig_mixed(lam, ref["lam"], n=5, rtol=1e-4)
    assert int(out["info"].min()) > 0
    print(f"jet L = 155 {precision}: leading-5 eigenvalue rel err {err:.2e} at 8 bins", flush=True)
    del out
    plan.close()
    torch.cuda.empty_cache()
