"""spod_csd_noalloc (the Gram without a caller workspace, for callers that
cannot allocate) against spod_csd, through the C ABI, MI355X only.

Two calls in a row on one device share the library's scratch array: a large
one (257 frequencies, so the slice count is cut to what the 64 MiB array
holds) and then a smaller one, each compared with spod_csd run with the same
slice count (identical arithmetic: bit-identical) and with spod_csd's own
slice count (FP64 summation order only), and with the oracle."""
import ctypes as C

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


def _noalloc(plan, qhat):
    from paper_2309_11808_amd.spod import lib, _check, _stream
    gram = torch.full((plan.nfreq, plan.nblocks, plan.nblocks), 7.0 + 7j, dtype=torch.complex128,
                      device="cuda")
    slices = C.c_int64(-1)
    _check(lib().spod_csd_noalloc(plan._h, C.c_void_p(qhat.data_ptr()), C.c_void_p(gram.data_ptr()),
                                  C.byref(slices), _stream(plan.device)))
    return gram, slices.value


def _plan(p, precision, **opt):
    from paper_2309_11808_amd import Plan
    return Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, weights=p.weights, precision=precision,
                options=opt or None)


@pytest.mark.parametrize("precision", ["fp16x4", "fp64"])
def test_noalloc_gram_matches_workspace_gram_twice(precision):
    from paper_2309_11808_amd import _native as N
    dtype = torch.float64 if precision == "fp64" else torch.float32
    cases = [  # (M, nt, nfft, noverlap): 257 bins and 31 blocks, then 65 bins and 15 blocks
        (20000, 8192, 512, 256),
        (5000, 1024, 128, 64),
    ]
    for M, nt, nfft, nov in cases:
        p = fields.random_rows(M, nt, nfft, nov, seed=M, dtype=dtype)
        plan = _plan(p, precision)
        K, L = plan.nfreq, plan.nblocks
        D = 16 * ((L + 15) // 16)
        qhat, _ = plan.blocks_fft(p.q.cuda())
        g_na, S = _noalloc(plan, qhat)
        torch.cuda.synchronize()
        per_slice = 16 * K * D * D
        assert 1 <= S <= N.SPOD_CSD_NOALLOC_MAX_BYTES // per_slice, (S, per_slice)
        # spod_csd with the same slice count: the same arithmetic
        ref_plan = _plan(p, precision, gram_split=S)
        qh2, _ = ref_plan.blocks_fft(p.q.cuda())
        g_ws = ref_plan.csd(qh2)
        # spod_csd with the plan's own slice count
        g_own = plan.csd(qhat)
        torch.cuda.synchronize()
        assert torch.equal(g_na, g_ws), f"M={M}: not identical to spod_csd with {S} slices"
        PT.check_gram(g_na, g_own, 1e-13)
        # and against the oracle's Gram of the library's own blocks
        qh = qhat.cpu().numpy().astype(np.complex128)
        PT.check_gram(g_na, O.gram(qh, p.weights), 1e-13 if precision == "fp64" else 2e-6)
        print(f"{precision} M={M} K={K} L={L}: {S} slices")
        ref_plan.close()
        plan.close()


def test_noalloc_rejects_what_does_not_fit():
    from paper_2309_11808_amd import _native as N
    from paper_2309_11808_amd.spod import lib, _stream
    # 1025 bins of 64 x 64 partials (67 MB per slice) do not fit the 64 MiB array
    p = fields.random_rows(8, 64 * 1024 + 1024, 2048, 1024, seed=3, dtype=torch.float32)
    plan = _plan(p, "fp16x4")
    assert plan.nblocks == 64 and plan.nfreq == 1025
    qhat = torch.zeros((plan.nfreq, plan.nblocks, plan.M), dtype=torch.complex64, device="cuda")
    gram = torch.zeros((plan.nfreq, 64, 64), dtype=torch.complex128, device="cuda")
    slices = C.c_int64(-1)
    st = lib().spod_csd_noalloc(plan._h, C.c_void_p(qhat.data_ptr()), C.c_void_p(gram.data_ptr()),
                                C.byref(slices), _stream(plan.device))
    assert st == N.SPOD_ERR_UNSUPPORTED and slices.value == 0
    assert lib().spod_csd_noalloc(plan._h, None, C.c_void_p(gram.data_ptr()), None,
                                  _stream(plan.device)) == N.SPOD_ERR_INVALID_ARG
    plan.close()
