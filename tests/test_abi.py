"""C ABI checks that need no GPU: the library loads, exports every function that
include/spod.h declares, and rejects bad arguments before touching HIP."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2309_11808_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(spod_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        pytest.fail("libspod.so is not built (run `python -m paper_2309_11808_amd.build`)")
    return N.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (spod_[a-z0-9_]+)$", out, flags=re.M))
    missing = declared - exported
    assert not missing, f"declared but not exported: {sorted(missing)}"
    for name in declared:
        assert hasattr(lib, name)


def test_binding_signature_table_matches_header():
    assert set(N.SIGNATURES) == _declared()


def test_status_strings(lib):
    for code, name in [(0, b"SPOD_OK"), (-1, b"SPOD_ERR_INVALID_ARG"), (-2, b"SPOD_ERR_UNSUPPORTED"),
                       (-3, b"SPOD_ERR_ALLOC"), (-4, b"SPOD_ERR_HIP"), (-5, b"SPOD_ERR_NUMERIC"),
                       (-6, b"SPOD_ERR_WORKSPACE"), (-7, b"SPOD_ERR_IO"),
                       (-8, b"SPOD_ERR_INTERNAL")]:
        assert lib.spod_status_string(code) == name
    assert lib.spod_status_string(-99) == b"SPOD_ERR_UNKNOWN"


def test_destroy_null_is_safe(lib):
    lib.spod_plan_destroy(None)


def test_shape_helper(lib):
    L, K = C.c_int64(), C.c_int64()
    assert lib.spod_shape(8192, 512, 256, C.byref(L), C.byref(K)) == 0
    assert (L.value, K.value) == (31, 257)
    assert lib.spod_shape(20000, 256, 128, C.byref(L), C.byref(K)) == 0 and L.value == 155
    assert lib.spod_shape(100, 64, 64, C.byref(L), C.byref(K)) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_shape(100, 1, 0, C.byref(L), C.byref(K)) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_shape(63, 64, 0, C.byref(L), C.byref(K)) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_shape(95, 64, 32, C.byref(L), C.byref(K)) == N.SPOD_ERR_INVALID_ARG   # L = 1
    assert lib.spod_shape(96, 64, 32, C.byref(L), C.byref(K)) == 0 and L.value == 2


def _create(lib, nspace=16, nvar=1, nt=256, nfft=64, nov=32, window=None, weights=None):
    h = C.c_void_p()
    w = None if window is None else (C.c_double * len(window))(*window)
    W = None if weights is None else (C.c_double * len(weights))(*weights)
    st = lib.spod_plan_create(nspace, nvar, nt, nfft, nov, w, W, C.byref(h))
    return st, h


@pytest.mark.parametrize("kw,expect", [
    (dict(nspace=0), N.SPOD_ERR_INVALID_ARG),
    (dict(nvar=0), N.SPOD_ERR_INVALID_ARG),
    (dict(nfft=1, nov=0), N.SPOD_ERR_INVALID_ARG),
    (dict(nov=64), N.SPOD_ERR_INVALID_ARG),
    (dict(nov=-1), N.SPOD_ERR_INVALID_ARG),
    (dict(nt=63), N.SPOD_ERR_INVALID_ARG),
    (dict(nt=64, nov=0), N.SPOD_ERR_INVALID_ARG),          # a single block: L - 1 = 0
    (dict(window=[0.0] * 64), N.SPOD_ERR_INVALID_ARG),
    (dict(window=[1.0] * 63 + [float("nan")]), N.SPOD_ERR_INVALID_ARG),
    (dict(weights=[1.0] * 15 + [-1.0]), N.SPOD_ERR_INVALID_ARG),
    (dict(weights=[0.0] * 16), N.SPOD_ERR_INVALID_ARG),
    (dict(weights=[1.0] * 15 + [float("inf")]), N.SPOD_ERR_INVALID_ARG),
    (dict(nfft=20481, nov=0, nt=40962), N.SPOD_ERR_UNSUPPORTED),   # above the LDS transform
    (dict(nfft=4, nov=2, nt=64), N.SPOD_ERR_UNSUPPORTED),
])
def test_plan_create_rejects_before_any_hip_call(lib, kw, expect):
    st, h = _create(lib, **kw)
    assert st == expect
    assert h.value is None
    assert lib.spod_last_error().startswith(lib.spod_status_string(expect))


def test_plan_create_null_out(lib):
    assert lib.spod_plan_create(16, 1, 256, 64, 32, None, None, None) == N.SPOD_ERR_INVALID_ARG


def test_null_plan_is_rejected_by_every_stage(lib):
    assert lib.spod_plan_set_precision(None, 0) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_plan_set_option(None, 0, 1) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_plan_query(None, None, None, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_blocks_fft(None, None, 0, None, None, None, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_csd(None, None, None, None, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_eig(None, None, None, None, None, None, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_modes(None, None, None, None, 1, None, None, None, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_backward(None, None, 0, None, None, None, None, None, 1, None, 0, None,
                             None, None, 0, None) == N.SPOD_ERR_INVALID_ARG


def test_valid_plan_without_gpu_reports_hip_error_or_succeeds(lib):
    st, h = _create(lib)
    if st == 0:                      # a GPU is present: the plan is usable
        L, K, ws = C.c_int64(), C.c_int64(), C.c_size_t()
        assert lib.spod_plan_query(h, C.byref(L), C.byref(K), C.byref(ws)) == 0
        assert (L.value, K.value) == (7, 33)
        lib.spod_plan_destroy(h)
    else:
        assert st == N.SPOD_ERR_HIP


def test_batch_entry_points_reject_null_and_bad_problems(lib):
    out = C.c_void_p()
    assert lib.spod_batch_create(None, 1, 0, 5, C.byref(out)) == N.SPOD_ERR_INVALID_ARG
    probs = (N.SpodProblem * 1)(N.SpodProblem(16, 1, 256, 64, 32, None, None))
    assert lib.spod_batch_create(probs, 1, 0, 5, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_create(probs, 0, 0, 5, C.byref(out)) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_create(probs, 1, 0, 0, C.byref(out)) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_create(probs, 1, 9, 5, C.byref(out)) == N.SPOD_ERR_INVALID_ARG
    # problem validation happens before any HIP call, with the problem's index
    bad = (N.SpodProblem * 2)(N.SpodProblem(16, 1, 256, 64, 32, None, None),
                              N.SpodProblem(16, 1, 256, 48, 24, None, None))
    st = lib.spod_batch_create(bad, 2, 0, 5, C.byref(out))
    assert st in (N.SPOD_ERR_UNSUPPORTED, N.SPOD_ERR_HIP)   # HIP: no device to create plan 0
    assert out.value is None
    assert lib.spod_batch_set_option(None, 0, 1) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_query(None, None, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_item_info(None, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_forward(None, None, 0, None, None, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_batch_autotune(None, None, 0, None, None, 0, None, None,
                                   None) == N.SPOD_ERR_INVALID_ARG
    lib.spod_batch_destroy(None)


def test_out_of_core_entry_points_reject_null(lib):
    out = C.c_void_p()
    assert lib.spod_ooc_create(None, 0, 256, 1, 0, C.byref(out)) == N.SPOD_ERR_INVALID_ARG
    assert out.value is None
    assert lib.spod_ooc_create(None, 0, 256, 1, 0, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_ooc_query(None, None, None, None, None, None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_ooc_forward(None, None, N.READ_FN(), None, None, None, None, None, None, None,
                                None) == N.SPOD_ERR_INVALID_ARG
    lib.spod_ooc_destroy(None)


def test_coefficient_entry_points_reject_null(lib):
    ws = C.c_size_t()
    assert lib.spod_coeffs_query(None, 1, 1, C.byref(ws)) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_coeffs(None, None, 0, None, None, 1, None, 1, 1, None, None, None, 0,
                           None) == N.SPOD_ERR_INVALID_ARG
    assert lib.spod_reconstruct(None, None, 1, None, 1, 1, None, None, None, 0,
                                None) == N.SPOD_ERR_INVALID_ARG
