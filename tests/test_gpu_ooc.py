"""Out-of-core SPOD (spod_ooc_*), MI355X only.

The snapshot matrix is streamed to the device in chunks of rows, twice.  The
results must match the FP64 oracle, whose chunked form is the same two-pass
spatial split.  With one chunk they must match the in-memory path bit for bit.
Every source (device memory, pinned or pageable host memory, a numpy array, a
reader) and every count of resident chunks runs the same kernels on the same
chunks, so those results must be bit-identical to each other.
"""
import numpy as np
import pytest
import torch

import oracle as O
from synth import fields
from tests import parity as PT

pytestmark = pytest.mark.gpu

KEYS = ("mean", "lam", "psi", "info", "phi", "n_valid")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2309_11808_amd  # noqa: F401
    yield


def _plan(p, precision):
    from paper_2309_11808_amd import Plan
    return Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, weights=p.weights, precision=precision)


def _cpu(t):
    return t.cpu() if isinstance(t, torch.Tensor) else torch.as_tensor(t)


def _same(a, b, what):
    for k in KEYS:
        x, y = _cpu(a[k]), _cpu(b[k])
        assert x.shape == y.shape, (what, k, x.shape, y.shape)
        assert torch.equal(x, y), f"{what}: {k} differs"


def _reader(qn, calls):
    def read(row0, nrows, out):
        calls.append((row0, nrows))
        out[:] = qn[row0:row0 + nrows]
    return read


def _sources(q):
    """Every way to hand the snapshots over: (name, forward kwargs, reader calls)."""
    qn = q.numpy()
    calls = []
    return [("device", {"q": q.cuda()}, None),
            ("pinned", {"q": q.pin_memory()}, None),
            ("pageable", {"q": q.clone()}, None),
            ("numpy", {"q": qn.copy()}, None),
            ("reader", {"reader": _reader(qn, calls)}, calls)]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x4", "fp16x4"])
def test_one_chunk_bit_identical_to_in_memory(precision):
    from paper_2309_11808_amd import OutOfCore
    dt = torch.float64 if precision == "fp64" else torch.float32
    p = fields.random_rows(1500, 21 * 32 + 40, 64, 32, seed=21, offset=0.5, dtype=dt)
    plan = _plan(p, precision)
    ref = plan.forward(p.q.cuda(), n_modes=4)
    torch.cuda.synchronize()
    ref = {k: ref[k].clone() for k in KEYS}
    o = OutOfCore(plan, dtype=dt, chunk_rows=1 << 20, n_modes=4)
    assert (o.n_chunks, o.chunk_rows) == (1, p.M)
    _same(o.forward(q=p.q.cuda()), ref, f"{precision} one chunk, device q")
    _same(o.forward(q=p.q.pin_memory()), ref, f"{precision} one chunk, pinned q")
    o.close()
    plan.close()


@pytest.fixture(scope="module")
def rows_fp64():
    # 2000 rows in chunks of 256: seven full chunks and a ragged one of 208
    p = fields.random_rows(2000, 19 * 32 + 64 + 5, 64, 32, seed=23, offset=0.3,
                           dtype=torch.float64)
    ref = O.spod(p.q.numpy(), 64, 32, weights=p.weights, n_modes=3)
    return p, ref


def test_chunks_fp64_match_oracle_for_every_source_and_residency(rows_fp64):
    from paper_2309_11808_amd import OutOfCore
    p, ref = rows_fp64
    plan = _plan(p, "fp64")
    chunks = [(r, min(256, p.M - r)) for r in range(0, p.M, 256)]
    first = None
    for resident in (0, 3, 8, 20):
        o = OutOfCore(plan, dtype=torch.float64, chunk_rows=200, n_modes=3, resident=resident)
        assert (o.chunk_rows, o.n_chunks, o.resident) == (256, 8, min(resident, 8))
        for name, kw, calls in _sources(p.q):
            out = o.forward(**kw)
            what = f"resident={resident} source={name}"
            if first is None:
                first = {k: out[k].clone() for k in KEYS}
                PT.check_eig(out["lam"], ref["lam"], rtol=1e-10)
                np.testing.assert_allclose(out["mean"].numpy(), ref["mean"], rtol=0,
                                           atol=1e-14 * float(np.abs(p.q.numpy()).max()))
                np.testing.assert_array_equal(out["n_valid"].cpu().numpy(), ref["n_valid"])
                PT.check_invalid_modes_zero(out["phi"], out["n_valid"].cpu().numpy())
                s, n = PT.check_modes(out["phi"], ref["phi"], ref["lam"], p.weights,
                                      ref["n_valid"], sin_tol=1e-8, elem_tol=1e-6, rel_gap=1e-6)
                assert n > 50
                assert int(out["info"].min()) > 0
            else:
                _same(out, first, what)
            if calls is not None:
                # pass 1 reads every chunk in order, pass 2 the ones not kept
                expect = chunks + chunks[:len(chunks) - o.resident]
                assert calls == expect, what
        o.close()
    plan.close()


def test_outputs_on_device_and_in_pageable_memory(rows_fp64):
    from paper_2309_11808_amd import OutOfCore
    p, _ = rows_fp64
    plan = _plan(p, "fp64")
    o = OutOfCore(plan, dtype=torch.float64, chunk_rows=512, n_modes=3, resident=1)
    base = o.forward(q=p.q.cuda())
    base = {k: v.clone() for k, v in base.items()}
    K, M = plan.nfreq, plan.M
    for phi, mean in ((torch.empty((K, 3, M), dtype=torch.complex128, device="cuda"),
                       torch.empty(M, dtype=torch.float64, device="cuda")),
                      (torch.empty((K, 3, M), dtype=torch.complex128),
                       torch.empty(M, dtype=torch.float64))):
        out = o.forward(q=p.q.pin_memory(), phi=phi, mean=mean)
        assert out["phi"] is phi and out["mean"] is mean
        _same(out, base, f"phi on {phi.device}")
    o.close()
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x4", "fp16x4"])
def test_chunks_mixed_match_oracle(precision):
    from paper_2309_11808_amd import OutOfCore
    p = fields.planted(nspace=3000, seed=5, sigma=0.1, dtype=torch.float32)
    o_ref = O.spod(p.q.numpy(), 128, 64, weights=p.weights, n_modes=5, eps=1e-6)
    plan = _plan(p, precision)
    o = OutOfCore(plan, dtype=torch.float32, chunk_rows=700, n_modes=5, resident=1)
    assert o.n_chunks == 4                           # 768, 768, 768, 696 rows
    out = o.forward(q=p.q.numpy())
    PT.check_eig_mixed(out["lam"], o_ref["lam"], p.M, n=5)
    s, n = PT.check_modes(out["phi"], o_ref["phi"], o_ref["lam"], p.weights, o_ref["n_valid"],
                          sin_tol=1e-3, elem_tol=1e-2, rel_gap=1e-3)
    assert n > 100
    # the same plan in memory: only the order of the Gram sums differs
    g = plan.forward(p.q.cuda(), n_modes=5)
    PT.check_eig_mixed(out["lam"], g["lam"], p.M, n=5, rtol=1e-5)
    o.close()
    plan.close()


def test_reader_failure_is_reported_and_the_object_stays_usable(rows_fp64):
    from paper_2309_11808_amd import OutOfCore, SpodError
    p, _ = rows_fp64
    plan = _plan(p, "fp64")
    o = OutOfCore(plan, dtype=torch.float64, chunk_rows=256, n_modes=3)
    qn = p.q.numpy()
    good = o.forward(q=p.q.cuda())
    good = {k: v.clone() for k, v in good.items()}
    for fail_at in (0, 5, 10):                       # pass 1 start, pass 1, pass 2
        seen = []

        def bad(row0, nrows, out):
            seen.append(row0)
            if len(seen) == fail_at + 1:
                raise OSError("disk went away")
            out[:] = qn[row0:row0 + nrows]
        with pytest.raises(SpodError) as ei:
            o.forward(reader=bad)
        assert ei.value.status == -7
        assert isinstance(ei.value.__cause__, OSError)
        assert len(seen) == fail_at + 1
    _same(o.forward(reader=_reader(qn, [])), good, "after reader failures")
    o.close()
    plan.close()


def test_bad_arguments():
    from paper_2309_11808_amd import OutOfCore, SpodError
    p = fields.random_rows(300, 512, 64, 32, seed=3, dtype=torch.float32)
    plan = _plan(p, "bf16x4")
    for kw in (dict(chunk_rows=0), dict(n_modes=0), dict(n_modes=plan.nblocks + 1),
               dict(resident=-1)):
        args = dict(dtype=torch.float32, chunk_rows=256, n_modes=2, resident=0)
        args.update(kw)
        with pytest.raises(SpodError) as ei:
            OutOfCore(plan, **args)
        assert ei.value.status == -1
    o = OutOfCore(plan, dtype=torch.float32, chunk_rows=256, n_modes=2)
    with pytest.raises(ValueError):
        o.forward()
    with pytest.raises(ValueError):
        o.forward(q=p.q, reader=lambda *a: None)
    with pytest.raises(TypeError):
        o.forward(q=p.q.double())
    with pytest.raises(ValueError):
        o.forward(q=p.q[:100])
    o.close()
    plan.close()


def test_chunks_with_a_general_block_length():
    """Out-of-core with N_f = 60 (the mixed-radix transform) against the oracle."""
    from paper_2309_11808_amd import OutOfCore
    p = fields.random_rows(900, 9 * 30 + 60, 60, 30, seed=61, offset=0.4, dtype=torch.float64)
    ref = O.spod(p.q.numpy(), 60, 30, weights=p.weights, n_modes=3)
    plan = _plan(p, "fp64")
    o = OutOfCore(plan, dtype=torch.float64, chunk_rows=256, n_modes=3, resident=1)
    assert o.n_chunks == 4
    out = o.forward(q=p.q.numpy())
    PT.check_eig(out["lam"], ref["lam"], rtol=1e-10)
    s, n = PT.check_modes(out["phi"], ref["phi"], ref["lam"], p.weights, ref["n_valid"],
                          sin_tol=1e-8, elem_tol=1e-6, rel_gap=1e-6)
    assert n > 20
    o.close()
    plan.close()
