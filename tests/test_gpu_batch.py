"""Batches of uneven problems (spod_batch_*), MI355X only.

A batch runs the single-problem kernels through grouped launches, so every
problem's results must be bit-identical to the single-problem path with the
same Gram split (except complex64 blocks of an odd M, which the batch stores
with an even row stride and sums in another order); the small problems are
also checked against the FP64 oracle.
"""
import json
import os

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


def _small_specs(count, seed, max_space=3000):
    """The batch generator's shape mix with nspace scaled down."""
    specs = fields.batch_specs(seed=seed, count=count)
    out = []
    for s in specs:
        s = dict(s)
        s["nspace"] = 50 + s["nspace"] % max_space
        out.append(s)
    return out


def _problems(specs, dtype=torch.float32):
    return [fields.batch_problem(s, dtype=dtype, device="cuda") for s in specs]


def _desc(p, window=None):
    return {"nspace": p.nspace, "nvar": p.nvar, "nt": p.nt, "nfft": p.nfft,
            "noverlap": p.noverlap, "weights": p.weights, "window": window}


def _single(p, precision, n_modes, window=None):
    from paper_2309_11808_amd import Plan
    plan = Plan(p.nspace, p.nvar, p.nt, p.nfft, p.noverlap, window=window, weights=p.weights,
                precision=precision)
    out = plan.forward(p.q, min(n_modes, plan.nblocks))
    torch.cuda.synchronize()
    res = {k: out[k].clone() for k in KEYS}
    plan.close()
    return res


def _close(a, b, precision, M, what):
    """Odd M with complex64 blocks: the grouped launch stores the blocks with an
    even row stride and takes the vectorised Gram, whose sum order differs from
    the single-problem path's; the rest of the path is the same arithmetic."""
    assert torch.equal(a["mean"], b["mean"]), f"{what}: mean"
    assert torch.equal(a["n_valid"], b["n_valid"]), f"{what}: n_valid"
    assert int(a["info"].min()) > 0
    PT.check_eig_mixed(a["lam"], b["lam"], M, n=a["phi"].shape[1], rtol=1e-5)


def _same(a, b, what):
    for k in KEYS:
        x, y = a[k], b[k]
        assert x.shape == y.shape, (what, k, x.shape, y.shape)
        assert torch.equal(x, y), f"{what}: {k} differs"


@pytest.mark.parametrize("precision", ["fp64", "bf16x4", "fp16x4", "fp32"])
def test_batch_bit_identical_to_single_path(precision):
    from paper_2309_11808_amd import Batch
    specs = _small_specs(16, seed=4)
    probs = _problems(specs)
    n_modes = 5
    ref = [_single(p, precision, n_modes) for p in probs]
    for grouped, graph in ((True, True), (True, False), (False, False), (False, True)):
        b = Batch([_desc(p) for p in probs], precision=precision, n_modes=n_modes,
                  grouped=grouped, graph=graph)
        res = b.forward([p.q for p in probs])
        torch.cuda.synchronize()
        for i, (r, s, p) in enumerate(zip(res, ref, probs)):
            what = f"{precision} grouped={grouped} graph={graph} problem {i}"
            if grouped and precision != "fp64" and p.M % 2 == 1:
                _close(r, s, precision, p.M, what)
            else:
                _same(r, s, what)
        b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x4"])
def test_batch_launch_shapes_bit_identical(precision):
    """The transform tile, the eigensolver's thread count and persistent
    workgroups change how the work is mapped, not the arithmetic."""
    from paper_2309_11808_amd import Batch
    specs = _small_specs(12, seed=9)
    probs = _problems(specs)
    descs = [_desc(p) for p in probs]
    base = Batch(descs, precision=precision, n_modes=4)
    ref = [{k: v.clone() for k, v in r.items()} for r in base.forward([p.q for p in probs])]
    torch.cuda.synchronize()
    base.close()
    for tile, nt, pers, graph in ((16, 256, True, True), (32, 1024, True, False),
                                  (32, 256, False, True), (16, 1024, True, True)):
        b = Batch(descs, precision=precision, n_modes=4, fft_tile=tile, eig_threads=nt,
                  persistent=pers, graph=graph)
        assert b.shapes()["fft_tile"] == tile and b.shapes()["persistent"] == int(pers)
        for rep in range(2):
            res = b.forward([p.q for p in probs])
            torch.cuda.synchronize()
            for i, (r, f) in enumerate(zip(res, ref)):
                _same(r, f, f"tile {tile} threads {nt} persistent {pers} graph {graph} "
                            f"pass {rep} problem {i}")
        b.close()


def test_batch_small_problems_match_oracle():
    from paper_2309_11808_amd import Batch
    specs = _small_specs(8, seed=11, max_space=400)
    probs = _problems(specs, dtype=torch.float64)
    b = Batch([_desc(p) for p in probs], precision="fp64", n_modes=3)
    res = b.forward([p.q for p in probs])
    torch.cuda.synchronize()
    for p, r in zip(probs, res):
        ref = O.spod(p.q.cpu().numpy(), p.nfft, p.noverlap, weights=p.weights, n_modes=3)
        PT.check_eig(r["lam"], ref["lam"], rtol=1e-10)
        np.testing.assert_allclose(r["mean"].cpu().numpy(), ref["mean"], rtol=0,
                                   atol=1e-14 * float(np.abs(p.q.cpu().numpy()).max()))
        PT.check_modes(r["phi"], ref["phi"], ref["lam"], p.weights, r["n_valid"].cpu().numpy(),
                       sin_tol=1e-8, elem_tol=1e-6, rel_gap=1e-6)
    b.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_graph_replays_and_new_buffers(persistent):
    """Replays see new values and stay equal; with persistent workgroups the
    queue counters are zeroed by a kernel inside the graph on every replay."""
    from paper_2309_11808_amd import Batch
    specs = _small_specs(10, seed=5)
    probs = _problems(specs)
    b = Batch([_desc(p) for p in probs], precision="bf16x4", n_modes=4, persistent=persistent)
    first = [{k: v.clone() for k, v in r.items()} for r in b.forward([p.q for p in probs])]
    torch.cuda.synchronize()
    for rep in range(3):
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        res = b.forward([p.q for p in probs])
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, (r, f) in enumerate(zip(res, first)):
            _same(r, f, f"replay {rep} problem {i}")
    # new input buffers (same values): tables rebuilt, graph recaptured
    qs2 = [p.q.clone() for p in probs]
    res = b.forward(qs2)
    torch.cuda.synchronize()
    for i, (r, f) in enumerate(zip(res, first)):
        _same(r, f, f"new buffers problem {i}")
    # new values in the same buffers: the graph sees them
    for q in qs2:
        q.mul_(2.0)
    res = b.forward(qs2)
    torch.cuda.synchronize()
    for i, (r, f) in enumerate(zip(res, first)):
        torch.testing.assert_close(r["lam"], 4.0 * f["lam"], rtol=1e-5, atol=1e-6 * float(f["lam"].max()))
    b.close()


def test_batch_windows_and_overlaps_fall_back_per_problem():
    """Problems the grouped transform does not take (a window with every DFT
    bin non-zero, 75% overlap) run their own transform inside the batch."""
    from paper_2309_11808_amd import Batch
    rng = np.random.Generator(np.random.PCG64(3))
    probs, descs, wins = [], [], []
    for i, (nfft, nov) in enumerate(((64, 32), (128, 96), (32, 16), (256, 128))):
        p = fields.random_rows(97 + 31 * i, 12 * nfft, nfft, nov, seed=i, dtype=torch.float32)
        p.q = p.q.cuda()
        win = rng.uniform(0.2, 1.0, nfft) if i % 2 == 0 else None
        probs.append(p)
        wins.append(win)
        descs.append(_desc(p, win))
    b = Batch(descs, precision="fp64", n_modes=2)
    res = b.forward([p.q for p in probs])
    torch.cuda.synchronize()
    for p, r, w in zip(probs, res, wins):
        _same(r, _single(p, "fp64", 2, w), "fallback")
    b.close()


def test_batch_autotune_and_cache(tmp_path):
    from paper_2309_11808_amd import Batch
    specs = _small_specs(6, seed=6)
    probs = _problems(specs)
    cache = str(tmp_path / "tune.jsonl")
    b = Batch([_desc(p) for p in probs], precision="bf16x4", n_modes=3)
    t = b.autotune([p.q for p in probs], cache_path=cache)
    assert t in (2048, 4096, 8192, 16384)
    lines = open(cache).read().strip().splitlines()
    rec = json.loads(lines[0])
    assert len(lines) == 1 and rec["gram_target"] == t
    shapes = b.shapes()
    assert shapes == {k: rec[k] for k in ("gram_target", "fft_tile", "eig_threads", "persistent")}
    assert shapes["fft_tile"] in (0, 16, 32) and shapes["eig_threads"] in (0, 256, 1024)
    # every candidate was timed: 4 targets, 2 tiles, 2 thread counts, persistent
    assert len(rec["ms"]) == 9 and all(v > 0 for v in rec["ms"].values())
    res = b.forward([p.q for p in probs])
    torch.cuda.synchronize()
    # the tuned split only changes the order of the Gram sums
    for p, r in zip(probs, res):
        s = _single(p, "bf16x4", 3)
        PT.check_eig_mixed(r["lam"], s["lam"], p.M, n=3, rtol=1e-5)
    b.close()
    # a second batch of the same shapes takes the cached choice without timing
    b2 = Batch([_desc(p) for p in probs], precision="bf16x4", n_modes=3)
    assert b2.autotune([p.q for p in probs], cache_path=cache) == t
    assert b2.shapes() == shapes
    assert len(open(cache).read().strip().splitlines()) == 1
    b2.close()
    os.remove(cache)


def test_batch_rejects_bad_arguments():
    from paper_2309_11808_amd import Batch, SpodError
    with pytest.raises(SpodError) as ei:
        Batch([{"nspace": 10, "nvar": 1, "nt": 50000, "nfft": 24000, "noverlap": 12000}])
    assert ei.value.status == -2
    with pytest.raises(SpodError) as ei:
        Batch([{"nspace": 10, "nvar": 1, "nt": 100, "nfft": 32, "noverlap": 32}])
    assert ei.value.status == -1
    p = fields.random_rows(40, 256, 32, 16, seed=1, dtype=torch.float32)
    b = Batch([_desc(p)], precision="fp32")
    with pytest.raises(ValueError):
        b.forward([p.q.cuda()[:20]])
    b.close()


def test_batch_with_general_block_lengths():
    """Problems whose N_f is not a power of two run their own transform inside
    the batch; everything else is the batch's grouped launches."""
    from paper_2309_11808_amd import Batch
    probs, descs = [], []
    for i, (nfft, nov) in enumerate(((64, 32), (60, 30), (128, 64), (100, 50), (73, 0))):
        p = fields.random_rows(150 + 37 * i, 10 * nfft, nfft, nov, seed=70 + i, dtype=torch.float64)
        p.q = p.q.cuda()
        probs.append(p)
        descs.append(_desc(p))
    b = Batch(descs, precision="fp64", n_modes=2)
    res = b.forward([p.q for p in probs])
    torch.cuda.synchronize()
    for i, (p, r) in enumerate(zip(probs, res)):
        _same(r, _single(p, "fp64", 2), f"problem {i} (N_f = {p.nfft})")
        if p.nfft in (60, 73):
            ref = O.spod(p.q.cpu().numpy(), p.nfft, p.noverlap, weights=p.weights, n_modes=2)
            PT.check_eig(r["lam"], ref["lam"], rtol=1e-10)
    b.close()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_of_long_problems_only(graph):
    """Only problems with more than 32 blocks: their chain runs alone on the
    caller's stream (no fork), with the same results as the single path."""
    from paper_2309_11808_amd import Batch
    probs = [fields.random_rows(200 + 61 * i, (40 + 7 * i) * 32 + 32, 64, 32, seed=90 + i,
                                dtype=torch.float32) for i in range(3)]
    for p in probs:
        p.q = p.q.cuda()
    b = Batch([_desc(p) for p in probs], precision="bf16x4", n_modes=4, graph=graph)
    assert [it.nblocks for it in b.items] == [40, 47, 54]
    for rep in range(2):
        res = b.forward([p.q for p in probs])
        torch.cuda.synchronize()
        for i, (r, p) in enumerate(zip(res, probs)):
            s = _single(p, "bf16x4", 4)
            if p.M % 2 == 1:
                _close(r, s, "bf16x4", p.M, f"graph={graph} rep {rep} problem {i}")
            else:
                _same(r, s, f"graph={graph} rep {rep} problem {i}")
    b.close()


def test_batch_full_size_problems_match_oracle():
    """The 64 problems of the batching workload at their real sizes (seed 4,
    46 GB of float32), grouped and replayed from the captured graph in the
    benchmark's precision.  Every problem's leading eigenvalues at three bins
    (low, middle, high) are compared with the oracle (streamed over chunks of
    rows, selected bins), and the modes of the middle bin with the oracle's
    where the problem is small enough to form them in full."""
    from paper_2309_11808_amd import Batch
    specs = fields.batch_specs(seed=4, count=64)
    probs = [fields.batch_problem(s, dtype=torch.float32, device="cuda") for s in specs]
    total = sum(p.q.numel() * 4 for p in probs)
    print(f"[batch full size] 64 problems, {total / 1e9:.1f} GB of float32", flush=True)
    b = Batch([_desc(p) for p in probs], precision="fp16x4", n_modes=5)
    res = b.forward([p.q for p in probs])
    res = b.forward([p.q for p in probs])             # a replay of the captured graph
    torch.cuda.synchronize()
    worst, compared = 0.0, 0
    for i, (p, r) in enumerate(zip(probs, res)):
        K = p.nfft // 2 + 1
        bins = sorted({1, K // 3, (2 * K) // 3})
        q_host = p.q.cpu().numpy()
        mid = K // 3
        rows = None if p.M <= 60000 else np.arange(0, p.M, max(1, p.M // 4096))
        ref = O.spod_chunked(q_host, p.nfft, p.noverlap, weights=p.weights, n_modes=5,
                             chunk=32768, bins=bins, mode_rows=rows)
        lam = r["lam"][bins].cpu().numpy()
        err = PT.check_eig_mixed(lam, ref["lam"], n=5, rtol=1e-4)
        assert int(r["info"].min()) > 0
        nv = r["n_valid"].cpu().numpy()[bins]
        np.testing.assert_array_equal(nv, (ref["lam"][:, :5] > 1e-6 * ref["lam"][:, :1]).sum(axis=1))
        ib = bins.index(mid)
        phi = r["phi"][mid].cpu().numpy()
        if rows is None:
            s, n = PT.check_modes(phi[None], ref["phi"][ib:ib + 1], ref["lam"][ib:ib + 1], p.weights,
                                  nv[ib:ib + 1], sin_tol=1e-3, elem_tol=1e-2, rel_gap=1e-3)
            compared += n
        else:
            for j in range(int(nv[ib])):
                if PT.separated(ref["lam"][ib], j, 1e-3):
                    o = ref["phi"][ib, j]
                    e = np.linalg.norm(phi[j, rows] - o) / np.linalg.norm(o)
                    assert e <= 1e-3, f"problem {i} mode {j}: sampled rows {e:.2e}"
        worst = max(worst, err)
        print(f"[batch full size] problem {i}: M={p.M} nt={p.nt} nfft={p.nfft} L={p.nt // (p.nfft // 2) - 1} "
              f"eigenvalue rel err {err:.2e}", flush=True)
    print(f"[batch full size] worst leading-5 eigenvalue rel err {worst:.2e}; "
          f"{compared} full modes compared", flush=True)
    b.close()
