"""Thin Python binding of libspod (include/spod.h).

Argument marshalling only: every step of the SPOD path runs in the library's
HIP kernels.  PyTorch provides device memory (output tensors are allocated
with torch.empty when not given) and the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _native as N

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = N.load()
    return _lib


PRECISIONS = {"fp64": N.SPOD_PREC_FP64, "fp32": N.SPOD_PREC_FP32, "bf16x4": N.SPOD_PREC_BF16X4,
              "fp16x4": N.SPOD_PREC_FP16X4}


def _check(status: int):
    if status != N.SPOD_OK:
        L = lib()
        msg = L.spod_last_error().decode() or L.spod_status_string(status).decode()
        raise N.SpodError(status, msg)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def shape(nt: int, nfft: int, noverlap: int):
    """(nblocks, nfreq) for a problem, validated by the library (host only)."""
    L, K = C.c_int64(), C.c_int64()
    _check(lib().spod_shape(nt, nfft, noverlap, C.byref(L), C.byref(K)))
    return L.value, K.value


class Plan:
    """A libspod plan: problem shape, window, weights, precision and options."""

    def __init__(self, nspace: int, nvar: int, nt: int, nfft: int, noverlap: int, window=None,
                 weights=None, precision: str = "fp64", options: Optional[dict] = None,
                 device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.nspace, self.nvar, self.nt, self.nfft, self.noverlap = nspace, nvar, nt, nfft, noverlap
        self.M = nspace * nvar
        self._win = None if window is None else np.ascontiguousarray(window, dtype=np.float64)
        self._w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        if self._win is not None and self._win.shape != (nfft,):
            raise ValueError("window must have nfft entries")
        if self._w is not None and self._w.shape != (self.M,):
            raise ValueError("weights must have nspace*nvar entries")
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().spod_plan_create(
                nspace, nvar, nt, nfft, noverlap,
                None if self._win is None else self._win.ctypes.data_as(C.c_void_p),
                None if self._w is None else self._w.ctypes.data_as(C.c_void_p), C.byref(h)))
        self._h = h
        self.precision = precision
        _check(lib().spod_plan_set_precision(self._h, PRECISIONS[precision]))
        self.packed = False
        for k, v in (options or {}).items():
            if k == "qhat_format":
                v = {"complex": N.SPOD_QHAT_COMPLEX, "bfp20": N.SPOD_QHAT_BFP20}[v]
                self.packed = v == N.SPOD_QHAT_BFP20
            opt = {"max_sweeps": N.SPOD_OPT_MAX_SWEEPS, "gram_split": N.SPOD_OPT_GRAM_SPLIT,
                   "fft_tile": N.SPOD_OPT_FFT_TILE, "qhat_format": N.SPOD_OPT_QHAT_FORMAT,
                   "modes_kernel": N.SPOD_OPT_MODES_KERNEL,
                   "general_passes": N.SPOD_OPT_GENERAL_PASSES}[k]
            if k == "modes_kernel":
                v = {"valu": 0, "mfma": 1}.get(v, v)
            _check(lib().spod_plan_set_option(self._h, opt, int(v)))
        L, K, ws = C.c_int64(), C.c_int64(), C.c_size_t()
        _check(lib().spod_plan_query(self._h, C.byref(L), C.byref(K), C.byref(ws)))
        self.nblocks, self.nfreq, self.workspace_bytes = L.value, K.value, ws.value
        qb = C.c_size_t()
        _check(lib().spod_plan_qhat_bytes(self._h, C.byref(qb)))
        self.qhat_bytes = qb.value
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self._ws = None

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().spod_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ------------------------------------------------------------
    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            self._ws = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=self.device)
        return self._ws

    def _dev(self, t: torch.Tensor, name: str, dtype, shape):
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _out(self, t, name, dtype, shape):
        if t is None:
            return torch.empty(shape, dtype=dtype, device=self.device)
        return self._dev(t, name, dtype, shape)

    def _q(self, q: torch.Tensor):
        if q.dtype not in (torch.float32, torch.float64):
            raise TypeError("q must be float32 or float64")
        self._dev(q, "q", q.dtype, (self.M, self.nt))
        return N.SPOD_F32 if q.dtype == torch.float32 else N.SPOD_F64

    def _qhat(self, qhat, name="qhat"):
        """qhat as the plan stores it: complex [K, L, M], or the packed
        20-bit layout as a uint8 tensor of qhat_bytes (SPOD_QHAT_BFP20)."""
        if self.packed:
            return self._out(qhat, name, torch.uint8, (self.qhat_bytes,))
        return self._out(qhat, name, self.cdtype, (self.nfreq, self.nblocks, self.M))

    # -- stages -------------------------------------------------------------
    def blocks_fft(self, q, qhat=None, mean=None, want_mean: bool = True):
        dt = self._q(q)
        qhat = self._qhat(qhat)
        if want_mean or mean is not None:
            mean = self._out(mean, "mean", torch.float64, (self.M,))
        ws = self.workspace()
        _check(lib().spod_blocks_fft(self._h, _ptr(q), dt, _ptr(qhat), _ptr(mean), _ptr(ws),
                                     ws.numel(), _stream(self.device)))
        return qhat, mean

    def csd(self, qhat, gram=None):
        self._qhat(qhat)
        gram = self._out(gram, "gram", torch.complex128, (self.nfreq, self.nblocks, self.nblocks))
        ws = self.workspace()
        _check(lib().spod_csd(self._h, _ptr(qhat), _ptr(gram), _ptr(ws), ws.numel(),
                              _stream(self.device)))
        return gram

    def eig(self, gram, lam=None, psi=None, info=None):
        L, K = self.nblocks, self.nfreq
        self._dev(gram, "gram", torch.complex128, (K, L, L))
        lam = self._out(lam, "lam", torch.float64, (K, L))
        psi = self._out(psi, "psi", torch.complex128, (K, L, L))
        info = self._out(info, "info", torch.int32, (K,))
        ws = self.workspace()
        _check(lib().spod_eig(self._h, _ptr(gram), _ptr(lam), _ptr(psi), _ptr(info), _ptr(ws),
                              ws.numel(), _stream(self.device)))
        return lam, psi, info

    def modes(self, qhat, lam, psi, n_modes: int, phi=None, n_valid=None):
        L, K = self.nblocks, self.nfreq
        self._qhat(qhat)
        self._dev(lam, "lam", torch.float64, (K, L))
        self._dev(psi, "psi", torch.complex128, (K, L, L))
        phi = self._out(phi, "phi", self.cdtype, (K, n_modes, self.M))
        n_valid = self._out(n_valid, "n_valid", torch.int32, (K,))
        ws = self.workspace()
        _check(lib().spod_modes(self._h, _ptr(qhat), _ptr(lam), _ptr(psi), n_modes, _ptr(phi),
                                _ptr(n_valid), _ptr(ws), ws.numel(), _stream(self.device)))
        return phi, n_valid

    def backward(self, q, lam, psi, g_lam=None, g_phi=None, n_modes: int = 0, bins=None,
                 qhat=None, g_qhat=None, g_q=None):
        """dE/dq from dE/dlam and dE/dphi (spod_backward).

        bins: optional increasing frequencies; g_lam [nb, L] and g_phi [nb, n, M]
        then hold only those rows.  qhat: the forward's Fourier blocks, or None
        to recompute them (selected bins only) into g_qhat."""
        dt = self._q(q)
        L, K = self.nblocks, self.nfreq
        self._dev(lam, "lam", torch.float64, (K, L))
        self._dev(psi, "psi", torch.complex128, (K, L, L))
        sel = None
        nb = K
        if bins is not None:
            sel = np.ascontiguousarray(np.asarray(bins, dtype=np.int32).reshape(-1))
            nb = int(sel.size)
        if g_lam is not None:
            self._dev(g_lam, "g_lam", torch.float64, (nb, L))
        if g_phi is not None:
            self._dev(g_phi, "g_phi", self.cdtype, (nb, n_modes, self.M))
        if qhat is not None:
            self._dev(qhat, "qhat", self.cdtype, (K, L, self.M))
        g_qhat = self._out(g_qhat, "g_qhat", self.cdtype, (nb, L, self.M))
        g_q = self._out(g_q, "g_q", q.dtype, (self.M, self.nt))
        ws = self.workspace()
        _check(lib().spod_backward(
            self._h, _ptr(q), dt, _ptr(qhat), _ptr(lam), _ptr(psi), _ptr(g_lam), _ptr(g_phi),
            n_modes, None if sel is None else sel.ctypes.data_as(C.c_void_p), nb, _ptr(g_qhat),
            _ptr(g_q), _ptr(ws), ws.numel(), _stream(self.device)))
        return g_q

    # -- expansion coefficients and reconstruction -------------------------
    def _bins(self, phi, bins, n_r):
        if phi.dim() != 3 or phi.shape[0] != self.nfreq or phi.shape[2] != self.M:
            raise ValueError(f"phi must have shape ({self.nfreq}, n_modes, {self.M})")
        self._dev(phi, "phi", self.cdtype, tuple(phi.shape))
        sel = np.ascontiguousarray(np.asarray(bins, dtype=np.int32))
        if sel.ndim != 1:
            raise ValueError("bins must be one-dimensional")
        return sel, len(sel) * int(n_r)

    def coeffs(self, q, mean, phi, bins, n_r: int, a=None, info=None):
        """Expansion coefficients A = (Phi_r^* W Phi_r)^{-1} Phi_r^* W (Q - qbar)
        over mode j < n_r of every frequency in bins (column i * n_r + j).
        Returns (a [R, nt] in phi's complex type, info [1] int32)."""
        dt = self._q(q)
        self._dev(mean, "mean", torch.float64, (self.M,))
        sel, R = self._bins(phi, bins, n_r)
        a = self._out(a, "a", self.cdtype, (R, self.nt))
        info = self._out(info, "info", torch.int32, (1,))
        wsb = C.c_size_t()
        _check(lib().spod_coeffs_query(self._h, len(sel), int(n_r), C.byref(wsb)))
        ws = torch.empty(max(1, wsb.value), dtype=torch.uint8, device=self.device)
        _check(lib().spod_coeffs(self._h, _ptr(q), dt, _ptr(mean), _ptr(phi), phi.shape[1],
                                 sel.ctypes.data_as(C.c_void_p), len(sel), int(n_r), _ptr(a),
                                 _ptr(info), _ptr(ws), ws.numel(), _stream(self.device)))
        return a, info

    def reconstruct(self, phi, bins, n_r: int, a, mean, q_rec=None, dtype=torch.float32):
        """Q~ = Re(Phi_r A) + qbar 1^T, [M, nt] of dtype."""
        sel, R = self._bins(phi, bins, n_r)
        self._dev(a, "a", self.cdtype, (R, self.nt))
        self._dev(mean, "mean", torch.float64, (self.M,))
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be float32 or float64")
        q_rec = self._out(q_rec, "q_rec", dtype, (self.M, self.nt))
        _check(lib().spod_reconstruct(self._h, _ptr(phi), phi.shape[1],
                                      sel.ctypes.data_as(C.c_void_p), len(sel), int(n_r), _ptr(a),
                                      _ptr(mean), _ptr(q_rec),
                                      N.SPOD_F32 if dtype == torch.float32 else N.SPOD_F64,
                                      _stream(self.device)))
        return q_rec

    def forward(self, q, n_modes: int = 5):
        """All stages: returns dict(mean, qhat, gram, lam, psi, info, phi, n_valid)."""
        qhat, mean = self.blocks_fft(q)
        gram = self.csd(qhat)
        lam, psi, info = self.eig(gram)
        phi, n_valid = self.modes(qhat, lam, psi, n_modes)
        return {"mean": mean, "qhat": qhat, "gram": gram, "lam": lam, "psi": psi, "info": info,
                "phi": phi, "n_valid": n_valid}


class Batch:
    """Many independent problems run with grouped launches (spod_batch_*).

    problems: sequence of dicts with nspace, nvar, nt, nfft, noverlap and
    optional window / weights.  forward(qs) returns, per problem, a dict of
    tensors viewing the batch's output buffer (mean, lam, psi, info, phi,
    n_valid); they are overwritten by the next forward call."""

    def __init__(self, problems, precision: str = "fp64", n_modes: int = 5, grouped: bool = True,
                 graph: bool = True, gram_target: Optional[int] = None,
                 fft_tile: Optional[int] = None, eig_threads: Optional[int] = None,
                 persistent: Optional[bool] = None, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.precision = precision
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        keep = []
        arr = (N.SpodProblem * len(problems))()
        for i, d in enumerate(problems):
            win = d.get("window")
            w = d.get("weights")
            win = None if win is None else np.ascontiguousarray(win, dtype=np.float64)
            w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
            keep += [win, w]
            arr[i] = N.SpodProblem(d["nspace"], d["nvar"], d["nt"], d["nfft"], d["noverlap"],
                                   None if win is None else win.ctypes.data,
                                   None if w is None else w.ctypes.data)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().spod_batch_create(arr, len(problems), PRECISIONS[precision], n_modes,
                                           C.byref(h)))
        self._h = h
        for opt, v in ((N.SPOD_BATCH_GROUPED, grouped), (N.SPOD_BATCH_GRAPH, graph),
                       (N.SPOD_BATCH_GRAM_TARGET, gram_target), (N.SPOD_BATCH_FFT_TILE, fft_tile),
                       (N.SPOD_BATCH_EIG_THREADS, eig_threads),
                       (N.SPOD_BATCH_PERSISTENT, persistent)):
            if v is not None:
                _check(lib().spod_batch_set_option(self._h, opt, int(v)))
        ws, out = C.c_size_t(), C.c_size_t()
        _check(lib().spod_batch_query(self._h, C.byref(ws), C.byref(out)))
        self.workspace_bytes, self.output_bytes = ws.value, out.value
        self.items = []
        for i in range(len(problems)):
            it = N.SpodBatchItem()
            _check(lib().spod_batch_item_info(self._h, i, C.byref(it)))
            self.items.append(it)
        self._ws = None
        self._out = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().spod_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def buffers(self):
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            self._out = torch.empty(self.output_bytes, dtype=torch.uint8, device=self.device)
        return self._ws, self._out

    def _qptrs(self, qs):
        if len(qs) != len(self.items):
            raise ValueError(f"expected {len(self.items)} inputs")
        dt = qs[0].dtype
        for q, it in zip(qs, self.items):
            if q.dtype != dt or q.device != self.device or not q.is_contiguous():
                raise ValueError("inputs must share a dtype and be contiguous on the batch's device")
            if q.dim() != 2 or q.shape[0] != it.M:
                raise ValueError("input rows do not match the problem's M")
        ptrs = (C.c_void_p * len(qs))(*[q.data_ptr() for q in qs])
        return ptrs, (N.SPOD_F32 if dt == torch.float32 else N.SPOD_F64)

    def _view(self, off, dtype, shape):
        n = int(np.prod(shape)) * torch.empty(0, dtype=dtype).element_size()
        return self._out[off:off + n].view(dtype).view(*shape)

    def results(self):
        out = []
        for it in self.items:
            K, L, M, n = it.nfreq, it.nblocks, it.M, it.n_modes
            out.append({"mean": self._view(it.mean, torch.float64, (M,)),
                        "lam": self._view(it.lam, torch.float64, (K, L)),
                        "psi": self._view(it.psi, torch.complex128, (K, L, L)),
                        "info": self._view(it.info, torch.int32, (K,)),
                        "phi": self._view(it.phi, self.cdtype, (K, n, M)),
                        "n_valid": self._view(it.n_valid, torch.int32, (K,))})
        return out

    def forward(self, qs):
        ptrs, dt = self._qptrs(qs)
        ws, out = self.buffers()
        _check(lib().spod_batch_forward(self._h, ptrs, dt, _ptr(out), _ptr(ws), ws.numel(),
                                        _stream(self.device)))
        return self.results()

    def autotune(self, qs, cache_path: Optional[str] = None) -> int:
        """Choose the launch shapes (spod_batch_autotune); returns the Gram
        target, and shapes() gives every choice."""
        ptrs, dt = self._qptrs(qs)
        ws, out = self.buffers()
        chosen = C.c_int64()
        _check(lib().spod_batch_autotune(self._h, ptrs, dt, _ptr(out), _ptr(ws), ws.numel(),
                                         _stream(self.device),
                                         None if cache_path is None else cache_path.encode(),
                                         C.byref(chosen)))
        return chosen.value

    def shapes(self) -> dict:
        """The launch shapes in use (options or the autotuner's choice)."""
        out = {}
        for name, opt in (("gram_target", N.SPOD_BATCH_GRAM_TARGET),
                          ("fft_tile", N.SPOD_BATCH_FFT_TILE),
                          ("eig_threads", N.SPOD_BATCH_EIG_THREADS),
                          ("persistent", N.SPOD_BATCH_PERSISTENT)):
            v = C.c_int64()
            _check(lib().spod_batch_get_option(self._h, opt, C.byref(v)))
            out[name] = v.value
        return out


def _host_or_device_ptr(t, name: str):
    """Data pointer of a contiguous torch tensor (CPU or the device) or numpy array."""
    if isinstance(t, np.ndarray):
        if not t.flags["C_CONTIGUOUS"]:
            raise ValueError(f"{name} must be C-contiguous")
        return C.c_void_p(t.ctypes.data)
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class OutOfCore:
    """Out-of-core SPOD (spod_ooc_*): the snapshot matrix stays in host memory
    and is streamed to the device in chunks of `chunk_rows` rows, twice (Gram
    pass, modes pass); the last `resident` chunks stay on the device between
    the passes.  The plan gives the shape, weights, window and precision and
    must stay open while this object is used."""

    def __init__(self, plan: Plan, dtype=torch.float32, chunk_rows: int = 32768, n_modes: int = 5,
                 resident: int = 0):
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be float32 or float64")
        self.plan = plan
        self.dtype = dtype
        self.n_modes = n_modes
        h = C.c_void_p()
        with torch.cuda.device(plan.device):
            _check(lib().spod_ooc_create(plan._h, N.SPOD_F32 if dtype == torch.float32 else N.SPOD_F64,
                                         int(chunk_rows), int(n_modes), int(resident), C.byref(h)))
        self._h = h
        rows, n, r, dev, pin = C.c_int64(), C.c_int64(), C.c_int64(), C.c_size_t(), C.c_size_t()
        _check(lib().spod_ooc_query(self._h, C.byref(rows), C.byref(n), C.byref(r), C.byref(dev),
                                    C.byref(pin)))
        self.chunk_rows, self.n_chunks, self.resident = rows.value, n.value, r.value
        self.device_bytes, self.pinned_bytes = dev.value, pin.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().spod_ooc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_q(self, q):
        p = self.plan
        dt = q.dtype if isinstance(q, torch.Tensor) else torch.from_numpy(q[:0]).dtype
        if dt != self.dtype:
            raise TypeError(f"q must be {self.dtype}, got {dt}")
        if tuple(q.shape) != (p.M, p.nt):
            raise ValueError(f"q must have shape {(p.M, p.nt)}, got {tuple(q.shape)}")
        if isinstance(q, torch.Tensor) and q.is_cuda and q.device != p.device:
            raise ValueError(f"q must be on the host or on {p.device}")

    def forward(self, q=None, reader=None, phi=None, mean=None):
        """One SPOD.  Exactly one of
          q      : [M, nt] torch tensor (host, pinned or not, or the plan's
                   device) or numpy array;
          reader : reader(row0, nrows, out) fills out (a numpy array
                   [nrows, nt] viewing pinned memory) with those rows of Q.
        phi ([K, n_modes, M] complex, host or device) and mean ([M] float64)
        are allocated when not given: phi in pinned host memory, mean on the
        host.  Returns dict(mean, lam, psi, info, phi, n_valid); lam, psi,
        info and n_valid are on the device."""
        p = self.plan
        if (q is None) == (reader is None):
            raise ValueError("give exactly one of q and reader")
        K, L, M, n = p.nfreq, p.nblocks, p.M, self.n_modes
        if q is not None:
            self._check_q(q)
        if phi is None:
            phi = torch.empty((K, n, M), dtype=p.cdtype, pin_memory=True)
        elif tuple(phi.shape) != (K, n, M) or phi.dtype != p.cdtype:
            raise ValueError(f"phi must be {p.cdtype} of shape {(K, n, M)}")
        if mean is None:
            mean = torch.empty(M, dtype=torch.float64)
        elif tuple(mean.shape) != (M,) or mean.dtype != torch.float64:
            raise ValueError(f"mean must be float64 of shape {(M,)}")
        lam = torch.empty((K, L), dtype=torch.float64, device=p.device)
        psi = torch.empty((K, L, L), dtype=torch.complex128, device=p.device)
        info = torch.empty(K, dtype=torch.int32, device=p.device)
        n_valid = torch.empty(K, dtype=torch.int32, device=p.device)

        err = []
        if reader is not None:
            nt, npdt = p.nt, (np.float32 if self.dtype == torch.float32 else np.float64)
            ct = C.c_float if self.dtype == torch.float32 else C.c_double

            def _read(user, row0, nrows, dst):
                try:
                    buf = (ct * (nrows * nt)).from_address(dst)
                    out = np.frombuffer(buf, dtype=npdt).reshape(nrows, nt)
                    reader(int(row0), int(nrows), out)
                    return 0
                except BaseException as e:  # reported through SPOD_ERR_IO
                    err.append(e)
                    return 1
            cb = N.READ_FN(_read)
        else:
            cb = N.READ_FN()
        with torch.cuda.device(p.device):
            _check_ooc(lib().spod_ooc_forward(
                self._h, None if q is None else _host_or_device_ptr(q, "q"), cb, None,
                _host_or_device_ptr(mean, "mean"), _ptr(lam), _ptr(psi), _ptr(info),
                _host_or_device_ptr(phi, "phi"), _ptr(n_valid), _stream(p.device)), err)
        return {"mean": mean, "lam": lam, "psi": psi, "info": info, "phi": phi, "n_valid": n_valid}


def _check_ooc(status: int, err: list):
    if status != N.SPOD_OK and err:
        L = lib()
        msg = L.spod_last_error().decode() or L.spod_status_string(status).decode()
        raise N.SpodError(status, f"{msg} ({err[0]!r})") from err[0]
    _check(status)
