"""Seeded synthetic snapshot matrices for the SPOD workloads.

This module only builds inputs: snapshot matrices Q [M, N_t] (degree of
freedom m = v * nspace + s, time contiguous per row) and diagonal quadrature
weights W [M].  It holds none of the SPOD arithmetic (no mean removal, no
blocking, no transform, no inner product), and both the FP64 oracle and the HIP
path consume exactly the arrays it returns.

Randomness comes from a seeded torch.Generator on the device the data is built
on, so a (seed, device) pair always gives the same array.  Arrays are formed in
float64 and rounded once to the stored dtype.

Workloads (stand-ins for the paper's LES jet and ERA5 data, which are not
available):
  * planted   - W-orthonormal random spatial modes times bin-centred cosines
                plus white noise (closed-form eigenvalues when sigma = 0).
  * jet_like  - 256 x 128 tanh-stretched grid, 3 variables, spatially
                correlated Gaussian random field (squared-exponential kernel,
                length 8 cells) driven by AR(1) in time, plus 4 travelling
                Gaussian wave packets at bin-centred frequencies.
  * era_like  - 1024 x 512 lat-lon grid, 2 variables, cos(latitude) weights,
                the same red noise plus 6 planted modes.
  * batch     - 64 independent problems of uneven sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

__all__ = ["Problem", "planted", "jet_like", "era_like", "random_rows", "batch_specs",
           "batch_problem", "block_count_of"]


@dataclass
class Problem:
    q: torch.Tensor                  # [M, N_t] snapshot rows (stored dtype) on its device
    weights: np.ndarray              # [M] float64 quadrature weights
    nspace: int
    nvar: int
    nfft: int
    noverlap: int
    meta: dict = field(default_factory=dict)

    @property
    def nt(self) -> int:
        return int(self.q.shape[1])

    @property
    def M(self) -> int:
        return int(self.q.shape[0])


def block_count_of(nt: int, nfft: int, noverlap: int) -> int:
    """Blocks that fit in nt snapshots (used only to size generated problems)."""
    return (nt - noverlap) // (nfft - noverlap)


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _w_orthonormal(x: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """Columns of x made orthonormal under diag(w): W^{-1/2} qr(W^{1/2} x)."""
    sw = torch.sqrt(w)[:, None]
    qm, _ = torch.linalg.qr(sw * x)
    return qm / sw


# ---------------------------------------------------------------------------
# planted modes (closed-form eigenvalues for sigma = 0)
# ---------------------------------------------------------------------------
def planted(nspace: int = 1024, nt: int = 1024, nfft: int = 128, noverlap: int = 64,
            bins=(5, 12, 30), amps=(3.0, 2.0, 1.0), sigma: float = 0.1, seed: int = 1,
            dtype=torch.float64, device="cpu", weights=None) -> Problem:
    """q = sum_i a_i phi_i cos(2 pi b_i t / N_f + theta_i) + sigma * eps.

    phi_i are W-orthonormal random vectors (W = 1/M by default), theta_i ~
    U[0, 2 pi), eps ~ N(0, 1).  Defaults: the 32 x 32, 1-variable, N_t = 1024,
    N_f = 128 parity workload.
    """
    g = _gen(seed, device)
    M = nspace
    w = torch.full((M,), 1.0 / M, dtype=torch.float64, device=device) if weights is None \
        else torch.as_tensor(np.asarray(weights, np.float64), device=device)
    x = torch.randn(M, len(bins), generator=g, dtype=torch.float64, device=device)
    phi = _w_orthonormal(x, w)
    theta = 2.0 * math.pi * torch.rand(len(bins), generator=g, dtype=torch.float64, device=device)
    t = torch.arange(nt, dtype=torch.float64, device=device)
    q = torch.zeros(M, nt, dtype=torch.float64, device=device)
    for i, (b, a) in enumerate(zip(bins, amps)):
        q += a * phi[:, i:i + 1] * torch.cos(2.0 * math.pi * b * t / nfft + theta[i])[None, :]
    if sigma > 0:
        q += sigma * torch.randn(M, nt, generator=g, dtype=torch.float64, device=device)
    return Problem(q=q.to(dtype), weights=w.cpu().numpy(), nspace=nspace, nvar=1, nfft=nfft,
                   noverlap=noverlap,
                   meta={"bins": tuple(bins), "amps": tuple(amps), "sigma": sigma,
                         "phi": phi.cpu().numpy(), "seed": seed})


# ---------------------------------------------------------------------------
# red noise: Gaussian random field in space, AR(1) in time
# ---------------------------------------------------------------------------
def _grf_filter(ny: int, nx: int, length: float, device) -> torch.Tensor:
    """Amplitude filter for a periodic squared-exponential field of unit variance."""
    fy = torch.fft.fftfreq(ny, device=device, dtype=torch.float64)
    fx = torch.fft.rfftfreq(nx, device=device, dtype=torch.float64)
    f2 = fy[:, None] ** 2 + fx[None, :] ** 2
    h = torch.exp(-(math.pi ** 2) * (length ** 2) * f2)        # sqrt of the Gaussian PSD
    # unit output variance for unit white input: mean of |H|^2 over the full grid
    full = torch.cat([h, torch.flip(h[:, 1:(nx + 1) // 2], dims=[1])], dim=1) if nx > 1 else h
    h = h / torch.sqrt(torch.mean(full ** 2))
    return h


class _RedNoise:
    """Streams time slices [nt_chunk, nvar, ny, nx] of a unit-variance field that
    is squared-exponential correlated in space and AR(1) in time."""

    def __init__(self, g, nvar, ny, nx, length, rho, device):
        self.g, self.nvar, self.ny, self.nx, self.rho, self.device = g, nvar, ny, nx, rho, device
        self.h = _grf_filter(ny, nx, length, device)
        self.state = torch.randn(nvar, ny, nx, generator=g, dtype=torch.float64, device=device)
        self.c = math.sqrt(1.0 - rho * rho)

    def take(self, n: int) -> torch.Tensor:
        eta = torch.randn(n, self.nvar, self.ny, self.nx, generator=self.g,
                          dtype=torch.float64, device=self.device)
        out = torch.empty_like(eta)
        a = self.state
        for i in range(n):
            a = self.rho * a + self.c * eta[i]
            out[i] = a
        self.state = a
        if self.ny == 1:
            # a line: the 1-D transform (the GPU FFT library rejects a 2-D
            # transform with a dimension of length one)
            spec = torch.fft.rfft(out, dim=-1) * self.h[0]
            return torch.fft.irfft(spec, n=self.nx, dim=-1)
        spec = torch.fft.rfft2(out) * self.h
        return torch.fft.irfft2(spec, s=(self.ny, self.nx))


# ---------------------------------------------------------------------------
# jet-like workload (256 x 128, 3 variables, N_t = 4096, N_f = 256)
# ---------------------------------------------------------------------------
def jet_like(seed: int = 2, nx: int = 256, ny: int = 128, nvar: int = 3, nt: int = 4096,
             nfft: int = 256, noverlap: int = 128, dtype=torch.float32, device="cpu",
             chunk: int = 256) -> Problem:
    g = _gen(seed, device)
    beta = 2.0
    xs = 2.0 * torch.arange(nx, dtype=torch.float64, device=device) / nx
    eta = 2.0 * torch.arange(ny, dtype=torch.float64, device=device) / (ny - 1) - 1.0
    ys = torch.tanh(beta * eta) / math.tanh(beta)
    wx = torch.full((nx,), 2.0 / nx, dtype=torch.float64, device=device)
    wy = torch.empty(ny, dtype=torch.float64, device=device)
    wy[1:-1] = 0.5 * (ys[2:] - ys[:-2])
    wy[0] = 0.5 * (ys[1] - ys[0])
    wy[-1] = 0.5 * (ys[-1] - ys[-2])
    w2 = (wy[:, None] * wx[None, :]).reshape(-1)
    weights = w2.repeat(nvar)
    nspace = nx * ny
    M = nspace * nvar
    # wave packets
    npk = 4
    pk_bins = torch.tensor([10.0, 20.0, 35.0, 50.0], dtype=torch.float64, device=device) * (256.0 / nfft)
    pk_amp = torch.tensor([2.0, 1.5, 1.2, 1.0], dtype=torch.float64, device=device)
    u = torch.rand(npk, 6, generator=g, dtype=torch.float64, device=device)
    x0 = 2.0 * u[:, 0]
    y0 = -0.6 + 1.2 * u[:, 1]
    speed = (0.5 + 1.5 * u[:, 2]) * 2.0 / nt              # crosses the domain 0.5..2 times
    kx = math.pi * torch.floor(2.0 + 5.0 * u[:, 3])          # integer wavenumbers on [0, 2)
    sx = 0.10 + 0.10 * u[:, 4]
    sy = 0.15 + 0.10 * u[:, 5]
    mix = (0.5 + torch.rand(nvar, npk, generator=g, dtype=torch.float64, device=device)) * \
        torch.where(torch.rand(nvar, npk, generator=g, device=device) < 0.5, -1.0, 1.0).to(torch.float64)
    noise = _RedNoise(g, nvar, ny, nx, 8.0, 0.95, device)
    q = torch.empty(M, nt, dtype=dtype, device=device)
    X = xs[None, None, :]
    Y = ys[None, :, None]
    for t0 in range(0, nt, chunk):
        n = min(chunk, nt - t0)
        f = noise.take(n)                                       # [n, nvar, ny, nx]
        t = torch.arange(t0, t0 + n, dtype=torch.float64, device=device)[:, None, None]
        for p in range(npk):
            dx = torch.remainder(X - x0[p] - speed[p] * t + 1.0, 2.0) - 1.0
            env = torch.exp(-dx * dx / (2 * sx[p] ** 2) - (Y - y0[p]) ** 2 / (2 * sy[p] ** 2))
            wave = pk_amp[p] * env * torch.cos(kx[p] * dx - 2.0 * math.pi * pk_bins[p] / nfft * t)
            f += mix[None, :, p, None, None] * wave[:, None, :, :]
        q[:, t0:t0 + n] = f.reshape(n, M).t().to(dtype)
    return Problem(q=q, weights=weights.cpu().numpy(), nspace=nspace, nvar=nvar, nfft=nfft,
                   noverlap=noverlap, meta={"seed": seed, "grid": (ny, nx),
                                            "packet_bins": pk_bins.cpu().numpy().tolist()})


# ---------------------------------------------------------------------------
# ERA-like workload (1024 x 512 lat-lon, 2 variables, N_t = 8192, N_f = 512)
# ---------------------------------------------------------------------------
def era_like(seed: int = 3, nlon: int = 1024, nlat: int = 512, nvar: int = 2, nt: int = 8192,
             nfft: int = 512, noverlap: int = 256, dtype=torch.float32, device="cpu",
             bins=(3, 8, 17, 40, 90, 200), amps=(6.0, 5.0, 4.0, 3.0, 2.0, 1.0),
             chunk: int = 128) -> Problem:
    g = _gen(seed, device)
    lat = -90.0 + (torch.arange(nlat, dtype=torch.float64, device=device) + 0.5) * 180.0 / nlat
    dlon = 2.0 * math.pi / nlon
    dlat = math.pi / nlat
    w2 = (torch.cos(torch.deg2rad(lat))[:, None] * dlon * dlat).expand(nlat, nlon).reshape(-1)
    weights = w2.repeat(nvar)
    nspace = nlat * nlon
    M = nspace * nvar
    # planted spatial modes: smooth random fields, W-orthonormal, scaled so that
    # their W-weighted mean square is 1 (amplitude a_i = multiple of the noise std)
    nm = len(bins)
    smooth = _grf_filter(nlat, nlon, 32.0, device)
    raw = torch.randn(nm, nvar, nlat, nlon, generator=g, dtype=torch.float64, device=device)
    raw = torch.fft.irfft2(torch.fft.rfft2(raw) * smooth, s=(nlat, nlon)).reshape(nm, M).t()
    phi = _w_orthonormal(raw, weights) * math.sqrt(float(weights.sum()))
    theta = 2.0 * math.pi * torch.rand(nm, generator=g, dtype=torch.float64, device=device)
    amp = torch.tensor(amps, dtype=torch.float64, device=device)
    fb = torch.tensor(bins, dtype=torch.float64, device=device) / nfft
    noise = _RedNoise(g, nvar, nlat, nlon, 8.0, 0.95, device)
    q = torch.empty(M, nt, dtype=dtype, device=device)
    for t0 in range(0, nt, chunk):
        n = min(chunk, nt - t0)
        f = noise.take(n).reshape(n, M)
        t = torch.arange(t0, t0 + n, dtype=torch.float64, device=device)
        c = amp[None, :] * torch.cos(2.0 * math.pi * fb[None, :] * t[:, None] + theta[None, :])
        f += c @ phi.t()
        q[:, t0:t0 + n] = f.t().to(dtype)
        del f
    return Problem(q=q, weights=weights.cpu().numpy(), nspace=nspace, nvar=nvar, nfft=nfft,
                   noverlap=noverlap, meta={"seed": seed, "grid": (nlat, nlon),
                                            "bins": tuple(bins), "amps": tuple(amps)})


# ---------------------------------------------------------------------------
# small random problems (edge cases, ragged shapes)
# ---------------------------------------------------------------------------
def random_rows(M: int, nt: int, nfft: int, noverlap: int, seed: int = 0, offset: float = 0.0,
                dtype=torch.float64, device="cpu", weights="random") -> Problem:
    """AR(1)-in-time rows (rho = 0.8) plus a per-row constant offset * U[-1, 1]."""
    g = _gen(seed, device)
    eta = torch.randn(M, nt, generator=g, dtype=torch.float64, device=device)
    x = torch.empty_like(eta)
    a = eta[:, 0]
    x[:, 0] = a
    c = math.sqrt(1 - 0.64)
    for t in range(1, nt):
        a = 0.8 * a + c * eta[:, t]
        x[:, t] = a
    if offset:
        x += offset * (2 * torch.rand(M, 1, generator=g, dtype=torch.float64, device=device) - 1)
    if weights == "random":
        w = (0.2 + torch.rand(M, generator=g, dtype=torch.float64, device=device)).cpu().numpy()
    else:
        w = np.full(M, 1.0 / M)
    return Problem(q=x.to(dtype), weights=w, nspace=M, nvar=1, nfft=nfft, noverlap=noverlap,
                   meta={"seed": seed})


# ---------------------------------------------------------------------------
# 64 uneven problems
# ---------------------------------------------------------------------------
def batch_specs(seed: int = 4, count: int = 64):
    """Sizes of the uneven batch: nspace log-uniform in [1e3, 2e5], nvar in
    {1, 2, 3}, N_f in {64, 128, 256}, N_t in {512, ..., 4096} (resampled until
    7 <= L <= 63), 50% overlap, periodic Hann, W = 1/M; kind alternates between
    planted modes and AR(1) red noise on a periodic line at random."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    specs = []
    while len(specs) < count:
        nspace = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        nvar = int(rng.integers(1, 4))
        nfft = int(rng.choice([64, 128, 256]))
        nt = int(rng.choice([512, 1024, 2048, 4096]))
        L = block_count_of(nt, nfft, nfft // 2)
        if not (7 <= L <= 63):
            continue
        kind = "planted" if rng.uniform() < 0.5 else "red"
        specs.append({"nspace": nspace, "nvar": nvar, "nfft": nfft, "noverlap": nfft // 2,
                      "nt": nt, "kind": kind, "seed": int(rng.integers(1 << 30))})
    return specs


def batch_problem(spec: dict, dtype=torch.float32, device="cpu") -> Problem:
    M = spec["nspace"] * spec["nvar"]
    nt, nfft = spec["nt"], spec["nfft"]
    if spec["kind"] == "planted":
        k = nfft // 2
        bins = (max(2, k // 10), max(5, k // 4), max(8, k // 2))
        p = planted(nspace=M, nt=nt, nfft=nfft, noverlap=spec["noverlap"], bins=bins,
                    amps=(3.0, 2.0, 1.0), sigma=0.1, seed=spec["seed"], dtype=dtype, device=device)
        p.nspace, p.nvar = spec["nspace"], spec["nvar"]
        return p
    g = _gen(spec["seed"], device)
    noise = _RedNoise(g, spec["nvar"], 1, spec["nspace"], 8.0, 0.95, device)
    f = noise.take(nt).reshape(nt, M)
    return Problem(q=f.t().contiguous().to(dtype), weights=np.full(M, 1.0 / M),
                   nspace=spec["nspace"], nvar=spec["nvar"], nfft=nfft,
                   noverlap=spec["noverlap"], meta=dict(spec))
