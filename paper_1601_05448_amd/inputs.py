"""Seeded synthetic inputs for the variable-density Poisson solve.

This module only draws and shapes input fields (density rho, right-hand side b,
request streams).  It holds none of the solver's arithmetic, imports nothing
from the GPU library or from the oracle, and is the one piece that both sides
share, so that they consume identical bytes.

All fields are float64 numpy arrays of shape (nz, ny, nx), x fastest, sampled at
cell centres x_i = (i + 1/2) h (scalars live at cell centres on the paper's
staggered grid, section "Spatial discretization").  Randomness comes from
numpy's PCG64 ``default_rng``; base seed 1601, workload c uses 1601*100 + c and
served request r uses 1601*1000 + r.

Workloads (the density contrasts follow the paper's motivation: particles heat
the gas, hot gas is light, section "Motivation and objectives"):
  1  32^3, [0,2pi)^3, rho = 1 + sin x sin y sin z / 2, b = discrete divergence
     of Gaussian face velocities.
  2  256^3, rho = exp(s), s band-limited |k| <= 8 and scaled to max/min = 4,
     b band-limited |k| <= 8.
  3  512^3, rho = 1/(1 + 9 d/max d), d = cloud-in-cell deposit of 10^6 uniform
     particles (the paper's linear particle-to-grid projection); b band-limited.
  4  served stream: 512 requests, Poisson arrivals, N in {64,96,128,192}, rho
     lognormal band-limited with contrast R ~ U[2,8], b band-limited.
  5  1024x512x512 on [0,4pi)x[0,2pi)^2, rho = 1/(1 + 19 f/max f), f = sum of
     10^5 periodic Gaussian blobs of width 2 cells; b band-limited.
  6  duct: 2N x N x N on [0,4pi)x[0,2pi)^2 (the inflow-outflow domain, twice as
     long in x as the box that feeds it), rho lognormal band-limited with
     max/min = 4, b band-limited; solved with zero-flux walls at the x ends.
     The fields are drawn as periodic ones; the walls only change the operator.
  8  warm-start chains: rho_t = exp(c s(x - U t)) with s band-limited and U half
     a cell per step in x and a quarter in y, b_t = cos(0.02 t) b1 + sin(0.02 t) b2;
     each solve of a chain starts from the previous solution.
  7  projection step: the predicted face momentum (three band-limited fields,
     |k| <= 8) and the divergence target (band-limited, scaled by 0.1) on the
     grid and density of the workload it accompanies; C dt = 5e-4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterator, List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 1601
TWO_PI = 2.0 * math.pi


def workload_seed(c: int) -> int:
    return BASE_SEED * 100 + c


def request_seed(r: int) -> int:
    return BASE_SEED * 1000 + r


def centres(n: int, length: float) -> np.ndarray:
    """Cell-centre coordinates (i + 1/2) h, h = length / n."""
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


def _bandlim_spectrum(shape: Sequence[int], lengths: Sequence[float], kmax: float,
                      rng: np.random.Generator, shift: Optional[Sequence[float]] = None):
    """Random coefficients and 1-D synthesis factors of a band-limited field;
    `shift` = (sx, sy, sz) evaluates the same field at x - s (the coefficients
    times exp(-i k.s)), so that fields drawn from equal seeds with growing shifts
    are one field carried along by a uniform flow."""
    nz, ny, nx = shape
    lx, ly, lz = lengths
    mx = int(math.floor(kmax * lx / TWO_PI))
    my = int(math.floor(kmax * ly / TWO_PI))
    mz = int(math.floor(kmax * lz / TWO_PI))
    ax = np.arange(-mx, mx + 1)
    ay = np.arange(-my, my + 1)
    az = np.arange(-mz, mz + 1)
    kz, ky, kx = np.meshgrid(TWO_PI * az / lz, TWO_PI * ay / ly, TWO_PI * ax / lx, indexing="ij")
    kk = kx * kx + ky * ky + kz * kz
    mask = (kk <= kmax * kmax * (1 + 1e-12)) & (kk > 0)
    coef = (rng.standard_normal(mask.shape) + 1j * rng.standard_normal(mask.shape)) * mask
    if shift is not None:
        coef = coef * np.exp(-1j * (kx * shift[0] + ky * shift[1] + kz * shift[2]))
    ex = np.exp(1j * np.outer(TWO_PI * ax / lx, centres(nx, lx)))  # (2mx+1, nx)
    ey = np.exp(1j * np.outer(TWO_PI * ay / ly, centres(ny, ly)))  # (2my+1, ny)
    ez = np.exp(1j * np.outer(TWO_PI * az / lz, centres(nz, lz)))  # (2mz+1, nz)
    t1 = coef @ ex  # (mz, my, nx)
    t2 = np.einsum("zyi,yj->zji", t1, ey).reshape(len(az), ny * nx)  # (mz, ny*nx)
    return t2, ez


def bandlim(shape: Sequence[int], lengths: Sequence[float], kmax: float,
            rng: np.random.Generator, z_chunk: int = 64) -> np.ndarray:
    """Gaussian random field band-limited to physical wavenumbers 0 < |k| <= kmax.

    Independent complex N(0,1) coefficients on every integer wavevector m with
    |2 pi m / L| <= kmax (m != 0); the field is the real part of their Fourier
    synthesis at cell centres, shifted to zero mean and scaled to unit RMS.
    The synthesis is separable (x, then y, then z) so it is independent of the
    grid resolution and cheap at any size.
    """
    nz, ny, nx = shape
    t2, ez = _bandlim_spectrum(shape, lengths, kmax, rng)
    t2r, t2i = np.ascontiguousarray(t2.real), np.ascontiguousarray(t2.imag)
    out = np.empty((nz, ny * nx))
    ezr, ezi = ez.real.T.copy(), ez.imag.T.copy()  # (nz, mz)
    for k0 in range(0, nz, z_chunk):
        k1 = min(nz, k0 + z_chunk)
        out[k0:k1] = ezr[k0:k1] @ t2r - ezi[k0:k1] @ t2i
    out = out.reshape(nz, ny, nx)
    out -= out.mean()
    rms = math.sqrt(float(np.mean(out * out)))
    if rms > 0:
        out /= rms
    return out


def bandlim_device(shape: Sequence[int], lengths: Sequence[float], kmax: float,
                   rng: np.random.Generator, device="cuda", shift: Optional[Sequence[float]] = None):
    """bandlim with the same random draws, its last synthesis step (the z
    contraction, the only large one) done as a float64 torch matmul on
    `device`; returns a torch tensor.  Values agree with bandlim up to the
    rounding order of the two matrix products."""
    import torch

    nz, ny, nx = shape
    t2, ez = _bandlim_spectrum(shape, lengths, kmax, rng, shift)
    t2r = torch.from_numpy(np.ascontiguousarray(t2.real)).to(device)
    t2i = torch.from_numpy(np.ascontiguousarray(t2.imag)).to(device)
    ezr = torch.from_numpy(ez.real.T.copy()).to(device)
    ezi = torch.from_numpy(ez.imag.T.copy()).to(device)
    out = (ezr @ t2r - ezi @ t2i).reshape(nz, ny, nx)
    out -= out.mean()
    rms = torch.sqrt(torch.mean(out * out))
    if float(rms) > 0:
        out /= rms
    return out.contiguous()


def contrast_exp(s: np.ndarray, ratio: float) -> np.ndarray:
    """rho = exp(c s) with c chosen so that max(rho)/min(rho) = ratio."""
    span = float(s.max() - s.min())
    return np.exp(s * (math.log(ratio) / span))


def face_divergence(shape: Sequence[int], lengths: Sequence[float],
                    rng: np.random.Generator) -> np.ndarray:
    """Divergence at cell centres of independent N(0,1) face velocities.

    u_d is stored on the face between cells i and i + e_d; the divergence is
    sum_d (u_d[i+1/2] - u_d[i-1/2]) / h_d, which sums to zero over the periodic
    box (telescoping)."""
    nz, ny, nx = shape
    hs = (lengths[0] / nx, lengths[1] / ny, lengths[2] / nz)
    out = np.zeros(shape)
    for d, axis in enumerate((2, 1, 0)):
        u = rng.standard_normal(shape)
        out += (u - np.roll(u, 1, axis=axis)) / hs[d]
    return out


def cic_deposit(shape: Sequence[int], lengths: Sequence[float], pos: np.ndarray) -> np.ndarray:
    """Cloud-in-cell (trilinear) deposit of unit-weight particles onto cell
    centres, periodic: the linear particle-to-grid projection the paper uses
    for two-way coupling (section "Physical model")."""
    nz, ny, nx = shape
    ns = (nx, ny, nz)
    idx = []
    wts = []
    for d in range(3):
        s = pos[:, d] * (ns[d] / lengths[d]) - 0.5
        i0 = np.floor(s)
        f = s - i0
        i0 = i0.astype(np.int64) % ns[d]
        idx.append((i0, (i0 + 1) % ns[d]))
        wts.append((1.0 - f, f))
    n = nx * ny * nz
    dep = np.zeros(n)
    for a in (0, 1):
        for bb in (0, 1):
            for c in (0, 1):
                flat = (idx[2][c] * ny + idx[1][bb]) * nx + idx[0][a]
                dep += np.bincount(flat, weights=wts[0][a] * wts[1][bb] * wts[2][c], minlength=n)
    return dep.reshape(shape)


def gaussian_blobs(shape: Sequence[int], lengths: Sequence[float], centres_xyz: np.ndarray,
                   sigma_cells: float, cut_sigmas: float = 4.0, batch: int = 4096) -> np.ndarray:
    """Sum of unit-amplitude periodic Gaussian blobs of width sigma_cells (in
    cells), truncated at cut_sigmas widths, evaluated at cell centres.  Each blob
    is separable, exp(-|x-c|^2 / (2 s^2)) = gx * gy * gz, so it is laid down as
    an outer product over its (2R+1)^3 support; batches of blobs are summed
    into the grid with bincount (a fixed summation order)."""
    nz, ny, nx = shape
    ns = (nx, ny, nz)
    hs = [lengths[d] / ns[d] for d in range(3)]
    R = int(math.ceil(cut_sigmas * sigma_cells))
    offs = np.arange(-R, R + 1)
    n = nx * ny * nz
    out = np.zeros(n)
    cen = np.asarray(centres_xyz, dtype=np.float64)
    for b0 in range(0, len(cen), batch):
        c = cen[b0:b0 + batch]
        gs, ids = [], []
        for d in range(3):
            s = c[:, d] / hs[d] - 0.5                     # position in cell-centre index units
            cells = np.floor(s).astype(np.int64)[:, None] + offs[None, :]
            dist = cells - s[:, None]
            g = np.exp(-0.5 * (dist / sigma_cells) ** 2)
            g[np.abs(dist) > cut_sigmas * sigma_cells] = 0.0
            gs.append(g)
            ids.append(cells % ns[d])
        w = gs[2][:, :, None, None] * gs[1][:, None, :, None] * gs[0][:, None, None, :]
        flat = (ids[2][:, :, None, None] * ny + ids[1][:, None, :, None]) * nx + ids[0][:, None, None, :]
        out += np.bincount(flat.ravel(), weights=w.ravel(), minlength=n)
    return out.reshape(shape)


@dataclass
class Problem:
    """One solve: grid shape (nz, ny, nx), box lengths (lx, ly, lz), fields."""
    name: str
    shape: Tuple[int, int, int]
    lengths: Tuple[float, float, float]
    rho: np.ndarray
    b: np.ndarray

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))


def workload1(n: int = 32) -> Problem:
    rng = np.random.default_rng(workload_seed(1))
    L = (TWO_PI,) * 3
    x = centres(n, TWO_PI)
    sz, sy, sx = np.sin(x)[:, None, None], np.sin(x)[None, :, None], np.sin(x)[None, None, :]
    rho = 1.0 + 0.5 * sz * sy * sx
    b = face_divergence((n, n, n), L, rng)
    return Problem(f"sinusoidal-rho {n}^3", (n, n, n), L, np.ascontiguousarray(rho), b)


def workload2(n: int = 256, ratio: float = 4.0, kmax: float = 8.0) -> Problem:
    rng = np.random.default_rng(workload_seed(2))
    L = (TWO_PI,) * 3
    s = bandlim((n, n, n), L, kmax, rng)
    rho = contrast_exp(s, ratio)
    b = bandlim((n, n, n), L, kmax, rng)
    return Problem(f"lognormal-rho {n}^3 ratio {ratio:g}", (n, n, n), L, rho, b)


def workload3_particles(particles: int = 10**6) -> np.ndarray:
    """The particle positions of workload 3, (particles, 3) as (x, y, z), the
    same draws workload3 uses."""
    rng = np.random.default_rng(workload_seed(3))
    return rng.uniform(0.0, TWO_PI, size=(particles, 3))


def workload3(n: int = 512, particles: int = 10**6, ratio: float = 10.0,
              kmax: float = 8.0) -> Problem:
    rng = np.random.default_rng(workload_seed(3))
    L = (TWO_PI,) * 3
    pos = rng.uniform(0.0, TWO_PI, size=(particles, 3))
    d = cic_deposit((n, n, n), L, pos)
    rho = 1.0 / (1.0 + (ratio - 1.0) * d / d.max())
    b = bandlim((n, n, n), L, kmax, rng)
    return Problem(f"particle-deposit-rho {n}^3 ratio {ratio:g}", (n, n, n), L, rho, b)


def workload3_b_device(n: int = 512, particles: int = 10**6, kmax: float = 8.0, device="cuda"):
    """b of workload 3 generated on `device` (a torch tensor), from the same
    seeded draws as workload3 (the particle positions are drawn first and
    skipped).  The density of workload 3 is the deposit of
    workload3_particles(), which a caller can build with the GPU's P."""
    rng = np.random.default_rng(workload_seed(3))
    rng.uniform(0.0, TWO_PI, size=(particles, 3))
    return bandlim_device((n, n, n), (TWO_PI,) * 3, kmax, rng, device)


def workload5_draws(shape=(512, 512, 1024), blobs: int = 10**5, kmax: float = 8.0, device=None):
    """The seeded draws of workload 5 without the blob sum: the box lengths, the
    blob centres (blobs, 3) as (x, y, z), and b (on `device` as a torch tensor
    when given, else on the host), from the same generator states as
    workload5."""
    rng = np.random.default_rng(workload_seed(5))
    nz, ny, nx = shape
    h = TWO_PI / ny
    L = (nx * h, ny * h, nz * h)
    cen = rng.uniform(0.0, 1.0, size=(blobs, 3)) * np.asarray(L)
    b = bandlim_device(shape, L, kmax, rng, device) if device is not None else bandlim(shape, L, kmax, rng)
    return L, cen, b


def workload5(shape=(512, 512, 1024), blobs: int = 10**5, ratio: float = 20.0,
              sigma_cells: float = 2.0, kmax: float = 8.0) -> Problem:
    rng = np.random.default_rng(workload_seed(5))
    nz, ny, nx = shape
    h = TWO_PI / ny
    L = (nx * h, ny * h, nz * h)
    cen = rng.uniform(0.0, 1.0, size=(blobs, 3)) * np.asarray(L)
    f = gaussian_blobs(shape, L, cen, sigma_cells)
    rho = 1.0 / (1.0 + (ratio - 1.0) * f / f.max())
    b = bandlim(shape, L, kmax, rng)
    return Problem(f"hot-blob-rho {nx}x{ny}x{nz} ratio {ratio:g}", tuple(shape), L, rho, b)


def workload_duct(n: int = 256, ratio: float = 4.0, kmax: float = 8.0) -> Problem:
    rng = np.random.default_rng(workload_seed(6))
    shape = (n, n, 2 * n)
    L = (2.0 * TWO_PI, TWO_PI, TWO_PI)
    s = bandlim(shape, L, kmax, rng)
    rho = contrast_exp(s, ratio)
    b = bandlim(shape, L, kmax, rng)
    return Problem(f"duct lognormal-rho {2 * n}x{n}x{n} ratio {ratio:g}", shape, L, rho, b)


def momentum_fields(shape: Sequence[int], lengths: Sequence[float], kmax: float = 8.0,
                    target_scale: float = 0.1, seed: int = 7):
    """Inputs of one pressure projection: the predicted face momentum (three
    band-limited fields, one per face direction) and the divergence target
    RHS^div (band-limited, scaled by `target_scale`)."""
    rng = np.random.default_rng(workload_seed(7) * 1000 + seed)
    mx, my, mz = (bandlim(shape, lengths, kmax, rng) for _ in range(3))
    rhs_div = target_scale * bandlim(shape, lengths, kmax, rng)
    return mx, my, mz, rhs_div


def advected_chain_device(n: int = 256, steps: int = 12, ratio: float = 4.0, kmax: float = 8.0,
                          shift_cells: Sequence[float] = (0.5, 0.25, 0.0), omega: float = 0.02,
                          chain: int = 0, device="cuda"):
    """A time series of solves whose inputs evolve slowly (workload 8): rho_t =
    exp(c s(x - U t)), s band-limited (|k| <= kmax) and carried by a uniform
    velocity U of `shift_cells` cells per step, c fixed by max/min rho_0 =
    `ratio`; b_t = cos(omega t) b1 + sin(omega t) b2 with b1, b2 band-limited.
    Generated on `device` (the last synthesis step as a matmul, see
    bandlim_device).  Returns (shape, lengths, [(rho_t, b_t)]) as torch tensors."""
    import torch

    shape, L = (n, n, n), (TWO_PI,) * 3
    h = TWO_PI / n
    seed = workload_seed(8) * 1000 + chain
    s0 = bandlim_device(shape, L, kmax, np.random.default_rng(seed), device)
    c = math.log(ratio) / float(s0.max() - s0.min())
    del s0
    rng_b = np.random.default_rng(seed + 500)
    b1 = bandlim_device(shape, L, kmax, rng_b, device)
    b2 = bandlim_device(shape, L, kmax, rng_b, device)
    out = []
    for t in range(steps):
        sh = tuple(v * h * t for v in shift_cells)
        s = bandlim_device(shape, L, kmax, np.random.default_rng(seed), device, shift=sh)
        rho = torch.exp(s * c).contiguous()
        del s
        b = (math.cos(omega * t) * b1 + math.sin(omega * t) * b2).contiguous()
        out.append((rho, b))
    return shape, L, out


SERVE_SIZES = (64, 96, 128, 192)


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    ratio: float


def request_stream(count: int = 512, rate_hz: float = 100.0,
                   sizes: Sequence[int] = SERVE_SIZES) -> List[Request]:
    """Poisson arrivals at a fixed rate; grid size uniform over `sizes`;
    density contrast uniform in [2, 8]."""
    rng = np.random.default_rng(workload_seed(4))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=count)
    ratios = rng.uniform(2.0, 8.0, size=count)
    return [Request(r, float(t[r]), int(ns[r]), float(ratios[r])) for r in range(count)]


def request_problem(req: Request, kmax: float = 8.0) -> Problem:
    """Fields of one served request: lognormal band-limited rho with the
    request's contrast, band-limited zero-mean b."""
    rng = np.random.default_rng(request_seed(req.rid))
    n = req.n
    L = (TWO_PI,) * 3
    s = bandlim((n, n, n), L, kmax, rng)
    rho = contrast_exp(s, req.ratio)
    b = bandlim((n, n, n), L, kmax, rng)
    return Problem(f"request {req.rid} {n}^3 ratio {req.ratio:.2f}", (n, n, n), L, rho, b)


def request_fields_device(req: Request, kmax: float = 8.0, device="cuda"):
    """Fields (rho, b) of one served request generated on `device` (torch
    tensors), from the same seeded draws as request_problem."""
    import torch

    rng = np.random.default_rng(request_seed(req.rid))
    n = req.n
    L = (TWO_PI,) * 3
    s = bandlim_device((n, n, n), L, kmax, rng, device)
    span = float(s.max() - s.min())
    rho = torch.exp(s * (math.log(req.ratio) / span))
    b = bandlim_device((n, n, n), L, kmax, rng, device)
    return rho.contiguous(), b


def small_problem(shape=(16, 12, 24), lengths=(TWO_PI, 3.0, 5.0), ratio: float = 3.0,
                  seed: int = 7, kmax: float = 3.0) -> Problem:
    """A small anisotropic problem (distinct nx, ny, nz and lx, ly, lz) for
    parity tests that must catch transposed axes."""
    rng = np.random.default_rng(seed)
    L3 = (lengths[0], lengths[1], lengths[2])
    s = bandlim(shape, L3, kmax, rng)
    rho = contrast_exp(s, ratio)
    b = bandlim(shape, L3, kmax, rng) + 0.3 * rng.standard_normal(shape)
    return Problem(f"small {shape}", tuple(shape), L3, rho, b)
