"""Workload fields built on the device with the library's own kernels.

The 512^3 particle workload's density is the trilinear deposit (the paper's
linear particle-to-grid projection P, section "Physical model") of its 10^6
seeded particles; building it with the GPU's P instead of the host recipe in
``inputs.workload3`` saves minutes of host time at this size.  Same draws as
the host recipe: the positions of ``inputs.workload3_particles`` and b from the
generator state after them.
"""
from __future__ import annotations

import math

from . import inputs
from . import poisson as P


class DeviceProblem:
    """A workload whose fields are torch tensors on the device."""

    def __init__(self, name, shape, lengths, rho, b):
        self.name, self.shape, self.lengths, self.rho, self.b = name, tuple(shape), tuple(lengths), rho, b

    @property
    def n(self) -> int:
        return int(self.shape[0] * self.shape[1] * self.shape[2])


def workload3_device(n: int = 512, ratio: float = 10.0) -> DeviceProblem:
    """rho = 1/(1 + (ratio - 1) d/max d) with d the GPU deposit (per unit
    volume; the ratio d/max d equals that of the raw weight sums), b
    band-limited (|k| <= 8)."""
    import torch

    shape, L = (n, n, n), (2.0 * math.pi,) * 3
    pos = torch.from_numpy(inputs.workload3_particles()).cuda()
    d = torch.empty(shape, dtype=torch.float64, device="cuda")
    with P.Solver(shape, L) as s:
        P.poisson_deposit(s.h, pos, None, d)
    rho = (1.0 / (1.0 + (ratio - 1.0) * d / d.max())).contiguous()
    del d, pos
    b = inputs.workload3_b_device(n)
    return DeviceProblem(f"particle-deposit-rho {n}^3 ratio {ratio:g}", shape, L, rho, b)


def gaussian_blobs_device(shape, lengths, centres_xyz, sigma_cells: float, cut_sigmas: float = 4.0,
                          batch: int = 2048, device="cuda"):
    """The blob sum of inputs.gaussian_blobs (unit-amplitude periodic Gaussians
    of width sigma_cells, truncated at cut_sigmas widths, at cell centres) on
    the device: each batch of blobs lays its separable (2R+1)^3 footprints into
    the grid with an accumulating index_put in torch's deterministic mode (a
    sort-based sum, the same bits every run)."""
    import torch

    nz, ny, nx = shape
    ns = (nx, ny, nz)
    hs = [lengths[d] / ns[d] for d in range(3)]
    R = int(math.ceil(cut_sigmas * sigma_cells))
    offs = torch.arange(-R, R + 1, device=device, dtype=torch.float64)
    out = torch.zeros(nx * ny * nz, dtype=torch.float64, device=device)
    cen = torch.as_tensor(centres_xyz, dtype=torch.float64, device=device)
    was = torch.are_deterministic_algorithms_enabled()
    torch.use_deterministic_algorithms(True)
    try:
        for b0 in range(0, cen.shape[0], batch):
            c = cen[b0:b0 + batch]
            gs, ids = [], []
            for d in range(3):
                s = c[:, d] / hs[d] - 0.5
                cells = torch.floor(s)[:, None] + offs[None, :]
                dist = cells - s[:, None]
                g = torch.exp(-0.5 * (dist / sigma_cells) ** 2)
                g = torch.where(dist.abs() > cut_sigmas * sigma_cells, torch.zeros_like(g), g)
                gs.append(g)
                ids.append(torch.remainder(cells.to(torch.int64), ns[d]))
            w = gs[2][:, :, None, None] * gs[1][:, None, :, None] * gs[0][:, None, None, :]
            flat = (ids[2][:, :, None, None] * ny + ids[1][:, None, :, None]) * nx + ids[0][:, None, None, :]
            out.index_put_((flat.reshape(-1),), w.reshape(-1), accumulate=True)
    finally:
        torch.use_deterministic_algorithms(was)
    return out.reshape(shape)


def workload5_device(shape=(512, 512, 1024), blobs: int = 10**5, ratio: float = 20.0,
                     sigma_cells: float = 2.0) -> DeviceProblem:
    """The 1024 x 512 x 512 hot-blob workload on the device: rho = 1/(1 + 19
    f/max f) with f the blob sum, b band-limited, from the host recipe's draws."""
    L, cen, b = inputs.workload5_draws(shape, blobs, device="cuda")
    f = gaussian_blobs_device(shape, L, cen, sigma_cells)
    rho = (1.0 / (1.0 + (ratio - 1.0) * f / f.max())).contiguous()
    del f
    nz, ny, nx = shape
    return DeviceProblem(f"hot-blob-rho {nx}x{ny}x{nz} ratio {ratio:g}", shape, L, rho, b)
