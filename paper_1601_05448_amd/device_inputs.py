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
