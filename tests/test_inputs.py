"""The seeded input generators against independent formulations of what they
produce (they hold none of the method's arithmetic; both the oracle and the
GPU path take their fields)."""
import math

import numpy as np

from paper_1601_05448_amd import inputs


def test_gaussian_blobs_against_direct_sum():
    """Sum over blobs of prod_d exp(-d_d^2 / (2 s^2)), d_d the signed distance
    (in cells) from the cell centre to the nearest periodic image of the blob
    centre, zero beyond 4 s; batches of any size give the same grid."""
    rng = np.random.default_rng(11)
    shape, L, sig = (16, 14, 20), (2.0, 1.5, 2.5), 1.3
    cen = rng.uniform(0, 1, size=(23, 3)) * np.asarray(L)
    got = inputs.gaussian_blobs(shape, L, cen, sig, batch=5)
    assert np.allclose(got, inputs.gaussian_blobs(shape, L, cen, sig, batch=1000), rtol=1e-14, atol=1e-14)
    nz, ny, nx = shape
    ns = (nx, ny, nz)
    want = np.zeros(shape)
    for c in cen:
        g = []
        for d in range(3):
            x = np.arange(ns[d]) + 0.5               # cell centres in cell units
            cc = c[d] * ns[d] / L[d]
            dist = (x - cc + ns[d] / 2) % ns[d] - ns[d] / 2
            g.append(np.where(np.abs(dist) <= 4 * sig, np.exp(-0.5 * (dist / sig) ** 2), 0.0))
        want += g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(want)


def test_cic_deposit_conserves_and_interpolates():
    """Each particle deposits total weight 1; a particle at a cell centre puts
    it all in that cell; one halfway between two centres splits it evenly."""
    shape, L = (8, 6, 10), (2.0, 3.0, 4.0)
    nz, ny, nx = shape
    h = (L[0] / nx, L[1] / ny, L[2] / nz)
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 1, size=(200, 3)) * np.asarray(L)
    assert abs(inputs.cic_deposit(shape, L, pos).sum() - 200) < 1e-10
    at_centre = np.array([[(3 + 0.5) * h[0], (2 + 0.5) * h[1], (5 + 0.5) * h[2]]])
    d = inputs.cic_deposit(shape, L, at_centre)
    assert abs(d[5, 2, 3] - 1.0) < 1e-12 and abs(d.sum() - 1.0) < 1e-12
    between = np.array([[(nx - 1 + 1.0) * h[0], 0.5 * h[1], 0.5 * h[2]]])  # halfway, wrapping in x
    d = inputs.cic_deposit(shape, L, between)
    assert abs(d[0, 0, nx - 1] - 0.5) < 1e-12 and abs(d[0, 0, 0] - 0.5) < 1e-12


def test_bandlim_is_band_limited_zero_mean_unit_rms():
    shape, L, kmax = (16, 12, 20), (2 * math.pi, 3.0, 5.0), 4.0
    f = inputs.bandlim(shape, L, kmax, np.random.default_rng(2))
    assert abs(f.mean()) < 1e-14 and abs(np.sqrt(np.mean(f * f)) - 1) < 1e-12
    F = np.fft.fftn(f)
    nz, ny, nx = shape
    kz = 2 * math.pi * np.fft.fftfreq(nz, 1 / nz) / L[2]
    ky = 2 * math.pi * np.fft.fftfreq(ny, 1 / ny) / L[1]
    kx = 2 * math.pi * np.fft.fftfreq(nx, 1 / nx) / L[0]
    kk = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    assert np.max(np.abs(F[kk > kmax * kmax * (1 + 1e-9)])) < 1e-9 * np.max(np.abs(F))


def test_shifted_bandlim_is_the_same_field_carried_along():
    """A shift of whole cells (any axis) is a roll of the unshifted field; the
    same draws with a fractional shift keep the band limit and the RMS."""
    shape, L, kmax = (12, 10, 16), (2 * math.pi, 2.5, 3.0), 3.0
    nz, ny, nx = shape
    h = (L[0] / nx, L[1] / ny, L[2] / nz)
    base = inputs.bandlim(shape, L, kmax, np.random.default_rng(9))

    def shifted(sh):
        t2, ez = inputs._bandlim_spectrum(shape, L, kmax, np.random.default_rng(9), sh)
        f = (ez.real.T @ t2.real - ez.imag.T @ t2.imag).reshape(shape)
        f -= f.mean()
        return f / math.sqrt(np.mean(f * f))

    got = shifted((3 * h[0], -2 * h[1], 5 * h[2]))
    want = np.roll(np.roll(np.roll(base, 3, axis=2), -2, axis=1), 5, axis=0)
    assert np.max(np.abs(got - want)) < 1e-12
    half = shifted((0.5 * h[0], 0.25 * h[1], 0.0))
    assert abs(np.sqrt(np.mean(half * half)) - 1) < 1e-12 and abs(half.mean()) < 1e-14


def test_duct_and_projection_inputs():
    """The duct is 2N x N x N on [0, 4pi) x [0, 2pi)^2 with max/min rho = ratio;
    the projection inputs are three band-limited momentum fields and a
    divergence target scaled by 0.1; both are deterministic."""
    p = inputs.workload_duct(8)
    assert p.shape == (8, 8, 16) and p.lengths == (4 * math.pi, 2 * math.pi, 2 * math.pi)
    assert abs(p.rho.max() / p.rho.min() - 4.0) < 1e-12
    assert np.array_equal(p.rho, inputs.workload_duct(8).rho)
    mx, my, mz, rd = inputs.momentum_fields((8, 6, 12), (2 * math.pi,) * 3)
    for m in (mx, my, mz):
        assert abs(np.sqrt(np.mean(m * m)) - 1) < 1e-12
    assert abs(np.sqrt(np.mean(rd * rd)) - 0.1) < 1e-12
    assert not np.array_equal(mx, my)
    assert np.array_equal(rd, inputs.momentum_fields((8, 6, 12), (2 * math.pi,) * 3)[3])


def test_workload3_particles_are_the_workload_draws():
    """workload3_particles returns the positions workload 3 deposits."""
    pos = inputs.workload3_particles(500)
    assert pos.shape == (500, 3) and pos.min() >= 0 and pos.max() < 2 * math.pi
    d = inputs.cic_deposit((8, 8, 8), (2 * math.pi,) * 3, pos)
    w = inputs.workload3(8, particles=500)
    assert np.allclose(w.rho, 1.0 / (1.0 + 9.0 * d / d.max()), rtol=0, atol=1e-15)


def test_device_blob_sum_matches_host_recipe():
    """The torch blob sum used to build the 1024 x 512 x 512 workload on the
    device equals the host recipe's (bincount) sum up to summation order."""
    import torch  # noqa: F401

    from paper_1601_05448_amd import device_inputs

    shape = (12, 16, 24)
    L, cen, _ = inputs.workload5_draws(shape, blobs=40)
    want = inputs.gaussian_blobs(shape, L, cen, 2.0)
    got = device_inputs.gaussian_blobs_device(shape, L, cen, 2.0, batch=16, device="cpu").numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(want)
