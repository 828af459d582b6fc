"""GPU parity at the two largest workloads, full size, in the launch
configuration the solver uses for them:

* 512^3, density from a trilinear deposit of 10^6 seeded particles,
  rho = 1/(1 + 9 d/max d) (ratio 10);
* 1024 x 512 x 512 on [0,4pi) x [0,2pi)^2, density from 10^5 seeded Gaussian
  blobs of width 2 cells, rho = 1/(1 + 19 f/max f) (ratio 20).

A full oracle solve at these sizes would take hours, so the checks are the
properties that hold at any size: the oracle's O(n) FP64 residual of the GPU
answer is <= 1e-10 and matches what the library reports; the reported
a-posteriori error bound is small; the FP64 and FP32+refinement answers agree
within the sum of their bounds; p has mean 0.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import announce, dev, host, rel_l2
from paper_1601_05448_amd import inputs
from paper_1601_05448_amd import poisson as P

pytestmark = pytest.mark.gpu
PRECISIONS = [P.POISSON_FP64, P.POISSON_FP32_REFINE]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()
    yield


@pytest.fixture(scope="module")
def deposit512():
    announce("generate particle-deposit 512^3")
    return inputs.workload3(512)


@pytest.fixture(scope="module")
def blobs1024():
    announce("generate hot-blob 1024x512x512")
    return inputs.workload5()


_answers = {}


def _solve_and_check(prob, precision, key):
    import torch

    announce("solve", prob.name, "precision", precision)
    rho, b = dev(prob.rho), dev(prob.b)
    p = torch.zeros(prob.shape, dtype=torch.float64, device="cuda")
    with P.Solver(prob.shape, prob.lengths, precision=precision) as s:
        st = s.solve(rho, b, p, 1e-10)
    ph = host(p)
    del rho, b, p
    torch.cuda.empty_cache()
    announce("residual", prob.name, "iters", st["iters"], "outer", st["outer_iters"])
    res = oracle.residual(prob.rho, prob.b, ph, prob.lengths)
    assert st["code"] == P.POISSON_OK, st
    assert res["rel"] <= 1e-10, res
    assert abs(st["rel_resid"] - res["rel"]) <= 1e-3 * res["rel"]
    assert st["err_bound_rel"] < 1e-6, st
    assert abs(ph.mean()) <= 1e-12 * np.max(np.abs(ph))
    _answers[(key, precision)] = (ph, st["err_bound_rel"])
    other = P.POISSON_FP64 if precision == P.POISSON_FP32_REFINE else P.POISSON_FP32_REFINE
    if (key, other) in _answers:
        po, bo = _answers.pop((key, other))
        _answers.pop((key, precision))
        assert rel_l2(ph, po) <= 1.01 * (st["err_bound_rel"] + bo) + 1e-14


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_size_512_particle_deposit(deposit512, precision):
    _solve_and_check(deposit512, precision, "deposit512")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_size_1024x512x512_hot_blobs(blobs1024, precision):
    _solve_and_check(blobs1024, precision, "blobs1024")
