"""GPU parity of the projection step around the solve (appendix A of
Pouransari, Mortazavi & Mani, arXiv:1601.05448: RHS of the pressure equation
from the divergence of the predicted momentum over the face density, chi from
its mean, the solve, and the momentum correction -C dt grad p) against the
FP64 CPU oracle, through the C ABI.

Tolerances:
  * divergence (FP64, the same sums up to rounding order; the GPU multiplies by
    1/h where the oracle divides by h): 1e-12 relative to the largest magnitude
    of the oracle's field;
  * projection: p as in the solver tests (relative residual <= 1e-10 by the
    oracle, error below the a-posteriori bound); chi to 1e-12 of max |RHS^div|;
    the corrected momentum differs from the oracle's by C dt times the face
    difference of the two pressures, so it is held to
    2 C dt max|p_gpu - p_oracle| / h_min + 1e-12 max|m|; and the oracle's
    divergence of the GPU's corrected momentum meets RHS^div - chi within
    C dt times 10 tol ||b~||.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import announce, dev, host, rel_l2
from paper_1601_05448_amd import inputs
from paper_1601_05448_amd import poisson as P

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi
C_DT = 5e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()
    yield


# (nz, ny, nx): partial z tiles (nz not a multiple of 16), rows shorter and
# longer than a block, a plane that is not a multiple of the block
@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 12), (24, 12, 24), (12, 4, 256), (6, 6, 96)])
@pytest.mark.parametrize("coef", [0, 1])
@pytest.mark.parametrize("bc", [P.POISSON_BC_PERIODIC, P.POISSON_BC_WALLS_X])
def test_divergence_matches_oracle(shape, coef, bc):
    announce("divergence", shape, coef, bc)
    rng = np.random.default_rng(sum(shape) + coef)
    L = (5.0, 3.0, TWO_PI)
    rho = np.exp(rng.uniform(-1.0, 1.0, shape))
    m = [rng.standard_normal(shape) for _ in range(3)]
    want = oracle.divergence(rho, *m, L, coef=coef, bcx=bc)
    h = P.poisson_create(shape, L, coef=coef, bc_x=bc)
    try:
        out = dev(np.zeros(shape))
        P.poisson_divergence(h, dev(rho), *(dev(x) for x in m), out)
    finally:
        P.poisson_destroy(h)
    assert np.max(np.abs(host(out) - want)) <= 1e-12 * np.max(np.abs(want))


def _project_gpu(prob, m, rd, precision=P.POISSON_FP64, coef=0, tol=1e-10, bc=P.POISSON_BC_PERIODIC):
    h = P.poisson_create(prob.shape, prob.lengths, precision=precision, coef=coef, bc_x=bc)
    try:
        dm = [dev(x) for x in m]
        p = dev(np.zeros(prob.shape))
        rc, chi = P.poisson_project(h, dev(prob.rho), *dm, dev(rd), C_DT, p, tol)
        st = P.poisson_get_stats(h)
    finally:
        P.poisson_destroy(h)
    return rc, chi, host(p), [host(x) for x in dm], st


def _check_projection(prob, m, rd, rc, chi, p, mg, st, coef=0, tol=1e-10, bc=P.POISSON_BC_PERIODIC):
    assert rc == P.POISSON_OK, st
    ref = oracle.project(prob.rho, *m, rd, C_DT, lengths=prob.lengths, coef=coef, tol=1e-13, bcx=bc)
    # chi
    assert abs(chi - ref["chi"]) <= 1e-12 * np.max(np.abs(rd))
    # the pressure: residual by the oracle and the a-posteriori bound
    b = (oracle.divergence(prob.rho, *m, prob.lengths, coef=coef, bcx=bc) - rd) / C_DT
    res = oracle.residual(prob.rho, b, p, prob.lengths, coef, bcx=bc)
    assert res["rel"] <= tol, res
    assert rel_l2(p, ref["p"]) <= st["err_bound_rel"] * (1 + 1e-6) + 1e-14
    # the corrected momentum
    nz, ny, nx = prob.shape
    hmin = min(prob.lengths[0] / nx, prob.lengths[1] / ny, prob.lengths[2] / nz)
    dp = np.max(np.abs(p - ref["p"]))
    for got, key in zip(mg, ("mx", "my", "mz")):
        want = ref[key]
        assert np.max(np.abs(got - want)) <= 2.0 * C_DT * dp / hmin + 1e-12 * np.max(np.abs(want)), key
    if bc == P.POISSON_BC_WALLS_X:  # the closed end faces keep their momentum, bit for bit
        assert np.array_equal(mg[0][:, :, -1], m[0][:, :, -1])
    # the divergence target
    d = oracle.divergence(prob.rho, *mg, prob.lengths, coef=coef, bcx=bc)
    bt = b - b.mean()
    assert np.linalg.norm(d - (rd - chi)) <= C_DT * 10 * tol * np.linalg.norm(bt)


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
@pytest.mark.parametrize("coef", [0, 1])
@pytest.mark.parametrize("bc", [P.POISSON_BC_PERIODIC, P.POISSON_BC_WALLS_X])
def test_project_matches_oracle(precision, coef, bc):
    announce("project", precision, coef, bc)
    prob = inputs.small_problem(shape=(24, 12, 64), lengths=(5.0, 3.0, TWO_PI))
    m0, m1, m2, rd = inputs.momentum_fields(prob.shape, prob.lengths)
    rd = rd + 0.37  # a target with a nonzero mean: chi must take it
    m = [m0, m1, m2]
    rc, chi, p, mg, st = _project_gpu(prob, m, rd, precision, coef, bc=bc)
    _check_projection(prob, m, rd, rc, chi, p, mg, st, coef, bc=bc)


def test_project_twice_changes_nothing():
    """The projected momentum already meets the target: a second projection
    finds (nearly) nothing to correct."""
    announce("project twice")
    prob = inputs.small_problem(shape=(16, 12, 24), lengths=(TWO_PI,) * 3)
    m0, m1, m2, rd = inputs.momentum_fields(prob.shape, prob.lengths, seed=3)
    h = P.poisson_create(prob.shape, prob.lengths)
    try:
        dm = [dev(x) for x in (m0, m1, m2)]
        p = dev(np.zeros(prob.shape))
        P.poisson_project(h, dev(prob.rho), *dm, dev(rd), C_DT, p, 1e-12)
        first = [host(x).copy() for x in dm]
        p2 = dev(np.zeros(prob.shape))
        rc, _ = P.poisson_project(h, dev(prob.rho), *dm, dev(rd), C_DT, p2, 1e-12)
        assert rc == P.POISSON_OK
        assert np.max(np.abs(host(p2))) <= 1e-9 * np.max(np.abs(host(p)))
        for a, x in zip(first, dm):
            assert np.max(np.abs(host(x) - a)) <= 1e-10 * np.max(np.abs(a))
    finally:
        P.poisson_destroy(h)


def test_project_rejects_bad_arguments():
    announce("project errors")
    prob = inputs.small_problem(shape=(8, 8, 16), lengths=(TWO_PI,) * 3)
    m = [dev(x) for x in inputs.momentum_fields(prob.shape, prob.lengths)[:3]]
    rho, rd, p = dev(prob.rho), dev(np.zeros(prob.shape)), dev(np.zeros(prob.shape))
    h = P.poisson_create(prob.shape, prob.lengths)
    try:
        for c_dt in (0.0, -1.0, float("nan")):
            with pytest.raises(P.PoissonError):
                P.poisson_project(h, rho, *m, rd, c_dt, p, 1e-10)
        with pytest.raises(P.PoissonError):  # p aliases a momentum component
            P.poisson_project(h, rho, m[0], m[1], m[2], rd, C_DT, m[1], 1e-10)
        with pytest.raises(P.PoissonError) as e:  # the divergence written over its input
            P.poisson_divergence(h, rho, m[0], m[1], m[2], m[2])
        assert e.value.code == P.POISSON_EINVAL
    finally:
        P.poisson_destroy(h)


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_full_size_projection_256(precision):
    """256^3 lognormal density with band-limited momentum, at full size: the
    oracle's divergence of the corrected momentum meets the target, and chi is
    the mean of the target."""
    announce("full size projection 256^3", precision)
    prob = inputs.workload2(256)
    m0, m1, m2, rd = inputs.momentum_fields(prob.shape, prob.lengths)
    rd = rd + 0.25
    tol = 1e-10
    rc, chi, p, mg, st = _project_gpu(prob, [m0, m1, m2], rd, precision)
    assert rc == P.POISSON_OK
    assert abs(chi - rd.mean()) <= 1e-10 * np.max(np.abs(rd))
    b = (oracle.divergence(prob.rho, m0, m1, m2, prob.lengths) - rd) / C_DT
    bt = b - b.mean()
    d = oracle.divergence(prob.rho, *mg, prob.lengths)
    assert np.linalg.norm(d - (rd - chi)) <= C_DT * 10 * tol * np.linalg.norm(bt)


def test_full_size_duct_projection():
    """The 512 x 256 x 256 duct (walls in x) at full size, FP32 sweeps with
    refinement: chi is the mean of the target (the closed box's divergence has
    zero mean), the closed end faces keep their momentum, and the oracle's
    divergence of the corrected momentum meets the target."""
    announce("full size duct projection 512x256x256")
    prob = inputs.workload_duct(256)
    m0, m1, m2, rd = inputs.momentum_fields(prob.shape, prob.lengths)
    rd = rd + 0.25
    tol = 1e-10
    bc = P.POISSON_BC_WALLS_X
    rc, chi, p, mg, st = _project_gpu(prob, [m0, m1, m2], rd, P.POISSON_FP32_REFINE, bc=bc)
    assert rc == P.POISSON_OK, st
    assert abs(chi - rd.mean()) <= 1e-10 * np.max(np.abs(rd))
    assert np.array_equal(mg[0][:, :, -1], m0[:, :, -1])
    b = (oracle.divergence(prob.rho, m0, m1, m2, prob.lengths, bcx=bc) - rd) / C_DT
    bt = b - b.mean()
    d = oracle.divergence(prob.rho, *mg, prob.lengths, bcx=bc)
    assert np.linalg.norm(d - (rd - chi)) <= C_DT * 10 * tol * np.linalg.norm(bt)
