"""GPU parity of libpoisson against the FP64 CPU oracle, through the C ABI.

Paper: Pouransari, Mortazavi & Mani (arXiv:1601.05448), section "Poisson
equation", eq. (Pois).  Tolerances:
  * operator, residual and L^+ sweeps (FP64): 1e-12 relative to the largest
    magnitude of the oracle's field (both sides are FP64; they differ only in
    the order of rounding, the GPU contracts to FMA);
  * solves: relative residual <= 1e-10 evaluated by the oracle on the GPU's p,
    and the relative L2 error against the oracle's solution below both the
    a-posteriori bound the library reports and a fixed 1e-8;
  * FP64 iteration histories agree with the oracle's to 1e-6 relative per
    iteration (same method, same iterates up to rounding).
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
LENGTHS = [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()
    yield


def _shapes_every_length():
    small = [4, 6, 8]
    out = []
    for n, L in enumerate(LENGTHS):
        a, b = small[n % 3], small[(n + 1) % 3]
        out += [(L, a, b), (a, L, b), (a, b, L)]
    return out


@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 12), (16, 12, 24), (12, 48, 32), (32, 32, 32), (6, 96, 8)])
@pytest.mark.parametrize("coef", [0, 1])
def test_apply_matches_oracle(shape, coef):
    announce("apply", shape, coef)
    rng = np.random.default_rng(11)
    L = (TWO_PI, 3.0, 5.0)
    rho = np.exp(rng.uniform(-1.0, 1.0, shape))
    p = rng.standard_normal(shape)
    want = oracle.apply(rho, p, L, coef)
    h = P.poisson_create(shape, L, coef=coef)
    try:
        out = dev(np.zeros(shape))
        P.poisson_apply(h, dev(rho), dev(p), out)
    finally:
        P.poisson_destroy(h)
    assert np.max(np.abs(host(out) - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("shape", _shapes_every_length())
def test_lap_pinv_matches_oracle(shape):
    """Every supported length along every axis (Hartley sweeps, radices 16/8/4/2/3)."""
    announce("lap_pinv", shape)
    rng = np.random.default_rng(sum(shape))
    L = (TWO_PI, 2.5, 4.0)
    q = rng.standard_normal(shape) + 0.7
    want = oracle.lap_pinv(q, L)
    h = P.poisson_create(shape, L)
    try:
        out = dev(np.zeros(shape))
        P.poisson_lap_pinv(h, dev(q), out)
    finally:
        P.poisson_destroy(h)
    got = host(out)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)), shape


def test_residual_matches_oracle():
    announce("residual")
    prob = inputs.small_problem()
    p = np.random.default_rng(2).standard_normal(prob.shape)
    want = oracle.residual(prob.rho, prob.b, p, prob.lengths, want_field=True)
    h = P.poisson_create(prob.shape, prob.lengths)
    try:
        r = dev(np.zeros(prob.shape))
        rn, bn = P.poisson_residual(h, dev(prob.rho), dev(prob.b), dev(p), r)
    finally:
        P.poisson_destroy(h)
    assert np.max(np.abs(host(r) - want["r"])) <= 1e-12 * np.max(np.abs(want["r"]))
    assert abs(rn - want["r_norm"]) <= 1e-12 * want["r_norm"]
    assert abs(bn - want["b_norm"]) <= 1e-12 * want["b_norm"]


def _solve_gpu(prob, precision=P.POISSON_FP64, coef=0, weight=0, tol=1e-10, p0=None, max_iter=0):
    h = P.poisson_create(prob.shape, prob.lengths, precision=precision, coef=coef, weight=weight,
                         max_iter=max_iter)
    try:
        p = dev(np.zeros(prob.shape) if p0 is None else p0)
        rc = P.poisson_solve(h, dev(prob.rho), dev(prob.b), p, tol)
        st = P.poisson_get_stats(h)
        hist = P.poisson_get_history(h)
    finally:
        P.poisson_destroy(h)
    st["code"] = rc
    return host(p), st, hist


def _check_solution(prob, p, st, ref, coef=0, tol=1e-10, ref_bound=0.0):
    """ref_bound: bound on the reference's own relative error (added to the
    GPU answer's bound when the reference is not much more accurate)."""
    res = oracle.residual(prob.rho, prob.b, p, prob.lengths, coef)
    assert st["code"] == P.POISSON_OK, st
    assert res["rel"] <= tol, res
    assert abs(st["rel_resid"] - res["rel"]) <= 1e-3 * res["rel"] + 1e-15
    err = rel_l2(p, ref)
    assert err <= st["err_bound_rel"] * (1 + 1e-6) + ref_bound + 1e-14, (err, st["err_bound_rel"], ref_bound)
    assert err <= 1e-8
    assert abs(p.mean()) <= 1e-12 * np.max(np.abs(p))
    return err


def test_solve_sinusoidal_32_matches_oracle():
    """The 32^3 workload (rho = 1 + sin x sin y sin z / 2, divergence b), FP64."""
    announce("solve sinusoidal 32^3")
    prob = inputs.workload1(32)
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-13)
    lit = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-10)
    p, st, hist = _solve_gpu(prob)
    _check_solution(prob, p, st, ref["p"])
    assert st["iters"] == lit["iters"]
    assert np.allclose(hist, lit["history"], rtol=1e-6, atol=0)
    assert abs(st["b_mean_removed"] - lit["b_mean"]) <= 1e-12 * max(1.0, abs(lit["b_mean"]))


@pytest.mark.parametrize("coef,weight", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_solve_anisotropic_modes(coef, weight):
    """Distinct nx, ny, nz and lx, ly, lz; both face coefficients and weights."""
    announce("solve anisotropic", coef, weight)
    prob = inputs.small_problem(shape=(24, 12, 48), lengths=(TWO_PI, 3.0, 5.0))
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, coef=coef, weight=weight, tol=1e-13)
    lit = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, coef=coef, weight=weight, tol=1e-10)
    p, st, hist = _solve_gpu(prob, coef=coef, weight=weight)
    _check_solution(prob, p, st, ref["p"], coef)
    assert st["iters"] == lit["iters"]
    assert np.allclose(hist, lit["history"], rtol=1e-6, atol=0)


@pytest.mark.parametrize("shape", [(6, 12, 256), (12, 24, 96), (64, 64, 64)])
def test_solve_ragged_tiles(shape):
    """Line counts that leave a partial last block in every sweep."""
    announce("solve ragged", shape)
    prob = inputs.small_problem(shape=shape, lengths=(TWO_PI, TWO_PI, TWO_PI), ratio=4.0)
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-13)
    p, st, _ = _solve_gpu(prob)
    _check_solution(prob, p, st, ref["p"])


@pytest.mark.parametrize("shape", [(48, 6, 768), (32, 4, 1024)])
def test_solve_fp64_long_rows(shape):
    """FP64 on rows of 768 and 1024 cells: the residual sweep marches four
    columns per thread (ragged z tiles: 48 and 32 planes)."""
    announce("solve fp64 long rows", shape)
    prob = inputs.small_problem(shape=shape, lengths=(TWO_PI, TWO_PI, TWO_PI), ratio=4.0)
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-14, max_iter=40, allow_noconv=True)
    rr = oracle.residual(prob.rho, prob.b, ref["p"], prob.lengths)
    ref_bound = oracle.error_bound(prob.shape, prob.lengths, float(prob.rho.max()), rr["r_norm"]) / \
        np.linalg.norm(ref["p"])
    p, st, _ = _solve_gpu(prob)
    _check_solution(prob, p, st, ref["p"], ref_bound=ref_bound)


@pytest.mark.parametrize("shape", [(6, 12, 128), (24, 6, 512), (24, 12, 64), (12, 8, 1024)])
def test_solve_fp32_refine_ragged_outer_tiles(shape):
    """FP32 refinement where the FP64 outer residual's column tiles are ragged:
    fewer planes than a tile, row-pair strips past the grid, two and four
    columns per thread."""
    announce("solve fp32 refine ragged", shape)
    prob = inputs.small_problem(shape=shape, lengths=(TWO_PI, TWO_PI, TWO_PI), ratio=4.0)
    # with 512 or 1024 cells along x and a few along y the FP64 rounding floor of
    # the relative residual is near 1e-12: the reference takes what 40
    # iterations reach, and its own a-posteriori bound joins the GPU's
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-14, max_iter=40, allow_noconv=True)
    rr = oracle.residual(prob.rho, prob.b, ref["p"], prob.lengths)
    ref_bound = oracle.error_bound(prob.shape, prob.lengths, float(prob.rho.max()), rr["r_norm"]) / \
        np.linalg.norm(ref["p"])
    p, st, _ = _solve_gpu(prob, precision=P.POISSON_FP32_REFINE)
    _check_solution(prob, p, st, ref["p"], ref_bound=ref_bound)


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_kernel_timer_counts_residual_sweeps(precision):
    """The event timer brackets every launch of P1 inside a solve, and the
    library counts the launches that did work."""
    announce("kernel timer", precision)
    prob = inputs.workload2(64)
    fp32 = precision == P.POISSON_FP32_REFINE
    with P.Solver(prob.shape, prob.lengths, precision=precision) as s:
        P.poisson_kernel_timer(s.h, 1, fp32)
        p = dev(np.zeros(prob.shape))
        st = s.solve(dev(prob.rho), dev(prob.b), p, 1e-10)
        ms, n = P.poisson_kernel_timer_read(s.h)
        P.poisson_kernel_timer(s.h, 0)
        st2 = s.solve(dev(prob.rho), dev(prob.b), p, 1e-10)
        assert P.poisson_kernel_timer_read(s.h) == (0.0, 0)
    assert st["code"] == P.POISSON_OK
    # FP64: one P1 per residual evaluation (iters updates + the final one).
    # FP32 on 64-cell rows: the outer residual sweep evaluates the first inner
    # residual of each step, so one P1 per inner update, less one for each step
    # whose end was predicted from the contraction (its confirming P1 idles)
    if fp32:
        assert st["iters"] - st["outer_iters"] <= st["p1_sweeps"] <= st["iters"], st
        assert n >= st["p1_sweeps"] and ms > 0.0
    else:
        assert st["p1_sweeps"] == st["iters"] + 1, st
        assert n >= st["p1_sweeps"] and ms > 0.0
    assert st2["code"] == P.POISSON_OK


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
@pytest.mark.parametrize("n", [32, 64])
def test_graph_replays_match_plain_launches(precision, n):
    """Captured HIP graphs of iteration chunks against the same kernels launched
    one by one: three solves each, with eager work on the caller's stream
    between them, bitwise equal results and equal iteration counts on every
    replay."""
    announce("graph replays", precision, n)
    import torch

    prob = inputs.workload2(n)
    rho, b = dev(prob.rho), dev(prob.b)
    outs = {}
    for plain in (True, False):
        with P.Solver(prob.shape, prob.lengths, precision=precision, use_graphs=not plain) as s:
            p = dev(np.zeros(prob.shape))
            runs = []
            for rep in range(3):
                p.zero_()
                junk = torch.sin(rho) * (rep + 1)  # eager work between replays
                st = s.solve(rho, b, p, 1e-10)
                assert float(junk.sum()) != 0.0
                runs.append((host(p).copy(), st["iters"], st["outer_iters"], st["rel_resid"]))
            outs[plain] = runs
    for (pa, ia, oa, ra), (pb, ib, ob, rb) in zip(outs[True], outs[False]):
        assert np.array_equal(pa, pb) and (ia, oa, ra) == (ib, ob, rb)
    assert all(np.array_equal(outs[False][0][0], r[0]) for r in outs[False])


@pytest.mark.parametrize("maker", ["sinusoidal32", "lognormal64", "deposit64"])
def test_solve_fp32_refine_matches_oracle(maker):
    """FP32 sweeps + FP64 refinement reach the same 1e-10 answer."""
    announce("solve fp32 refine", maker)
    if maker == "sinusoidal32":
        prob = inputs.workload1(32)
    elif maker == "lognormal64":
        prob = inputs.workload2(64)
    else:
        prob = inputs.workload3(64, particles=2000)
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-13)
    p, st, hist = _solve_gpu(prob, precision=P.POISSON_FP32_REFINE)
    _check_solution(prob, p, st, ref["p"])
    assert st["outer_iters"] >= 1 and len(hist) == st["outer_iters"] + 1


def test_constant_b_gives_zero():
    announce("constant b")
    prob = inputs.small_problem()
    prob.b[...] = 3.25
    p, st, _ = _solve_gpu(prob, p0=np.ones(prob.shape))
    assert st["code"] == P.POISSON_OK and st["iters"] == 0
    assert np.all(p == 0.0)


@pytest.mark.parametrize("bad", ["rho_negative", "rho_zero", "rho_nan", "b_inf", "ratio"])
def test_invalid_fields_edomain_and_p_untouched(bad):
    announce("edomain", bad)
    prob = inputs.small_problem()
    if bad == "rho_negative":
        prob.rho[3, 2, 1] = -0.5
    elif bad == "rho_zero":
        prob.rho[0, 0, 0] = 0.0
    elif bad == "rho_nan":
        prob.rho[1, 1, 1] = np.nan
    elif bad == "b_inf":
        prob.b[2, 2, 2] = np.inf
    else:  # density ratio beyond what the scaled reciprocals of the sweeps support
        prob.rho[4, 4, 4] = prob.rho.max() * 1e21
    p0 = np.random.default_rng(1).standard_normal(prob.shape)
    for prec in (P.POISSON_FP64, P.POISSON_FP32_REFINE):
        p, st, _ = _solve_gpu(prob, precision=prec, p0=p0)
        assert st["code"] == P.POISSON_EDOMAIN
        assert np.array_equal(p, p0)


def test_large_density_ratio_within_limits():
    """Ratios up to the documented limits solve (1e6 FP64 with the face average
    of rho; 1e6 FP32_REFINE with the diagonal weight)."""
    announce("large ratio")
    prob = inputs.small_problem(shape=(16, 16, 16), lengths=(TWO_PI,) * 3, ratio=1e6)
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, weight=1, tol=1e-13)
    for prec in (P.POISSON_FP64, P.POISSON_FP32_REFINE):
        p, st, _ = _solve_gpu(prob, precision=prec, weight=1, max_iter=5000)
        _check_solution(prob, p, st, ref["p"])


def test_iteration_cap_returns_last_iterate():
    announce("enoconv")
    prob = inputs.small_problem()
    lit = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-30, max_iter=3, allow_noconv=True)
    p, st, hist = _solve_gpu(prob, tol=1e-30, max_iter=3)
    assert st["code"] == P.POISSON_ENOCONV and st["iters"] == 3
    assert np.allclose(hist, lit["history"], rtol=1e-9, atol=0)
    assert rel_l2(p, lit["p"]) <= 1e-11


def test_warm_start_and_mean_gauge():
    announce("warm start")
    prob = inputs.small_problem()
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-13)["p"]
    p, st, _ = _solve_gpu(prob, p0=ref + 4.0)
    assert st["iters"] == 0 and st["code"] == P.POISSON_OK
    assert np.max(np.abs(p - ref)) <= 1e-12 * np.max(np.abs(ref))
    p, st, _ = _solve_gpu(prob, p0=np.full(prob.shape, -2.0))  # mean removed by the first update
    assert abs(p.mean()) <= 1e-12 * np.max(np.abs(p))
    _check_solution(prob, p, st, ref)


def test_argument_errors():
    announce("argument errors")
    import torch

    prob = inputs.small_problem()
    h = P.poisson_create(prob.shape, prob.lengths)
    try:
        rho, b, p = dev(prob.rho), dev(prob.b), dev(np.zeros(prob.shape))
        for tol in (0.0, -1.0, float("nan")):
            with pytest.raises(P.PoissonError) as e:
                P.poisson_solve(h, rho, b, p, tol)
            assert e.value.code == P.POISSON_EINVAL
        big = torch.zeros(2 * prob.n, dtype=torch.float64, device="cuda")
        with pytest.raises(P.PoissonError):  # b overlaps p
            P.poisson_solve(h, rho, big[: prob.n].view(prob.shape), big[prob.n // 2: prob.n // 2 + prob.n].view(prob.shape), 1e-10)
    finally:
        P.poisson_destroy(h)


def test_deterministic():
    announce("determinism")
    prob = inputs.workload2(64)
    a, _, _ = _solve_gpu(prob)
    b, _, _ = _solve_gpu(prob)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_full_size_256_lognormal(precision):
    """The 256^3 lognormal workload at full size, in the benchmark's launch
    configuration: the oracle's O(n) residual of the GPU answer <= 1e-10, and the
    a-posteriori bound on the error."""
    announce("full size 256^3", precision)
    prob = inputs.workload2(256)
    p, st, _ = _solve_gpu(prob, precision=precision)
    res = oracle.residual(prob.rho, prob.b, p, prob.lengths)
    assert st["code"] == P.POISSON_OK
    assert res["rel"] <= 1e-10
    assert abs(st["rel_resid"] - res["rel"]) <= 1e-3 * res["rel"]
    assert st["err_bound_rel"] < 1e-8


def _lap_min(shape, lengths):
    """Smallest nonzero eigenvalue magnitude of the periodic 7-point Laplacian."""
    nz, ny, nx = shape
    return min(4.0 * math.sin(math.pi / n) ** 2 / (l / n) ** 2 for n, l in zip((nx, ny, nz), lengths))


@pytest.mark.parametrize("shape", _shapes_every_length())
def test_lap_pinv_fp32_matches_oracle(shape):
    """The FP32 sweeps of the refinement path (the transforms the inner
    iterations run, register-resident at 256 along y and z) on their own, every
    length along every axis, element by element against the oracle's FP64 L^+.

    Bound derived from the arithmetic: with u = 2^-24, each length-N FFT adds
    at most about u log2 N of the norm of what it transforms; the path rounds
    q to FP32, transforms along x, y and z, divides by the FP32 symbol and
    transforms back, so the spectrum carries at most u (2 + 2 sum_d log2 N_d)
    ||q~||, and dividing by the symbol (>= lambda_min) bounds the error of
    delta in the 2-norm, hence element by element, by that over lambda_min
    (taken with a factor 4)."""
    announce("lap_pinv fp32", shape)
    rng = np.random.default_rng(sum(shape) + 1)
    L = (TWO_PI, 2.5, 4.0)
    q = rng.standard_normal(shape) + 0.7
    want = oracle.lap_pinv(q, L)
    h = P.poisson_create(shape, L, precision=P.POISSON_FP32_REFINE)
    try:
        out = dev(np.zeros(shape))
        P.poisson_lap_pinv_fp32(h, dev(q), out)
    finally:
        P.poisson_destroy(h)
    got = host(out)
    u = 2.0 ** -24
    passes = 2 + 2 * sum(math.log2(n) for n in shape)
    bound = 4 * u * passes * np.linalg.norm(q - q.mean()) / _lap_min(shape, L)
    assert np.max(np.abs(got - want)) <= bound, shape
    assert np.linalg.norm(got - want) <= bound, shape
    assert abs(got.mean()) <= bound / math.sqrt(q.size)


def test_lap_pinv_fp32_smooth_256_cube():
    """FP32 L^+ at 256^3 (the headline grid, the register-resident 256-point
    transforms along y and z) on a band-limited right-hand side, against the
    oracle, with the bound above."""
    announce("lap_pinv fp32 256^3")
    shape, L = (256, 256, 256), (TWO_PI,) * 3
    q = inputs.bandlim(shape, L, 8.0, np.random.default_rng(99))
    want = oracle.lap_pinv(q, L)
    h = P.poisson_create(shape, L, precision=P.POISSON_FP32_REFINE)
    try:
        out = dev(np.zeros(shape))
        P.poisson_lap_pinv_fp32(h, dev(q), out)
    finally:
        P.poisson_destroy(h)
    got = host(out)
    u = 2.0 ** -24
    bound = 4 * u * (2 + 2 * 3 * 8) * np.linalg.norm(q) / _lap_min(shape, L)
    assert np.linalg.norm(got - want) <= bound
    assert np.max(np.abs(got - want)) <= bound
    # in practice far inside the bound: a few FP32 ulps of the result
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))


def test_lap_pinv_fp32_needs_fp32_handle():
    announce("lap_pinv fp32 on an FP64 handle")
    shape = (8, 8, 8)
    h = P.poisson_create(shape, (TWO_PI,) * 3)
    try:
        with pytest.raises(P.PoissonError) as e:
            P.poisson_lap_pinv_fp32(h, dev(np.ones(shape)), dev(np.zeros(shape)))
        assert e.value.code == P.POISSON_EINVAL
    finally:
        P.poisson_destroy(h)


@pytest.mark.parametrize("scale", [1e-7, 1e10])
@pytest.mark.parametrize("shape", [(256, 8, 8), (512, 8, 8), (8, 512, 8)])
def test_lap_pinv_extreme_spacings(shape, scale):
    """L^+ on boxes 1e7 times smaller and 1e10 times larger than the unit box,
    with 256- and 512-cell lines along z and y (the register-resident
    transforms): the z sweep takes the inverse symbols of a row pair from one
    reciprocal of a product of two symbols, formed after scaling them by a
    power of two; unscaled, that product (times 2 n) would overflow FP32 at
    the small box (symbols up to 7e18) and leave FP32's normal range at the
    large one (symbols down to 2.5e-20).  Element by element against the oracle,
    with the bounds of the tests above."""
    announce("lap_pinv extreme spacing", shape, scale)
    rng = np.random.default_rng(int(math.log10(scale)) + sum(shape))
    L = (TWO_PI * scale, 2.5 * scale, 4.0 * scale)
    q = rng.standard_normal(shape) + 0.7
    want = oracle.lap_pinv(q, L)
    for precision in (P.POISSON_FP64, P.POISSON_FP32_REFINE):
        h = P.poisson_create(shape, L, precision=precision)
        try:
            out = dev(np.zeros(shape))
            if precision == P.POISSON_FP64:
                P.poisson_lap_pinv(h, dev(q), out)
            else:
                P.poisson_lap_pinv_fp32(h, dev(q), out)
        finally:
            P.poisson_destroy(h)
        got = host(out)
        assert np.all(np.isfinite(got)), (shape, scale, precision)
        if precision == P.POISSON_FP64:
            assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)), (shape, scale)
        else:
            passes = 2 + 2 * sum(math.log2(n) for n in shape)
            bound = 4 * 2.0 ** -24 * passes * np.linalg.norm(q - q.mean()) / _lap_min(shape, L)
            assert np.max(np.abs(got - want)) <= bound, (shape, scale)


@pytest.mark.parametrize("shape", [(12, 8, 256), (8, 256, 12), (256, 8, 12)])
def test_solve_fp32_refine_axis_256(shape):
    """FP32 sweeps + FP64 refinement with a 256-long axis along x, y or z (the
    headline row and column length), element by element against the oracle."""
    announce("solve fp32 refine 256 axis", shape)
    prob = inputs.small_problem(shape=shape, lengths=(TWO_PI, TWO_PI, TWO_PI), ratio=4.0)
    ref = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-14, max_iter=60, allow_noconv=True)
    rr = oracle.residual(prob.rho, prob.b, ref["p"], prob.lengths)
    ref_bound = oracle.error_bound(prob.shape, prob.lengths, float(prob.rho.max()), rr["r_norm"]) / \
        np.linalg.norm(ref["p"])
    p, st, _ = _solve_gpu(prob, precision=P.POISSON_FP32_REFINE)
    err = _check_solution(prob, p, st, ref["p"], ref_bound=ref_bound)
    assert np.max(np.abs(p - ref["p"])) <= (st["err_bound_rel"] + ref_bound) * np.linalg.norm(ref["p"]) + 1e-14
    assert err <= 1e-8


def test_fp32_refine_check_that_does_not_end_the_solve():
    """The final check of a host round (the outer residual's sums alone) can
    find the residual still above the tolerance; the solve must then go on
    with a full refinement step, planned from the residual the check measured.
    This 128^3 problem at 1e-12 ends its third step at 6e-12 (measured), so its
    check fails once."""
    announce("fp32 refine failed check")
    prob = inputs.small_problem(shape=(128, 128, 128), lengths=(TWO_PI,) * 3, ratio=4.0, seed=9)
    p, st, _ = _solve_gpu(prob, precision=P.POISSON_FP32_REFINE, tol=1e-12)
    assert st["code"] == P.POISSON_OK, st
    assert 4 <= st["outer_iters"] <= 6, st
    res = oracle.residual(prob.rho, prob.b, p, prob.lengths)
    assert res["rel"] <= 1e-12, res
    assert abs(st["rel_resid"] - res["rel"]) <= 1e-3 * res["rel"]


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_rough_density_diverges(precision):
    """The oracle's divergent case (face mean of 1/rho, w = rho, cell-to-cell
    rough density on 8^3): both paths stop with EDIVERGED, and the FP64 path
    follows the oracle's residual history up to the divergence."""
    announce("ediverged", precision)
    rng = np.random.default_rng(6)
    shape, L = (8, 8, 8), (TWO_PI,) * 3
    rho = np.exp(rng.uniform(-0.8, 0.8, shape))
    b = rng.standard_normal(shape)
    lit = oracle.solve(rho, b, lengths=L, coef=1, weight=0, tol=1e-12, allow_diverged=True)
    assert lit["code"] == oracle.EDIVERGED
    h = P.poisson_create(shape, L, precision=precision, coef=1, weight=0, max_iter=5000)
    try:
        p = dev(np.zeros(shape))
        rc = P.poisson_solve(h, dev(rho), dev(b), p, 1e-12)
        st = P.poisson_get_stats(h)
        hist = P.poisson_get_history(h)
    finally:
        P.poisson_destroy(h)
    assert rc == P.POISSON_EDIVERGED and st["status"] == P.POISSON_EDIVERGED, st
    if precision == P.POISSON_FP64:
        assert st["iters"] == lit["iters"]
        k = len(hist) - 1  # the last entry is the divergent one: compare the contracting part closely
        assert np.allclose(hist[:k], lit["history"][:k], rtol=1e-6, atol=0)
        assert hist[k] > 1e8 and lit["history"][k] > 1e8
