"""Warm-start chains: time series of dependent solves whose density and
right-hand side evolve slowly, each solve starting from the previous solution
(the paper's estimate p_g of eq. (Pois) is the pressure of the previous step;
section "Poisson equation").  Against the FP64 CPU oracle, through the C ABI.

Checks: every warm-started solve meets the tolerance by the oracle's residual
and matches the oracle's cold solution within the a-posteriori bound; a warm
FP64 solve takes the oracle's iteration count from the same starting field
(the GPU's previous answer) with the same residual history (1e-6 relative or
1e-14 absolute, the rounding floor in units of ||b~||); warm chains need fewer
iterations than cold ones; chains served through the server (one request in
flight per chain) give bitwise the answers of the same chains solved one by
one.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import announce, host, rel_l2
from paper_1601_05448_amd import inputs
from paper_1601_05448_amd import poisson as P
from paper_1601_05448_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()
    yield


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_warm_chain_matches_oracle(precision):
    announce("warm chain 32^3", precision)
    import torch

    shape, L, steps = inputs.advected_chain_device(32, steps=5, shift_cells=(2.0, 1.0, 0.0), omega=0.1)
    p = torch.zeros(shape, dtype=torch.float64, device="cuda")
    iters = []
    with P.Solver(shape, L, precision=precision) as s:
        for t, (rho, b) in enumerate(steps):
            p0 = host(p).copy()
            st = s.solve(rho, b, p, 1e-10)
            hist = s.history()
            assert st["code"] == P.POISSON_OK, (t, st)
            rh, bh, ph = host(rho), host(b), host(p)
            res = oracle.residual(rh, bh, ph, L)
            assert res["rel"] <= 1e-10
            ref = oracle.solve(rh, bh, lengths=L, tol=1e-13)
            assert rel_l2(ph, ref["p"]) <= st["err_bound_rel"] * (1 + 1e-6) + 1e-14
            if precision == P.POISSON_FP64:
                lit = oracle.solve(rh, bh, p0=p0, lengths=L, tol=1e-10)
                assert st["iters"] == lit["iters"], t
                assert np.allclose(hist, lit["history"], rtol=1e-6, atol=1e-14), t
            iters.append(st["iters"])
    # from the second step on the previous answer is a better start than zero:
    # fewer FP64 iterations; the FP32 path counts inner sweeps, which fall only
    # when the head start saves part of a refinement step, so there no more
    if precision == P.POISSON_FP64:
        assert max(iters[1:]) < iters[0], iters
    else:
        assert max(iters[1:]) <= iters[0], iters


def _chain_fields(n, chains, steps):
    out = []
    for c in range(chains):
        shape, L, st = inputs.advected_chain_device(n, steps=steps, chain=c)
        out.append((shape, L, st))
    return out


def test_served_chains_bitwise_equal_to_sequential():
    announce("served chains 64^3")
    import torch

    fields = _chain_fields(64, 3, 4)
    # one by one
    alone = []
    for shape, L, st in fields:
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        res = []
        with P.Solver(shape, L) as s:
            for rho, b in st:
                r = s.solve(rho, b, p, 1e-10)
                res.append((host(p).copy(), r["iters"]))
        alone.append(res)
    # served: all chains in flight together
    chains = [serve.Chain(shape, L, st, torch.zeros(shape, dtype=torch.float64, device="cuda"))
              for shape, L, st in fields]
    with serve.Server(1 << 32, 8) as srv:
        out = serve.run_chains(srv, chains)
    for c, ch in enumerate(chains):
        assert [s["iters"] for s in out.stats[c]] == [a[1] for a in alone[c]]
        assert all(s["status"] == P.POISSON_OK for s in out.stats[c])
        assert np.array_equal(host(ch.p), alone[c][-1][0])


def test_warm_chains_take_fewer_iterations_than_cold():
    announce("warm vs cold chains 64^3")
    import torch

    fields = _chain_fields(64, 2, 5)
    tot = {}
    for warm in (False, True):
        chains = [serve.Chain(shape, L, st, torch.zeros(shape, dtype=torch.float64, device="cuda"), warm=warm)
                  for shape, L, st in fields]
        with serve.Server(1 << 32, 8) as srv:
            out = serve.run_chains(srv, chains)
        tot[warm] = sum(s["iters"] for ch in out.stats for s in ch[1:])
    assert tot[True] < tot[False], tot


def test_fp32_warm_chain_saves_inner_sweeps():
    """FP32 sweeps with refinement on the slowly evolving chain (half a cell
    of advection per step, the benchmark's chain) at 64^3: the warm start
    begins within a few percent of the answer, so the refinement steps'
    adaptive inner stop needs fewer inner sweeps than from zero, on every step
    after the first."""
    announce("fp32 warm vs cold 64^3")
    import torch

    shape, L, steps = inputs.advected_chain_device(64, steps=6)
    its = {}
    for warm in (False, True):
        p = torch.zeros(shape, dtype=torch.float64, device="cuda")
        its[warm] = []
        with P.Solver(shape, L, precision=P.POISSON_FP32_REFINE) as s:
            for rho, b in steps:
                if not warm:
                    p.zero_()
                st = s.solve(rho, b, p, 1e-10)
                assert st["code"] == P.POISSON_OK
                its[warm].append(st["iters"])
    assert its[True][0] == its[False][0], its
    assert all(w < c for w, c in zip(its[True][1:], its[False][1:])), its
