"""GPU tests of the serving engine (continuous batching of many solves).

Each request's result must be the same alone and in the mix: the batched
kernels give every request its own fields, workspace, state and fixed-order
reductions, so the stated tolerance is 0 (bitwise identical p and identical
iteration counts).  This is the solver-level analogue of the paper's check that
results do not depend on the domain decomposition (section "Effect of domain
partitioning").
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import announce, dev, host
from paper_1601_05448_amd import inputs
from paper_1601_05448_amd import poisson as P
from paper_1601_05448_amd import serve

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()
    yield


def _mix(count=12):
    shapes = [(16, 16, 16), (24, 24, 24), (32, 32, 32), (12, 16, 24)]
    lens = [(TWO_PI,) * 3, (TWO_PI,) * 3, (TWO_PI,) * 3, (TWO_PI, 3.0, 5.0)]
    probs = []
    for k in range(count):
        sh, L = shapes[k % 4], lens[k % 4]
        probs.append(inputs.small_problem(shape=sh, lengths=L, ratio=2.0 + (k % 5), seed=100 + k))
    return probs


def _alone(prob, precision):
    h = P.poisson_create(prob.shape, prob.lengths, precision=precision)
    try:
        p = dev(np.zeros(prob.shape))
        P.poisson_solve(h, dev(prob.rho), dev(prob.b), p, 1e-10)
        st = P.poisson_get_stats(h)
    finally:
        P.poisson_destroy(h)
    return host(p), st


def _served(probs, precision, budget=1 << 33, slots=64, tols=None, use_graphs=False):
    jobs = []
    for k, pr in enumerate(probs):
        jobs.append(serve.Job(0.0, pr.shape, pr.lengths, dev(pr.rho), dev(pr.b), dev(np.zeros(pr.shape)),
                              tol=1e-10 if tols is None else tols[k], tag=k))
    with serve.Server(budget, slots, precision=precision, use_graphs=use_graphs) as s:
        res = serve.replay(s, jobs, realtime=False)
    out = [None] * len(probs)
    for o in res.outcomes:
        out[o.job.tag] = (host(o.job.p), o.stats)
    return out, res


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_same_bits_when_the_batch_shrinks_the_grids(precision):
    """128^3 requests: alone a sweep gets every resident block, in a batch of four
    each request gets a quarter, so the blocks cover different tiles; the
    residual sums are kept per tile, so the answers are the same bits."""
    announce("serve 128^3 batch invariance", precision)
    probs = [inputs.small_problem(shape=(128, 128, 128), lengths=(TWO_PI,) * 3, ratio=2.0 + k, seed=300 + k)
             for k in range(4)]
    mixed, res = _served(probs, precision)
    assert len(res.outcomes) == len(probs)
    for k, pr in enumerate(probs):
        p_alone, st_alone = _alone(pr, precision)
        p_mix, st_mix = mixed[k]
        assert st_mix["status"] == 0 and st_alone["status"] == 0
        assert st_mix["iters"] == st_alone["iters"] and st_mix["outer_iters"] == st_alone["outer_iters"]
        assert np.array_equal(p_mix, p_alone), k


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_each_result_same_alone_and_in_the_mix(precision):
    announce("serve mix invariance", precision)
    probs = _mix()
    mixed, res = _served(probs, precision)
    assert len(res.outcomes) == len(probs)
    for k, pr in enumerate(probs):
        p_alone, st_alone = _alone(pr, precision)
        p_mix, st_mix = mixed[k]
        assert st_mix["status"] == 0 and st_alone["status"] == 0
        assert st_mix["iters"] == st_alone["iters"] and st_mix["outer_iters"] == st_alone["outer_iters"]
        assert np.array_equal(p_mix, p_alone), k
        assert oracle.residual(pr.rho, pr.b, p_mix, pr.lengths)["rel"] <= 1e-10


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_same_bits_when_a_large_class_splits_the_cus(precision):
    """A 64^3 request with 16^3 requests: 64 times larger, so while both are
    active the server runs it on one half of the CUs and the small ones on the
    other (CU-masked streams where available), with other launch grids; every
    answer is still the same bits as alone."""
    announce("serve split CUs", precision)
    probs = [inputs.small_problem(shape=(64, 64, 64), lengths=(TWO_PI,) * 3, ratio=4.0, seed=610)]
    probs += [inputs.small_problem(shape=(16, 16, 16), lengths=(TWO_PI,) * 3, ratio=2.0 + k, seed=611 + k)
              for k in range(6)]
    mixed, res = _served(probs, precision)
    assert len(res.outcomes) == len(probs)
    for k, pr in enumerate(probs):
        p_alone, st_alone = _alone(pr, precision)
        p_mix, st_mix = mixed[k]
        assert st_mix["status"] == 0 and st_alone["status"] == 0
        assert st_mix["iters"] == st_alone["iters"] and st_mix["outer_iters"] == st_alone["outer_iters"]
        assert np.array_equal(p_mix, p_alone), k


def test_budget_admits_one_at_a_time_and_all_finish():
    announce("serve tight budget")
    probs = _mix(6)
    # footprint of the largest request (32^3): three fields plus about 8 B/cell of
    # workspace; the budget holds one such request, not two
    one = 32 ** 3 * 8 * 4 + (1 << 20)
    mixed, res = _served(probs, P.POISSON_FP64, budget=int(1.5 * one))
    for k, pr in enumerate(probs):
        p_alone, _ = _alone(pr, P.POISSON_FP64)
        assert np.array_equal(mixed[k][0], p_alone)


def test_admission_reuses_a_pooled_workspace_when_the_budget_is_tight():
    """Regression test of admission with a pooled workspace: a 32^3 request
    arrives while the server holds an idle pooled 32^3 workspace and a resident
    request of another size, and the budget lies in the window where the new
    request's fields fit only if that pooled workspace were released.  The
    request must wait for the other resident to retire and then reuse its own
    class's workspace; every answer equals the solve alone, bit for bit."""
    announce("serve admission window")
    a = inputs.small_problem(shape=(32, 32, 32), lengths=(TWO_PI,) * 3, ratio=3.0, seed=501)
    o = inputs.small_problem(shape=(24, 32, 32), lengths=(TWO_PI,) * 3, ratio=5.0, seed=502)
    probe = serve.Server(1 << 30, 4)
    f_a = P.poisson_server_footprint(probe.h, a.shape)
    f_o = P.poisson_server_footprint(probe.h, o.shape)
    probe.close()
    fields_a = 24 * a.n
    ws_a = f_a - fields_a
    assert ws_a > 0 and f_o >= ws_a
    # window: fields_a + f_o <= budget < f_a + f_o; and the request alone fits
    budget = fields_a + f_o + ws_a // 2
    assert fields_a + f_o <= budget < f_a + f_o and f_a <= budget
    p_a_alone, _ = _alone(a, P.POISSON_FP64)
    p_o_alone, _ = _alone(o, P.POISSON_FP64)
    with serve.Server(budget, 8) as s:
        # first request of the 32^3 class: afterwards its workspace is pooled
        first = serve.replay(s, [serve.Job(0.0, a.shape, a.lengths, dev(a.rho), dev(a.b), dev(np.zeros(a.shape)),
                                           tag="first")], realtime=False)
        # the other-size request and a second 32^3 request arrive together
        res = serve.replay(s, [serve.Job(0.0, o.shape, o.lengths, dev(o.rho), dev(o.b), dev(np.zeros(o.shape)),
                                         tag="other"),
                               serve.Job(0.0, a.shape, a.lengths, dev(a.rho), dev(a.b), dev(np.zeros(a.shape)),
                                         tag="second")], realtime=False)
    got = {oc.job.tag: (host(oc.job.p), oc.stats) for oc in first.outcomes + res.outcomes}
    assert set(got) == {"first", "other", "second"}
    for tag, want in (("first", p_a_alone), ("other", p_o_alone), ("second", p_a_alone)):
        assert got[tag][1]["status"] == P.POISSON_OK, (tag, got[tag][1])
        assert np.array_equal(got[tag][0], want), tag


def test_request_too_big_for_budget():
    announce("serve etoobig")
    pr = _mix(1)[0]
    with serve.Server(1024, 4) as s:
        with pytest.raises(P.PoissonError) as e:
            s.submit(pr.shape, pr.lengths, dev(pr.rho), dev(pr.b), dev(np.zeros(pr.shape)), 1e-10)
        assert e.value.code == P.POISSON_ETOOBIG


def test_bad_request_does_not_disturb_the_mix():
    announce("serve edomain in mix")
    probs = _mix(8)
    probs[3].rho[1, 2, 3] = -1.0
    mixed, _ = _served(probs, P.POISSON_FP64)
    assert mixed[3][1]["status"] == P.POISSON_EDOMAIN
    for k in (0, 1, 2, 4, 5, 6, 7):
        p_alone, _ = _alone(probs[k], P.POISSON_FP64)
        assert mixed[k][1]["status"] == 0
        assert np.array_equal(mixed[k][0], p_alone)


def test_per_request_tolerance():
    announce("serve per-request tol")
    probs = _mix(4)
    mixed, _ = _served(probs, P.POISSON_FP64, tols=[1e-4, 1e-6, 1e-8, 1e-10])
    for k, tol in enumerate([1e-4, 1e-6, 1e-8, 1e-10]):
        st = mixed[k][1]
        assert st["rel_resid"] <= tol
        assert oracle.residual(probs[k].rho, probs[k].b, mixed[k][0], probs[k].lengths)["rel"] <= tol


def test_poisson_arrival_stream_of_served_sizes():
    """A short real-time stream with the served grid sizes (64^3, 96^3), fields
    generated on the device; every request reaches 1e-10."""
    announce("serve realtime stream")
    import torch

    reqs = [r for r in inputs.request_stream(48, rate_hz=400.0) if r.n in (64, 96)][:16]
    jobs = []
    for r in reqs:
        rho, b = inputs.request_fields_device(r)
        jobs.append(serve.Job(r.arrival_s, (r.n,) * 3, (TWO_PI,) * 3, rho, b,
                              torch.zeros((r.n,) * 3, dtype=torch.float64, device="cuda"), tag=r))
    with serve.Server(1 << 33, 32) as s:
        res = serve.replay(s, jobs, realtime=True)
    assert len(res.outcomes) == len(jobs)
    for o in res.outcomes:
        assert o.stats["status"] == 0 and o.stats["rel_resid"] <= 1e-10 and o.latency_ms > 0
    o = res.outcomes[0]
    chk = oracle.residual(host(o.job.rho), host(o.job.b), host(o.job.p), o.job.lengths)
    assert chk["rel"] <= 1e-10


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_duct_and_box_requests_in_one_mix(precision):
    """Requests with walls in x (the duct) and periodic ones of the same grid
    are separate classes; each is served with its own condition and gives the
    same bits as a solve of that request alone (checked by the oracle with the
    matching condition)."""
    announce("serve duct and box", precision)
    W = P.POISSON_BC_WALLS_X
    probs = [inputs.small_problem(shape=(16, 16, 64), lengths=(TWO_PI,) * 3, ratio=2.0 + k, seed=500 + k)
             for k in range(6)]
    bcs = [W if k % 2 else P.POISSON_BC_PERIODIC for k in range(6)]
    jobs = [serve.Job(0.0, pr.shape, pr.lengths, dev(pr.rho), dev(pr.b), dev(np.zeros(pr.shape)), tag=k,
                      bc_x=bcs[k]) for k, pr in enumerate(probs)]
    with serve.Server(1 << 33, 16, precision=precision) as s:
        res = serve.replay(s, jobs, realtime=False)
    assert len(res.outcomes) == len(probs)
    for o in res.outcomes:
        k = o.job.tag
        pr = probs[k]
        h = P.poisson_create(pr.shape, pr.lengths, precision=precision, bc_x=bcs[k])
        try:
            p = dev(np.zeros(pr.shape))
            P.poisson_solve(h, dev(pr.rho), dev(pr.b), p, 1e-10)
            st = P.poisson_get_stats(h)
        finally:
            P.poisson_destroy(h)
        assert o.stats["status"] == 0 and st["status"] == 0
        assert o.stats["iters"] == st["iters"]
        assert np.array_equal(host(o.job.p), host(p)), k
        assert oracle.residual(pr.rho, pr.b, host(p), pr.lengths, bcx=bcs[k])["rel"] <= 1e-10


def test_server_rejects_unknown_boundary_condition():
    announce("serve bad bc")
    pr = inputs.small_problem(shape=(8, 8, 16), lengths=(TWO_PI,) * 3)
    with serve.Server(1 << 30, 4) as s:
        with pytest.raises(P.PoissonError) as e:
            s.submit(pr.shape, pr.lengths, dev(pr.rho), dev(pr.b), dev(np.zeros(pr.shape)), 1e-10, bc_x=3)
        assert e.value.code == P.POISSON_EINVAL


def test_server_footprint_query():
    """The footprint the budget charges: three FP64 fields plus the workspace
    (8 B/cell and more for FP64, 24 B/cell and more for FP32 refinement)."""
    announce("serve footprint")
    for prec, ws_min in ((P.POISSON_FP64, 8), (P.POISSON_FP32_REFINE, 24)):
        with serve.Server(1 << 30, 4, precision=prec) as s:
            n = 32 ** 3
            f = P.poisson_server_footprint(s.h, (32, 32, 32))
            assert f >= (24 + ws_min) * n and f < (24 + ws_min) * n + (4 << 20)
            with pytest.raises(P.PoissonError) as e:
                P.poisson_server_footprint(s.h, (32, 32, 33))
            assert e.value.code == P.POISSON_EINVAL


@pytest.mark.parametrize("precision", [P.POISSON_FP64, P.POISSON_FP32_REFINE])
def test_graph_replays_give_the_same_bits(precision):
    """Chunks captured once per (batch size, chunk, share) and replayed: every
    request's answer and iteration counts equal its solve alone, bit for bit,
    across a stream whose batch sizes change as requests come and go (several
    replays of the same graphs with the slot table rewritten between them)."""
    announce("serve graphs", precision)
    probs = _mix(16)
    mixed, res = _served(probs, precision, slots=6, use_graphs=True)
    assert len(res.outcomes) == len(probs)
    for k, pr in enumerate(probs):
        p_alone, st_alone = _alone(pr, precision)
        p_mix, st_mix = mixed[k]
        assert st_mix["status"] == 0
        assert (st_mix["iters"], st_mix["outer_iters"]) == (st_alone["iters"], st_alone["outer_iters"])
        assert np.array_equal(p_mix, p_alone), k


def test_served_timing_breakdown():
    """Served requests report their queue time (submit to admission) within
    their latency (submit to done)."""
    announce("serve timing breakdown")
    mixed, _ = _served(_mix(10), P.POISSON_FP64, slots=2)
    for _, st in mixed:
        assert 0.0 <= st["queue_ms"] <= st["ms"]
    assert max(st["queue_ms"] for _, st in mixed) > 0.0  # with two slots some requests waited
