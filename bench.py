"""Throughput of the variable-density Poisson solve on one MI355X.

Workload: 256^3 periodic cube [0, 2pi)^3, rho = exp(s) with s a seeded Gaussian
field band-limited to |k| <= 8 scaled to max/min rho = 4, b band-limited
|k| <= 8; tolerance 1e-10 on ||b~ - A p|| / ||b~||.  One step = one complete
solve from p = 0 (the zeroing of p included), inputs resident in HBM.  Both
arithmetic paths are timed (FP64, and FP32 sweeps with FP64 refinement); the
headline value is the faster path.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Poisson solves/s at 256^3 to 1e-10 resid (FP64 vs FP32+refine); p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell of each sweep (FP64, FP32): read inputs once,
# write outputs once
SWEEP_BYTES = {1: (32, 16), 2: (16, 8), 3: (16, 8), 5: (24, 12)}
SWEEP_NAMES = {1: "k_resid_dhtx_z", 2: "k_dht_cols", 3: "k_dht_z_solve", 5: "k_dhtx_update"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel, size):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or None when
    there is none for this kernel and size or the kernel sources have changed
    since the counters were taken."""
    from paper_1601_05448_amd import profile_summary

    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(f"{kernel}@{size}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != profile_summary.kernel_source_hash():
        return None
    return rec["bytes_per_launch"]


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    f, c = math.floor(k), math.ceil(k)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def model_bytes_per_cell(fp32, iters, outer_iters, p1_sweeps=None):
    """Modelled HBM bytes per cell of one whole solve from p = 0 (each sweep
    reads its inputs once and writes its outputs once).
    FP64, K iterations: setup 16 + K x 104 + the final residual sweep 32.
    FP32 + refinement, S refinement steps, K inner updates and E inner residual
    sweeps that ran (the first evaluation of each step is fused into the FP64
    outer residual): setup 20 (rho, b read, rho32 written); per step the fused
    outer residual 32, the rest of its first inner sweep 32 (y, z, y 8 each,
    the x pass 8) and the FP64 update 20; 36 per further inner update (y, z, y,
    x update) and 16 per inner residual sweep; the final outer residual, which
    checks the result and writes nothing on rows that take the fused sweep (all
    the workloads here), 24: 44 + 48 S + 36 K + 16 E, which is 44 + 48 S + 52 K
    when every step ends with a confirming residual sweep (E = K)."""
    if fp32:
        e = iters if p1_sweeps is None else p1_sweeps
        return 44 + 48 * outer_iters + 36 * iters + 16 * e
    return 48 + 104 * iters


def time_path(P, torch, prob, precision, steps, warmup, tol, bc_x=0, keep_p=False):
    """Warm up, then time `steps` solves from p = 0.  Inside the timed region
    every launch of the path's residual sweep P1 (the dominant kernel) is
    bracketed by HIP events on the solver's stream (poisson_kernel_timer).
    prob.rho and prob.b are numpy arrays or device tensors."""
    fp32 = precision == P.POISSON_FP32_REFINE
    rho = prob.rho if torch.is_tensor(prob.rho) else torch.from_numpy(prob.rho).cuda()
    b = prob.b if torch.is_tensor(prob.b) else torch.from_numpy(prob.b).cuda()
    p = torch.zeros(prob.shape, dtype=torch.float64, device="cuda")
    s = P.Solver(prob.shape, prob.lengths, precision=precision, bc_x=bc_x)
    stats = None
    for _ in range(warmup):
        p.zero_()
        stats = s.solve(rho, b, p, tol)
    torch.cuda.synchronize()
    P.poisson_kernel_timer(s.h, 1, fp32)
    lat = []
    p1_work = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        p.zero_()
        stats = s.solve(rho, b, p, tol)
        lat.append((time.perf_counter() - a) * 1e3)
        p1_work += stats["p1_sweeps"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = P.poisson_kernel_timer_read(s.h)
    P.poisson_kernel_timer(s.h, 0)
    if stats["status"] != 0:
        raise RuntimeError(f"solve failed: {stats}")
    bytes_p1 = SWEEP_BYTES[1][1 if fp32 else 0] * prob.n
    bpc = model_bytes_per_cell(fp32, stats["iters"], stats["outer_iters"], stats["p1_sweeps"])
    out = dict(solves_per_s=steps / (t1 - t0), ms_per_solve=(t1 - t0) * 1e3 / steps,
               model_bytes_per_cell=bpc,
               # whole-solve roofline fraction: modelled bytes per solve x solves/s over the peak
               solve_frac=bpc * prob.n * steps / (t1 - t0) / (HBM_PEAK_GBS * 1e9),
               p50_ms=percentile(lat, 0.5), p99_ms=percentile(lat, 0.99), iters=stats["iters"],
               outer_iters=stats["outer_iters"], rel_resid=stats["rel_resid"],
               err_bound_rel=stats["err_bound_rel"], device_ms=stats["ms"],
               p1=dict(kernel=("f32:" if fp32 else "f64:") + SWEEP_NAMES[1], launches=k_launches,
                       working_launches=p1_work, total_ms=k_ms, avg_launch_us=1e3 * k_ms / max(k_launches, 1),
                       bytes_per_launch=bytes_p1,
                       # algorithmic bytes of the launches that did work over the time of all launches
                       gbs=bytes_p1 * p1_work / (k_ms * 1e6) if k_ms > 0 else 0.0))
    # each sweep alone, back to back between two HIP events on the solver's stream
    sweeps = {}
    for sw in (1, 2, 3, 5):
        for f32 in ((False, True) if fp32 else (False,)):
            ms = P.poisson_time_sweep(s.h, sw, f32, rho, b, p, 20)
            nbytes = SWEEP_BYTES[sw][1 if f32 else 0] * prob.n
            sweeps[f"{'f32' if f32 else 'f64'}:{SWEEP_NAMES[sw]}"] = dict(
                ms=ms, bytes=nbytes, gbs=nbytes / ms / 1e6)
    if keep_p:
        # the last timed solve's answer (the sweep timings above used p as scratch)
        p.zero_()
        s.solve(rho, b, p, tol)
        out["_p"] = p.cpu().numpy()
    s.close()
    out["sweeps"] = sweeps
    return out


def serve_leg(P, torch, count, budget_gb, slots, precision, fracs=(0.3, 0.5, 0.7, 0.9)):
    """The served stream (Poisson arrivals, grids drawn from 64^3..192^3, each
    with its own lognormal rho): first all requests at once to measure the
    capacity, then in real time at `fracs` x that rate; latency = arrival to
    done, split into the wait before submission (the replay loop), the queue
    (submit to admission) and the rest (admission to done).  Both with direct
    launches and with each size class's chunks replayed from captured graphs;
    the headline figures are the 0.7 x capacity point of the faster mode."""
    from paper_1601_05448_amd import inputs, serve

    reqs = inputs.request_stream(count)
    fields = [inputs.request_fields_device(r) for r in reqs]
    budget = int(budget_gb * (1 << 30))

    def jobs_for(stream):
        return [serve.Job(r.arrival_s, (r.n,) * 3, (2 * math.pi,) * 3, f[0], f[1],
                          torch.zeros((r.n,) * 3, dtype=torch.float64, device="cuda"))
                for r, f in zip(stream, fields)]

    def point(res, rate):
        bad = [o for o in res.outcomes if o.stats["status"] != 0 or o.stats["rel_resid"] > 1e-10]
        if bad or len(res.outcomes) != count:
            raise RuntimeError(f"served solves failed: {len(bad)} bad of {len(res.outcomes)}")
        lat = res.latencies()
        queue = [o.stats["queue_ms"] for o in res.outcomes]
        run = [o.stats["ms"] - o.stats["queue_ms"] for o in res.outcomes]
        before = [lt - o.stats["ms"] for lt, o in zip(lat, res.outcomes)]
        p50, p99 = percentile(lat, 0.5), percentile(lat, 0.99)
        by_size = {}
        for n in inputs.SERVE_SIZES:
            ls = [lt for lt, o in zip(lat, res.outcomes) if o.job.shape[0] == n]
            by_size[str(n)] = {"p50_ms": percentile(ls, 0.5), "p99_ms": percentile(ls, 0.99)}
        return {"rate_hz": rate, "solves_per_s": len(lat) / res.wall_s, "p50_ms": p50, "p99_ms": p99,
                "p99_over_p50": p99 / p50, "mean_submit_wait_ms": sum(before) / len(before),
                "queue_p50_ms": percentile(queue, 0.5), "queue_p99_ms": percentile(queue, 0.99),
                "run_p50_ms": percentile(run, 0.5), "run_p99_ms": percentile(run, 0.99), "by_size": by_size}

    def solo():
        """Latency of each size served alone (one request at a time, nothing
        else resident): the floor under that size's latency in the mix."""
        out = {}
        with serve.Server(budget, slots, precision=precision) as srv:
            for n in inputs.SERVE_SIZES:
                ks = [k for k, r in enumerate(reqs) if r.n == n][:6]
                jobs = [serve.Job(0.0, (n,) * 3, (2 * math.pi,) * 3, fields[k][0], fields[k][1],
                                  torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")) for k in ks]
                lat = []
                for j in jobs:
                    res = serve.replay(srv, [j], realtime=False)
                    lat.append(res.outcomes[0].latency_ms)
                out[str(n)] = percentile(lat[1:], 0.5)  # the first one warms the class up
        return out

    modes = {}
    capacity = None
    for graphs in (False, True):
        with serve.Server(budget, slots, precision=precision, use_graphs=graphs) as srv:
            serve.replay(srv, jobs_for(reqs[: min(16, count)]), realtime=False)  # warm-up
            torch.cuda.synchronize()
            cap = serve.replay(srv, jobs_for(reqs), realtime=False)
            cap_rate = len(cap.outcomes) / cap.wall_s
            if capacity is None:
                capacity = cap_rate  # the direct mode's capacity sets the arrival rates of both
            sweep = {}
            for f in (fracs if not graphs else (0.7,)):
                rate = f * capacity
                stream = inputs.request_stream(count, rate_hz=rate)
                sweep[f"{f:g}"] = point(serve.replay(srv, jobs_for(stream), realtime=True), rate)
        modes["graphs" if graphs else "direct"] = {"capacity_solves_per_s": cap_rate, "load": sweep}
    solo_ms = solo()
    best = "graphs" if modes["graphs"]["load"]["0.7"]["p99_ms"] < modes["direct"]["load"]["0.7"]["p99_ms"] \
        else "direct"
    head = modes[best]["load"]["0.7"]
    return {"requests": count, "sizes": list(inputs.SERVE_SIZES), "budget_gb": budget_gb, "slots": slots,
            "precision": "fp64" if precision == P.POISSON_FP64 else "fp32_refine", "tol": 1e-10,
            "capacity_solves_per_s": modes[best]["capacity_solves_per_s"], "mode": best,
            "rate_hz": head["rate_hz"], "solves_per_s": head["solves_per_s"], "p50_ms": head["p50_ms"],
            "p99_ms": head["p99_ms"], "solo_p50_ms_by_size": solo_ms, "modes": modes}


def serve_mixed(P, torch, big, count, budget_gb):
    """A stream of 128^3 requests (FP32+refine) served alone, then with the
    1024x512x512 hot-blob solve `big` (device fields) admitted at the start of
    the same stream: p50/p99 of the small requests both ways and the big
    solve's latency."""
    from paper_1601_05448_amd import inputs, serve

    reqs = inputs.request_stream(count, sizes=(128,))
    fields = [inputs.request_fields_device(r) for r in reqs]
    big_rho, big_b = big.rho, big.b
    budget = int(budget_gb * (1 << 30))

    def jobs_for(stream):
        return [serve.Job(r.arrival_s, (128,) * 3, (2 * math.pi,) * 3, f[0], f[1],
                          torch.zeros((128,) * 3, dtype=torch.float64, device="cuda"), tag="small")
                for r, f in zip(stream, fields)]

    out = {"small": "128^3 lognormal rho (ratio 2-8), FP32+refine, tol 1e-10",
           "big": big.name + ", FP32+refine, tol 1e-10", "requests": count, "budget_gb": budget_gb}
    with serve.Server(budget, 64, precision=P.POISSON_FP32_REFINE) as srv:
        serve.replay(srv, jobs_for(reqs[:8]), realtime=False)  # warm-up
        cap = serve.replay(srv, jobs_for(reqs), realtime=False)
        rate = 0.5 * len(cap.outcomes) / cap.wall_s
        stream = inputs.request_stream(count, rate_hz=rate, sizes=(128,))
        alone = serve.replay(srv, jobs_for(stream), realtime=True)
        jobs = jobs_for(stream)
        jobs.insert(0, serve.Job(0.0, big.shape, big.lengths, big_rho, big_b,
                                 torch.zeros(big.shape, dtype=torch.float64, device="cuda"), tag="big"))
        mixed = serve.replay(srv, jobs, realtime=True)
    for res in (alone, mixed):
        bad = [o for o in res.outcomes if o.stats["status"] != 0 or o.stats["rel_resid"] > 1e-10]
        if bad:
            raise RuntimeError(f"served solves failed: {len(bad)}")
    small_mixed = [o.latency_ms for o in mixed.outcomes if o.job.tag == "small"]
    big_ms = [o.latency_ms for o in mixed.outcomes if o.job.tag == "big"][0]
    out.update(rate_hz=rate, alone_p50_ms=percentile(alone.latencies(), 0.5),
               alone_p99_ms=percentile(alone.latencies(), 0.99),
               with_big_p50_ms=percentile(small_mixed, 0.5), with_big_p99_ms=percentile(small_mixed, 0.99),
               big_latency_ms=big_ms)
    return out


PROJ_CDT = 5e-4


def time_projection(P, torch, prob, precision, steps, warmup, tol, bc_x=0):
    """The projection step around the solve (RHS from the divergence of the
    predicted momentum, the solve from the previous pressure, momentum
    correction): `steps` projections, each from the same predicted momentum and
    p = 0, timed on the host around poisson_project (which blocks); the copy
    that restores the predicted momentum is outside the timed calls."""
    from paper_1601_05448_amd import inputs

    rho = torch.from_numpy(prob.rho).cuda()
    m_np = inputs.momentum_fields(prob.shape, prob.lengths)
    m0 = [torch.from_numpy(x).cuda() for x in m_np[:3]]
    rd = torch.from_numpy(m_np[3]).cuda()
    m = [x.clone() for x in m0]
    p = torch.zeros(prob.shape, dtype=torch.float64, device="cuda")
    out = torch.empty_like(p)
    with P.Solver(prob.shape, prob.lengths, precision=precision, bc_x=bc_x) as s:
        total, lat, st = 0.0, [], None
        for it in range(warmup + steps):
            for a, b in zip(m, m0):
                a.copy_(b)
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, chi = P.poisson_project(s.h, rho, *m, rd, PROJ_CDT, p, tol)
            dt = time.perf_counter() - t0
            st = P.poisson_get_stats(s.h)
            if it >= warmup:
                total += dt
                lat.append(dt * 1e3)
        # the divergence kernel alone: 32 B/cell read (rho and three momentum
        # components), 8 B/cell written
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        P.poisson_divergence(s.h, rho, *m, out)
        e0.record()
        reps = 10
        for _ in range(reps):
            P.poisson_divergence(s.h, rho, *m, out)
        e1.record()
        torch.cuda.synchronize()
        div_ms = e0.elapsed_time(e1) / reps
    return dict(projections_per_s=steps / total, ms_per_projection=total * 1e3 / steps,
                p50_ms=percentile(lat, 0.5), p99_ms=percentile(lat, 0.99), iters=st["iters"],
                outer_iters=st["outer_iters"], solve_ms=st["ms"], chi=chi,
                divergence_kernel=dict(ms=div_ms, bytes=40 * prob.n, gbs=40 * prob.n / div_ms / 1e6))


def warm_chain_leg(P, torch, n, steps, tol):
    """A chain of `steps` dependent solves with slowly evolving rho and b
    (advected density, rotating right-hand side), each step from p = 0 (cold)
    or from the previous solution (warm), both paths.  Inputs are generated on
    the device before the timed region."""
    from paper_1601_05448_amd import inputs

    shape, L, fields = inputs.advected_chain_device(n, steps)
    out = {}
    for name, prec in (("fp64", P.POISSON_FP64), ("fp32_refine", P.POISSON_FP32_REFINE)):
        res = {}
        with P.Solver(shape, L, precision=prec) as s:
            p = torch.zeros(shape, dtype=torch.float64, device="cuda")
            s.solve(fields[0][0], fields[0][1], p, tol)  # warm-up
            for warm in (False, True):
                p.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                its = []
                for rho, b in fields:
                    if not warm:
                        p.zero_()
                    st = s.solve(rho, b, p, tol)
                    its.append(st["iters"])
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                res["warm" if warm else "cold"] = dict(ms_per_solve=dt * 1e3 / steps, iters=its,
                                                       mean_iters_after_first=sum(its[1:]) / max(1, steps - 1))
        res["speedup"] = res["cold"]["ms_per_solve"] / res["warm"]["ms_per_solve"]
        out[name] = res
    del fields
    return out


def served_chains_leg(P, torch, n, chains, steps, tol):
    """`chains` chains of `steps` solves each served at once through the
    server (one request in flight per chain, the next submitted when the
    previous is done), warm against cold; FP64."""
    from paper_1601_05448_amd import inputs, serve

    fields = [inputs.advected_chain_device(n, steps, chain=c) for c in range(chains)]
    out = {}
    for warm in (False, True):
        cs = [serve.Chain(shape, L, st, torch.zeros(shape, dtype=torch.float64, device="cuda"), tol=tol, warm=warm)
              for shape, L, st in fields]
        with serve.Server(16 << 30, 64) as srv:
            r = serve.run_chains(srv, cs)
        its = [s["iters"] for ch in r.stats for s in ch[1:]]
        out["warm" if warm else "cold"] = dict(solves_per_s=r.solves() / r.wall_s, wall_s=r.wall_s,
                                               mean_iters_after_first=sum(its) / max(1, len(its)))
    out["speedup"] = out["warm"]["solves_per_s"] / out["cold"]["solves_per_s"]
    return out


def deposit_leg(P, torch, n, reps):
    """The particle-to-grid projection P of workload 3 (10^6 uniform particles
    onto n^3, unit values): `reps` calls of poisson_deposit (each blocks),
    positions resident on the device; algorithmic bytes = the grid written once
    (8 B/cell) + the positions read once (24 B/particle)."""
    from paper_1601_05448_amd import inputs

    pos = torch.from_numpy(inputs.workload3_particles()).cuda()
    shape, L = (n, n, n), (2.0 * math.pi,) * 3
    out = torch.empty(shape, dtype=torch.float64, device="cuda")
    with P.Solver(shape, L) as s:
        P.poisson_deposit(s.h, pos, None, out)  # warm-up (grows the particle buffers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            P.poisson_deposit(s.h, pos, None, out)
        dt = (time.perf_counter() - t0) / reps
    nbytes = 8 * n ** 3 + 24 * pos.shape[0]
    return dict(ms=dt * 1e3, particles=int(pos.shape[0]), particles_per_s=pos.shape[0] / dt,
                bytes=nbytes, gbs=nbytes / dt / 1e9)


def copy_ceiling(torch, mib=1024, reps=10):
    """Rate of a plain device-to-device copy of `mib` MiB (read + write bytes per
    second): the practical HBM ceiling next to the published peak."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 8 / ms / 1e6


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class CpuBaseline:
    """The cpu_baseline leg: the oracle (single-threaded C, FP64) timed on the
    host's cores, as it stands.

    * One full oracle solve of the headline workload from p = 0 to the same
      tolerance, in a background process started before the GPU legs so that
      its minutes of host time overlap them; the same process continues that
      solve to a relative residual of 1e-12, and the result is the reference
      against which the GPU answers' error is measured.
    * After the GPU legs: 5 repeated solves of the 32^3 workload on one core
      (median, min), then the same on `procs` concurrent processes (aggregate
      solves/s of the host)."""

    def __init__(self, prob, small, tol):
        import subprocess
        import tempfile

        import numpy as np

        self.prob, self.small, self.tol = prob, small, tol
        self.dir = tempfile.mkdtemp(prefix="bench_oracle_")
        self.big_dir = os.path.join(self.dir, "big")
        self.small_dir = os.path.join(self.dir, "small")
        for d, pr in ((self.big_dir, prob), (self.small_dir, small)):
            os.makedirs(d)
            np.save(os.path.join(d, "rho.npy"), pr.rho)
            np.save(os.path.join(d, "b.npy"), pr.b)
        self.log = open(os.path.join(self.dir, "solve.log"), "w")
        self.proc = subprocess.Popen([sys.executable, "-m", "oracle.jobs", "solve", self.big_dir,
                                      *(repr(v) for v in prob.lengths), repr(tol), "1e-12"],
                                     cwd=ROOT, stdout=self.log, stderr=subprocess.STDOUT)

    def _repeat(self, procs, repeats):
        import subprocess

        cmd = lambda k: [sys.executable, "-m", "oracle.jobs", "repeat", self.small_dir,
                         *(repr(v) for v in self.small.lengths), repr(self.tol), str(repeats), f"{procs}_{k}"]
        t0 = time.perf_counter()
        ps = [subprocess.Popen(cmd(k), cwd=ROOT) for k in range(procs)]
        for q in ps:
            if q.wait() != 0:
                raise RuntimeError("oracle repeat job failed")
        wall = time.perf_counter() - t0
        runs = []
        for k in range(procs):
            with open(os.path.join(self.small_dir, f"repeat_{procs}_{k}.json")) as f:
                runs.append(json.load(f))
        return wall, runs

    def finish(self, answers):
        """answers: {path name: GPU p (numpy)} of the headline workload.
        Returns (cpu_baseline dict, {path name: error dict})."""
        import shutil

        import numpy as np

        t0 = time.perf_counter()
        while self.proc.poll() is None:
            time.sleep(1.0)
            if time.perf_counter() - t0 > 30:
                print("bench: waiting for the oracle solve", file=sys.stderr, flush=True)
                t0 = time.perf_counter()
        self.log.close()
        if self.proc.returncode != 0:
            with open(os.path.join(self.dir, "solve.log")) as f:
                raise RuntimeError("oracle solve failed: " + f.read()[-2000:])
        with open(os.path.join(self.big_dir, "solve.json")) as f:
            big = json.load(f)
        p_ref = np.load(os.path.join(self.big_dir, "p_ref.npy"))
        errors = {}
        for name, p in answers.items():
            d = p - p_ref
            errors[name] = {"rel_l2": float(np.linalg.norm(d) / big["ref_norm"]), "max_abs": float(np.max(np.abs(d))),
                            "max_abs_rel": float(np.max(np.abs(d)) / np.max(np.abs(p_ref))),
                            "reference": f"oracle solve to {big['ref_rel']:.1e} relative residual "
                                         f"(its own error bound {big['ref_err_bound_abs'] / big['ref_norm']:.1e})"}
        del p_ref
        _, one = self._repeat(1, 5)
        times = sorted(one[0]["seconds"])
        procs = min(16, len(os.sched_getaffinity(0)))
        _, runs = self._repeat(procs, 20)
        shutil.rmtree(self.dir, ignore_errors=True)
        n = self.prob.shape[0]
        base = {"value": 1.0 / big["seconds"], "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"one full oracle solve of the {n}^3 workload from p = 0 to {self.tol:g} "
                          f"({big['iters']} iterations, {big['seconds']:.1f} s, single-threaded FP64 C)",
                "cpu_model": cpu_model(), "nproc": os.cpu_count(), "cores_available": len(os.sched_getaffinity(0)),
                "small_32": {"workload": "32^3 sinusoidal rho, divergence b, tol %g" % self.tol,
                             "iters": one[0]["iters"][0], "median_s": times[len(times) // 2], "min_s": times[0],
                             "solves_per_s_one_core": 1.0 / times[len(times) // 2],
                             # the processes run side by side: the sum of their rates
                             "procs": procs, "aggregate_solves_per_s": sum(len(r["seconds"]) / sum(r["seconds"])
                                                                           for r in runs)}}
        return base, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512, help="0 skips the served stream")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--no-512", action="store_true",
                    help="skip the 512^3 particle-deposit workload (fields beyond the 256 MB MALL)")
    ap.add_argument("--no-blobs", action="store_true",
                    help="skip the 1024x512x512 hot-blob workload (alone, and served beside a 128^3 stream)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see the design notes on "
              "sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1601_05448_amd import inputs
    from paper_1601_05448_amd import poisson as P

    torch.cuda.set_device(0)
    prob = inputs.workload2(args.size)
    cpu = None if args.no_cpu_baseline else CpuBaseline(prob, inputs.workload1(32), args.tol)
    fp64 = time_path(P, torch, prob, P.POISSON_FP64, args.steps, args.warmup, args.tol, keep_p=cpu is not None)
    fp32 = time_path(P, torch, prob, P.POISSON_FP32_REFINE, args.steps, args.warmup, args.tol,
                     keep_p=cpu is not None)
    answers = {name: r.pop("_p") for name, r in (("fp64", fp64), ("fp32_refine", fp32)) if "_p" in r}
    best_name, best = ("fp32_refine", fp32) if fp32["solves_per_s"] > fp64["solves_per_s"] else ("fp64", fp64)

    # dominant kernel of the headline path: its residual sweep P1, timed live
    dom = best["p1"]
    roofline = {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dom["gbs"] / HBM_PEAK_GBS,
                "traffic": measured_traffic(dom["kernel"], args.size),
                "bytes_per_launch": dom["bytes_per_launch"], "avg_launch_us": dom["avg_launch_us"],
                "launches": dom["launches"], "working_launches": dom["working_launches"]}
    roofline["copy_ceiling_gbs"] = copy_ceiling(torch)
    roofline["frac_of_copy"] = dom["gbs"] / roofline["copy_ceiling_gbs"]
    # whole solves: modelled bytes per solve x solves/s over the peak
    roofline["solve_frac"] = {"fp64": fp64["solve_frac"], "fp32_refine": fp32["solve_frac"]}

    line = {
        "metric": METRIC,
        "value": best["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sweeps + f64 refinement" if best_name == "fp32_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.size}^3 lognormal rho (max/min 4), band-limited b, tol {args.tol:g}",
                   "path": best_name, "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"]},
        "paths": {"fp64": fp64, "fp32_refine": fp32},
        "roofline": roofline,
    }
    # the projection step around the solve (same density), both paths
    psteps, pwarm = max(5, args.steps // 5), max(1, args.warmup // 2)
    line["projection"] = {"workload": f"{args.size}^3 lognormal rho, band-limited face momentum and divergence "
                                      f"target, C dt {PROJ_CDT:g}, tol {args.tol:g}",
                          "fp64": time_projection(P, torch, prob, P.POISSON_FP64, psteps, pwarm, args.tol),
                          "fp32_refine": time_projection(P, torch, prob, P.POISSON_FP32_REFINE, psteps, pwarm,
                                                         args.tol)}
    # warm-start chains: slowly evolving rho and b, each solve from the previous answer
    line["warm_chain"] = {"workload": f"{args.size}^3 chain of 12 solves, rho advected by half a cell per step, "
                                      f"b rotating slowly, tol {args.tol:g}",
                          **warm_chain_leg(P, torch, args.size, 12, args.tol)}
    line["warm_chain"]["served"] = {"workload": "8 chains x 6 steps at 128^3 through the server, FP64",
                                    **served_chains_leg(P, torch, 128, 8, 6, args.tol)}
    # the particle-to-grid projection that builds the 512^3 workload's density
    line["deposit"] = {"workload": "10^6 uniform particles onto 512^3, trilinear weights per unit volume "
                                   "(the density of the 512^3 particle workload)",
                       **deposit_leg(P, torch, 512, 10)}
    # the inflow-outflow duct: zero-flux walls at the x ends, cosine transform along x
    duct = inputs.workload_duct(args.size)
    dsteps, dwarm = max(5, args.steps // 5), max(1, args.warmup // 2)
    line["duct"] = {"workload": f"{2 * args.size}x{args.size}x{args.size} duct, walls in x, lognormal rho "
                                f"(max/min 4), band-limited b, tol {args.tol:g}",
                    "fp64": time_path(P, torch, duct, P.POISSON_FP64, dsteps, dwarm, args.tol, P.POISSON_BC_WALLS_X),
                    "fp32_refine": time_path(P, torch, duct, P.POISSON_FP32_REFINE, dsteps, dwarm, args.tol,
                                             P.POISSON_BC_WALLS_X),
                    # the projection step on the duct (closed x end faces), FP32 sweeps with refinement
                    "projection_fp32_refine": time_projection(P, torch, duct, P.POISSON_FP32_REFINE, psteps, pwarm,
                                                              args.tol, P.POISSON_BC_WALLS_X)}
    del duct
    if not args.no_512:
        from paper_1601_05448_amd import device_inputs

        big = device_inputs.workload3_device(512)
        lg = {"workload": "512^3 particle-deposit rho (10^6 uniform particles, trilinear deposit by the GPU's P, "
                          "rho = 1/(1 + 9 d/max d), ratio 10), band-limited b, tol %g" % args.tol,
              "fp64": time_path(P, torch, big, P.POISSON_FP64, 5, 1, args.tol),
              "fp32_refine": time_path(P, torch, big, P.POISSON_FP32_REFINE, 5, 1, args.tol)}
        lg["fp32_speedup"] = lg["fp32_refine"]["solves_per_s"] / lg["fp64"]["solves_per_s"]
        line["large"] = lg
        del big
        torch.cuda.empty_cache()
    if not args.no_blobs:
        from paper_1601_05448_amd import device_inputs

        blobs = device_inputs.workload5_device()
        bl = {"workload": "1024x512x512 box [0,4pi)x[0,2pi)^2, 10^5 Gaussian hot blobs (sigma 2 cells), "
                          "rho = 1/(1 + 19 f/max f) (ratio 20), band-limited b, tol %g" % args.tol,
              "fp64": time_path(P, torch, blobs, P.POISSON_FP64, 3, 1, args.tol),
              "fp32_refine": time_path(P, torch, blobs, P.POISSON_FP32_REFINE, 3, 1, args.tol)}
        bl["fp32_speedup"] = bl["fp32_refine"]["solves_per_s"] / bl["fp64"]["solves_per_s"]
        bl["served_alongside"] = serve_mixed(P, torch, blobs, 128, 32.0)
        line["blobs"] = bl
        del blobs
        torch.cuda.empty_cache()
    if args.serve_requests > 0:
        line["serving"] = serve_leg(P, torch, args.serve_requests, args.serve_budget_gb, 64, P.POISSON_FP64)
    if cpu is not None:
        line["cpu_baseline"], errors = cpu.finish(answers)
        for name, e in errors.items():
            line["paths"][name]["err_vs_oracle"] = e
    print(json.dumps(line))


if __name__ == "__main__":
    main()
