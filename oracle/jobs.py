"""Oracle runs in a process of their own (test infrastructure).

The benchmark's CPU-baseline leg starts these so that the oracle's host time
overlaps the GPU measurements.  Inputs are read from .npy files that the
caller wrote (this module imports numpy and the oracle only); results go to
.npy and .json files, the .json last, so that its presence means the run is
complete.

    python -m oracle.jobs solve DIR LX LY LZ TOL_TIMED TOL_REF
        rho.npy, b.npy in DIR -> p_ref.npy, solve.json: the paper's iteration
        (section "Poisson equation", eq. (Pois)) from p = 0 timed to TOL_TIMED,
        then continued from that iterate to TOL_REF (the same iteration, whose
        state is p alone, so this equals one solve to TOL_REF).
    python -m oracle.jobs repeat DIR LX LY LZ TOL REPEATS TAG
        rho.npy, b.npy in DIR -> repeat_TAG.json: REPEATS timed solves from p = 0.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import error_bound, residual, solve


def _write_json(path: str, obj) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(obj, f)
    os.replace(tmp, path)


def run_solve(d: str, lengths, tol_timed: float, tol_ref: float) -> None:
    rho = np.load(os.path.join(d, "rho.npy"))
    b = np.load(os.path.join(d, "b.npy"))
    print(f"oracle solve {rho.shape}: started", flush=True)
    t0 = time.perf_counter()
    first = solve(rho, b, lengths=lengths, tol=tol_timed, max_iter=500)
    t_timed = time.perf_counter() - t0
    print(f"oracle solve: {first['iters']} iterations to {first['rel']:.2e} in {t_timed:.1f} s", flush=True)
    t1 = time.perf_counter()
    ref = solve(rho, b, p0=first["p"], lengths=lengths, tol=tol_ref, max_iter=500)
    t_more = time.perf_counter() - t1
    rr = residual(rho, b, ref["p"], lengths)
    bound = error_bound(rho.shape, lengths, float(rho.max()), rr["r_norm"])
    np.save(os.path.join(d, "p_ref.npy"), ref["p"])
    _write_json(os.path.join(d, "solve.json"),
                dict(shape=list(rho.shape), iters=first["iters"], rel=first["rel"], seconds=t_timed,
                     ref_more_iters=ref["iters"], ref_rel=ref["rel"], ref_seconds=t_more, ref_err_bound_abs=bound,
                     ref_norm=float(np.linalg.norm(ref["p"]))))
    print(f"oracle solve: reference at {ref['rel']:.2e} after {ref['iters']} more iterations", flush=True)


def run_repeat(d: str, lengths, tol: float, repeats: int, tag: str) -> None:
    rho = np.load(os.path.join(d, "rho.npy"))
    b = np.load(os.path.join(d, "b.npy"))
    times, iters = [], []
    for _ in range(repeats):
        t0 = time.perf_counter()
        r = solve(rho, b, lengths=lengths, tol=tol, max_iter=500)
        times.append(time.perf_counter() - t0)
        iters.append(r["iters"])
    _write_json(os.path.join(d, f"repeat_{tag}.json"), dict(seconds=times, iters=iters))


def main(argv) -> None:
    cmd, d = argv[0], argv[1]
    lengths = tuple(float(v) for v in argv[2:5])
    if cmd == "solve":
        run_solve(d, lengths, float(argv[5]), float(argv[6]))
    elif cmd == "repeat":
        run_repeat(d, lengths, float(argv[5]), int(argv[6]), argv[7])
    else:
        raise SystemExit(f"unknown job {cmd}")


if __name__ == "__main__":
    main(sys.argv[1:])
