"""Background job of the full-size parity test (test infrastructure).

Computes, on the host and with the oracle only, the reference solution of the
256^3 lognormal workload (rho = exp(s), s band-limited |k| <= 8 scaled to
max/min = 4, b band-limited |k| <= 8): the paper's iteration (section "Poisson
equation", eq. (Pois)) from p = 0 to a relative residual of 1e-12.  The GPU
answer is never an input.  Writes rho.npy, b.npy (the generated inputs, so that
the test solves exactly these bytes on the GPU), p.npy and result.json into the
output directory, printing one line per step.

    python tests/oracle_ref_job.py OUT_DIR [N]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(out_dir: str, n: int = 256) -> None:
    import numpy as np

    import oracle
    from paper_1601_05448_amd import inputs

    t0 = time.perf_counter()
    prob = inputs.workload2(n)
    np.save(os.path.join(out_dir, "rho.npy"), prob.rho)
    np.save(os.path.join(out_dir, "b.npy"), prob.b)
    print(f"oracle job: inputs generated in {time.perf_counter() - t0:.1f} s", flush=True)
    t1 = time.perf_counter()
    res = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-12, max_iter=200)
    t_solve = time.perf_counter() - t1
    rr = oracle.residual(prob.rho, prob.b, res["p"], prob.lengths)
    bound = oracle.error_bound(prob.shape, prob.lengths, float(prob.rho.max()), rr["r_norm"])
    np.save(os.path.join(out_dir, "p.npy"), res["p"])
    info = dict(n=n, iters=res["iters"], rel=res["rel"], history=list(res["history"]), seconds=t_solve,
                err_bound_abs=bound, p_norm=float(np.linalg.norm(res["p"])))
    with open(os.path.join(out_dir, "result.tmp"), "w") as f:
        json.dump(info, f)
    os.replace(os.path.join(out_dir, "result.tmp"), os.path.join(out_dir, "result.json"))
    print(f"oracle job: {res['iters']} iterations to {res['rel']:.2e} in {t_solve:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 256)
