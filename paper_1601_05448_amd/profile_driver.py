"""Launches for profiling under rocprofv3: every sweep of the iteration alone
(FP64 and FP32), one full solve per path, and a device copy of known size that
calibrates the HBM byte counters.

    python -m paper_1601_05448_amd.profile_driver --size 256 --reps 5
    python -m paper_1601_05448_amd.profile_driver --size 256 --duct   # 2N x N x N, walls in x
    python -m paper_1601_05448_amd.profile_driver --size 512 --deposit  # the 512^3 particle workload
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--paths", default="fp64,fp32")
    ap.add_argument("--inner-tols", default="", help="comma list: extra FP32+refine solves at these inner tolerances")
    ap.add_argument("--duct", action="store_true", help="the duct workload with walls in x instead of the cube")
    ap.add_argument("--periodic", action="store_true", help="with --duct: periodic in x instead of walls")
    ap.add_argument("--deposit", action="store_true",
                    help="the particle-deposit workload (density built with the GPU's P) instead of the lognormal cube")
    args = ap.parse_args()

    import torch

    from paper_1601_05448_amd import inputs
    from paper_1601_05448_amd import poisson as P

    torch.cuda.set_device(0)
    if args.deposit:
        from paper_1601_05448_amd import device_inputs

        prob = device_inputs.workload3_device(args.size)
    else:
        prob = inputs.workload_duct(args.size) if args.duct else inputs.workload2(args.size)
    bc_x = P.POISSON_BC_WALLS_X if args.duct and not args.periodic else P.POISSON_BC_PERIODIC
    rho = prob.rho if torch.is_tensor(prob.rho) else torch.from_numpy(prob.rho).cuda()
    b = prob.b if torch.is_tensor(prob.b) else torch.from_numpy(prob.b).cuda()
    p = torch.zeros(prob.shape, dtype=torch.float64, device="cuda")
    for name in args.paths.split(","):
        prec = P.POISSON_FP64 if name == "fp64" else P.POISSON_FP32_REFINE
        with P.Solver(prob.shape, prob.lengths, precision=prec, bc_x=bc_x) as s:
            fp32 = prec == P.POISSON_FP32_REFINE
            for sw in (1, 2, 3, 5, 6) if fp32 else (1, 2, 3, 5):
                ms = P.poisson_time_sweep(s.h, sw, fp32 and sw != 6, rho, b, p, args.reps)
                print(f"{name} sweep {sw}: {ms * 1e3:.1f} us", flush=True)
            p.zero_()
            st = s.solve(rho, b, p, 1e-10)
            print(f"{name} solve: {st['ms']:.3f} ms iters {st['iters']} outer {st['outer_iters']}", flush=True)
    for it in (float(v) for v in args.inner_tols.split(",") if v):
        with P.Solver(prob.shape, prob.lengths, precision=P.POISSON_FP32_REFINE, inner_tol=it, bc_x=bc_x) as s:
            for _ in range(3):
                p.zero_()
                st = s.solve(rho, b, p, 1e-10)
            print(f"fp32 inner_tol {it:g} solve: {st['ms']:.3f} ms iters {st['iters']} outer {st['outer_iters']} "
                  f"rel {st['rel_resid']:.2e}", flush=True)
    n = args.copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy: {args.copy_mib} MiB read + {args.copy_mib} MiB written per launch", flush=True)


if __name__ == "__main__":
    main()
