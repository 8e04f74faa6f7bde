"""Benchmark: time-to-solve of the 3-field FSI-like system on one MI355X.

One step = one full pass of the hot path on the device-resident system:
rebuild the whole preconditioner from the blocks already in HBM (node graphs,
MIS-2 aggregation, prolongators, Galerkin products, SIMPLE diagonal and Schur
complement, smoothers, coarse inverses) and solve with GMRES(50) to
rtol 1e-8.  value = steps per second (solves/s, setup included, as the
paper's times include the preconditioner setup).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
[--workload fsi3d|tsi2d] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    # 3-field FSI-like system: Q1 elastic slab 40x40x8 (S), ALE vector
    # Laplacian (G) and PSPG Q1-Q1 Oseen flow (F) on a 40^3 hex box
    "fsi3d": dict(make=lambda seed: __import__("nfgen").fsi3d(n=40, layers=8, seed=seed),
                  spec="SIMPLE(BGS(AMG);AMG[smoother=sgs,omega=0.69])", opts=dict(split=[0, 0, 1])),
    # 2-field thermo-structure-like system on a 32x32 Q1 mesh
    "tsi2d": dict(make=lambda seed: __import__("nfgen").tsi2d(nel=32, seed=seed),
                  spec="BGS(AMG)", opts=dict(sweeps=2, order="bwd")),
}


def cpu_baseline(sys_, spec, opts, gpu_iters, budget_its=20):
    """The CPU oracle on a bounded sample of the same workload: its full setup
    plus the first `budget_its` GMRES iterations, scaled to the GPU's
    iteration count."""
    import oracle
    t0 = time.perf_counter()
    o = oracle.Oracle(sys_.fields, sys_.blocks, spec, **opts)
    t_setup = time.perf_counter() - t0
    its = max(1, min(budget_its, gpu_iters))
    t0 = time.perf_counter()
    _, st = o.gmres(sys_.rhs[0], restart=50, maxit=its, rtol=1e-8)
    t_its = time.perf_counter() - t0
    per_it = t_its / max(st["iters"], 1)
    t_solve = t_setup + per_it * gpu_iters
    return dict(value=1.0 / t_solve, unit="solves/s", cores=1, kind="oracle",
                sample=f"oracle setup ({t_setup:.2f} s) + first {st['iters']} GMRES iterations "
                       f"({t_its:.2f} s) of the same system, scaled to {gpu_iters} iterations",
                setup_s=t_setup, s_per_iter=per_it)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fsi3d", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-form", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "layout is described in DESIGN.md and not measured.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1605_01522_amd import nfield
    from paper_1605_01522_amd.nfield import NField

    W = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    s = W["make"](args.seed)
    t_gen = time.perf_counter() - t0
    print(f"# generated {args.workload}: n={s.n} nnz={s.nnz()} in {t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver = NField(s.fields, s.blocks, W["spec"], **W["opts"])
    torch.cuda.synchronize()
    t_first_setup = time.perf_counter() - t0     # includes the host -> device upload
    b = torch.tensor(s.rhs[0], device=dev)
    x = torch.zeros_like(b)

    def step():
        solver.rebuild()
        x.zero_()
        _, st = solver.gmres_solve(b, x, restart=50, rtol=1e-8)
        return st[0]

    for w in range(args.warmup):
        st = step()
        print(f"# warmup {w}: iters {st['iters']} setup {1e3 * st['setup_s']:.1f} ms "
              f"solve {1e3 * st['solve_s']:.1f} ms", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(step())
        print(f"# step {k}: iters {stats[-1]['iters']} setup {1e3 * stats[-1]['setup_s']:.1f} ms "
              f"solve {1e3 * stats[-1]['solve_s']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # kernel timing: the same steps again with HIP events recorded on the
    # launch stream around every SpMV launch and every Gauss-Seidel sweep
    # (kept out of the timed steps above so that they do not slow them)
    nfield.nfield_prof_enable(1)
    for k in range(max(1, min(args.steps, 2))):
        step()
    torch.cuda.synchronize()
    prof = nfield.nfield_prof_read()
    nfield.nfield_prof_enable(0)

    xs = x.cpu().numpy()
    A = s.assembled()
    relres = float(np.linalg.norm(s.rhs[0] - A @ xs) / np.linalg.norm(s.rhs[0]))

    # precision form: FP32 hierarchy and smoothers inside FP64 flexible GMRES
    prec = None
    if not args.no_precision_form:
        solver32 = NField(s.fields, s.blocks, W["spec"], hier_fp32=1, **W["opts"])
        x32 = torch.zeros_like(b)

        def step32():
            solver32.rebuild()
            x32.zero_()
            _, st = solver32.gmres_solve(b, x32, restart=50, flexible=1, rtol=1e-8)
            return st[0]

        step32()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st32 = [step32() for _ in range(args.steps)]
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t0
        x32h = x32.cpu().numpy()
        prec = dict(value=round(args.steps / el32, 4), unit="solves/s",
                    setup_ms=round(1e3 * float(np.median([t["setup_s"] for t in st32])), 3),
                    solve_ms=round(1e3 * float(np.median([t["solve_s"] for t in st32])), 3),
                    gmres_iters=st32[-1]["iters"],
                    relres=float(np.linalg.norm(s.rhs[0] - A @ x32h) / np.linalg.norm(s.rhs[0])),
                    rel_err_vs_fp64=float(np.linalg.norm(x32h - xs) / np.linalg.norm(xs)),
                    footprint_mb=round(solver32.footprint_bytes() / 2**20, 1),
                    fp64_footprint_mb=round(solver.footprint_bytes() / 2**20, 1))
        solver32.close()
    ms_per_step = 1e3 * elapsed / args.steps
    dom = max(prof, key=lambda p: p["ms"]) if prof else None
    roofline = None
    if dom:
        achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                        frac=round(achieved / PEAK_HBM_GBS, 4), traffic=None,
                        kernel=nfield.kernel_name(dom),
                        launches=dom["launches"], avg_us=round(1e3 * dom["ms"] / dom["launches"], 2),
                        bytes_per_launch=round(dom["bytes"] / dom["launches"]))
    iters = stats[-1]["iters"]
    out = {
        "metric": "time-to-solve + HBM GB/s of GMRES/BGS-AMG; solves/s, p50/p99 latency",
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={s.n} dofs, nnz={s.nnz()}, spec {W['spec']}, "
                               f"GMRES(50) rtol 1e-8, seed {args.seed}",
                   "fields": [f.ndof for f in s.fields]},
        "setup_ms": round(1e3 * float(np.median([t["setup_s"] for t in stats])), 3),
        "solve_ms": round(1e3 * float(np.median([t["solve_s"] for t in stats])), 3),
        "first_setup_with_upload_ms": round(1e3 * t_first_setup, 3),
        "gmres_iters": iters,
        "relres": relres,
        "roofline": roofline,
        "precision_form": prec,
        "spmv_profile": [dict(p, gbps=round(p["bytes"] / (p["ms"] * 1e-3) / 1e9, 1)) for p in
                         sorted(prof, key=lambda p: -p["ms"])[:6]],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, W["spec"], W["opts"], iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
