"""Benchmark: time-to-solve of the 3-field FSI-like system on one MI355X.

One step = one full pass of the hot path on the device-resident system:
rebuild the whole preconditioner from the blocks already in HBM (node graphs,
MIS-2 aggregation, prolongators, Galerkin products, SIMPLE diagonal and Schur
complement, smoothers, coarse inverses) and solve with GMRES(50) to
rtol 1e-8.  value = steps per second (solves/s, setup included, as the
paper's times include the preconditioner setup).

Besides the main workload the line carries a "lung" record (the lung-like
saddle system, SIMPLE(AMG(BGS);LU)), a "lung_monolithic" record (AMG(SIMPLE)
with coupled coarse levels on the lung-like system with 8 constraints), the
TSI-like system's own timing, the coupling-strength sweep and a "serving"
record (continuous batching of 512 TSI-like requests against sequential
plain FP64 solves).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
[--workload fsi3d|tsi2d|lung3d] [--no-cpu-baseline] [--no-precision-form]
[--no-lung] [--no-lung-mono] [--no-tsi] [--no-alpha-sweep] [--no-variants]
[--no-serving]
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
    # Laplacian (G) and PSPG Q1-Q1 Oseen flow (F) on a 40^3 hex box; degree-1
    # Chebyshev on S and G, damped multicolour Gauss-Seidel on F with the
    # paper's fluid damping omega 0.69, two forward sweeps before the coarse
    # correction and two backward after (48 iterations, 69.3 ms per step;
    # one sweep each way with omega 0.85: 68 and 72.4 ms; two each way with
    # omega 0.8: 46 and 67.1 ms, 0.9: 57, 1.0: no convergence; three each way
    # 41 iterations and 72.8 ms), the SIMPLE diagonal D~ = diag(A11), coarse
    # direct solves up to 2,000 dofs (the slab's second level, 1,932 dofs)
    # and the degree-1 Chebyshev interval [lambda/4, 1.1 lambda] on S and G
    "fsi3d": dict(make=lambda seed: __import__("nfgen").fsi3d(n=40, layers=8, seed=seed),
                  spec="SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.69,half=1,steps=2])",
                  opts=dict(split=[0, 0, 1], simplec_mode=2, coarse_max=2000, cheb_ratio=4.0, max_rhs=1)),
    # the same system with the paper's own fluid smoother, DD(GS) (one
    # workgroup per aggregate, Gauss-Seidel inside in colour order; levels
    # with fewer than 256 aggregates are one subdomain)
    "fsi3d_dd": dict(make=lambda seed: __import__("nfgen").fsi3d(n=40, layers=8, seed=seed),
                     spec="SIMPLE(BGS(AMG[degree=1]);AMG[smoother=ddgs,omega=0.69,half=1,steps=2])",
                     opts=dict(split=[0, 0, 1], simplec_mode=2, coarse_max=2000, cheb_ratio=4.0, max_rhs=1)),
    # the same system with Petrov-Galerkin transfers on the fluid (the
    # paper's fluid AMG, after Sala and Tuminaro)
    "fsi3d_pg": dict(make=lambda seed: __import__("nfgen").fsi3d(n=40, layers=8, seed=seed),
                     spec="SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.69,half=1,steps=2,pg=1])",
                     opts=dict(split=[0, 0, 1], simplec_mode=2, coarse_max=2000, cheb_ratio=4.0, max_rhs=1)),
    # 2-field thermo-structure-like system on a 32x32 Q1 mesh
    "tsi2d": dict(make=lambda seed: __import__("nfgen").tsi2d(nel=32, seed=seed),
                  spec="BGS(AMG)", opts=dict(sweeps=2, order="bwd", max_rhs=1)),
    # lung-like saddle system: Q1 tissue on a 64^3 box, airway tree of depth
    # 12, 4096 acinus volume constraints; outer SIMPLE (D~ = diag(A11);
    # the absolute row sums take more iterations) with the monolithic
    # AMG(BGS) on tissue + airway: damped Gauss-Seidel (the paper's omega
    # 0.79) on the finest level, two forward sweeps before the coarse
    # correction and two backward after, degree-3 Chebyshev over
    # [lambda/8, 1.1 lambda] on the coarser level (127 iterations, 272 ms
    # per step; one symmetric sweep pair each way: 150 and 308 ms; Gauss-
    # Seidel on both levels as well: 154 and 371 ms, one launch per colour
    # on the coarse tissue level); a dense inverse of the 4096 x 4096 S~;
    # coarse direct solves up to 1,000 dofs (three levels; four levels with
    # 200: more set-up)
    "lung3d": dict(make=lambda seed: __import__("nfgen").lung3d(n=64, depth=12, acinus=8, seed=seed),
                   spec="SIMPLE(AMG[smoother=sgs,omega=0.79,half=1,steps=2,cheb_from=1,degree=3](BGS);LU)",
                   opts=dict(split=[0, 0, 1], simplec_mode=2, coarse_max=1000, cheb_ratio=8.0, max_rhs=1)),
}
SERVE_SPEC = "BGS(AMG)"
# two backward BGS sweeps; Chebyshev interval [lambda/8, 1.1 lambda] (one
# GMRES iteration fewer than [lambda/30, 1.1 lambda] on the 32^2-128^2 grids)
SERVE_OPTS = dict(sweeps=2, order="bwd", cheb_ratio=8.0)


# HBM traffic summaries (FETCH_SIZE / WRITE_SIZE counter runs) of the
# dominant kernel per workload, and the source segments of that kernel and
# the helpers it inlines whose digest the summary records
TRAFFIC_PROFILES = {
    "fsi3d": (os.path.join(ROOT, "profiles", "k_sgs_color_fsi3d_traffic.md"),
              [("template <int G, int NR, class T, int U = (NR == 1 ? 8 : 4)>\n__device__ __forceinline__ void row_dot(",
                "template <int G, int MODE, int NR, class T>"),
               ("template <int NR, class T>\n__device__ __forceinline__ void sgs_row_load(",
                "// A whole sweep over every colour of a small level")]),
    "lung3d": (os.path.join(ROOT, "profiles", "k_sgs_color_bsr_lung3d_traffic.md"),
               [("template <int B, class T>\n__device__ __forceinline__ void bsr_block_rows(",
                 "// SpMV from the block copy"),
                ("template <int B, int G, class T>\n__global__ __launch_bounds__(256) void k_sgs_color_bsr(",
                 "template <class T> static DBuf<T>& bsr_store(")]),
}


def kernel_source_digest(workload="fsi3d"):
    """sha256 (first 16 hex digits) of the source of a workload's dominant
    kernel and the helpers it inlines."""
    import hashlib
    s = open(os.path.join(ROOT, "paper_1605_01522_amd", "csrc", "kernels.hip")).read()

    def seg(a, b):
        i = s.index(a)
        return s[i:s.index(b, i)]
    text = "".join(seg(a, b) for a, b in TRAFFIC_PROFILES[workload][1])
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary,
    if it is for this kernel and the kernel's source has not changed since."""
    if workload not in TRAFFIC_PROFILES:
        return None
    try:
        fields = dict(line.split(": ", 1) for line in open(TRAFFIC_PROFILES[workload][0]).read().splitlines()
                      if line.startswith(("kernel: ", "source_sha256_16: ", "traffic_bytes_per_launch: ")))
        if fields.get("kernel") != kernel or fields.get("source_sha256_16") != kernel_source_digest(workload):
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


_COPY_GBPS = None


def measured_copy_gbps():
    """A device-to-device copy of a 1 GiB buffer (torch, HIP events on the
    current stream), bytes read plus written per second: what a plain
    streaming kernel reaches on this device, beside the nominal peak."""
    global _COPY_GBPS
    if _COPY_GBPS is None:
        import torch
        n = 1 << 27
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        _COPY_GBPS = 2 * 8 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del a, b
        torch.cuda.empty_cache()
    return _COPY_GBPS


def cpu_baseline(sys_, spec, opts, gpu_iters, budget_its=20):
    """The CPU oracle on a bounded sample of the same workload: its full setup
    plus the first `budget_its` GMRES iterations, scaled to the GPU's
    iteration count."""
    import oracle
    # launch-shape options of the library (columns per launch sequence) do
    # not change the arithmetic and the oracle has none
    opts = {k: v for k, v in opts.items() if k in oracle.DEFAULT_OPTS}
    # the (single-threaded) oracle pinned to one of this process's cores
    allowed = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(allowed) if allowed else None
    if core is not None:
        os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        o = oracle.Oracle(sys_.fields, sys_.blocks, spec, **opts)
        t_setup = time.perf_counter() - t0
        its = max(1, min(budget_its, gpu_iters))
        t0 = time.perf_counter()
        _, st = o.gmres(sys_.rhs[0], restart=50, maxit=its, rtol=1e-8)
        t_its = time.perf_counter() - t0
    finally:
        if core is not None:
            os.sched_setaffinity(0, allowed)
    per_it = t_its / max(st["iters"], 1)
    t_solve = t_setup + per_it * gpu_iters
    host = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                host = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=1.0 / t_solve, unit="solves/s", cores=1, kind="oracle",
                sample=f"oracle setup ({t_setup:.2f} s) + first {st['iters']} GMRES iterations "
                       f"({t_its:.2f} s) of the same system, scaled to {gpu_iters} iterations",
                setup_s=t_setup, s_per_iter=per_it, host_cpu=host, host_threads=os.cpu_count(), pinned_core=core)


# the paper's own figures (other problems, other hardware): context only
PAPER_CONTEXT = {
    "note": "different problems, meshes and hardware (Leibniz Supercomputing Centre processors; CPU model, "
            "clock and node layout not stated); Trilinos MueLu/ML with DD(GS) smoothers and KLU; times "
            "include preconditioner setup; context, not a target",
    "lung": "patient-specific lung, 2,197,952 dofs incl. 5 constraints, 64 processors, GMRES rtol 1e-6: "
            "SIMPLE(BGS(AMG)) about 20 iterations, 14.9 s per linear solve; SIMPLE(AMG(BGS)) 16.6 s",
    "tsi": "thermo-structure (second Danilovskaya problem), GMRES rtol 1e-8: BGS(AMG) 85,184 dofs on 2 "
           "processors 33 iterations / 7.7 s; 1,331,000 dofs on 32 processors 56 iterations / 25.7 s",
    "fsi": "pressure-wave FSI: results only in figures, no numbers recoverable",
}


def run_workload(name, steps, warmup, seed, precision_form):
    """Generate the workload, build its solver once (upload included), then
    time `steps` full steps (rebuild + GMRES(50) to rtol 1e-8) after `warmup`
    untimed ones; a separate profiled pass gives per-kernel HIP-event times."""
    import numpy as np
    import torch
    from paper_1605_01522_amd import nfield
    from paper_1605_01522_amd.nfield import NField

    W = WORKLOADS[name]
    t0 = time.perf_counter()
    s = W["make"](seed)
    t_gen = time.perf_counter() - t0
    print(f"# generated {name}: n={s.n} nnz={s.nnz()} in {t_gen:.1f} s", file=sys.stderr, flush=True)
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

    for w in range(warmup):
        st = step()
        print(f"# warmup {w}: iters {st['iters']} setup {1e3 * st['setup_s']:.1f} ms "
              f"solve {1e3 * st['solve_s']:.1f} ms", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        stats.append(step())
        print(f"# step {k}: iters {stats[-1]['iters']} setup {1e3 * stats[-1]['setup_s']:.1f} ms "
              f"solve {1e3 * stats[-1]['solve_s']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # kernel timing: the same steps again with HIP events recorded on the
    # launch stream around every SpMV launch and every Gauss-Seidel sweep
    # (kept out of the timed steps above so that they do not slow them)
    nfield.nfield_prof_enable(1)
    for k in range(max(1, min(steps, 2))):
        step()
    torch.cuda.synchronize()
    prof = nfield.nfield_prof_read()
    nfield.nfield_prof_enable(0)

    xs = x.cpu().numpy()
    A = s.assembled()
    relres = float(np.linalg.norm(s.rhs[0] - A @ xs) / np.linalg.norm(s.rhs[0]))

    # precision form: FP32 hierarchy and smoothers inside FP64 flexible GMRES
    prec = None
    if precision_form:
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
        st32 = [step32() for _ in range(steps)]
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t0
        x32h = x32.cpu().numpy()
        prec = dict(value=round(steps / el32, 4), unit="solves/s",
                    setup_ms=round(1e3 * float(np.median([t["setup_s"] for t in st32])), 3),
                    solve_ms=round(1e3 * float(np.median([t["solve_s"] for t in st32])), 3),
                    gmres_iters=st32[-1]["iters"],
                    relres=float(np.linalg.norm(s.rhs[0] - A @ x32h) / np.linalg.norm(s.rhs[0])),
                    rel_err_vs_fp64=float(np.linalg.norm(x32h - xs) / np.linalg.norm(xs)),
                    footprint_mb=round(solver32.footprint_bytes() / 2**20, 1),
                    fp64_footprint_mb=round(solver.footprint_bytes() / 2**20, 1),
                    precond_mb=round(solver32.precond_bytes() / 2**20, 1),
                    fp64_precond_mb=round(solver.precond_bytes() / 2**20, 1))
        solver32.close()
    ms_per_step = 1e3 * elapsed / steps
    dom = max(prof, key=lambda p: p["ms"]) if prof else None
    roofline = None
    if dom:
        achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
        kname = nfield.kernel_name(dom)
        traffic = measured_traffic(name, kname)
        copy = measured_copy_gbps()
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                        frac=round(achieved / PEAK_HBM_GBS, 4),
                        traffic=None if traffic is None else round(traffic),
                        copy_gbps=round(copy, 1), frac_of_copy=round(achieved / copy, 4),
                        kernel=kname,
                        launches=dom["launches"], avg_us=round(1e3 * dom["ms"] / dom["launches"], 2),
                        bytes_per_launch=round(dom["bytes"] / dom["launches"]))
    footprint_mb = round(solver.footprint_bytes() / 2**20, 1)
    solver.close()
    return dict(system=s, stats=stats, elapsed=elapsed, roofline=roofline, prec=prec, prof=prof,
                relres=relres, t_first_setup=t_first_setup, spec=W["spec"], opts=W["opts"],
                footprint_mb=footprint_mb)


def tsi_config0(steps=50, warmup=5, seed=0):
    """The 2-field TSI-like system as its configuration states it (FP64,
    GMRES(50) rtol 1e-8, two backward BGS sweeps with per-field SA-AMG,
    degree-2 Chebyshev, coarse direct solves up to 200 dofs): BGS(AMG), and
    the monolithic AMG(BGS) whose coarse levels carry the coupling blocks
    R_i A_ij P_j, and the paper's single-level comparator BGS(DD(GS))
    (omega 0.79, the level's aggregates as subdomains); median of `steps`
    steps (rebuild + solve) each."""
    import numpy as np
    import torch
    import nfgen
    from paper_1605_01522_amd.nfield import NField
    s = nfgen.tsi2d(nel=32, seed=seed)
    b = torch.tensor(s.rhs[0], device="cuda")
    A = s.assembled()
    out = {}
    for spec in ("BGS(AMG)", "AMG(BGS)", "BGS(DDGS[omega=0.79,ddmin=1])"):
        # a small, launch-bound system: the preconditioner replayed as a HIP
        # graph captured after each rebuild (5.9 -> 5.5 ms per BGS(AMG) step)
        g = NField(s.fields, s.blocks, spec, sweeps=2, order="bwd", max_rhs=1, graphs=1)
        x = torch.zeros_like(b)
        ts, st = [], None
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.rebuild()
            x.zero_()
            _, st = g.gmres_solve(b, x, rtol=1e-8)
            torch.cuda.synchronize()
            if k >= warmup:
                ts.append(time.perf_counter() - t0)
        xs = x.cpu().numpy()
        rec = dict(gmres_iters=st[0]["iters"], status=st[0]["status"],
                   median_ms_per_step=round(1e3 * float(np.median(ts)), 3),
                   solves_per_s=round(len(ts) / sum(ts), 2),
                   setup_ms=round(1e3 * st[0]["setup_s"], 3), solve_ms=round(1e3 * st[0]["solve_s"], 3),
                   relres=float(np.linalg.norm(s.rhs[0] - A @ xs) / np.linalg.norm(s.rhs[0])),
                   levels=g.nlevels(0) if g.hier_count() else 0,
                   op_complexity=[round(g.complexity(h)[0], 3) for h in range(g.hier_count())])
        if spec == "AMG(BGS)":
            rec["coupled_coarse_nnz"] = [[g.matrix(0, l, "A", 0, 1).nnz, g.matrix(0, l, "A", 1, 0).nnz]
                                         for l in range(g.nlevels(0))]
        out[spec] = rec
        g.close()
    return dict(workload=f"tsi2d: n={s.n} dofs, nnz={s.nnz()}, two backward BGS sweeps, degree-2 Chebyshev "
                         f"over [lambda/30, 1.1 lambda], coarse direct solves up to 200 dofs, FP64 GMRES(50) "
                         f"rtol 1e-8, seed {seed}; a step = rebuild + solve (the preconditioner replayed as a HIP "
                         f"graph); {steps} steps after {warmup} warm-up",
                **out)


# monolithic AMG over all three lung-like fields with SIMPLE as the level
# smoother (the multipliers not coarsened, every coarse level carrying the
# coupling blocks R_i A_ij P_j), on the full-size tissue and a depth-3 airway
# tree: 8 acinus constraints, a few as in the paper's lung, against the 4,096
# of the lung3d workload, where the coarse levels have fewer tissue dofs
# than constraints and AMG(SIMPLE) does not converge
LUNG_MONO = dict(make=lambda seed: __import__("nfgen").lung3d(n=64, depth=3, acinus=8, seed=seed),
                 specs=("AMG[smoother=sgs,omega=0.79,half=1,steps=2,cheb_from=1,degree=3](SIMPLE)",
                        "SIMPLE(AMG[smoother=sgs,omega=0.79,half=1,steps=2,cheb_from=1,degree=3](BGS);LU)"),
                 opts=dict(split=[0, 0, 1], simplec_mode=2, coarse_max=1000, cheb_ratio=8.0, max_rhs=1))


def lung_monolithic(steps=5, warmup=1, seed=0):
    """AMG(SIMPLE) with coupled coarse levels on the lung-like system with 8
    constraints, beside SIMPLE(AMG(BGS);LU) on the same system: iterations,
    median step time (rebuild + solve), the hierarchy's level sizes per field
    and the nonzeros of the coarse coupling blocks tissue-multiplier and
    airway-multiplier on every level."""
    import numpy as np
    import torch
    from paper_1605_01522_amd.nfield import NField
    s = LUNG_MONO["make"](seed)
    b = torch.tensor(s.rhs[0], device="cuda")
    A = s.assembled()
    out = {}
    for spec in LUNG_MONO["specs"]:
        g = NField(s.fields, s.blocks, spec, **LUNG_MONO["opts"])
        x = torch.zeros_like(b)
        ts, st = [], None
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.rebuild()
            x.zero_()
            _, st = g.gmres_solve(b, x, rtol=1e-8, maxit=1000)
            torch.cuda.synchronize()
            if k >= warmup:
                ts.append(time.perf_counter() - t0)
        xs = x.cpu().numpy()
        rec = dict(gmres_iters=st[0]["iters"], status=st[0]["status"],
                   median_ms_per_step=round(1e3 * float(np.median(ts)), 3),
                   solves_per_s=round(len(ts) / sum(ts), 2),
                   setup_ms=round(1e3 * st[0]["setup_s"], 3), solve_ms=round(1e3 * st[0]["solve_s"], 3),
                   relres=float(np.linalg.norm(s.rhs[0] - A @ xs) / np.linalg.norm(s.rhs[0])),
                   level_sizes=[[g.level_size(0, l, f) for f in range(g.nfields(0))] for l in range(g.nlevels(0))])
        if spec.startswith("AMG"):
            nf = g.nfields(0)
            rec["coupled_coarse_nnz"] = [[g.matrix(0, l, "A", i, nf - 1).nnz for i in range(nf - 1)]
                                         for l in range(g.nlevels(0))]
        out[spec] = rec
        g.close()
    return dict(workload=f"lung3d with 8 constraints: n={s.n} dofs ({', '.join(str(f.ndof) for f in s.fields)}), "
                         f"nnz={s.nnz()}, {opts_text(LUNG_MONO['opts'])}, FP64 GMRES(50) rtol 1e-8, seed {seed}; "
                         f"a step = rebuild + solve; {steps} steps after {warmup} warm-up",
                **out)


def alpha_sweep(steps=3, seed=0):
    """Coupling-strength sweep on the TSI-like system (the paper's robustness
    experiment, Sec. 7.1): both coupling blocks scale with alpha; per alpha
    and preconditioner, GMRES(50) iterations to rtol 1e-8 (maxit 1000) and
    the median step time (rebuild + solve)."""
    import numpy as np
    import torch
    import nfgen
    from paper_1605_01522_amd.nfield import NField
    specs = {"BGS(AMG)": dict(sweeps=2, order="bwd"), "BGS[order=sym](AMG)": dict(sweeps=2),
             "AMG(BGS)": dict(sweeps=2, order="bwd"), "SIMPLE(AMG;AMG)": {}}
    rows = []
    for alpha in nfgen.ALPHA_SWEEP:
        s = nfgen.tsi2d_alpha(alpha, nel=32, seed=seed)
        b = torch.tensor(s.rhs[0], device="cuda")
        row = dict(alpha=alpha)
        for spec, o in specs.items():
            g = NField(s.fields, s.blocks, spec, max_rhs=1, **o)
            ts, st = [], None
            for _ in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.rebuild()
                _, st = g.gmres_solve(b, rtol=1e-8, maxit=1000)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            row[spec] = dict(iters=st[0]["iters"], status=st[0]["status"],
                             ms=round(1e3 * float(np.median(ts)), 2))
            g.close()
        rows.append(row)
        print(f"# alpha {alpha}: " + ", ".join(f"{k} {v['iters']}" for k, v in row.items() if k != "alpha"),
              file=sys.stderr, flush=True)
    return dict(workload="tsi2d 32 x 32, C_AB = alpha int B^T m N, C_BA = -0.1 alpha int N div N_u; "
                         "GMRES(50) rtol 1e-8, maxit 1000 (status 1 = not converged), median of "
                         f"{steps} steps (rebuild + solve)", rows=rows)


def opts_text(opts):
    """The setup options of a workload other than the field split, as text."""
    names = {"simplec_mode": {0: "SIMPLE D~ = abs row sums", 1: "SIMPLE D~ = |row sums|", 2: "SIMPLE D~ = diag(A11)"}}
    parts = []
    for k, v in opts.items():
        if k == "split":
            continue
        parts.append(names[k][v] if k in names else f"{k}={v}")
    return ", ".join(parts)


def profile_rows(prof, k):
    """The k kernel variants with the most event time in the profiled pass:
    launches, time, algorithmic bytes and GB/s, with the kernel's name."""
    from paper_1605_01522_amd import nfield
    return [dict(p, kernel=nfield.kernel_name(p), gbps=round(p["bytes"] / (p["ms"] * 1e-3) / 1e9, 1))
            for p in sorted(prof, key=lambda p: -p["ms"])[:k]]


def summary(name, r, steps, seed):
    """Compact record of a secondary workload run."""
    import numpy as np
    s, stats = r["system"], r["stats"]
    extra = opts_text(WORKLOADS[name]["opts"])
    return dict(workload=f"{name}: n={s.n} dofs, nnz={s.nnz()}, spec {r['spec']}"
                         f"{', ' + extra if extra else ''}, GMRES(50) rtol 1e-8, seed {seed}",
                fields=[f.ndof for f in s.fields], value=round(steps / r["elapsed"], 4), unit="solves/s",
                setup_ms=round(1e3 * float(np.median([t["setup_s"] for t in stats])), 3),
                solve_ms=round(1e3 * float(np.median([t["solve_s"] for t in stats])), 3),
                gmres_iters=stats[-1]["iters"], relres=r["relres"], footprint_mb=r["footprint_mb"],
                roofline=r["roofline"], precision_form=r["prec"],
                spmv_profile=profile_rows(r["prof"], 8))


def serving(n_requests=512, seed=0, workers=4, loads=(0.5, 0.8, 1.0, 1.2), no_cache_sample=48):
    """Continuous-batching leg: 512 requests of 2-field TSI-like systems on
    grids {16..128}^2 with 1-8 right-hand sides each, served with
    iteration-level batching (columns join and leave running slot batches
    at Arnoldi step boundaries).  (1) capacity: every request queued at
    once, contexts already cached; (2) the same requests with Poisson
    arrivals at each of `loads` x capacity, replayed in real time, for
    p50/p99 latency; (3) baselines: the same requests served one
    right-hand side at a time with plain FP64 GMRES, contexts cached; and
    without a context cache (every request builds its hierarchy, then
    solves), on the first `no_cache_sample` requests."""
    import numpy as np
    import torch
    import nfgen
    from paper_1605_01522_amd.nfield import NField
    from paper_1605_01522_amd.serve import Server, summarize

    systems = {g: nfgen.tsi2d(nel=g) for g in nfgen.SERVE_GRIDS}

    def rhs_for(req):
        return nfgen.request_rhs(req, systems[req["grid"]].n)

    def trace(rate):
        t = nfgen.request_trace(n_requests, rate=rate, seed=seed)
        for q in t:
            q["key"] = q["grid"]
        return t

    rnd = lambda d: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}
    srv = Server(lambda g: systems[g], SERVE_SPEC, SERVE_OPTS, workers=workers, max_cols=8, hier_fp32=True)
    t0 = time.perf_counter()
    srv.run(trace(1e9), rhs_for, time_scale=0.0)          # builds the cached contexts
    t_warm = time.perf_counter() - t0
    cap = summarize(srv.run(trace(1e9), rhs_for, time_scale=0.0))
    print(f"# serving capacity: {cap['solves_per_s']:.1f} solves/s", file=sys.stderr, flush=True)
    at_load = []
    worst = 0.0
    assembled = {g: systems[g].assembled() for g in systems}
    for load in loads:
        items = srv.run(trace(load * cap["requests_per_s"]), rhs_for, time_scale=1.0)
        live = summarize(items)
        print(f"# serving at {load}x capacity: p50 {live['p50_ms']:.2f} ms p99 {live['p99_ms']:.2f} ms",
              file=sys.stderr, flush=True)
        at_load.append(dict(rnd(live), load=load))
        # accuracy of the served solutions
        for it in items:
            A = assembled[it.req["grid"]]
            B = rhs_for(it.req)
            for k in range(B.shape[0]):
                worst = max(worst, float(np.linalg.norm(B[k] - A @ it.x[k]) / np.linalg.norm(B[k])))
    srv.close()
    # baseline: sequential plain FP64, one column per solve, contexts cached
    ctx = {g: NField(systems[g].fields, systems[g].blocks, SERVE_SPEC, **SERVE_OPTS) for g in systems}
    tr = trace(1e9)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in tr:
        tq = time.perf_counter()
        B = torch.tensor(rhs_for(q), device="cuda")
        for k in range(B.shape[0]):
            ctx[q["grid"]].gmres_solve(B[k].contiguous(), rtol=1e-8)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - tq)
    el = time.perf_counter() - t0
    for c in ctx.values():
        c.close()
    cols = sum(q["nrhs"] for q in tr)
    seq = dict(solves_per_s=round(cols / el, 2), requests_per_s=round(len(tr) / el, 2),
               service_p50_ms=round(1e3 * float(np.percentile(lat, 50)), 3),
               service_p99_ms=round(1e3 * float(np.percentile(lat, 99)), 3))
    # baseline without a context cache: each request sets up its own context
    # (FP32 hierarchy) and solves its columns in one multi-column call
    sample = tr[:no_cache_sample]
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in sample:
        tq = time.perf_counter()
        sysq = systems[q["grid"]]
        c = NField(sysq.fields, sysq.blocks, SERVE_SPEC, hier_fp32=1, max_rhs=8, **SERVE_OPTS)
        B = torch.tensor(rhs_for(q), device="cuda")
        c.gmres_solve(B, flexible=1, rtol=1e-8)
        torch.cuda.synchronize()
        c.close()
        lat.append(time.perf_counter() - tq)
    el = time.perf_counter() - t0
    cols = sum(q["nrhs"] for q in sample)
    nocache = dict(requests=len(sample), solves_per_s=round(cols / el, 2),
                   requests_per_s=round(len(sample) / el, 2),
                   service_p50_ms=round(1e3 * float(np.percentile(lat, 50)), 3),
                   service_p99_ms=round(1e3 * float(np.percentile(lat, 99)), 3))
    return dict(workload=f"{n_requests} requests, tsi2d grids {list(nfgen.SERVE_GRIDS)}^2, 1-8 rhs each, "
                         f"spec {SERVE_SPEC}, {opts_text(SERVE_OPTS)}, FP32 hierarchy in FP64 flexible GMRES(50) "
                         f"rtol 1e-8, "
                         f"{workers} streams, 8-slot batches joined and left at Arnoldi step boundaries",
                capacity=rnd(cap), at_load=at_load, max_relres=worst,
                context_build_s=round(t_warm, 3), sequential_plain_fp64=seq, no_context_cache=nocache,
                speedup_solves_per_s=round(cap["solves_per_s"] / seq["solves_per_s"], 2),
                speedup_vs_no_cache=round(cap["solves_per_s"] / nocache["solves_per_s"], 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fsi3d", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-form", action="store_true")
    ap.add_argument("--no-lung", action="store_true", help="skip the lung-like saddle system leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the continuous-batching leg")
    ap.add_argument("--no-tsi", action="store_true", help="skip the TSI-like system's own timing")
    ap.add_argument("--no-alpha-sweep", action="store_true", help="skip the coupling-strength sweep")
    ap.add_argument("--no-lung-mono", action="store_true",
                    help="skip AMG(SIMPLE) on the lung-like system with 8 constraints")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FSI-like variants (DD(GS) fluid smoother, Petrov-Galerkin fluid AMG)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this solver is built and "
              "measured on a single GPU; no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1605_01522_amd import nfield
    from paper_1605_01522_amd.nfield import NField

    W = WORKLOADS[args.workload]
    r = run_workload(args.workload, args.steps, args.warmup, args.seed, not args.no_precision_form)
    s, stats, elapsed, roofline, prec, prof = r["system"], r["stats"], r["elapsed"], r["roofline"], r["prec"], r["prof"]
    relres, ms_per_step = r["relres"], 1e3 * r["elapsed"] / args.steps
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
        "config": {"workload": f"{args.workload}: n={s.n} dofs, nnz={s.nnz()}, spec {W['spec']}"
                               f"{', ' + opts_text(W['opts']) if opts_text(W['opts']) else ''}, "
                               f"GMRES(50) rtol 1e-8, seed {args.seed}",
                   "fields": [f.ndof for f in s.fields]},
        "setup_ms": round(1e3 * float(np.median([t["setup_s"] for t in stats])), 3),
        "solve_ms": round(1e3 * float(np.median([t["solve_s"] for t in stats])), 3),
        "first_setup_with_upload_ms": round(1e3 * r["t_first_setup"], 3),
        "gmres_iters": iters,
        "relres": relres,
        "roofline": roofline,
        "precision_form": prec,
        "spmv_profile": profile_rows(prof, 16),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, W["spec"], W["opts"], iters)
    out["paper_context"] = PAPER_CONTEXT
    del r, s
    if not args.no_lung and args.workload != "lung3d":
        out["lung"] = summary("lung3d", run_workload("lung3d", 5, 1, args.seed, not args.no_precision_form),
                              5, args.seed)
    if not args.no_variants and args.workload == "fsi3d":
        # the paper's own fluid components on the same system, 5 steps each
        out["variants"] = {v: summary(v, run_workload(v, 5, 1, args.seed, False), 5, args.seed)
                           for v in ("fsi3d_dd", "fsi3d_pg")}
    if not args.no_lung_mono:
        out["lung_monolithic"] = lung_monolithic(seed=args.seed)
    if not args.no_tsi:
        out["tsi2d"] = tsi_config0(seed=args.seed)
    if not args.no_alpha_sweep:
        out["alpha_sweep"] = alpha_sweep(seed=args.seed)
    if not args.no_serving:
        out["serving"] = serving(seed=args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
