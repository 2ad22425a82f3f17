"""Benchmark of the curl-div solver on one MI355X.

A step solves one right-hand side of the 3D workload (p = 3, n = 128
intervals per direction: 6,440,067 unknowns; alpha = 1, beta = 1e-6; Gaussian
right-hand side) to relative residual 1e-8 with the mixed-precision solver
(FP32 V-cycle inside FP64 flexible CG).  Right-hand sides are resident in HBM
before the timed region; solver setup is outside it and reported apart.  The
same right-hand sides are then solved by the plain FP64 path, and the two
solutions are compared.  The other workloads (2D p=2 n=16 latency, 2D p=3
n=256, 3D p=2 n=64, the serving stream) are reported as extra keys.  Prints
one JSON line.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROF_PERIOD = 8  # outer iterations per timed one in the timed region
HEADLINE = "c4_3d_p3_n128"

# HBM-side traffic per launch of the level-0 FP32 Chebyshev step at the
# headline workload: rocprofv3 FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (KiB
# per dispatch, factors from a 256 MiB copy) in runs of
# `bench.py --pmc-pass --copy-cal`, summarised with the commands in
# profiles/c4_3d_p3_n128_solve_kernels.txt.  It holds only for the kernel
# sources it was measured on (their SHA-256 below); after any change to them
# the line reports null until the counters are taken again.
CHEB_TRAFFIC = {"fetch_kib": 71376.4, "write_kib": 30660.0, "fetch_factor": 2.000, "write_factor": 1.000,
                "sources": ["paper_1805_10058_amd/csrc/apply3d.hip", "paper_1805_10058_amd/csrc/apply_common.hpp"],
                "sha256": "9b37aa47d8ff3da93f72ea8b6e08bb3f7b9a4234efd163c915e25cfda757964e"}


def cheb_traffic_bytes():
    """Counted HBM bytes per launch of the roofline kernel, or None when its
    sources differ from those the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in CHEB_TRAFFIC["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != CHEB_TRAFFIC["sha256"]:
        return None
    c = CHEB_TRAFFIC
    return 1024.0 * (c["fetch_kib"] * c["fetch_factor"] + c["write_kib"] * c["write_factor"])


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    k = (len(v) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def finest_apply_equivalents(opt, p, levels, coarse_degree):
    """Operator applies of one outer iteration, in units of a finest-level
    apply: on level 0 the Chebyshev steps after the first (the first rides on
    the input conversion), the residual before the coarse correction, the
    GMRES post-smoother's residual and p Krylov applies, and the outer
    iteration's A d; on each smoothed coarser level l two smoothing
    applications and a residual, weighted by the level's size 8^-l (3D,
    knot insertion halves n per axis)."""
    fine = (opt.cheb_degree - 1) + 1 + 1 + p + 1
    coarse = 0.0
    for l in range(1, levels - 1):
        coarse += (2 * coarse_degree - 1 + 1) * 8.0 ** (-l)
    return fine + coarse


def cpu_baseline(its_gpu, levels, coarse_degree):
    """The oracle's tier-2 Kronecker apply (FP64, one host thread) timed at
    the 3D p=3 n=128 size, times the operator applies one outer iteration of
    the method needs, times the outer iterations the GPU solver took: a
    projection of the oracle's solve time that counts operator applies only
    (T-solves, transfers and vector updates left out, so it favours the
    host)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import curldiv_inputs as ci
    from oracle import assembly as asm
    from oracle import matrices as mt
    from paper_1805_10058_amd import capi

    d, p, n, alpha, betas, dist, tol = ci.CONFIGS[HEADLINE]
    x = ci.rhs(d, p, n, 99, dist)
    reps = 5
    with threadpool_limits(limits=1):
        M, A, S = mt.mass_adv_stiff(n, p)
        asm.kron_apply({"M": M, "A": A, "S": S}, x, d, alpha, betas[0])  # warm
        t0 = time.perf_counter()
        for _ in range(reps):
            asm.kron_apply({"M": M, "A": A, "S": S}, x, d, alpha, betas[0])
        t_apply = (time.perf_counter() - t0) / reps
    opt = capi.options()
    per_iter = finest_apply_equivalents(opt, p, levels, coarse_degree)
    t_solve = t_apply * per_iter * its_gpu
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cores_available": len(os.sched_getaffinity(0)),
            "sample": f"{reps} FP64 oracle Kronecker applies y = A x at 3D p=3 n=128 (6,440,067 unknowns) on one "
                      f"thread, {t_apply:.3f} s each, times {per_iter:.1f} finest-level-equivalent applies per outer "
                      f"iteration times {its_gpu} outer iterations (the GPU solver's count); T-solves, transfers "
                      f"and vector updates not counted",
            "oracle_apply_s": t_apply, "projected_solve_s": t_solve}


def headline(capi, torch, st, steps, warmup):
    """The 3D p=3 n=128 workload: `warmup` + `steps` mixed solves of distinct
    seeded right-hand sides, live kernel timing of the FP32 operator applies
    in the timed solves, then the FP64 path on the timed right-hand sides."""
    import numpy as np

    import curldiv_inputs as ci

    d, p, n, alpha, betas, dist, tol = ci.CONFIGS[HEADLINE]
    beta = betas[0]
    N = ci.num_dofs(d, p, n)
    prob = capi.problem(d, p, n, alpha, beta)
    nsteps = warmup + steps
    rhs = [torch.as_tensor(ci.rhs(d, p, n, 2000 + k, dist)).cuda() for k in range(nsteps)]
    xm = [torch.zeros(N, dtype=torch.float64, device="cuda") for _ in range(nsteps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mixed = capi.Solver(prob, capi.options(precision=capi.CD_MIXED_FP32, rtol=tol), st)
    torch.cuda.synchronize()
    setup_mixed = time.perf_counter() - t0
    levels = mixed.num_levels()
    coarse_degree = mixed.coarse_degree()
    # live timing on from the warm-up on, so that the timed region replays
    # graphs captured (with their timing nodes) before it
    mixed.profile_enable(True, PROF_PERIOD)
    for k in range(warmup):
        r = mixed.solve(rhs[k].data_ptr(), xm[k].data_ptr())
        log(f"warm-up solve {k}: {r.iterations} iterations, status {r.status}")
    mixed.profile_enable(False)
    mixed.profile_enable(True, PROF_PERIOD)
    lat, res = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup, nsteps):
        ts = time.perf_counter()
        r = mixed.solve(rhs[k].data_ptr(), xm[k].data_ptr())
        lat.append(time.perf_counter() - ts)
        res.append(r)
        log(f"timed solve {k}: {r.iterations} iterations, {lat[-1]:.3f} s, status {r.status}")
        if r.status != capi.CD_OK:
            raise RuntimeError(f"mixed solve did not converge: status {r.status}")
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    cheb = mixed.profile_read_smoother(0, True)
    per_level = {}
    for lvl in range(levels):
        a = mixed.profile_read(lvl, True)
        per_level[str(lvl)] = {"launches": a.launches, "avg_us": 1e3 * a.total_ms / max(a.launches, 1),
                               "GB_s": a.bytes / (a.total_ms * 1e-3) / 1e9 if a.total_ms > 0 else 0.0}
    ts = mixed.profile_read_tsolve(True)
    mixed.profile_enable(False)
    launches = mixed.graph_launches()[0]
    mixed_degree0 = mixed.get_smoother(0)[0]
    mixed.close()

    # plain FP64 path on the same right-hand sides
    t0 = time.perf_counter()
    fp64 = capi.Solver(prob, capi.options(precision=capi.CD_FP64, rtol=tol), st)
    torch.cuda.synchronize()
    setup_fp64 = time.perf_counter() - t0
    x64 = torch.zeros(N, dtype=torch.float64, device="cuda")
    lat64, res64, err = [], [], []
    t0 = time.perf_counter()
    for k in range(warmup, nsteps):
        ts0 = time.perf_counter()
        r = fp64.solve(rhs[k].data_ptr(), x64.data_ptr())
        lat64.append(time.perf_counter() - ts0)
        res64.append(r)
        err.append(float(torch.linalg.vector_norm(xm[k] - x64) / torch.linalg.vector_norm(x64)))
        log(f"fp64 solve {k}: {r.iterations} iterations, {lat64[-1]:.3f} s, |x_mixed - x_64|/|x_64| = {err[-1]:.2e}")
    torch.cuda.synchronize()
    T64 = time.perf_counter() - t0
    fp64.close()

    ach = cheb.bytes / (cheb.total_ms * 1e-3) / 1e9 if cheb.total_ms > 0 else 0.0
    flops = 22 * (2 * p + 1) * N  # 33 band contractions of 2p+1 terms per point, 2 flops each
    out = {
        "value": steps / T,
        "ms_per_step": 1e3 * T / steps,
        "config": {"workload": "3D curl-div, p=3, n=128 (6,440,067 unknowns), alpha=1, beta=1e-6, Gaussian RHS, "
                               "rel. residual 1e-8, FP32 V-cycle in FP64 flexible CG",
                   "dim": d, "degree": p, "n": n, "beta": beta, "solves_per_step": 1},
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
        "iterations": [r.iterations for r in res],
        "kernel_launches_per_outer_iteration": launches,
        "smoother": {"degree_finest": mixed_degree0, "degree_coarse": coarse_degree, "note": "default options: "
                     "the coarse-level degree is chosen from beta / alpha (32 below 1e-5, 16 up to 1e-2, 8 above)"},
        "coarse_degree": coarse_degree,
        "max_true_rel_residual": max(r.true_rel_residual for r in res),
        "kappa_estimate": [r.kappa_estimate for r in res],
        "setup_ms": 1e3 * setup_mixed,
        "levels": levels,
        "fp64_path": {"solves_per_s": steps / T64, "p50_ms": 1e3 * percentile(lat64, 50),
                      "p99_ms": 1e3 * percentile(lat64, 99), "iterations": [r.iterations for r in res64],
                      "max_true_rel_residual": max(r.true_rel_residual for r in res64),
                      "kappa_estimate": [r.kappa_estimate for r in res64], "setup_ms": 1e3 * setup_fp64},
        "error_vs_fp64": {"max_rel_diff": max(err), "per_solve": err,
                          "note": "||x_mixed - x_fp64||_2 / ||x_fp64||_2 per right-hand side; both solutions meet "
                                  "rel. residual 1e-8, and the forward error of each is at most kappa_2(A) times "
                                  "its residual"},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": cheb_traffic_bytes(),
                     "traffic_note": "HBM-side bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE runs on the "
                                     "same kernel sources, calibrated by a 256 MiB copy (null: sources changed "
                                     "since)",
                     "kernel": "FP32 Chebyshev-step operator apply k_apply3d<float,3,2> on level 0, inside the timed "
                               f"solves (every {PROF_PERIOD}th outer iteration timed by the kernel's own stamps)",
                     "bytes_per_unit": "4 N s per step (read x_k, x_{k-1}, b; write x_{k+1}), N = 6,440,067, s = 4",
                     "launches": cheb.launches, "avg_us": 1e3 * cheb.total_ms / max(cheb.launches, 1),
                     "bytes_per_launch": cheb.bytes / max(cheb.launches, 1),
                     "TFLOP_s": flops * cheb.launches / (cheb.total_ms * 1e-3) / 1e12 if cheb.total_ms > 0 else 0.0},
        "fp32_applies_per_level": per_level,
        "tsolve": {"kernel": "FP32 T-solve axis passes k_tsolve_line<float,2,*>", "launches": ts.launches,
                   "avg_us": 1e3 * ts.total_ms / max(ts.launches, 1),
                   "GB_s": ts.bytes / (ts.total_ms * 1e-3) / 1e9 if ts.total_ms > 0 else 0.0},
    }
    return out, levels


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--serve", type=int, default=32, help="requests of the serving stream to run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=8.0, help="Poisson arrival rate of the stream, 1/s (0: burst)")
    ap.add_argument("--serve-max-iter", type=int, default=4000)
    ap.add_argument("--serve-stream", type=int, default=0, metavar="N",
                    help="run only the full serving workload on N requests: capacity from a burst, Poisson "
                         "arrivals at 0.5x and 0.9x of it, and the plain FP64 path one at a time")
    ap.add_argument("--batched", type=int, default=8,
                    help="also solve this many right-hand sides of the 2D p=3 n=256 workload at once through the "
                         "continuous-batching server (0: skip)")
    ap.add_argument("--only-c4-apply", action="store_true",
                    help="run only the operator-apply measurement at 3D p=3 n=128 (FP64 and FP32)")
    ap.add_argument("--only-c4-solve", type=int, default=0, metavar="MAX_ITER",
                    help="run only one mixed solve of the headline workload, cut at MAX_ITER outer iterations "
                         "(a short program for profiling)")
    ap.add_argument("--only-c2-solve", action="store_true",
                    help="run only three mixed solves of the 2D p=3 n=256 workload at beta = 1e-4 (a short "
                         "program for profiling)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="only run 6 eager outer iterations of the headline mixed solve (and --copy-cal): a short "
                         "program for the HBM byte counters of the V-cycle kernels")
    ap.add_argument("--copy-cal", action="store_true",
                    help="also run a plain 256 MiB device copy 5 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (--gpus 1 only)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import curldiv_inputs as ci
    from paper_1805_10058_amd import capi

    torch.cuda.set_device(0)
    st = torch.cuda.current_stream().cuda_stream
    if args.copy_cal:
        copy_calibration(torch)
    if args.only_c4_apply:
        print(json.dumps({"operator_apply_c4": c4_apply(capi, torch, st)}), flush=True)
        return
    if args.serve_stream > 0:
        print(json.dumps({"serving_stream": serve_stream(capi, torch, st, args.serve_stream, args.serve_max_iter,
                                                         log)}), flush=True)
        return
    if args.only_c2_solve:
        print(json.dumps({"solve_c2": c2_solve(capi, torch, st)}), flush=True)
        return
    if args.only_c4_solve or args.pmc_pass:
        print(json.dumps({"solve_c4": c4_solve(capi, torch, st, args.only_c4_solve or 6,
                                                graphs=0 if args.pmc_pass else 1)}), flush=True)
        return

    out = {"metric": "solves/sec + p50/p99 latency to rel. residual 1e-8; operator-apply HBM GB/s",
           "value": None, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic"}
    head, levels = headline(capi, torch, st, args.steps, args.warmup)
    out.update(head)

    if not args.no_extras:
        out["operator_apply_c4"] = c4_apply(capi, torch, st)
        log(f"3D p=3 n=128 operator apply: {out['operator_apply_c4']}")
        out["c4_symbol_bounds"] = {
            "note": "one mixed solve of the headline workload with smoother bounds from the spectral symbol "
                    "(1.5 x its maximum) instead of 20 Lanczos steps per level; setup_ms and iterations against "
                    "the headline's",
            **c4_solve(capi, torch, st, 4000, bounds=1)}
        log(f"3D p=3 n=128 with symbol bounds: {out['c4_symbol_bounds']}")
        out["c1_2d_p2_n16"] = c1_latency(capi, torch, st)
        log(f"2D p=2 n=16: {out['c1_2d_p2_n16']}")
        out["c2_2d_p3_n256"] = c2_solves(capi, torch, st, args.steps, args.warmup)
        log(f"2D p=3 n=256: {out['c2_2d_p3_n256']}")
        out["c3_3d_p2_n64"] = c3_solves(capi, torch, st)
        log(f"3D p=2 n=64: {out['c3_3d_p2_n64']}")
        if args.batched > 0:
            out["batched"] = c2_batched(capi, torch, ci.CONFIGS["c2_2d_p3_n256"], args.batched, log)
            log(f"batched: {out['batched']}")
        if args.serve > 0:
            # Poisson arrivals measure latency under load (throughput is then the
            # arrival rate); a burst of the same requests measures capacity.
            out["serving"] = serve_bench(capi, torch, st, args.serve, args.serve_max_iter, log, args.serve_rate)
            log(f"serving: {out['serving']}")
            if args.serve_rate > 0:
                out["serving"]["burst"] = serve_bench(capi, torch, st, args.serve, args.serve_max_iter, log, 0.0)
                log(f"serving burst: {out['serving']['burst']}")

    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(int(percentile(out["iterations"], 50)), levels, out["coarse_degree"])
    print(json.dumps(out), flush=True)


def run_solves(capi, torch, st, name, precision, seeds, **kw):
    """Solve the workload `name` once per seed (per beta of the workload);
    returns (wall seconds, latencies, results)."""
    import curldiv_inputs as ci

    d, p, n, alpha, betas, dist, tol = ci.CONFIGS[name]
    N = ci.num_dofs(d, p, n)
    solvers = {b: capi.Solver(capi.problem(d, p, n, alpha, b), capi.options(precision=precision, rtol=tol, **kw), st)
               for b in betas}
    rhs = [[torch.as_tensor(ci.rhs(d, p, n, s * 10 + j, dist)).cuda() for j in range(len(betas))] for s in seeds]
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    for j, b in enumerate(betas):  # warm-up: graph capture
        solvers[b].solve(rhs[0][j].data_ptr(), x.data_ptr())
    torch.cuda.synchronize()
    lat, res = [], []
    t0 = time.perf_counter()
    for k in range(len(seeds)):
        for j, b in enumerate(betas):
            ts = time.perf_counter()
            r = solvers[b].solve(rhs[k][j].data_ptr(), x.data_ptr())
            lat.append(time.perf_counter() - ts)
            res.append((b, r))
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    launches = {str(b): s.graph_launches()[0] for b, s in solvers.items()}
    for s in solvers.values():
        s.close()
    return T, lat, res, launches


def summarize(capi, T, lat, res, launches=None):
    out = {"solves_per_s": len(lat) / T, "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
           "iterations": {str(b): r.iterations for b, r in res},
           "converged": sum(1 for _, r in res if r.status == capi.CD_OK), "solves": len(res),
           "max_true_rel_residual": max(r.true_rel_residual for _, r in res)}
    if launches:
        out["kernel_launches_per_outer_iteration"] = launches
    return out


def c1_latency(capi, torch, st, reps=100):
    """2D p=2 n=16 (512 unknowns), FP64 to rel. residual 1e-10: latency of
    one solve, with the outer iterations replayed from a HIP graph and
    launched one kernel at a time."""
    out = {}
    for graphs in (1, 0):
        # a 32-unknown coarsest level (3 levels), so the solve runs the V-cycle
        # rather than the dense coarse solve alone
        T, lat, res, launches = run_solves(capi, torch, st, "c1_2d_p2_n16", capi.CD_FP64, list(range(reps)),
                                           graphs=graphs, coarse_max_dofs=64)
        out["graph" if graphs else "eager"] = summarize(capi, T, lat, res, launches if graphs else None)
    out["workload"] = ("2D p=2 n=16 (512 unknowns), alpha=beta=1, FP64, rel. residual 1e-10, one solve at a time, "
                       "3 levels (coarsest 32 unknowns)")
    return out


def c2_solves(capi, torch, st, steps, warmup):
    """2D p=3 n=256 (132,098 unknowns), beta in {1, 1e-4}: mixed and FP64."""
    seeds = list(range(max(steps, 3)))
    out = {"workload": "2D p=3 n=256 (132,098 unknowns), alpha=1, beta in {1, 1e-4}, rel. residual 1e-8"}
    for name, prec in (("mixed", capi.CD_MIXED_FP32), ("fp64", capi.CD_FP64)):
        out[name] = summarize(capi, *run_solves(capi, torch, st, "c2_2d_p3_n256", prec, seeds))
    return out


def c3_solves(capi, torch, st):
    """3D p=2 n=64 (786,432 unknowns), beta in {1, 1e-2}: mixed and FP64."""
    out = {"workload": "3D p=2 n=64 (786,432 unknowns), alpha=1, beta in {1, 1e-2}, rel. residual 1e-8"}
    for name, prec in (("mixed", capi.CD_MIXED_FP32), ("fp64", capi.CD_FP64)):
        out[name] = summarize(capi, *run_solves(capi, torch, st, "c3_3d_p2_n64", prec, [0, 1, 2]))
    return out


def c2_batched(capi, torch, cfg, count, log):
    """`count` right-hand sides of the 2D workload (betas alternating), all
    submitted at t = 0 to the mixed-precision server: the device's capacity
    when independent solves overlap, next to the one-at-a-time headline.
    Solver setup is included."""
    import curldiv_inputs as ci

    d, p, n, alpha, betas, dist, tol = cfg
    rhs = [torch.as_tensor(ci.rhs(d, p, n, 5000 + k, dist)).cuda() for k in range(count)]
    xs = [torch.zeros_like(b) for b in rhs]
    torch.cuda.synchronize()
    srv = capi.Server(max_active=count)
    opt = capi.options(precision=capi.CD_MIXED_FP32, rtol=tol)
    t0 = time.perf_counter()
    for k in range(count):
        srv.submit(capi.problem(d, p, n, alpha, betas[k % len(betas)]), opt, rhs[k].data_ptr(), xs[k].data_ptr())
    done = []
    while True:
        a, q = srv.step()
        done += srv.poll()
        if a == 0 and q == 0:
            break
    T = time.perf_counter() - t0
    srv.close()
    ok = sum(1 for c in done if c.result.status == capi.CD_OK)
    lat = [c.t_done - c.t_submit for c in done]
    return {"solves": count, "betas": betas, "solves_per_s": count / T, "converged": ok,
            "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "note": "all submitted at t=0 to the continuous-batching server; includes solver setup"}


def serve_data(capi, torch, count):
    """The serving stream's requests with their right-hand sides resident in HBM."""
    import curldiv_inputs as ci

    data = []
    for r in ci.serving_stream(count, seed=7, rate=1.0):
        prob = capi.problem(r["dim"], r["p"], r["n"], r["alpha"], r["beta"])
        b = torch.as_tensor(ci.rhs(r["dim"], r["p"], r["n"], r["seed"])).cuda()
        data.append({"prob": prob, "b": b, "x": torch.zeros_like(b), "gap1": r["arrival"], "req": r})
    torch.cuda.synchronize()
    return data


def serve_run(capi, data, arrivals, max_iter, max_active=64):
    """Serve the requests with the continuous-batching mixed-precision server,
    each submitted at its arrival time (seconds from the start).  Latency =
    completion - arrival, solver set-up included."""
    count = len(data)
    srv = capi.Server(max_active=max_active)
    opt = capi.options(precision=capi.CD_MIXED_FP32, rtol=1e-8, max_iter=max_iter)
    ticket, done = {}, {}
    nxt = 0
    peak = 0
    t0 = time.perf_counter()
    while len(done) < count:
        now = time.perf_counter() - t0
        while nxt < count and arrivals[nxt] <= now:
            tk = srv.submit(data[nxt]["prob"], opt, data[nxt]["b"].data_ptr(), data[nxt]["x"].data_ptr())
            ticket[tk] = nxt
            nxt += 1
        a, q = srv.step()
        peak = max(peak, a)
        for c in srv.poll():
            done[ticket[c.ticket]] = (c, time.perf_counter() - t0)
        if a == 0 and q == 0 and nxt < count:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    T = time.perf_counter() - t0
    srv.close()
    lat = [t_done - arrivals[i] for i, (c, t_done) in done.items()]
    its = [c.result.iterations for c, _ in done.values()]
    return {"solves_per_s": count / T, "wall_s": T, "converged": sum(1 for c, _ in done.values()
                                                                     if c.result.status == capi.CD_OK),
            "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "iterations_min_max": [min(its), max(its)], "peak_in_flight": peak,
            "max_true_rel_residual": max(c.result.true_rel_residual for c, _ in done.values())}


def fp64_sequential(capi, data, arrivals, st, max_iter):
    """The same requests, one at a time, by the plain FP64 single-solve path."""
    t1 = time.perf_counter()
    lat, ok = [], 0
    for d, arr in zip(data, arrivals):
        wait = arr - (time.perf_counter() - t1)
        if wait > 0:
            time.sleep(wait)
        s = capi.Solver(d["prob"], capi.options(rtol=1e-8, max_iter=max_iter), st)
        r = s.solve(d["b"].data_ptr(), d["x"].data_ptr())
        s.close()
        lat.append(time.perf_counter() - t1 - arr)
        ok += int(r.status == capi.CD_OK)
    T = time.perf_counter() - t1
    return {"solves_per_s": len(data) / T, "wall_s": T, "converged": ok,
            "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99)}


def serve_bench(capi, torch, st, count, max_iter, log, rate):
    """`count` requests of the serving stream (2D/3D, p in {2,3,4}, n
    log-uniform, beta log-uniform in [1e-6, 1]) arriving as a Poisson process
    of `rate` requests per second (0: all at t = 0), served by the
    continuous-batching server, then the same schedule one request at a time
    by the plain FP64 single-solve path."""
    data = serve_data(capi, torch, count)
    arrivals = [d["gap1"] / rate if rate > 0 else 0.0 for d in data]
    srv = serve_run(capi, data, arrivals, max_iter)
    log(f"server: {srv}")
    seq = fp64_sequential(capi, data, arrivals, st, max_iter)
    mode = (f"Poisson arrivals at {rate:g}/s" if rate > 0 else "burst (all arrive at t=0)") + \
        ", continuous batching, mixed FP32/FP64, one stream per solve, set-up on a worker thread"
    out = {"requests": count, "mode": mode, **srv, "max_iter": max_iter, "fp64_sequential": seq,
           "speedup_vs_fp64_sequential": seq["wall_s"] / srv["wall_s"]}
    return out


def serve_stream(capi, torch, st, count, max_iter, log):
    """The full serving workload: capacity from a burst of `count` requests,
    then the same requests arriving as Poisson processes at 0.5x and 0.9x that
    capacity; the plain FP64 path one request at a time on the burst and on
    the 0.5x schedule."""
    data = serve_data(capi, torch, count)
    out = {"requests": count}
    burst = serve_run(capi, data, [0.0] * count, max_iter)
    out["burst"] = burst
    log(f"stream burst: {burst}")
    cap = burst["solves_per_s"]
    for frac in (0.5, 0.9):
        arr = [d["gap1"] / (frac * cap) for d in data]
        out[f"poisson_{frac:g}x"] = {"rate_per_s": frac * cap, **serve_run(capi, data, arr, max_iter)}
        log(f"stream at {frac}x capacity: {out[f'poisson_{frac:g}x']}")
    out["fp64_sequential_burst"] = fp64_sequential(capi, data, [0.0] * count, st, max_iter)
    log(f"fp64 sequential burst: {out['fp64_sequential_burst']}")
    arr = [d["gap1"] / (0.5 * cap) for d in data]
    out["fp64_sequential_0.5x"] = fp64_sequential(capi, data, arr, st, max_iter)
    log(f"fp64 sequential at 0.5x: {out['fp64_sequential_0.5x']}")
    out["speedup_burst_vs_fp64_sequential"] = out["fp64_sequential_burst"]["wall_s"] / burst["wall_s"]
    return out


def copy_calibration(torch, mib=256, reps=5):
    """A plain device-to-device copy of known size: its FETCH_SIZE and
    WRITE_SIZE counters per dispatch calibrate those of the solver kernels."""
    a = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)  # an elementwise kernel of its own name: reads and writes mib MiB
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: {reps} copies of {mib} MiB", file=sys.stderr, flush=True)


def c4_apply(capi, torch, st, reps=20):
    """Operator apply A x at the 3D p=3 n=128 size (6,440,067 unknowns),
    FP64 and FP32, kernel time from the kernels' own wall-clock stamps."""
    d, p, n = 3, 3, 128
    opt = capi.options(method=capi.CD_METHOD_CG)
    s = capi.Solver(capi.problem(d, p, n, 1.0, 1e-6), opt, st)
    N = capi.num_dofs(s.prob)
    res = {}
    for prec, dt, fn in (("fp64", torch.float64, s.apply), ("fp32", torch.float32, s.apply_f32)):
        x = torch.rand(N, dtype=dt, device="cuda")
        y = torch.empty(N, dtype=dt, device="cuda")
        fn(0, x.data_ptr(), y.data_ptr())
        s.profile_enable(True)
        for _ in range(reps):
            fn(0, x.data_ptr(), y.data_ptr())
        stt = s.profile_read(0, prec == "fp32")
        s.profile_enable(False)
        gbs = stt.bytes / (stt.total_ms * 1e-3) / 1e9
        flops = (22 * (2 * p + 1)) * N * stt.launches  # 33 band contractions per point
        res[prec] = {"avg_us": 1e3 * stt.total_ms / stt.launches, "GB_s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                     "TFLOP_s": flops / (stt.total_ms * 1e-3) / 1e12}
    s.close()
    return res


def c4_solve(capi, torch, st, max_iter, graphs=1, bounds=0):
    """One mixed-precision solve of the 3D p=3 n=128 workload (beta = 1e-6,
    Gaussian right-hand side, rel. residual 1e-8): setup and solve times.
    bounds: the smoother's eigenvalue bounds (0 Lanczos, 1 symbol)."""
    import curldiv_inputs as ci

    d, p, n, alpha, betas, dist, tol = ci.CONFIGS["c4_3d_p3_n128"]
    N = ci.num_dofs(d, p, n)
    b = torch.as_tensor(ci.rhs(d, p, n, 0, dist)).cuda()
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = capi.Solver(capi.problem(d, p, n, alpha, betas[0]),
                    capi.options(precision=capi.CD_MIXED_FP32, rtol=tol, max_iter=max_iter, graphs=graphs,
                                 eig_bounds=bounds), st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = s.solve(b.data_ptr(), x.data_ptr())
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"unknowns": N, "beta": betas[0], "levels": s.num_levels(), "iterations": r.iterations,
           "status": r.status, "true_rel_residual": r.true_rel_residual, "setup_ms": 1e3 * (t1 - t0),
           "solve_s": t2 - t1, "ms_per_iteration": 1e3 * (t2 - t1) / max(r.iterations, 1)}
    s.close()
    return out


def c2_solve(capi, torch, st, solves=3):
    """Mixed-precision solves of the 2D p=3 n=256 workload at its small beta
    (1e-4, uniform right-hand side, rel. residual 1e-8), from the captured
    graph after a first solve: iterations, launches and time per solve."""
    import curldiv_inputs as ci

    d, p, n, alpha, betas, dist, tol = ci.CONFIGS["c2_2d_p3_n256"]
    beta = min(betas)
    N = ci.num_dofs(d, p, n)
    b = torch.as_tensor(ci.rhs(d, p, n, 0, dist)).cuda()
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    s = capi.Solver(capi.problem(d, p, n, alpha, beta), capi.options(precision=capi.CD_MIXED_FP32, rtol=tol), st)
    s.solve(b.data_ptr(), x.data_ptr())
    torch.cuda.synchronize()
    ts = []
    for _ in range(solves):
        t0 = time.perf_counter()
        r = s.solve(b.data_ptr(), x.data_ptr())
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    out = {"unknowns": N, "beta": beta, "levels": s.num_levels(), "iterations": r.iterations, "status": r.status,
           "kernel_launches_per_outer_iteration": s.graph_launches()[0],
           "ms_per_solve": [1e3 * t for t in ts], "ms_per_iteration": 1e3 * min(ts) / max(r.iterations, 1)}
    s.close()
    return out


if __name__ == "__main__":
    main()
