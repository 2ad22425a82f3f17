"""Benchmark of the curl-div solver on one MI355X.

A step solves one batch of the 2D workload (p = 3, n = 256 intervals per
direction, alpha = 1, beta in {1, 1e-4}, uniform [-1, 1] right-hand sides)
to relative residual 1e-8 with the mixed-precision solver (FP32 V-cycle
inside FP64 flexible CG).  Right-hand sides are resident in HBM before the
timed region; solver setup is outside it.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROF_PERIOD = 8  # outer iterations per timed one in the timed region


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    k = (len(v) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


# HBM bytes per launch of the FP32 V-cycle applies of the 2D p=3 n=256 mixed
# solve (all levels, the timed solves' launch mix), from FETCH_SIZE and
# WRITE_SIZE counter runs scaled by a plain copy kernel's readings (factors
# 2.000 and 1.000): 581.9 KiB x 2 + 537.0 KiB.  The counters were read with
# the kernels of this source; a change to k_apply2d voids the figure.
C2_APPLY_HBM_BYTES_PER_LAUNCH = 1741471


def cpu_baseline(cfg, its_gpu):
    """Oracle timed on the host: one full solve at beta = 1 and a bounded
    number of outer iterations at beta = 1e-4, projected to the iteration
    count the GPU solver needed (setup excluded on both sides)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import curldiv_inputs as ci
    from oracle import method
    from paper_1805_10058_amd import capi

    d, p, n, alpha, betas, dist, tol = cfg
    opt = capi.options()  # the GPU solver's defaults, so both run the same method
    times = []
    with threadpool_limits(limits=1):
        for beta in betas:
            meth = method.Method(d, p, n, alpha, beta, coarse_max_dofs=opt.coarse_max_dofs, nu=opt.cheb_degree,
                                 nu_coarse=opt.cheb_degree_coarse if opt.cheb_degree_coarse > 0 else None,
                                 ratio=opt.cheb_ratio, lanczos_steps=opt.lanczos_steps)
            b = ci.rhs(d, p, n, 0, dist)
            cap = 6 if beta < 1e-2 else 10000
            t0 = time.perf_counter()
            _, it, _ = meth.solve(b, tol, maxiter=cap)
            dt = time.perf_counter() - t0
            target = its_gpu.get(beta, it)
            times.append(dt / it * max(it, target))
    return {"value": len(betas) / sum(times), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle P_MIM (FCG + V-cycle, same algorithm) on the {d}D p={p} n={n} workload, "
                      f"one solve per beta in {betas}; beta=1 run to completion, beta<1e-2 run for 6 outer "
                      f"iterations and projected to the GPU iteration count; setup excluded; 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the 3D p=3 n=128 operator-apply measurement")
    ap.add_argument("--only-c4", action="store_true", help="run only the 3D p=3 n=128 operator-apply measurement")
    ap.add_argument("--serve", type=int, default=32, help="requests of the serving stream to run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=8.0, help="Poisson arrival rate of the stream, 1/s (0: burst)")
    ap.add_argument("--serve-max-iter", type=int, default=4000)
    ap.add_argument("--batched", type=int, default=8,
                    help="also solve this many right-hand sides of the 2D workload at once through the "
                         "continuous-batching server (0: skip)")
    ap.add_argument("--only-c4-solve", action="store_true",
                    help="run only the mixed solve of the 3D p=3 n=128 workload (beta = 1e-6)")
    ap.add_argument("--c4-max-iter", type=int, default=20000,
                    help="outer-iteration cap of that solve (a small cap gives a short profiling run)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="only run 6 eager outer iterations of each mixed 2D workload solve (and --copy-cal): a "
                         "short program for the HBM byte counters of the V-cycle kernels")
    ap.add_argument("--copy-cal", action="store_true",
                    help="also run a plain 256 MiB device copy 5 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (--gpus 1 only)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import curldiv_inputs as ci
    from paper_1805_10058_amd import capi

    torch.cuda.set_device(0)
    st = torch.cuda.current_stream().cuda_stream
    if args.copy_cal:
        copy_calibration(torch)
    if args.only_c4:
        print(json.dumps({"operator_apply_c4": c4_apply(capi, torch, st)}), flush=True)
        return
    if args.only_c4_solve:
        print(json.dumps({"solve_c4": c4_solve(capi, torch, st, args.c4_max_iter)}), flush=True)
        return
    name = "c2_2d_p3_n256"
    cfg = ci.CONFIGS[name]
    d, p, n, alpha, betas, dist, tol = cfg
    N = ci.num_dofs(d, p, n)

    def make(beta, precision):
        opt = capi.options(precision=precision, rtol=tol)
        return capi.Solver(capi.problem(d, p, n, alpha, beta), opt, st)

    if args.pmc_pass:
        # the same kernels and per-iteration launch mix as the timed solves,
        # launched eagerly and cut to a few outer iterations
        b0 = torch.as_tensor(ci.rhs(d, p, n, 0, dist)).cuda()
        x0 = torch.zeros(N, dtype=torch.float64, device="cuda")
        for beta in betas:
            opt = capi.options(precision=capi.CD_MIXED_FP32, rtol=tol, max_iter=6, graphs=0)
            s = capi.Solver(capi.problem(d, p, n, alpha, beta), opt, st)
            r = s.solve(b0.data_ptr(), x0.data_ptr())
            s.close()
            print(f"[bench] counter pass: beta={beta} iterations={r.iterations}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return

    mixed = {beta: make(beta, capi.CD_MIXED_FP32) for beta in betas}
    fp64 = {beta: make(beta, capi.CD_FP64) for beta in betas}
    nsteps = args.warmup + args.steps
    rhs = [[torch.as_tensor(ci.rhs(d, p, n, 1000 * k + j, dist)).cuda() for j in range(len(betas))]
           for k in range(nsteps)]
    xs = [torch.zeros(N, dtype=torch.float64, device="cuda") for _ in betas]
    torch.cuda.synchronize()

    def step(k, solvers, lat, its, res_out):
        for j, beta in enumerate(betas):
            t0 = time.perf_counter()
            r = solvers[beta].solve(rhs[k][j].data_ptr(), xs[j].data_ptr())
            lat.append(time.perf_counter() - t0)
            its[beta] = r.iterations
            res_out.append(r.true_rel_residual)
            if r.status != capi.CD_OK:
                raise RuntimeError(f"solve did not converge: beta={beta} status={r.status}")

    lat, its, tres = [], {}, []
    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # live timing on from the warm-up on, so that the timed region replays
    # graphs that were captured (with their timing event nodes) before it;
    # every PROF_PERIOD-th outer iteration carries the timing events
    for s in mixed.values():
        s.profile_enable(True, PROF_PERIOD)
    for k in range(args.warmup):
        step(k, mixed, [], its, [])
        log(f"warmup step {k} done, iterations {its}")
    for s in mixed.values():  # restart the counters
        s.profile_enable(False)
        s.profile_enable(True, PROF_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, nsteps):
        step(k, mixed, lat, its, tres)
        log(f"timed step {k} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = t1 - t0
    nsolves = args.steps * len(betas)

    # live kernel timing (stamps written by the kernels themselves, sampled
    # outer iterations of the timed region) of the FP32 V-cycle operator apply
    # (k_apply2d<float, 3, *> on every level), the kernel that takes the most
    # GPU time in the timed solves, and of the FP32 T-solve passes
    nlev = {beta: mixed[beta].num_levels() for beta in betas}
    tot_ms = tot_b = 0.0
    launches = 0
    per_level = {}
    ts_ms = ts_b = 0.0
    ts_n = 0
    for beta, s in mixed.items():
        for lvl in range(nlev[beta]):
            stt = s.profile_read(lvl, True)
            tot_ms += stt.total_ms
            tot_b += stt.bytes
            launches += stt.launches
            pl = per_level.setdefault(lvl, [0, 0.0, 0.0])
            pl[0] += stt.launches
            pl[1] += stt.total_ms
            pl[2] += stt.bytes
        tst = s.profile_read_tsolve(True)
        ts_ms += tst.total_ms
        ts_b += tst.bytes
        ts_n += tst.launches
        s.profile_enable(False)
    ach = (tot_b / (tot_ms * 1e-3)) / 1e9 if tot_ms > 0 else 0.0
    ts_gbs = (ts_b / (ts_ms * 1e-3)) / 1e9 if ts_ms > 0 else 0.0

    # plain FP64 single-solve path on the same inputs (comparison, not the headline)
    lat64, its64, tres64 = [], {}, []
    step(0, fp64, [], its64, [])
    t2 = time.perf_counter()
    for k in range(args.warmup, nsteps):
        step(k, fp64, lat64, its64, tres64)
    torch.cuda.synchronize()
    T64 = time.perf_counter() - t2
    log(f"fp64 comparison done, iterations {its64}")

    out = {
        "metric": "solves/sec + p50/p99 latency to rel. residual 1e-8; operator-apply HBM GB/s",
        "value": nsolves / T,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "2D curl-div, p=3, n=256 (132,098 unknowns), alpha=1, beta in {1, 1e-4}, "
                               "uniform[-1,1] RHS, rel. residual 1e-8, FP32 V-cycle in FP64 flexible CG",
                   "dim": d, "degree": p, "n": n, "betas": betas, "solves_per_step": len(betas)},
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
        "iterations": {str(b): its[b] for b in betas},
        "max_true_rel_residual": max(tres),
        "fp64_path": {"solves_per_s": nsolves / T64, "p50_ms": 1e3 * percentile(lat64, 50),
                      "p99_ms": 1e3 * percentile(lat64, 99), "iterations": {str(b): its64[b] for b in betas},
                      "max_true_rel_residual": max(tres64)},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": C2_APPLY_HBM_BYTES_PER_LAUNCH,
                     "kernel": "FP32 V-cycle operator apply k_apply2d<float,3,*>, all levels, inside the timed solves "
                               f"(every {PROF_PERIOD}th outer iteration timed)",
                     "launches": launches, "avg_us": 1e3 * tot_ms / max(launches, 1),
                     "bytes_per_launch": tot_b / max(launches, 1),
                     "per_level": {str(l): {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1),
                                            "GB_s": (v[2] / (v[1] * 1e-3)) / 1e9 if v[1] > 0 else 0.0}
                                   for l, v in sorted(per_level.items())}},
        "tsolve": {"kernel": "FP32 T-solve axis passes k_tsolve_line<float,2,*>", "launches": ts_n,
                   "avg_us": 1e3 * ts_ms / max(ts_n, 1), "GB_s": ts_gbs, "hbm_frac": ts_gbs / HBM_PEAK_GBS},
    }

    if args.batched > 0:
        out["batched"] = c2_batched(capi, torch, cfg, args.batched, log)
        log(f"batched: {out['batched']}")

    if not args.no_c4:
        out["operator_apply_c4"] = c4_apply(capi, torch, st)
        log(f"3D p=3 n=128 operator apply: {out['operator_apply_c4']}")
        out["solve_c4"] = c4_solve(capi, torch, st, args.c4_max_iter)
        log(f"3D p=3 n=128 solve: {out['solve_c4']}")

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
        out["cpu_baseline"] = cpu_baseline(cfg, its)
    print(json.dumps(out), flush=True)


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


def serve_bench(capi, torch, st, count, max_iter, log, rate):
    """The serving workload: `count` seeded requests of the stream (2D/3D,
    p in {2,3,4}, n log-uniform, beta log-uniform in [1e-6, 1]) arriving as a
    Poisson process of `rate` requests per second (0: all at t = 0), served
    by the continuous-batching mixed-precision server; then the same arrival
    schedule served one request at a time by the plain FP64 single-solve
    path.  Latency = completion - arrival; both include solver setup; the
    right-hand sides are resident in HBM before timing starts."""
    import curldiv_inputs as ci

    reqs = ci.serving_stream(count, seed=7, rate=rate if rate > 0 else None)
    data = []
    for r in reqs:
        prob = capi.problem(r["dim"], r["p"], r["n"], r["alpha"], r["beta"])
        b = torch.as_tensor(ci.rhs(r["dim"], r["p"], r["n"], r["seed"])).cuda()
        data.append((prob, b, torch.zeros_like(b), torch.zeros_like(b), r["arrival"]))
    torch.cuda.synchronize()
    srv = capi.Server(max_active=32)
    opt = capi.options(precision=capi.CD_MIXED_FP32, rtol=1e-8, max_iter=max_iter)
    ticket, done, arrival_of = {}, {}, {}
    nxt = 0
    t0 = time.perf_counter()
    while len(done) < count:
        now = time.perf_counter() - t0
        while nxt < count and data[nxt][4] <= now:
            prob, b, x, _, arr = data[nxt]
            tk = srv.submit(prob, opt, b.data_ptr(), x.data_ptr())
            ticket[tk] = nxt
            arrival_of[nxt] = arr
            nxt += 1
        a, q = srv.step()
        for c in srv.poll():
            done[ticket[c.ticket]] = (c, time.perf_counter() - t0)
        if a == 0 and q == 0 and nxt < count:
            time.sleep(max(0.0, data[nxt][4] - (time.perf_counter() - t0)))
    T = time.perf_counter() - t0
    srv.close()
    lat = [t_done - arrival_of[i] for i, (c, t_done) in done.items()]
    ok = sum(1 for c, _ in done.values() if c.result.status == capi.CD_OK)
    its = [c.result.iterations for c, _ in done.values()]
    log(f"server done in {T:.2f}s; converged {ok}/{count}")
    ok64, lat64 = 0, []
    t1 = time.perf_counter()
    for prob, b, _, x, arr in data:
        wait = arr - (time.perf_counter() - t1)
        if wait > 0:
            time.sleep(wait)
        s = capi.Solver(prob, capi.options(rtol=1e-8, max_iter=max_iter), st)
        r = s.solve(b.data_ptr(), x.data_ptr())
        s.close()
        lat64.append(time.perf_counter() - t1 - arr)
        ok64 += int(r.status == capi.CD_OK)
    T64 = time.perf_counter() - t1
    mode = (f"Poisson arrivals at {rate:g}/s" if rate > 0 else "burst (all arrive at t=0)") + \
        ", continuous batching, mixed FP32/FP64, max 32 in flight"
    return {"requests": count, "mode": mode,
            "solves_per_s": count / T, "converged": ok, "p50_ms": 1e3 * percentile(lat, 50),
            "p99_ms": 1e3 * percentile(lat, 99), "iterations_min_max": [min(its), max(its)],
            "max_iter": max_iter,
            "fp64_sequential": {"solves_per_s": count / T64, "converged": ok64,
                                "p50_ms": 1e3 * percentile(lat64, 50), "p99_ms": 1e3 * percentile(lat64, 99)},
            "speedup_vs_fp64_sequential": T64 / T}


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


def c4_solve(capi, torch, st, max_iter):
    """One mixed-precision solve of the 3D p=3 n=128 workload (beta = 1e-6,
    Gaussian right-hand side, rel. residual 1e-8): setup and solve times."""
    import curldiv_inputs as ci

    d, p, n, alpha, betas, dist, tol = ci.CONFIGS["c4_3d_p3_n128"]
    N = ci.num_dofs(d, p, n)
    b = torch.as_tensor(ci.rhs(d, p, n, 0, dist)).cuda()
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = capi.Solver(capi.problem(d, p, n, alpha, betas[0]),
                    capi.options(precision=capi.CD_MIXED_FP32, rtol=tol, max_iter=max_iter), st)
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


if __name__ == "__main__":
    main()
