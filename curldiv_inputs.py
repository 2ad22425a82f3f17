"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only names the workload
configurations and draws right-hand sides and arrival streams from numpy's
PCG64 generator.  The configurations follow the problem sizes named for the
benchmark (sizes n per direction, degree p, weights alpha and beta).
"""
import numpy as np

# name -> (dim, degree p, intervals n, alpha, list of beta, rhs distribution, relative tolerance)
CONFIGS = {
    "c1_2d_p2_n16": (2, 2, 16, 1.0, [1.0], "uniform", 1e-10),
    "c2_2d_p3_n256": (2, 3, 256, 1.0, [1.0, 1e-4], "uniform", 1e-8),
    "c3_3d_p2_n64": (3, 2, 64, 1.0, [1.0, 1e-2], "uniform", 1e-8),
    "c4_3d_p3_n128": (3, 3, 128, 1.0, [1e-6], "normal", 1e-8),
}


def num_dofs(dim, p, n):
    return dim * (n + p - 2) ** dim


def rhs(dim, p, n, seed, dist="uniform"):
    """Right-hand side coefficient vector: i.i.d. U[-1, 1] or N(0, 1) from ``seed``."""
    rng = np.random.default_rng(seed)
    N = num_dofs(dim, p, n)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, N)
    if dist == "normal":
        return rng.standard_normal(N)
    raise ValueError(dist)


def serving_stream(count=512, seed=2024, rate=None, round_n=False):
    """Requests of the serving workload: dimension 2/3 with equal probability,
    p in {2,3,4}, n log-uniform in [32,256] (2D) or [16,96] (3D) (rounded to
    the nearest integer; with round_n to the nearest c * 2^k, c in 4..7),
    beta log-uniform in [1e-6, 1], alpha = 1, and Poisson arrival times (rate
    requests per second; None = all at t = 0).  The arrival gaps are unit
    exponentials divided by the rate, so streams of one seed at different
    rates differ only in their time scale."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(count):
        d = 2 if rng.random() < 0.5 else 3
        p = int(rng.integers(2, 5))
        lo, hi = (32, 256) if d == 2 else (16, 96)
        n_raw = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        if round_n:
            cands = sorted({c * 2**k for c in range(4, 8) for k in range(0, 8) if lo <= c * 2**k <= hi})
            n = min(cands, key=lambda v: abs(v - n_raw))
        else:
            n = int(round(n_raw))
        beta = float(10.0 ** rng.uniform(-6.0, 0.0))
        gap = float(rng.exponential(1.0))
        if rate:
            t += gap / rate
        out.append({"id": i, "dim": d, "p": p, "n": n, "alpha": 1.0, "beta": beta, "arrival": t,
                    "seed": 10_000 + i})
    return out
