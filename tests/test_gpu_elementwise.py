"""Element-by-element GPU parity of every step of the V-cycle against the
FP64 oracle, in FP64 and in FP32, including the 3D operator kernel marching
over several x1 planes per block in every mode.

Error measures (both element-wise):
* linear maps y = L x with an explicit oracle matrix (operator, transfers):
  the row-scaled error max_i |y_i - (L x)_i| / (|L| |x|)_i, which bounds the
  rounding of any summation order by gamma_k = k u / (1 - k u), k the number
  of terms a row sums (at most 3 (2p+1)^3 + 3 (2p+1)^2 for the operator,
  (p+2)^d for a transfer);
* the other steps (smoother, T-solve, V-cycle): the max-norm error relative to
  the largest entry of the oracle's result, max_i |y_i - y*_i| / max_i |y*_i|.

Tolerances: FP64 (u = 1.1e-16): operator 1e-13 row-scaled, transfers 1e-14,
smoother 1e-11 and V-cycle 1e-10 (the 2-norm bounds of the other parity
tests, now entry by entry), T-solve 1e-13 kappa(T).  FP32 (u = 6.0e-8, with
FP32 coefficients): operator 2e-5 and transfers 2e-6 row-scaled (gamma_k
with k a few hundred and a few tens), T-solve 2e-6 kappa(T) (a backward
stable banded solve loses kappa(T) times a small multiple of u), smoother
1e-4 (up to 48 Chebyshev steps; the three-term recurrence is stable on the
smoothing interval, so rounding grows about linearly with the step count:
48 x 30 u) and V-cycle 1e-3 (the smoother's error passed through the
transfers, the coarse solve and the GMRES post-smoother, whose small least
squares problem amplifies it by its condition number, measured below 10 on
these cases).
"""
import numpy as np
import pytest

from tests.gpu_util import dev, empty, gpu_ok, host, stream, torch

pytestmark = pytest.mark.gpu

if not gpu_ok():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import method  # noqa: E402
from paper_1805_10058_amd import capi  # noqa: E402

# (dim, p, n, beta, transfer, coarse_max, x1 chunk of the 3D kernel (0 =
# automatic), 3D kernel variant)
CASES = [
    (2, 2, 40, 0.05, "knot", 100, 0, "auto"),
    (2, 3, 64, 1e-2, "knot", 300, 0, "auto"),
    (2, 4, 24, 0.5, "paper", 80, 0, "auto"),
    (3, 2, 20, 0.1, "knot", 500, 3, "auto"),
    (3, 3, 16, 0.01, "knot", 700, 3, "auto"),
    (3, 3, 16, 0.01, "knot", 700, 5, "auto"),
    (3, 4, 10, 1.0, "paper", 600, 4, "auto"),
    (3, 6, 8, 0.3, "knot", 2000, 3, "auto"),
    (3, 2, 20, 0.1, "knot", 500, 0, "auto"),
    # n_l = nu_l n (anisotropic grids), an odd n (its axis coarsens with the
    # paper's prolongator), and an axis that stops at one point
    (2, 3, (24, 40), 0.05, "knot", 300, 0, "auto"),
    (3, 2, (8, 12, 16), 0.1, "knot", 500, 3, "auto"),
    (2, 3, 25, 0.1, "knot", 60, 0, "auto"),
    (3, 2, (7, 8, 6), 0.2, "knot", 30, 2, "auto"),
    (2, 2, (4, 64), 0.3, "knot", 10, 0, "auto"),
    # the grouped-march variant of the 3D kernel: its own geometry, one range
    # over the whole x1 axis (several phases, the last one partly idle),
    # ragged ranges, p = 6 and an anisotropic grid
    (3, 3, 16, 0.01, "knot", 700, 0, "group"),
    (3, 3, 16, 0.01, "knot", 700, 17, "group"),
    (3, 2, 20, 0.1, "knot", 500, 7, "group"),
    (3, 4, 10, 1.0, "paper", 600, 0, "group"),
    (3, 6, 8, 0.3, "knot", 2000, 0, "group"),
    (3, 2, (8, 12, 16), 0.1, "knot", 500, 0, "group"),
]
KERNELS = {"auto": capi.CD_APPLY3D_AUTO, "march": capi.CD_APPLY3D_MARCH, "short": capi.CD_APPLY3D_SHORT,
           "group": capi.CD_APPLY3D_GROUP}


def _nid(n):
    return "x".join(map(str, n)) if isinstance(n, tuple) else str(n)


IDS = [f"d{c[0]}p{c[1]}n{_nid(c[2])}b{c[3]}{c[4]}x{c[6]}{'' if c[7] == 'auto' else c[7]}" for c in CASES]
U64, U32 = 2.0 ** -53, 2.0 ** -24

_cache = {}


def setup(case, precision=capi.CD_FP64):
    d, p, n, beta, xfer, cmax, chunk, kern = case
    key = (case, precision)
    if key not in _cache:
        tr = capi.CD_XFER_KNOT if xfer == "knot" else capi.CD_XFER_PAPER
        opt = capi.options(transfer=tr, coarse_max_dofs=cmax, precision=precision, apply_x1_chunk=chunk,
                           apply3d_kernel=KERNELS[kern])
        s = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
        m = method.Method(d, p, n, 1.0, beta, transfer=xfer, coarse_max_dofs=cmax, nu=opt.cheb_degree,
                          ratio=opt.cheb_ratio, lanczos_steps=opt.lanczos_steps, nu_coarse=s.coarse_degree())
        # both sides estimate the smoother's eigenvalue bound independently (checked
        # below); the oracle then takes the GPU's estimate so that the smoother and
        # V-cycle comparisons measure the kernels' arithmetic, not the last bits of
        # two Lanczos recurrences, which the Chebyshev coefficients pass on
        for l, L in enumerate(m.levels[:-1]):
            lam = s.get_lambda(l)
            assert abs(lam - L.lam) <= 1e-9 * L.lam, (l, lam, L.lam)
            L.lam, L.hi = lam, 1.1 * lam
            L.lo = L.hi / opt.cheb_ratio
        _cache[key] = (s, m)
    return _cache[key]


def rowscaled(y, ref, scale):
    return np.max(np.abs(y - ref) / np.where(scale > 0, scale, 1.0))


def maxrel(y, ref):
    return np.max(np.abs(y - ref)) / max(np.max(np.abs(ref)), 1e-300)


def kappa_T(p):
    return max(1.0, (np.pi / 2) ** (2 * (p - 1)))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_operator_every_level(case):
    s, m = setup(case)
    rng = np.random.default_rng(41)
    for l, L in enumerate(m.levels):
        Ka = abs(L.K)
        x = rng.uniform(-1, 1, L.K.shape[0])
        xd, y = dev(x), empty(x.size)
        s.apply(l, xd.data_ptr(), y.data_ptr())
        assert rowscaled(host(y), L.K @ x, Ka @ np.abs(x)) <= 1e-13, l
        x32 = x.astype(np.float32)
        xf, yf = dev(x32, torch.float32), empty(x.size, torch.float32)
        s.apply_f32(l, xf.data_ptr(), yf.data_ptr())
        x64 = x32.astype(np.float64)
        assert rowscaled(host(yf), L.K @ x64, Ka @ np.abs(x64)) <= 2e-5, l


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_transfers_entrywise(case):
    s, m = setup(case)
    rng = np.random.default_rng(42)
    for l in range(len(m.levels) - 1):
        Pb = m._prolong_block(l)
        Pa = abs(Pb)
        rf = rng.uniform(-1, 1, Pb.shape[0])
        ec = rng.uniform(-1, 1, Pb.shape[1])
        x0 = rng.uniform(-1, 1, Pb.shape[0])
        for dt, tol_r, tol_p in ((torch.float64, 1e-14, 1e-14), (torch.float32, 2e-6, 2e-6)):
            rfd, rc = dev(rf, dt), empty(Pb.shape[1], dt)
            ecd, xt = dev(ec, dt), dev(x0, dt)
            if dt == torch.float64:
                s.restrict(l, rfd.data_ptr(), rc.data_ptr())
                s.prolong_add(l, ecd.data_ptr(), xt.data_ptr())
                rfx, ecx, x0x = rf, ec, x0
            else:
                s.restrict_f32(l, rfd.data_ptr(), rc.data_ptr())
                s.prolong_add_f32(l, ecd.data_ptr(), xt.data_ptr())
                rfx, ecx, x0x = (v.astype(np.float32).astype(np.float64) for v in (rf, ec, x0))
            assert rowscaled(host(rc), Pb.T @ rfx, Pa.T @ np.abs(rfx)) <= tol_r, (l, dt)
            assert rowscaled(host(xt), x0x + Pb @ ecx, np.abs(x0x) + Pa @ np.abs(ecx)) <= tol_p, (l, dt)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tsolve_entrywise(case):
    s, m = setup(case)
    v = np.random.default_rng(43).uniform(-1, 1, m.K.shape[0])
    ref = m.Tsolve(v)
    vd, z = dev(v), empty(v.size)
    s.tsolve(vd.data_ptr(), z.data_ptr())
    assert maxrel(host(z), ref) <= 1e-13 * kappa_T(case[1])
    v32 = v.astype(np.float32)
    vf, zf = dev(v32, torch.float32), empty(v.size, torch.float32)
    s.tsolve_f32(vf.data_ptr(), zf.data_ptr())
    assert maxrel(host(zf), m.Tsolve(v32.astype(np.float64))) <= 2e-6 * kappa_T(case[1])


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_smoother_entrywise(case):
    s, m = setup(case)
    rng = np.random.default_rng(44)
    for l, L in enumerate(m.levels[:-1]):
        b = rng.uniform(-1, 1, L.K.shape[0])
        x0 = rng.uniform(-1, 1, L.K.shape[0])
        ref = method.chebyshev(L, x0, b)
        bd, xd, out = dev(b), dev(x0), empty(b.size)
        s.smooth(l, bd.data_ptr(), xd.data_ptr(), out.data_ptr())
        assert maxrel(host(out), ref) <= 1e-11, l
        b32, x32 = b.astype(np.float32), x0.astype(np.float32)
        ref32 = method.chebyshev(L, x32.astype(np.float64), b32.astype(np.float64))
        bf, xf, of = dev(b32, torch.float32), dev(x32, torch.float32), empty(b.size, torch.float32)
        s.smooth_f32(l, bf.data_ptr(), xf.data_ptr(), of.data_ptr())
        assert maxrel(host(of), ref32) <= 1e-4, l


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_vcycle_entrywise(case):
    s, m = setup(case)
    s32, _ = setup(case, capi.CD_MIXED_FP32)
    r = np.random.default_rng(45).uniform(-1, 1, m.K.shape[0])
    ref = m.vcycle(r)
    rd, z = dev(r), empty(r.size)
    s.precondition(rd.data_ptr(), z.data_ptr())
    assert maxrel(host(z), ref) <= 1e-10
    z32 = empty(r.size)
    s32.precondition(rd.data_ptr(), z32.data_ptr())
    err = maxrel(host(z32), ref)
    print(f"FP32 V-cycle max-norm error {err:.2e}")
    assert err <= 1e-3


CHUNKED = [(c, i) for c, i in zip(CASES, IDS)
           if c[0] == 3 and c[6] > 0 and c[7] == "auto" and not isinstance(c[2], tuple)]


@pytest.mark.parametrize("case", [c for c, _ in CHUNKED], ids=[i for _, i in CHUNKED])
def test_x1_chunk_solve_matches_automatic(case):
    # the launch geometry changes only the per-block partial sums of the dot
    # products: solves agree to the solver tolerance and take the same count
    s, m = setup(case)
    auto = case[:6] + (0, "auto")
    s0, _ = setup(auto)
    b = np.random.default_rng(46).uniform(-1, 1, m.K.shape[0])
    bd, x1, x0 = dev(b), empty(b.size), empty(b.size)
    r1 = s.solve(bd.data_ptr(), x1.data_ptr())
    r0 = s0.solve(bd.data_ptr(), x0.data_ptr())
    assert r1.status == capi.CD_OK and r0.status == capi.CD_OK
    assert abs(r1.iterations - r0.iterations) <= 1
    assert maxrel(host(x1), host(x0)) <= 1e-6


@pytest.mark.parametrize("d,p,n", [(3, 3, 12), (3, 2, (9, 14, 20)), (3, 1, 10), (3, 3, 16)])
def test_short_march_variant_matches_marching_kernel(d, p, n):
    # small grids take the variant of the 3D kernel that processes a block's
    # 2 HB + 1 input planes side by side (automatic launch geometry); forcing
    # one-plane ranges selects the marching kernel: y = A x is bitwise the
    # same, in FP64 and in FP32, on every level
    prob = capi.problem(d, p, n, 1.0, 0.2)
    auto = capi.Solver(prob, capi.options(coarse_max_dofs=50), stream())
    march = capi.Solver(prob, capi.options(coarse_max_dofs=50, apply_x1_chunk=1), stream())
    rng = np.random.default_rng(47)
    for l in range(auto.num_levels()):
        _, nl = auto.level_shape(l)
        x = rng.uniform(-1, 1, nl)
        for dt, fn in ((torch.float64, "apply"), (torch.float32, "apply_f32")):
            xd, ya, ym = dev(x, dt), empty(nl, dt), empty(nl, dt)
            getattr(auto, fn)(l, xd.data_ptr(), ya.data_ptr())
            getattr(march, fn)(l, xd.data_ptr(), ym.data_ptr())
            np.testing.assert_array_equal(host(ya), host(ym))
    auto.close()
    march.close()


@pytest.mark.parametrize("d,p,n,chunk", [(3, 3, 12, 0), (3, 2, (9, 14, 20), 0), (3, 1, 10, 0), (3, 3, 16, 0),
                                         (3, 3, 16, 5), (3, 4, (10, 7, 12), 0), (3, 5, (9, 11, 8), 0), (3, 6, 8, 0),
                                         (3, 2, 34, 0)])
def test_apply3d_variants_agree(d, p, n, chunk):
    # every variant of the 3D kernel (marching, short-march, grouped march)
    # sums each output entry's terms in the same order: y = A x bitwise equal
    # on every level in FP64 and FP32; the Chebyshev smoother within the
    # rounding of its update (the FP32 step may round its last bit
    # differently, and 48 steps pass that on)
    prob = capi.problem(d, p, n, 1.0, 0.2)
    solvers = {k: capi.Solver(prob, capi.options(coarse_max_dofs=50, apply_x1_chunk=chunk, apply3d_kernel=v),
                              stream())
               for k, v in (("march", capi.CD_APPLY3D_MARCH), ("short", capi.CD_APPLY3D_SHORT),
                            ("group", capi.CD_APPLY3D_GROUP), ("auto", capi.CD_APPLY3D_AUTO))}
    ref = solvers["march"]
    rng = np.random.default_rng(48)
    for l in range(ref.num_levels()):
        _, nl = ref.level_shape(l)
        x, b = rng.uniform(-1, 1, nl), rng.uniform(-1, 1, nl)
        for dt, fn, sm, tol in ((torch.float64, "apply", "smooth", 1e-13), (torch.float32, "apply_f32", "smooth_f32", 1e-5)):
            xd, bd = dev(x, dt), dev(b, dt)
            ym, zm = empty(nl, dt), empty(nl, dt)
            getattr(ref, fn)(l, xd.data_ptr(), ym.data_ptr())
            if l < ref.num_levels() - 1:
                getattr(ref, sm)(l, bd.data_ptr(), xd.data_ptr(), zm.data_ptr())
            for k, s in solvers.items():
                if k == "march":
                    continue
                y, z = empty(nl, dt), empty(nl, dt)
                getattr(s, fn)(l, xd.data_ptr(), y.data_ptr())
                np.testing.assert_array_equal(host(y), host(ym), err_msg=f"{k} level {l} {dt}")
                if l < ref.num_levels() - 1:
                    getattr(s, sm)(l, bd.data_ptr(), xd.data_ptr(), z.data_ptr())
                    assert maxrel(host(z), host(zm)) <= tol, (k, l, dt)
    for s in solvers.values():
        s.close()
