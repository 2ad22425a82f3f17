"""GPU parity tests: every kernel of libcurldiv (through the C ABI) against the
FP64 oracle on the same seeded inputs.

Tolerances: linear maps in FP64 to 1e-12 relative (the operator, transfers,
T-solve, coarse solve, one smoother application), whole V-cycles to 1e-10
relative (the GMRES post-smoother's least-squares step amplifies rounding
by the conditioning of its small Hessenberg problem), FP32 operator applies
to 2e-5 relative (FP32 rounding of 2p+1-term sums across three axes).
"""
import numpy as np
import pytest

from tests.gpu_util import dev, empty, gpu_ok, host, relerr, stream, torch

pytestmark = pytest.mark.gpu

if not gpu_ok():  # collected on CPU with -m "not gpu" deselected anyway
    pytest.skip("no GPU", allow_module_level=True)

from oracle import assembly as asm  # noqa: E402
from oracle import loadvec, method, solvers  # noqa: E402
from oracle import matrices as mt  # noqa: E402
from paper_1805_10058_amd import capi  # noqa: E402

# (dim, p, n, beta, transfer, coarse_max): sizes span several tiles with ragged tails
CASES = [
    (2, 1, 20, 0.3, "knot", 60),
    (2, 2, 40, 0.05, "knot", 100),
    (2, 3, 64, 1e-2, "knot", 300),
    (2, 4, 24, 0.5, "paper", 80),
    (2, 6, 18, 0.1, "knot", 400),
    (3, 1, 12, 0.2, "knot", 400),
    (3, 2, 20, 0.1, "knot", 500),
    (3, 3, 16, 0.01, "knot", 700),
    (3, 4, 10, 1.0, "paper", 600),
    (3, 6, 8, 0.3, "knot", 2000),
]
IDS = [f"d{c[0]}p{c[1]}n{c[2]}b{c[3]}{c[4]}" for c in CASES]

_cache = {}


def setup_case(case, precision=capi.CD_FP64, **kw):
    d, p, n, beta, xfer, cmax = case
    key = (case, precision, tuple(sorted(kw.items())))
    if key not in _cache:
        tr = capi.CD_XFER_KNOT if xfer == "knot" else capi.CD_XFER_PAPER
        opt = capi.options(transfer=tr, coarse_max_dofs=cmax, precision=precision, **kw)
        s = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
        m = method.Method(d, p, n, 1.0, beta, transfer=xfer, coarse_max_dofs=cmax,
                          nu=opt.cheb_degree, ratio=opt.cheb_ratio, lanczos_steps=opt.lanczos_steps,
                          krylov_steps=None if opt.krylov_steps < 0 else opt.krylov_steps,
                          nu_coarse=s.coarse_degree())
        _cache[key] = (s, m)
    return _cache[key]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_setup_matrices(case):
    s, m = setup_case(case)
    assert s.num_levels() == len(m.levels)
    d = case[0]
    for l, L in enumerate(m.levels):
        shape, ndofs = s.level_shape(l)
        assert ndofs == L.K.shape[0]
        assert shape[:d] == (L.m,) * d
        for ax in range(d):
            for w, X in (("M", L.M), ("A", L.A), ("S", L.S)):
                G = np.array(s.get_matrix(l, ax, w, L.m, L.m)).reshape(L.m, L.m)
                assert np.abs(G - X).max() <= 1e-13 * max(1.0, np.abs(X).max()), (l, ax, w)
            if L.P is not None:
                G = np.array(s.get_matrix(l, ax, "P", L.P.shape[0], L.P.shape[1])).reshape(L.P.shape)
                assert np.abs(G - L.P).max() <= 1e-13
    T = np.array(s.get_matrix(0, 0, "T", m.levels[0].m, m.levels[0].m)).reshape(m.levels[0].m, -1)
    assert np.abs(T - mt.toeplitz_T(m.levels[0].m, case[1])).max() <= 1e-15


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_apply_every_level_fp64(case):
    s, m = setup_case(case)
    rng = np.random.default_rng(1)
    for l, L in enumerate(m.levels):
        x = rng.uniform(-1, 1, L.K.shape[0])
        xd, y = dev(x), empty(L.K.shape[0])
        s.apply(l, xd.data_ptr(), y.data_ptr())
        assert relerr(host(y), L.K @ x) <= 1e-12, l


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_apply_fp32(case):
    s, m = setup_case(case)
    rng = np.random.default_rng(2)
    L = m.levels[0]
    x = rng.uniform(-1, 1, L.K.shape[0]).astype(np.float32)
    xd, y = dev(x, torch.float32), empty(L.K.shape[0], torch.float32)
    s.apply_f32(0, xd.data_ptr(), y.data_ptr())
    assert relerr(host(y), L.K @ x.astype(np.float64)) <= 2e-5


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_transfers(case):
    s, m = setup_case(case)
    d = case[0]
    rng = np.random.default_rng(3)
    for l in range(len(m.levels) - 1):
        Pb = m._prolong_block(l)
        rf = rng.uniform(-1, 1, Pb.shape[0])
        rfd, rc = dev(rf), empty(Pb.shape[1])
        s.restrict(l, rfd.data_ptr(), rc.data_ptr())
        assert relerr(host(rc), Pb.T @ rf) <= 1e-13
        ec = rng.uniform(-1, 1, Pb.shape[1])
        x0 = rng.uniform(-1, 1, Pb.shape[0])
        xt, ecd = dev(x0), dev(ec)
        s.prolong_add(l, ecd.data_ptr(), xt.data_ptr())
        assert relerr(host(xt), x0 + Pb @ ec) <= 1e-13
    assert d in (2, 3)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_tsolve(case):
    s, m = setup_case(case)
    rng = np.random.default_rng(4)
    v = rng.uniform(-1, 1, m.K.shape[0])
    vd, z = dev(v), empty(m.K.shape[0])
    s.tsolve(vd.data_ptr(), z.data_ptr())
    # backward-stable banded solves: error <= c kappa(T) u, kappa(T) <= (pi/2)^(2(p-1))
    kappa = (np.pi / 2) ** (2 * (case[1] - 1))
    assert relerr(host(z), m.Tsolve(v)) <= 1e-13 * max(1.0, kappa)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_coarse_solve(case):
    s, m = setup_case(case)
    C = m.levels[-1]
    r = np.random.default_rng(5).uniform(-1, 1, C.K.shape[0])
    rd, z = dev(r), empty(C.K.shape[0])
    s.coarse_solve(rd.data_ptr(), z.data_ptr())
    # explicit inverse (GPU) vs LU solve (oracle): both backward stable, so they
    # agree to a small multiple of kappa(K_c) u
    Kd = C.K.toarray()
    kappa = np.linalg.cond(Kd)
    assert relerr(host(z), np.linalg.solve(Kd, r)) <= max(1e-13, 50 * kappa * 2.2e-16)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_smoother_and_eigenvalue_bound(case):
    s, m = setup_case(case)
    rng = np.random.default_rng(6)
    for l, L in enumerate(m.levels[:-1]):
        # both sides compute the bound from the same definition (Lanczos from the
        # same start vector, largest Ritz value), independently
        assert abs(s.get_lambda(l) - L.lam) <= 1e-10 * L.lam
        b = rng.uniform(-1, 1, L.K.shape[0])
        x0 = rng.uniform(-1, 1, L.K.shape[0])
        bd, xd, out = dev(b), dev(x0), empty(L.K.shape[0])
        s.smooth(l, bd.data_ptr(), xd.data_ptr(), out.data_ptr())
        assert relerr(host(out), method.chebyshev(L, x0, b)) <= 1e-11, l


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_vcycle(case):
    s, m = setup_case(case)
    r = np.random.default_rng(7).uniform(-1, 1, m.K.shape[0])
    rd, z = dev(r), empty(m.K.shape[0])
    s.precondition(rd.data_ptr(), z.data_ptr())
    assert relerr(host(z), m.vcycle(r)) <= 1e-10


@pytest.mark.parametrize("alpha,beta,expect", [(1.0, 1.0, 8), (2.0, 0.05, 8), (1.0, 5e-3, 16), (1.0, 1e-5, 16),
                                                (10.0, 1.1e-4, 16), (10.0, 9e-5, 32), (1.0, 1e-6, 32)])
def test_default_coarse_degree_follows_beta_over_alpha(alpha, beta, expect):
    # cheb_degree_coarse < 0 resolves from beta / alpha at creation: 8 from
    # 1e-2 up, 16 from 1e-5 to 1e-2, 32 below; the finest level keeps cheb_degree
    s = capi.Solver(capi.problem(2, 2, 16, alpha, beta), capi.options(coarse_max_dofs=40), stream())
    assert s.num_levels() > 2
    assert s.coarse_degree() == expect
    assert s.get_smoother(0)[0] == 48
    s.close()
    for set_to, got in ((0, 48), (5, 5)):
        s = capi.Solver(capi.problem(2, 2, 16, alpha, beta), capi.options(coarse_max_dofs=40, cheb_degree_coarse=set_to),
                        stream())
        assert s.coarse_degree() == got
        s.close()


@pytest.mark.parametrize("case", [CASES[2], CASES[4], CASES[7]], ids=[IDS[2], IDS[4], IDS[7]])
def test_vcycle_light_smoothing_one_degree_everywhere(case):
    # cheb_degree_coarse = 0 keeps the finest level's degree on every level
    s, m = setup_case(case, cheb_degree=3, cheb_degree_coarse=0, cheb_ratio=30.0)
    assert all(L.nu == 3 for L in m.levels[:-1])
    rng = np.random.default_rng(17)
    for l, L in enumerate(m.levels[:-1]):
        b, x0 = rng.uniform(-1, 1, L.K.shape[0]), rng.uniform(-1, 1, L.K.shape[0])
        bd, xd, out = dev(b), dev(x0), empty(L.K.shape[0])
        s.smooth(l, bd.data_ptr(), xd.data_ptr(), out.data_ptr())
        assert relerr(host(out), method.chebyshev(L, x0, b)) <= 1e-11, l
    r = rng.uniform(-1, 1, m.K.shape[0])
    rd, z = dev(r), empty(m.K.shape[0])
    s.precondition(rd.data_ptr(), z.data_ptr())
    assert relerr(host(z), m.vcycle(r)) <= 1e-10


@pytest.mark.parametrize("case", [(2, 1, 8, 0.3, "knot", 1), (2, 1, 4, 0.5, "knot", 1)],
                         ids=["d2p1n8b0.3", "d2p1n4b0.5"])
def test_lanczos_breakdown_restart_on_tiny_levels(case):
    # levels of 18 unknowns: the Lanczos recurrence from the symmetric start
    # vector breaks down there and restarts from the fixed vector, the same
    # way on both sides
    s, m = setup_case(case)
    for l, L in enumerate(m.levels[:-1]):
        assert abs(s.get_lambda(l) - L.lam) <= 1e-10 * L.lam, l
    r = np.random.default_rng(19).uniform(-1, 1, m.K.shape[0])
    rd, z = dev(r), empty(m.K.shape[0])
    s.precondition(rd.data_ptr(), z.data_ptr())
    assert relerr(host(z), m.vcycle(r)) <= 1e-10


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_solve_matches_direct(case):
    s, m = setup_case(case, rtol=1e-12)
    b = np.random.default_rng(8).uniform(-1, 1, m.K.shape[0])
    bd, x = dev(b), empty(m.K.shape[0])
    res = s.solve(bd.data_ptr(), x.data_ptr())
    assert res.status == capi.CD_OK
    xd = solvers.solve_direct(m.K, b)
    assert relerr(host(x), xd) <= 1e-9
    # the recursive residual reached 1e-12; the true residual may drift above it
    # by rounding (largest for p = 6)
    assert res.true_rel_residual <= 5e-11
    _, it_o, _ = m.solve(b, 1e-12)
    assert abs(res.iterations - it_o) <= 1


def test_c1_configuration():
    # 2D, p = 2, n = 16, alpha = beta = 1, uniform RHS, FCG + V-cycle to 1e-10
    from curldiv_inputs import rhs
    d, p, n = 2, 2, 16
    opt = capi.options(rtol=1e-12, coarse_max_dofs=64)
    s = capi.Solver(capi.problem(d, p, n, 1.0, 1.0), opt, stream())
    assert s.num_levels() >= 3
    for seed in range(4):
        b = rhs(d, p, n, seed)
        bd, x = dev(b), empty(b.size)
        res = s.solve(bd.data_ptr(), x.data_ptr())
        assert res.status == capi.CD_OK
        # alpha = beta: exact solution by fast diagonalization (independent of assembly)
        assert relerr(host(x), solvers.fast_diag_solve(d, p, n, 1.0, b)) <= 1e-10


@pytest.mark.parametrize("d,p,n,beta,cg_paper", [(2, 2, 15, 0.1, 40), (2, 3, 30, 0.01, 201),
                                                 (3, 2, 7, 0.1, 29), (3, 3, 14, 0.01, 102)])
def test_plain_cg_reproduces_paper_counts(d, p, n, beta, cg_paper):
    # CG column of Tables 1-4 with the manufactured right-hand side (Sec. 6.2)
    opt = capi.options(method=capi.CD_METHOD_CG, rtol=1e-7)
    s = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
    b = loadvec.load_vector(d, p, n, 1.0, beta)
    bd, x = dev(b), empty(b.size)
    res = s.solve(bd.data_ptr(), x.data_ptr())
    assert abs(res.iterations - cg_paper) <= 2


@pytest.mark.parametrize("case", [CASES[2], CASES[7]], ids=[IDS[2], IDS[7]])
def test_mixed_precision_solve(case):
    s64, m = setup_case(case, rtol=1e-8)
    s32, _ = setup_case(case, precision=capi.CD_MIXED_FP32, rtol=1e-8)
    b = np.random.default_rng(9).uniform(-1, 1, m.K.shape[0])
    bd, x64, x32 = dev(b), empty(b.size), empty(b.size)
    r64 = s64.solve(bd.data_ptr(), x64.data_ptr())
    r32 = s32.solve(bd.data_ptr(), x32.data_ptr())
    assert r64.status == capi.CD_OK and r32.status == capi.CD_OK
    xo = host(x32)
    # true FP64 residual recomputed by the oracle
    assert np.linalg.norm(b - m.K @ xo) <= 1e-8 * np.linalg.norm(b) * 1.01
    assert r32.true_rel_residual <= 1e-8 * 1.01
    assert r32.iterations <= r64.iterations + 3


def test_edge_cases():
    st = stream()
    opt = capi.options()
    # invalid parameters are rejected before any device work
    with pytest.raises(capi.CurldivError):
        capi.Solver(capi.problem(2, 2, 8, 1.0, 0.0), opt, st)
    with pytest.raises(capi.CurldivError):
        capi.Solver(capi.problem(4, 2, [8, 8, 8], 1.0, 1.0), opt, st)
    with pytest.raises(capi.CurldivError):
        capi.Solver(capi.problem(2, 7, 8, 1.0, 1.0), opt, st)
    with pytest.raises(capi.CurldivError):
        capi.Solver(capi.problem(2, 1, 1, 1.0, 1.0), opt, st)  # n + p - 2 = 0 unknowns
    s = capi.Solver(capi.problem(2, 2, 8, 1.0, 0.5), opt, st)
    N = capi.num_dofs(s.prob)
    # zero right-hand side: x = 0 after zero iterations
    x, zero = empty(N) + 7.0, empty(N)
    res = s.solve(zero.data_ptr(), x.data_ptr())
    assert res.status == capi.CD_OK and res.iterations == 0 and np.all(host(x) == 0.0)
    # non-finite right-hand side: clean error
    b = np.ones(N)
    b[3] = np.nan
    bd, xn = dev(b), empty(N)
    with pytest.raises(capi.CurldivError):
        s.solve(bd.data_ptr(), xn.data_ptr())
    # max_iter = 1: not converged, x holds the first iterate
    s1 = capi.Solver(capi.problem(2, 2, 8, 1.0, 0.01),
                     capi.options(max_iter=1, coarse_max_dofs=30, rtol=1e-14), st)
    ones = dev(np.ones(N))
    res = s1.solve(ones.data_ptr(), x.data_ptr())
    assert res.status == capi.CD_NOT_CONVERGED and res.iterations == 1
    # a single level: the preconditioner is the exact coarse solve, one iteration
    s2 = capi.Solver(capi.problem(2, 3, 6, 1.0, 0.2), capi.options(coarse_max_dofs=5000, rtol=1e-10), st)
    assert s2.num_levels() == 1
    b = np.random.default_rng(0).uniform(-1, 1, capi.num_dofs(s2.prob))
    bd, x = dev(b), empty(b.size)
    res = s2.solve(bd.data_ptr(), x.data_ptr())
    assert res.iterations <= 2
    assert relerr(host(x), solvers.solve_direct(asm.curl_div_matrix(2, 3, 6, 1.0, 0.2), b)) <= 1e-11


@pytest.mark.parametrize("case", [CASES[2], CASES[7]], ids=[IDS[2], IDS[7]])
@pytest.mark.parametrize("precision", [capi.CD_FP64, capi.CD_MIXED_FP32])
def test_graph_replay_equals_eager(case, precision):
    # outer iterations replayed from a captured HIP graph (with host
    # synchronisation between replays) give bitwise the eager result
    s_g, m = setup_case(case, precision=precision, rtol=1e-9, graphs=1)
    s_e, _ = setup_case(case, precision=precision, rtol=1e-9, graphs=0)
    b = np.random.default_rng(11).uniform(-1, 1, m.K.shape[0])
    bd, xg, xe = dev(b), empty(b.size), empty(b.size)
    for _ in range(2):  # second solve replays the graph captured in the first
        rg = s_g.solve(bd.data_ptr(), xg.data_ptr())
        re = s_e.solve(bd.data_ptr(), xe.data_ptr())
        assert rg.iterations == re.iterations and rg.iterations >= 3
        np.testing.assert_array_equal(host(xg), host(xe))
    # the captured iteration's launch count: the kernels of one outer
    # iteration (the eager handle captured nothing)
    kg, ng = s_g.graph_launches()
    assert 10 <= kg <= ng
    assert s_e.graph_launches() == (0, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("graphs", [1, 0])
def test_live_timing_counts_and_leaves_results_unchanged(graphs):
    # kernel-side timing of the applies and T-solve passes: results are bitwise
    # those of an untimed solve, every timed launch is counted once, and the
    # algorithmic bytes follow the launch kinds (2D p=3: 2 T-solve passes per
    # solve of T, one solve per Krylov step, 3 Krylov steps per outer iteration)
    case = CASES[2]
    d, p, n, beta, _, cmax = case
    opt = capi.options(coarse_max_dofs=cmax, precision=capi.CD_MIXED_FP32, rtol=1e-9, graphs=graphs)
    s_t = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
    s_u = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
    b = np.random.default_rng(5).uniform(-1, 1, capi.num_dofs(s_t.prob))
    bd, xt, xu = dev(b), empty(b.size), empty(b.size)
    s_t.profile_enable(True, 1)
    rt = s_t.solve(bd.data_ptr(), xt.data_ptr())
    ru = s_u.solve(bd.data_ptr(), xu.data_ptr())
    assert rt.iterations == ru.iterations
    np.testing.assert_array_equal(host(xt), host(xu))
    ts = s_t.profile_read_tsolve(True)
    assert ts.launches == rt.iterations * p * d
    assert abs(ts.bytes - ts.launches * 2 * capi.num_dofs(s_t.prob) * 4) < 1
    assert ts.total_ms > 0
    a0 = s_t.profile_read(0, True)
    assert a0.launches >= rt.iterations * (p + 2) and a0.total_ms > 0 and a0.bytes > 0
    # sampled: every 2nd outer iteration
    s_t.profile_enable(True, 2)
    rt2 = s_t.solve(bd.data_ptr(), xt.data_ptr())
    ts2 = s_t.profile_read_tsolve(True)
    assert ts2.launches == ((rt2.iterations + 1) // 2) * p * d
    s_t.profile_enable(False)


# alpha != 1, including beta > alpha (the curl weight below the div weight)
ALPHA_CASES = [(2, 3, 24, 2.5, 0.05), (3, 2, 10, 0.4, 3.0), (2, 2, 30, 0.3, 7.0)]


@pytest.mark.parametrize("case", ALPHA_CASES, ids=[f"d{c[0]}p{c[1]}n{c[2]}a{c[3]}b{c[4]}" for c in ALPHA_CASES])
def test_alpha_not_one(case):
    d, p, n, alpha, beta = case
    opt = capi.options(coarse_max_dofs=200, rtol=1e-12)
    s = capi.Solver(capi.problem(d, p, n, alpha, beta), opt, stream())
    m = method.Method(d, p, n, alpha, beta, coarse_max_dofs=200, nu=opt.cheb_degree,
                      nu_coarse=s.coarse_degree(),
                      ratio=opt.cheb_ratio, lanczos_steps=opt.lanczos_steps)
    assert s.num_levels() == len(m.levels)
    rng = np.random.default_rng(23)
    for l, L in enumerate(m.levels):
        x = rng.uniform(-1, 1, L.K.shape[0])
        xd, y = dev(x), empty(L.K.shape[0])
        s.apply(l, xd.data_ptr(), y.data_ptr())
        assert relerr(host(y), L.K @ x) <= 1e-12, l
        if l + 1 < len(m.levels):
            assert abs(s.get_lambda(l) - L.lam) <= 1e-10 * L.lam, l
    r = rng.uniform(-1, 1, m.K.shape[0])
    rd, z = dev(r), empty(m.K.shape[0])
    s.precondition(rd.data_ptr(), z.data_ptr())
    assert relerr(host(z), m.vcycle(r)) <= 1e-10
    x = empty(m.K.shape[0])
    res = s.solve(rd.data_ptr(), x.data_ptr())
    assert res.status == capi.CD_OK
    assert relerr(host(x), solvers.solve_direct(m.K, r)) <= 1e-9
    s.close()


@pytest.mark.parametrize("d,p,n,beta", [(2, 2, 10, 0.05), (3, 2, 4, 0.1)])
def test_kappa_estimate_against_the_spectrum(d, p, n, beta):
    # Unpreconditioned CG: the Lanczos matrix of its coefficients has Ritz
    # values inside the spectrum of A, reaching its ends once CG has run long
    # enough; with a linear SPD preconditioner (the V-cycle without the Krylov
    # post-smoother) the same holds for B A, B the oracle's V-cycle matrix.
    K = asm.curl_div_matrix(d, p, n, 1.0, beta)
    N = K.shape[0]
    ev = np.linalg.eigvalsh(K.toarray())
    b = np.random.default_rng(31).uniform(-1, 1, N)
    bd, x = dev(b), empty(N)
    opt = capi.options(method=capi.CD_METHOD_CG, rtol=1e-13, max_iter=5000)
    s = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
    r = s.solve(bd.data_ptr(), x.data_ptr())
    kap = ev[-1] / ev[0]
    assert r.status == capi.CD_OK
    assert 0.9 * kap <= r.kappa_estimate <= kap * (1 + 1e-6), (r.kappa_estimate, kap)
    s.close()
    kw = dict(krylov_steps=0, cheb_degree=3, cheb_ratio=30.0, cheb_degree_coarse=0, coarse_max_dofs=60)
    opt = capi.options(rtol=1e-13, **kw)
    s = capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())
    r = s.solve(bd.data_ptr(), x.data_ptr())
    m = method.Method(d, p, n, 1.0, beta, coarse_max_dofs=60, nu=3, ratio=30.0, krylov_steps=0,
                      lanczos_steps=opt.lanczos_steps)
    B = np.column_stack([m.vcycle(e) for e in np.eye(N)])
    evb = np.sort(np.linalg.eigvals(B @ K.toarray()).real)
    kapb = evb[-1] / evb[0]
    assert r.status == capi.CD_OK
    assert 0.8 * kapb <= r.kappa_estimate <= kapb * (1 + 1e-3), (r.kappa_estimate, kapb)
    s.close()
