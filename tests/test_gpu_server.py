"""GPU tests of the serving loop: continuous batching of independent solves."""
import numpy as np
import pytest

from tests.gpu_util import dev, empty, gpu_ok, host, relerr, stream, torch

pytestmark = pytest.mark.gpu

if not gpu_ok():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import assembly, solvers  # noqa: E402
from paper_1805_10058_amd import capi  # noqa: E402

MIX = [  # (dim, p, n, beta, precision)
    (2, 2, 32, 0.1, capi.CD_FP64),
    (2, 3, 40, 1e-2, capi.CD_MIXED_FP32),
    (3, 2, 12, 0.5, capi.CD_FP64),
    (2, 4, 24, 1.0, capi.CD_MIXED_FP32),
    (3, 3, 10, 1e-3, capi.CD_MIXED_FP32),
    (2, 1, 48, 0.05, capi.CD_FP64),
]


def _run_server(reqs, budget=0, max_active=0, streams=0, tol=1e-10, seeds=None):
    srv = capi.Server(hbm_budget_bytes=budget, max_active=max_active, num_streams=streams)
    bufs, tickets = [], {}
    for i, (d, p, n, beta, prec) in enumerate(reqs):
        prob = capi.problem(d, p, n, 1.0, beta)
        opt = capi.options(precision=prec, rtol=tol, coarse_max_dofs=300)
        seed = 100 + (seeds[i] if seeds is not None else i)
        b = np.random.default_rng(seed).uniform(-1, 1, capi.num_dofs(prob))
        bd, x = dev(b), empty(b.size)
        bufs.append((b, bd, x, prob))
        torch.cuda.synchronize()
        tickets[srv.submit(prob, opt, bd.data_ptr(), x.data_ptr())] = i
    out = {}
    peak_active = 0
    for _ in range(100000):
        a, q = srv.step()
        peak_active = max(peak_active, a)
        for c in srv.poll():
            out[tickets[c.ticket]] = c
        if a == 0 and q == 0:
            break
    srv.close()
    return out, bufs, peak_active


def test_each_result_same_alone_and_in_mix():
    mix, bufs, peak = _run_server(MIX)
    assert peak >= 2  # work of different requests was in flight together
    for i, req in enumerate(MIX):
        alone, abufs, _ = _run_server([req], seeds=[i])
        c, ca = mix[i], alone[0]
        assert c.result.status == capi.CD_OK and ca.result.status == capi.CD_OK
        assert c.result.iterations == ca.result.iterations
        xm, xa = host(bufs[i][2]), host(abufs[0][2])
        np.testing.assert_array_equal(xm, xa)  # bitwise: no cross-request arithmetic
        # and the answer is the solution of the system (oracle direct solve)
        d, p, n, beta, prec = req
        K = assembly.curl_div_matrix(d, p, n, 1.0, beta)
        xd = solvers.solve_direct(K, bufs[i][0])
        assert np.linalg.norm(bufs[i][0] - K @ xm) <= 1.01e-10 * np.linalg.norm(bufs[i][0])
        assert relerr(xm, xd) <= 1e-5


def test_admission_respects_budget_and_slots():
    reqs = [(2, 2, 32, 0.1, capi.CD_FP64)] * 6
    prob = capi.problem(2, 2, 32, 1.0, 0.1)
    fp = capi.footprint_bytes(prob, capi.options(rtol=1e-10, coarse_max_dofs=300))
    assert fp > 0
    out, _, peak = _run_server(reqs, budget=2 * fp + fp // 2, max_active=8)
    assert peak <= 2  # only two fit in the budget at a time
    assert len(out) == 6 and all(c.result.status == capi.CD_OK for c in out.values())
    for c in out.values():
        assert c.t_submit <= c.t_admit <= c.t_done
    out, _, peak = _run_server(reqs, max_active=3)
    assert peak <= 3 and len(out) == 6


def test_request_larger_than_budget_is_refused():
    srv = capi.Server(hbm_budget_bytes=1 << 20)
    prob = capi.problem(3, 3, 32, 1.0, 0.1)
    b, x = empty(capi.num_dofs(prob)), empty(capi.num_dofs(prob))
    with pytest.raises(capi.CurldivError) as e:
        srv.submit(prob, capi.options(), b.data_ptr(), x.data_ptr())
    assert e.value.code == capi.CD_ENOMEM
    with pytest.raises(capi.CurldivError) as e:
        srv.submit(capi.problem(3, 3, 32, 1.0, -1.0), capi.options(), b.data_ptr(), x.data_ptr())
    assert e.value.code == capi.CD_EINVAL
    srv.close()


@pytest.mark.parametrize("case", [(2, 3, 64, capi.CD_MIXED_FP32), (2, 6, 40, capi.CD_FP64),
                                  (3, 2, 20, capi.CD_FP64), (3, 4, 12, capi.CD_MIXED_FP32)])
def test_footprint_covers_device_bytes(case):
    # the server admits by cd_footprint_bytes: it must cover what a solver
    # really holds (and not overstate it grossly)
    d, p, n, prec = case
    prob = capi.problem(d, p, n, 1.0, 0.1)
    opt = capi.options(precision=prec)
    fp = capi.footprint_bytes(prob, opt)
    s = capi.Solver(prob, opt, stream())
    b = np.random.default_rng(0).uniform(-1, 1, capi.num_dofs(prob))
    bd, x = dev(b), empty(b.size)
    s.solve(bd.data_ptr(), x.data_ptr())
    held = s.device_bytes()
    assert held <= fp <= 2 * held + (2 << 20)
    s.close()
