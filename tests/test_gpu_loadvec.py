"""The manufactured-solution load vector and the L2 error on the GPU
(cd_load_vector, cd_l2_error; Sec. 6.2) against the oracle, and the
discretization error of GPU solutions converging at order p + 1.

Tolerances: the load vector is a sum of positive-weight quadrature terms of
bounded fields; FP64 rounding of the sum-factorized order against the
oracle's is below 1e-13 relative to the largest entry.  The L2 error is a
square root of a sum of squares: relative 1e-10 (the squares of differences
lose up to half the digits where u_h is close to u).
"""
import numpy as np
import pytest

from tests.gpu_util import dev, empty, gpu_ok, host, stream

pytestmark = pytest.mark.gpu

if not gpu_ok():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import loadvec  # noqa: E402
from paper_1805_10058_amd import capi  # noqa: E402


def _solver(d, p, n, beta=0.1, **kw):
    opt = capi.options(rtol=1e-12, **kw)
    return capi.Solver(capi.problem(d, p, n, 1.0, beta), opt, stream())


@pytest.mark.parametrize("d,p,n,beta", [(2, 2, 16, 0.1), (2, 3, (24, 40), 0.01), (3, 2, 8, 0.1),
                                        (3, 3, (6, 8, 10), 1e-3), (2, 5, 12, 1.0)])
def test_load_vector_and_l2_error(d, p, n, beta):
    s = _solver(d, p, n, beta)
    N = capi.num_dofs(s.prob)
    b = empty(N)
    s.load_vector(b.data_ptr())
    ref = loadvec.load_vector(d, p, n, 1.0, beta)
    got = host(b)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    x = np.random.default_rng(61).uniform(-1, 1, N) * 1e-2
    e = s.l2_error(dev(x).data_ptr())
    e_ref = loadvec.l2_error(d, p, n, x)
    assert abs(e - e_ref) <= 1e-10 * e_ref
    s.close()


def test_load_vector_full_size_samples():
    # 3D p=3 n=128 (6,440,067 unknowns): sampled entries (boundary and
    # interior of each component) against the oracle's entry-by-entry sums
    d, p, n, beta = 3, 3, 128, 1e-6
    s = _solver(d, p, n, beta)
    N = capi.num_dofs(s.prob)
    b = empty(N)
    s.load_vector(b.data_ptr())
    G = N // 3
    rng = np.random.default_rng(62)
    rows = np.unique(np.concatenate([np.arange(0, 300), G + np.arange(0, 300), 2 * G - 300 + np.arange(300),
                                     N - 300 + np.arange(300), rng.integers(0, N, 300)]))
    ref = loadvec.load_vector_rows(d, p, n, 1.0, beta, rows)
    got = host(b)[rows]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    s.close()


@pytest.mark.parametrize("d,p,ns", [(2, 2, (16, 32, 64)), (2, 3, (16, 32, 64)), (3, 2, (8, 16, 32))])
def test_gpu_solutions_converge_at_order_p_plus_1(d, p, ns):
    # the discretization error of the solutions the GPU solver computes from the
    # GPU load vector: ||u - u_h|| falls like h^(p+1)
    errs = []
    for n in ns:
        s = _solver(d, p, n, 0.1)
        N = capi.num_dofs(s.prob)
        b, x = empty(N), empty(N)
        s.load_vector(b.data_ptr())
        res = s.solve(b.data_ptr(), x.data_ptr())
        assert res.status == capi.CD_OK
        errs.append(s.l2_error(x.data_ptr()))
        s.close()
    print(f"L2 errors {d}D p={p} n={ns}: {errs}")
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 >= 0.85 * 2 ** (p + 1), errs
