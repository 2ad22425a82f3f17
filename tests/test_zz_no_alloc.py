"""cd_tsolve_noalloc (the T-solve entry point for callers that cannot
allocate) against cd_tsolve, through the C ABI: the same kernels, so the
results must be bitwise equal; two calls in a row share the static
workspace, the second on a smaller problem; in-place calls; the size limit."""
import numpy as np
import pytest

from tests.gpu_util import dev, empty, gpu_ok, host, stream

pytestmark = pytest.mark.gpu

MAX_DOFS = 1 << 20


def _solver(d, p, n):
    from paper_1805_10058_amd import capi

    opt = capi.options(method=capi.CD_METHOD_CG)  # the T factor is built for every method
    return capi.Solver(capi.problem(d, p, n, 1.0, 0.1), opt, stream())


@pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")
def test_noalloc_tsolve_equals_tsolve_twice_in_a_row():
    from paper_1805_10058_amd import capi

    # first a larger 3D problem, then a smaller 2D one: the second call must
    # not see anything the first left in the shared workspace
    for (d, p, n), seed in (((3, 3, 40), 1), ((2, 4, 30), 2)):
        s = _solver(d, p, n)
        N = capi.num_dofs(s.prob)
        print(f"noalloc case d={d} p={p} n={n} N={N}", flush=True)
        v = np.random.default_rng(seed).uniform(-1, 1, N)
        vd = dev(v)
        z_ref, z_new = empty(N), empty(N)
        z_new.fill_(np.nan)
        s.tsolve(vd.data_ptr(), z_ref.data_ptr())
        s.tsolve_noalloc(vd.data_ptr(), z_new.data_ptr())
        a, b = host(z_ref), host(z_new)
        assert np.array_equal(a, b), np.abs(a - b).max()
        # in place
        zi = dev(v)
        s.tsolve_noalloc(zi.data_ptr(), zi.data_ptr())
        assert np.array_equal(host(zi), a)
        assert np.array_equal(host(vd), v)  # input untouched
        s.close()


@pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")
def test_noalloc_tsolve_rejects_problems_beyond_the_workspace():
    from paper_1805_10058_amd import capi

    s = _solver(2, 2, 1024)  # 2 * 1024^2 unknowns
    N = capi.num_dofs(s.prob)
    assert N > MAX_DOFS
    v, z = empty(N), empty(N)
    with pytest.raises(RuntimeError, match="static workspace"):
        s.tsolve_noalloc(v.data_ptr(), z.data_ptr())
    s.close()
