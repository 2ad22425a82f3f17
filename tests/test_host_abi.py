"""Host-side checks of the C-ABI library (no GPU): every function the header
declares is exported and bound, the binding's structures have the header's
layout, and the host logic (defaults, option validation, unknown counts,
footprint estimate) behaves as documented."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from oracle import assembly
from paper_1805_10058_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "curldiv.h")


def declared_functions():
    text = open(HEADER).read()
    return set(re.findall(r"^(?:const\s+)?(?:int|void|size_t|char\s*\*)\s*\**\s*(cd_\w+)\s*\(", text, re.M))


def test_every_declared_function_is_exported_and_bound():
    names = declared_functions()
    assert len(names) >= 30
    assert names == set(capi.SIGNATURES), names ^ set(capi.SIGNATURES)
    lib = ctypes.CDLL(capi.LIB_PATH)
    for name in sorted(names):
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="no fallback"):
        capi.load(str(tmp_path / "libcurldiv.so"))


STRUCTS = [capi.cd_problem, capi.cd_options, capi.cd_result, capi.cd_kernel_stats, capi.cd_server_options,
           capi.cd_completion]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a C compiler")
def test_binding_structs_have_the_header_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "curldiv.h"', 'int main(void) {']
    expect = []
    for S in STRUCTS:
        lines.append(f'printf("%zu\\n", sizeof({S.__name__}));')
        expect.append(ctypes.sizeof(S))
        for f in S._fields_:
            lines.append(f'printf("%zu\\n", offsetof({S.__name__}, {f[0]}));')
            expect.append(getattr(S, f[0]).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_default_options():
    o = capi.options()
    assert (o.method, o.transfer, o.precision) == (capi.CD_METHOD_PMIM, capi.CD_XFER_KNOT, capi.CD_FP64)
    assert o.rtol == 1e-8 and o.max_iter == 10000 and o.coarse_max_dofs == 2500
    assert (o.cheb_degree, o.cheb_degree_coarse, o.cheb_ratio, o.lanczos_steps) == (48, -1, 1000.0, 20)
    assert o.krylov_steps < 0 and o.graphs == 1
    assert o.eig_bounds == capi.CD_BOUNDS_LANCZOS and o.bound_safety == 0.0
    assert o.apply3d_kernel == capi.CD_APPLY3D_AUTO and o.apply_x1_chunk == 0


@pytest.mark.parametrize("field,value", [
    ("cheb_degree", 0), ("cheb_degree", 129), ("cheb_degree_coarse", 129), ("lanczos_steps", 0),
    ("lanczos_steps", 201), ("cheb_ratio", 1.0), ("rtol", 0.0), ("max_iter", 0), ("precision", 7),
    ("method", 9), ("transfer", 5), ("eig_bounds", 2), ("bound_safety", 0.5), ("bound_safety", 11.0),
    ("apply3d_kernel", -1), ("apply3d_kernel", 4), ("apply_x1_chunk", -1),
])
def test_invalid_options_are_rejected(field, value):
    prob = capi.problem(2, 3, 32, 1.0, 0.1)
    assert capi.validate(prob, capi.options()) == capi.CD_OK
    assert capi.validate(prob, capi.options(**{field: value})) == capi.CD_EINVAL
    assert capi.lib().cd_last_error()


@pytest.mark.parametrize("args", [(0, 3, 8), (4, 3, 8), (2, 0, 8), (2, 3, 0), (2, 9, 8)])
def test_invalid_problems_are_rejected(args):
    d, p, n = args
    prob = capi.cd_problem(d, p, (ctypes.c_int * 3)(n, n, n), 1.0, 0.1)
    assert capi.validate(prob, capi.options()) == capi.CD_EINVAL


def test_negative_beta_is_rejected():
    assert capi.validate(capi.problem(2, 3, 8, 1.0, -1.0), capi.options()) == capi.CD_EINVAL


@pytest.mark.parametrize("d,p,n", [(2, 1, 5), (2, 3, 16), (2, 6, 9), (3, 2, 4), (3, 4, 3)])
def test_num_dofs_matches_the_assembled_system(d, p, n):
    K = assembly.curl_div_matrix(d, p, n, 1.0, 0.5)
    assert capi.num_dofs(capi.problem(d, p, n, 1.0, 0.5)) == K.shape[0]


def test_footprint_grows_with_size_and_precision():
    o64, o32 = capi.options(), capi.options(precision=capi.CD_MIXED_FP32)
    prev = 0
    for n in (32, 64, 128, 256):
        prob = capi.problem(2, 3, n, 1.0, 1e-3)
        f64, f32 = capi.footprint_bytes(prob, o64), capi.footprint_bytes(prob, o32)
        N = capi.num_dofs(prob)
        assert f64 > 5 * N * 8 and f32 > 5 * N * 8
        assert f64 > f32
        assert f64 > prev
        prev = f64
    assert capi.footprint_bytes(capi.problem(2, 3, 32, 1.0, 0.1), capi.options(cheb_degree=0)) == 0


# The symbol bound is host logic (cd_symbol_bound runs without a device): it
# must equal the oracle's, which reads the symbol off the central rows of the
# assembled level operators (oracle/symbols.py, pinned against the paper's
# symbol in test_oracle_symbol_bound).  Cases: 2D and 3D, both transfers (the
# paper prolongator's Galerkin levels are not re-discretizations), P_WL (no
# off-diagonal blocks), an anisotropic grid, and levels too short for an
# interior row (bound 0, Lanczos takes over).
@pytest.mark.parametrize("d,p,n,alpha,beta,transfer,method", [
    (2, 3, 32, 1.0, 0.01, "knot", "P_MIM"), (3, 3, 16, 1.0, 1.0, "knot", "P_MIM"),
    (3, 2, (8, 12, 16), 1.0, 0.1, "knot", "P_MIM"), (2, 2, 30, 1.0, 0.1, "paper", "P_MIM"),
    (2, 3, 25, 1.0, 0.1, "knot", "P_WL"), (3, 4, 12, 0.5, 2.0, "knot", "P_MIM"),
])
def test_symbol_bound_matches_the_oracle(d, p, n, alpha, beta, transfer, method):
    from oracle import method as om
    from oracle import symbols
    meth = {"P_MIM": capi.CD_METHOD_PMIM, "P_WL": capi.CD_METHOD_PWL}[method]
    tr = capi.CD_XFER_KNOT if transfer == "knot" else capi.CD_XFER_PAPER
    opt = capi.options(transfer=tr, method=meth, eig_bounds=capi.CD_BOUNDS_SYMBOL, coarse_max_dofs=60)
    prob = capi.problem(d, p, n, alpha, beta)
    levels = om.build_hierarchy(d, p, n, alpha, beta, transfer=transfer, coarse_max_dofs=60,
                                blockdiag=(method == "P_WL"), lanczos_steps=2)
    for lvl, L in enumerate(levels[:-1]):
        got = capi.symbol_bound(prob, opt, lvl)
        if min(L.ms) < 2 * p + 1:
            assert got == 0.0
        else:
            ref = symbols.symbol_bound(L.K, d, L.ms, om.symbol_samples(d))
            assert abs(got - ref) <= 1e-13 * ref, (lvl, got, ref)
    with pytest.raises(capi.CurldivError):
        capi.symbol_bound(prob, opt, len(levels) - 1)
