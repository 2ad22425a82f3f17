"""Pins of the grid-transfer matrices (Sec. 6.1) and the coarse operators."""
import math

import numpy as np
import pytest

from oracle import bspline as bs
from oracle import matrices as mt
from oracle import transfer as tr


@pytest.mark.parametrize("p", range(1, 7))
@pytest.mark.parametrize("nf", [2, 4, 10, 16])
def test_knot_insertion_is_exact_embedding(nf, p):
    # coarse B-splines are exactly reproduced by fine B-splines
    P = tr.knot_insertion_prolongator(nf, p, full=True)
    x = np.random.default_rng(nf + p).random(300)
    np.testing.assert_allclose(bs.basis(nf, p, x) @ P, bs.basis(nf // 2, p, x), atol=1e-14)
    # partition of unity is preserved: columns sum to ... rows of P sum to 1
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 7))
def test_knot_insertion_interior_stencil(p):
    # two-scale relation of uniform B-splines: 2^{-p} C(p+1, k), k = 0..p+1
    nf = 4 * p + 16
    P = tr.knot_insertion_prolongator(nf, p)
    j = (nf // 2 + p - 2) // 2
    col = P[:, j]
    nz = col[np.abs(col) > 0]
    expect = np.array([math.comb(p + 1, k) for k in range(p + 2)]) / 2.0**p
    np.testing.assert_allclose(nz, expect, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 7))
def test_galerkin_equals_rediscretization(p):
    # with the knot-insertion prolongator, P^T X_n P = X_{n/2} (same Galerkin space)
    nf = 12
    P = tr.knot_insertion_prolongator(nf, p)
    fine = mt.mass_adv_stiff(nf, p)
    coarse = mt.mass_adv_stiff(nf // 2, p)
    for Xf, Xc in zip(fine, coarse):
        np.testing.assert_allclose(P.T @ Xf @ P, Xc, atol=1e-12 * max(1.0, np.abs(Xc).max()))


@pytest.mark.parametrize("m", [1, 2, 3, 7, 8, 15, 16])
def test_paper_prolongator(m):
    P = tr.paper_prolongator(m)
    assert P.shape == (m, m // 2)
    for j in range(m // 2):
        col = P[:, j]
        i = 2 * j + 1  # zero-based fine index of the coarse node
        assert col[i] == 1.0 and col[i - 1] == 0.5
        if i + 1 < m:
            assert col[i + 1] == 0.5
        assert np.count_nonzero(col) == (3 if i + 1 < m else 2)
    # P = T_m(1 + cos theta) K^T with K selecting the even (one-based) indices
    T = np.eye(m) + 0.5 * (np.eye(m, k=1) + np.eye(m, k=-1))
    K = np.zeros((m // 2, m))
    for j in range(m // 2):
        K[j, 2 * j + 1] = 1.0
    np.testing.assert_array_equal(P, T @ K.T)
