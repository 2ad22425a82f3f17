"""Load vectors of the manufactured solutions used in the numerical examples
of Sec. 6.2.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

2D: u = (sin(2 pi g), cos(2 pi g) - 1), g = x1(1-x1) x2(1-x2).
3D: u = (sin(2 pi g), cos(2 pi g) - 1, u1 + u2), g = prod_i x_i(1-x_i).
Both fields vanish on the boundary, so the load vector of f = L_{alpha,beta} u
against a test field psi in the Dirichlet space equals
alpha (curl u, curl psi) + beta (div u, div psi) (integration by parts of the
weak form of the curl-div operator, Sec. 1); only first derivatives of u are
needed.  Quadrature: (p+3)-point Gauss-Legendre per element and direction.
"""
import numpy as np

from .bspline import basis, basis_deriv
from .matrices import gauss_points


def _grad_u(d, X):
    """Jacobian du_c/dx_j of the manufactured field at points X (list of d
    arrays).  Returns J with J[c][j] an array like X[0]."""
    f = [x * (1 - x) for x in X]
    df = [1 - 2 * x for x in X]
    g = np.prod(f, axis=0)
    dg = []
    for j in range(d):
        t = df[j].copy()
        for l in range(d):
            if l != j:
                t = t * f[l]
        dg.append(t)
    c1 = 2 * np.pi * np.cos(2 * np.pi * g)
    c2 = -2 * np.pi * np.sin(2 * np.pi * g)
    J = [[c1 * dg[j] for j in range(d)], [c2 * dg[j] for j in range(d)]]
    if d == 3:
        J.append([J[0][j] + J[1][j] for j in range(d)])
    return J


def load_vector(d, p, n, alpha, beta):
    """Load vector in the component-major layout of the system matrix."""
    x, w = gauss_points(n, p + 3)
    B = basis(n, p, x)[:, 1 : n + p - 1]
    Dv = basis_deriv(n, p, x)[:, 1 : n + p - 1]
    X = np.meshgrid(*([x] * d), indexing="ij")
    W = np.prod(np.meshgrid(*([w] * d), indexing="ij"), axis=0)
    J = _grad_u(d, X)
    div = sum(J[c][c] for c in range(d)) * W
    out = []
    if d == 2:
        curl = (J[1][0] - J[0][1]) * W
        # psi^1 = (phi, 0): curl = -d2 phi, div = d1 phi
        b1 = -alpha * np.einsum("ab,ai,bj->ij", curl, B, Dv, optimize=True) + beta * np.einsum("ab,ai,bj->ij", div, Dv, B, optimize=True)
        # psi^2 = (0, phi): curl = d1 phi, div = d2 phi
        b2 = alpha * np.einsum("ab,ai,bj->ij", curl, Dv, B, optimize=True) + beta * np.einsum("ab,ai,bj->ij", div, B, Dv, optimize=True)
        out = [b1, b2]
    elif d == 3:
        cu = [(J[2][1] - J[1][2]) * W, (J[0][2] - J[2][0]) * W, (J[1][0] - J[0][1]) * W]
        Bs = [B, Dv]

        def proj(field, derivs):
            ops = [Bs[k] for k in derivs]
            return np.einsum("abc,ai,bj,ck->ijk", field, *ops, optimize=True)

        # psi^c = phi e_c: curl psi^c = grad phi x e_c; div psi^c = d_c phi
        # e1: curl = (0, d3 phi, -d2 phi); e2: (-d3 phi, 0, d1 phi); e3: (d2 phi, -d1 phi, 0)
        b1 = alpha * (proj(cu[1], (0, 0, 1)) - proj(cu[2], (0, 1, 0))) + beta * proj(div, (1, 0, 0))
        b2 = alpha * (-proj(cu[0], (0, 0, 1)) + proj(cu[2], (1, 0, 0))) + beta * proj(div, (0, 1, 0))
        b3 = alpha * (proj(cu[0], (0, 1, 0)) - proj(cu[1], (1, 0, 0))) + beta * proj(div, (0, 0, 1))
        out = [b1, b2, b3]
    else:
        raise ValueError("d must be 2 or 3")
    return np.concatenate([o.ravel() for o in out])
