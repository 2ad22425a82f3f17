"""Load vectors of the manufactured solutions used in the numerical examples
of Sec. 6.2, and the L2 error of a discrete field against them.

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


def _axes(d, p, n):
    """Per-axis quadrature points, weights, and Dirichlet basis values and
    derivatives there ((p+3)-point Gauss-Legendre per element); n is the
    interval count of every axis or one per axis."""
    ns = [n] * d if np.isscalar(n) else list(n)
    out = []
    for nl in ns:
        x, w = gauss_points(nl, p + 3)
        out.append((x, w, basis(nl, p, x)[:, 1 : nl + p - 1], basis_deriv(nl, p, x)[:, 1 : nl + p - 1]))
    return out


def load_vector(d, p, n, alpha, beta):
    """Load vector in the component-major layout of the system matrix
    (n: intervals of every axis, or one count per axis)."""
    ax = _axes(d, p, n)
    X = np.meshgrid(*[a[0] for a in ax], indexing="ij")
    W = np.prod(np.meshgrid(*[a[1] for a in ax], indexing="ij"), axis=0)
    Bs = [[a[2] for a in ax], [a[3] for a in ax]]  # [value or derivative][axis]
    J = _grad_u(d, X)
    div = sum(J[c][c] for c in range(d)) * W
    out = []
    if d == 2:
        curl = (J[1][0] - J[0][1]) * W

        def proj2(field, derivs):
            return np.einsum("ab,ai,bj->ij", field, Bs[derivs[0]][0], Bs[derivs[1]][1], optimize=True)

        # psi^1 = (phi, 0): curl = -d2 phi, div = d1 phi
        b1 = -alpha * proj2(curl, (0, 1)) + beta * proj2(div, (1, 0))
        # psi^2 = (0, phi): curl = d1 phi, div = d2 phi
        b2 = alpha * proj2(curl, (1, 0)) + beta * proj2(div, (0, 1))
        out = [b1, b2]
    elif d == 3:
        cu = [(J[2][1] - J[1][2]) * W, (J[0][2] - J[2][0]) * W, (J[1][0] - J[0][1]) * W]

        def proj(field, derivs):
            ops = [Bs[k][l] for l, k in enumerate(derivs)]
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


def load_vector_rows(d, p, n, alpha, beta, rows):
    """Selected entries of the load vector (flat indices), each summed over
    the quadrature points of its basis function's support only: for checking
    full-size results on samples."""
    ax = _axes(d, p, n)
    ms = [a[2].shape[1] for a in ax]
    G = int(np.prod(ms))
    qn = p + 3
    out = np.empty(len(rows))
    for r, flat in enumerate(rows):
        c, rem = divmod(int(flat), G)
        idx = np.unravel_index(rem, ms)
        sl = []
        for l, i in enumerate(idx):  # Dirichlet function i = full function i+1, on elements i+1-p .. i+1
            nl = ax[l][0].size // qn
            e0, e1 = max(0, i + 1 - p), min(nl - 1, i + 1)
            sl.append(slice(e0 * qn, (e1 + 1) * qn))
        X = np.meshgrid(*[ax[l][0][sl[l]] for l in range(d)], indexing="ij")
        W = np.prod(np.meshgrid(*[ax[l][1][sl[l]] for l in range(d)], indexing="ij"), axis=0)
        J = _grad_u(d, X)
        val = [ax[l][2][sl[l], idx[l]] for l in range(d)]
        der = [ax[l][3][sl[l], idx[l]] for l in range(d)]

        def tens(ds):  # product of value / derivative factors on the local grid
            f = [der[l] if ds[l] else val[l] for l in range(d)]
            return np.prod(np.meshgrid(*f, indexing="ij"), axis=0)

        # grad of the test function phi e_c, component j: tens with the derivative on axis j
        gphi = [tens(tuple(1 if l == j else 0 for l in range(d))) for j in range(d)]
        div_u = sum(J[e][e] for e in range(d))
        if d == 2:
            curl_u = J[1][0] - J[0][1]
            curl_psi = -gphi[1] if c == 0 else gphi[0]  # (phi, 0): -d2 phi; (0, phi): d1 phi
            val_ = alpha * curl_u * curl_psi + beta * div_u * gphi[c]
        else:
            cu = [J[2][1] - J[1][2], J[0][2] - J[2][0], J[1][0] - J[0][1]]
            # curl(phi e_c) = grad phi x e_c
            e = np.zeros(3)
            e[c] = 1.0
            cp = [gphi[(k + 1) % 3] * e[(k + 2) % 3] - gphi[(k + 2) % 3] * e[(k + 1) % 3] for k in range(3)]
            val_ = alpha * sum(cu[k] * cp[k] for k in range(3)) + beta * div_u * gphi[c]
        out[r] = float(np.sum(W * val_))
    return out


def l2_error(d, p, n, x):
    """||u - u_h||_{L2((0,1)^d)} of the discrete field with coefficients x
    (component-major, Dirichlet basis) against the manufactured solution,
    by (p+3)-point Gauss-Legendre quadrature per element and direction."""
    ax = _axes(d, p, n)
    ms = [a[2].shape[1] for a in ax]
    G = int(np.prod(ms))
    X = np.meshgrid(*[a[0] for a in ax], indexing="ij")
    W = np.prod(np.meshgrid(*[a[1] for a in ax], indexing="ij"), axis=0)
    g = np.prod([t * (1 - t) for t in X], axis=0)
    u = [np.sin(2 * np.pi * g), np.cos(2 * np.pi * g) - 1]
    if d == 3:
        u.append(u[0] + u[1])
    B = [a[2] for a in ax]
    total = 0.0
    for c in range(d):
        C = x[c * G : (c + 1) * G].reshape(ms)
        if d == 2:
            uh = np.einsum("ai,bj,ij->ab", B[0], B[1], C, optimize=True)
        else:
            uh = np.einsum("ai,bj,ck,ijk->abc", B[0], B[1], B[2], C, optimize=True)
        total += float(np.sum(W * (u[c] - uh) ** 2))
    return np.sqrt(total)
