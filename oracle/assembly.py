"""Block matrices of the curl-div problem and their Kronecker-form apply.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Vector layout (Sec. 4.1): component-major; inside a component the unknowns
u_{i_1,...,i_d}, i_l = 2..n+p-1, are ordered lexicographically with i_1
slowest, which is the row ordering of the Kronecker product X_1 (x) ... (x) X_d.
"""
import numpy as np
import scipy.sparse as sp

from .matrices import mass_adv_stiff


def _kron(*mats):
    out = sp.csr_matrix(mats[0])
    for X in mats[1:]:
        out = sp.kron(out, sp.csr_matrix(X), format="csr")
    return out


def curl_div_matrix(d, p, n, alpha, beta, mats=None):
    """The system matrix alpha*A^{curl} + beta*A^{div}, written term by term as
    in Sec. 4.1 (d = 2, 2x2 blocks) and Sec. 4.2 (d = 3, 3x3 blocks).
    ``mats`` may supply the 1D (M, A, S) triple (default: assembled at n, p).
    Returns a scipy CSR matrix of size d*m^d."""
    M, A, S = mats if mats is not None else mass_adv_stiff(n, p)
    At = A.T
    if d == 2:
        curl = [
            [_kron(M, S), -_kron(At, A)],
            [-_kron(A, At), _kron(S, M)],
        ]
        div = [
            [_kron(S, M), _kron(A, At)],
            [_kron(At, A), _kron(M, S)],
        ]
    elif d == 3:
        curl = [
            [_kron(M, M, S) + _kron(M, S, M), -_kron(At, A, M), -_kron(At, M, A)],
            [-_kron(A, At, M), _kron(S, M, M) + _kron(M, M, S), -_kron(M, At, A)],
            [-_kron(A, M, At), -_kron(M, A, At), _kron(S, M, M) + _kron(M, S, M)],
        ]
        div = [
            [_kron(S, M, M), _kron(A, At, M), _kron(A, M, At)],
            [_kron(At, A, M), _kron(M, S, M), _kron(M, A, At)],
            [_kron(At, M, A), _kron(M, At, A), _kron(M, M, S)],
        ]
    else:
        raise ValueError("d must be 2 or 3")
    Kc = sp.bmat(curl, format="csr")
    Kd = sp.bmat(div, format="csr")
    return (alpha * Kc + beta * Kd).tocsr()


def simplified_blocks(d, alpha, beta):
    """Block structure obtained from the literal form using A^T = -A
    (skew-symmetry, Sec. 3.2): block (c,c) = beta*D_c + alpha*sum_{e!=c} D_e,
    where D_e has S on axis e and M elsewhere; block (c,e), e != c, equals
    (alpha-beta) times the product with A on axes c and e and M elsewhere.
    Returned as {(c, e): [(coef, (X_1, ..., X_d)), ...]} with X in 'MAS'."""
    blocks = {}
    for c in range(d):
        terms = []
        for e in range(d):
            coef = beta if e == c else alpha
            terms.append((coef, tuple("S" if l == e else "M" for l in range(d))))
        blocks[(c, c)] = terms
        for e in range(d):
            if e != c:
                blocks[(c, e)] = [
                    (alpha - beta, tuple("A" if l in (c, e) else "M" for l in range(d)))
                ]
    return blocks


def kron_apply_axis(X, U, axis):
    """Apply the 1D matrix X along ``axis`` of the tensor U (the Kronecker
    identity (I (x) X (x) I) vec(U) = vec(U x_axis X))."""
    return np.moveaxis(np.tensordot(X, U, axes=([1], [axis])), 0, axis)


def kron_apply(mats1d, x, d, alpha, beta):
    """Matrix-free y = K x from the simplified block form, one Kronecker
    product at a time (no fusion).  ``mats1d`` is {'M': M, 'A': A, 'S': S}
    (1D matrices of size m) or a list of such dicts, one per axis."""
    if isinstance(mats1d, dict):
        mats1d = [mats1d] * d
    shape = tuple(mats1d[l]["M"].shape[0] for l in range(d))
    G = int(np.prod(shape))
    xs = [x[c * G : (c + 1) * G].reshape(shape) for c in range(d)]
    y = np.zeros_like(x)
    for (c, e), terms in simplified_blocks(d, alpha, beta).items():
        acc = np.zeros(shape)
        for coef, names in terms:
            U = xs[e]
            for l in range(d):
                U = kron_apply_axis(mats1d[l][names[l]], U, l)
            acc += coef * U
        y[c * G : (c + 1) * G] += acc.ravel()
    return y
