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


def axis_matrices(d, p, n, mats=None):
    """Per-axis 1D (M, A, S) triples: ``n`` is one interval count for every
    axis or one per axis (n_l = nu_l n in Sec. 5); ``mats`` may supply one
    triple for every axis or a list of d triples."""
    if mats is not None:
        if len(mats) == 3 and not isinstance(mats[0], (list, tuple)):
            return [tuple(mats)] * d
        return [tuple(t) for t in mats]
    ns = [n] * d if np.isscalar(n) else list(n)
    return [mass_adv_stiff(int(nl), p) for nl in ns]


def curl_div_matrix(d, p, n, alpha, beta, mats=None):
    """The system matrix alpha*A^{curl} + beta*A^{div}, written term by term as
    in Sec. 4.1 (d = 2, 2x2 blocks) and Sec. 4.2 (d = 3, 3x3 blocks): every
    block is a sum of Kronecker products X_1 (x) ... (x) X_d of 1D matrices of
    the axes 1..d in order.  ``n`` is the number of intervals of every axis or
    one per axis; ``mats`` may supply the 1D (M, A, S) triple(s).
    Returns a scipy CSR matrix of size d * prod_l m_l."""
    ax = axis_matrices(d, p, n, mats)
    M = [t[0] for t in ax]
    A = [t[1] for t in ax]
    S = [t[2] for t in ax]
    At = [X.T for X in A]
    if d == 2:
        curl = [
            [_kron(M[0], S[1]), -_kron(At[0], A[1])],
            [-_kron(A[0], At[1]), _kron(S[0], M[1])],
        ]
        div = [
            [_kron(S[0], M[1]), _kron(A[0], At[1])],
            [_kron(At[0], A[1]), _kron(M[0], S[1])],
        ]
    elif d == 3:
        curl = [
            [_kron(M[0], M[1], S[2]) + _kron(M[0], S[1], M[2]), -_kron(At[0], A[1], M[2]), -_kron(At[0], M[1], A[2])],
            [-_kron(A[0], At[1], M[2]), _kron(S[0], M[1], M[2]) + _kron(M[0], M[1], S[2]), -_kron(M[0], At[1], A[2])],
            [-_kron(A[0], M[1], At[2]), -_kron(M[0], A[1], At[2]), _kron(S[0], M[1], M[2]) + _kron(M[0], S[1], M[2])],
        ]
        div = [
            [_kron(S[0], M[1], M[2]), _kron(A[0], At[1], M[2]), _kron(A[0], M[1], At[2])],
            [_kron(At[0], A[1], M[2]), _kron(M[0], S[1], M[2]), _kron(M[0], A[1], At[2])],
            [_kron(At[0], M[1], A[2]), _kron(M[0], At[1], A[2]), _kron(M[0], M[1], S[2])],
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


def kron_apply_rows(mats1d, x, d, alpha, beta, rows):
    """Selected entries (K x)_i, i in ``rows`` (flat indices in the
    component-major layout), from the simplified block form, one entry at a
    time: entry (c, i_1..i_d) of block (c, e) term X_1 (x) ... (x) X_d is
    sum_j prod_l X_l[i_l, j_l] x_e[j_1..j_d].  For checking full-size results
    on samples without forming K.  ``mats1d`` as for kron_apply."""
    if isinstance(mats1d, dict):
        mats1d = [mats1d] * d
    shape = tuple(mats1d[l]["M"].shape[0] for l in range(d))
    G = int(np.prod(shape))
    xs = [x[c * G : (c + 1) * G].reshape(shape) for c in range(d)]
    blocks = simplified_blocks(d, alpha, beta)
    out = np.empty(len(rows))
    for r, flat in enumerate(rows):
        c, rem = divmod(int(flat), G)
        idx = np.unravel_index(rem, shape)
        acc = 0.0
        for e in range(d):
            for coef, names in blocks[(c, e)]:
                U = xs[e]
                for l in range(d):  # contract axis l with row idx[l] of its matrix (its nonzero span)
                    row = mats1d[l][names[l]][idx[l]]
                    nz = np.nonzero(row)[0]
                    if nz.size == 0:
                        U = None
                        break
                    lo, hi = nz[0], nz[-1] + 1
                    U = np.tensordot(row[lo:hi], U[lo:hi], axes=([0], [0]))
                if U is not None:
                    acc += coef * float(U)
        out[r] = acc
    return out
