"""The paper's multi-iterative method with exact (sequential) Gauss-Seidel,
for iteration-count context (Sec. 6.1, setting of Sec. 6.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Setting of Sec. 6.2: V-cycle with the block prolongator I_d (x) P (x) ... (x) P
of the (1/2)[1 2 1] stencil, Galerkin coarse matrices, one forward
Gauss-Seidel pre-smoothing sweep on every level, p post-smoothing steps of
PGMRES (MIM, P_MIM) or PCG (P_WL) with preconditioner T at the finest level,
one Gauss-Seidel post-smoothing sweep on the other levels.  Levels are
coarsened until m = 1 (log2(n+p-1) levels when m = 2^k - 1), where the
system is solved exactly.  P_WL runs the same cycle on the block-diagonal
part D of A (Sec. 6.1).  The outer CG of P_MIM / P_WL is taken as flexible
CG (FCG(1)) because the Krylov post-smoother makes the cycle nonlinear.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import curl_div_matrix
from .method import _kron, gmres_T, pcg_T, t_operator
from .transfer import paper_prolongator


def _block_diag_part(K, d):
    G = K.shape[0] // d
    blocks = [K[c * G:(c + 1) * G, c * G:(c + 1) * G] for c in range(d)]
    return sp.block_diag(blocks, format="csr")


class PaperMIM:
    def __init__(self, d, p, n, alpha, beta, variant="P_MIM", K=None):
        self.d, self.p, self.variant = d, p, variant
        K = curl_div_matrix(d, p, n, alpha, beta) if K is None else K
        self.K = K
        A0 = _block_diag_part(K, d) if variant == "P_WL" else K
        m = n + p - 2
        self.ops, self.Ps, self.lower = [A0.tocsr()], [], []
        while m >= 2:
            P1 = paper_prolongator(m)
            Pb = _kron(*([np.eye(d)] + [P1] * d))
            self.Ps.append(Pb)
            self.ops.append((Pb.T @ self.ops[-1] @ Pb).tocsr())
            m = m // 2
        self.lower = [sp.tril(A, format="csr") for A in self.ops]
        self.coarse = spla.splu(self.ops[-1].tocsc())
        _, self.Tsolve = t_operator(d, p, n + p - 2)

    def _gs(self, l, x, b):
        return x + spla.spsolve_triangular(self.lower[l], b - self.ops[l] @ x, lower=True)

    def vcycle(self, b, l=0):
        A = self.ops[l]
        if l == len(self.ops) - 1:
            return self.coarse.solve(b)
        x = self._gs(l, np.zeros_like(b), b)
        r = b - A @ x
        x = x + self.Ps[l] @ self.vcycle(self.Ps[l].T @ r, l + 1)
        if l == 0:
            post = pcg_T if self.variant == "P_WL" else gmres_T
            x = x + post(A, self.Tsolve, b - A @ x, self.p)
        else:
            x = self._gs(l, x, b)
        return x

    def solve(self, b, tol=1e-7, maxiter=3000):
        K = self.K
        x = np.zeros_like(b)
        r = b.copy()
        r0 = np.linalg.norm(r)
        if self.variant == "MIM":
            for k in range(1, maxiter + 1):
                x = x + self.vcycle(r)
                r = b - K @ x
                if np.linalg.norm(r) < tol * r0:
                    return x, k
            return x, maxiter
        dprev = qprev = None
        for k in range(1, maxiter + 1):
            z = self.vcycle(r)
            dk = z if dprev is None else z - (z @ qprev) / (dprev @ qprev) * dprev
            q = K @ dk
            a = (dk @ r) / (dk @ q)
            x += a * dk
            r -= a * q
            if np.linalg.norm(r) < tol * r0:
                return x, k
            dprev, qprev = dk, q
        return x, maxiter
