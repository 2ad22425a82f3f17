"""The solver the GPU library computes, written out plainly (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's multi-iterative method (Sec. 6.1), used as preconditioner of a
conjugate-gradient iteration (Remark 6.1 and the P_MIM label of Sec. 6.2),
with these readings, each also listed with its reason in the design notes:

1. Grid hierarchy.  Level 0 is A^{p,alpha,beta}_n.  Coarse operators are the
   Galerkin products P^T A P with the block prolongator I_d (x) P (x) ... (x) P
   (Sec. 6.1); because every block of A is a sum of Kronecker products of 1D
   matrices, the coarse operator has the same form with the 1D matrices
   P^T M P, P^T A P, P^T S P.  P is either the knot-insertion prolongator
   (n -> n/2, default) or the paper's (1/2)[1 2 1] stencil.  Coarsening stops
   when the level has at most ``coarse_max_dofs`` unknowns or cannot be
   coarsened further; that coarsest level is solved exactly.
2. Smoother.  The paper's Gauss-Seidel sweeps are sequential; this method uses
   Chebyshev smoothing of degree ``nu`` on D^{-1} A_l (D = diag A_l), on the
   interval [hi/ratio, hi], hi = 1.1 * lambda_est.  lambda_est is the
   largest Ritz value of ``lanczos_steps`` steps of the Lanczos process on
   D^{-1} A_l in the D inner product (no reorthogonalisation), started from
   v0 = (-1)^{i_1+...+i_d} in every component and restarted from a fixed
   vector when the recurrence breaks down.  One smoothing application (degree nu) replaces each of the
   paper's Gauss-Seidel sweeps: before the coarse correction on every level,
   and after it on all levels but the finest.  Levels below the finest may
   use their own degree ``nu_coarse`` (None: the same nu everywhere).
3. Finest-level post-smoother: ``krylov_steps`` (default p) steps of GMRES on
   the error equation with zero initial guess, right-preconditioned by
   T = I_d (x) T_m(m_{p-1})^{(x) d} (Sec. 6.1), Arnoldi by classical
   Gram-Schmidt, update T^{-1}(V y) with y the least-squares solution of the
   (s+1) x s Hessenberg problem.
4. Outer iteration: flexible CG with one stored direction (Notay's FCG(1)),
   x_0 = 0, stop when ||r_k||_2 / ||r_0||_2 < tol (Sec. 6.2).  FCG(1) equals
   PCG for a fixed SPD preconditioner; the GMRES post-smoother makes the
   preconditioner nonlinear.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import curl_div_matrix
from .symbols import symbol_bound
from .matrices import mass_adv_stiff, toeplitz_T
from .transfer import knot_insertion_prolongator, paper_prolongator


def _kron(*mats):
    out = sp.csr_matrix(mats[0])
    for X in mats[1:]:
        out = sp.kron(out, sp.csr_matrix(X), format="csr")
    return out


class Level:
    """One level: per-axis interval counts ``ns`` (None below the finest level
    with the paper's transfer) and per-axis 1D (M, A, S) triples; the
    attributes n, m, M, A, S, P are those of axis 1 (all axes alike on a
    uniform grid)."""

    def __init__(self, d, p, ns, alpha, beta, mats, blockdiag=False):
        self.d, self.p = d, p
        self.ns = list(ns)
        self.mats = [tuple(t) for t in mats]
        self.ms = tuple(t[0].shape[0] for t in self.mats)
        self.n, self.m = self.ns[0], self.ms[0]
        self.M, self.A, self.S = self.mats[0]
        self.K = curl_div_matrix(d, p, None, alpha, beta, mats=self.mats)
        if blockdiag:  # the block-diagonal part D of the level operator (Sec. 6.1, eq. diag)
            G = self.K.shape[0] // d
            self.K = sp.block_diag([self.K[c * G:(c + 1) * G, c * G:(c + 1) * G] for c in range(d)], format="csr")
        self.D = self.K.diagonal().copy()
        self.Ps = None  # per-axis 1D prolongators from the next level to this one
        self.P = None
        self.lam = None


def build_hierarchy(d, p, n, alpha, beta, transfer="knot", coarse_max_dofs=1000,
                    lanczos_steps=20, nu=3, ratio=30.0, nu_coarse=None, blockdiag=False,
                    bounds="lanczos", safety=1.5):
    """List of Level objects, finest first.  ``n``: intervals of every axis,
    or one count per axis.  Each level coarsens every axis that can be:
    by knot insertion (n -> n/2) while the transfer is "knot" and the axis's
    n is even, otherwise by the paper's prolongator (m -> floor(m/2)), which
    the axis keeps from then on; an axis with one point is left as it is.
    The hierarchy stops when a level has at most coarse_max_dofs unknowns or
    no axis can be coarsened.  blockdiag: every level holds the block-diagonal
    part of its operator (P_WL); the block prolongator keeps it block diagonal,
    so the Galerkin coarse operator of D is the block-diagonal part of the
    coarse operator.  bounds="symbol": each smoothed level whose axes all have
    at least 2p+1 points takes hi = safety x the symbol maximum of
    diag(K_l)^{-1} K_l (Sec. 5, symbols.symbol_bound); the others, and
    bounds="lanczos", hi = 1.1 x the Lanczos estimate."""
    ns = [n] * d if np.isscalar(n) else [int(v) for v in n]
    levels = [Level(d, p, ns, alpha, beta, [mass_adv_stiff(nl, p) for nl in ns], blockdiag)]
    if transfer not in ("knot", "paper"):
        raise ValueError(transfer)
    knot = [transfer == "knot"] * d
    while True:
        L = levels[-1]
        if d * int(np.prod(L.ms)) <= coarse_max_dofs:
            break
        Ps, ncs = [], []
        for l in range(d):
            nl, ml = L.ns[l], L.ms[l]
            if knot[l] and nl % 2 == 0 and nl // 2 + p - 2 >= 1:
                Ps.append(knot_insertion_prolongator(nl, p))
                ncs.append(nl // 2)
            elif ml // 2 >= 1:
                knot[l] = False
                Ps.append(paper_prolongator(ml))
                ncs.append(None)
            else:
                Ps.append(np.eye(ml))
                ncs.append(nl)
        if all(P.shape[0] == P.shape[1] for P in Ps):
            break
        L.Ps, L.P = Ps, Ps[0]
        cm = [tuple(P.T @ X @ P for X in trip) for P, trip in zip(Ps, L.mats)]
        levels.append(Level(d, p, ncs, alpha, beta, cm, blockdiag))
    if bounds not in ("lanczos", "symbol"):
        raise ValueError(bounds)
    for l, L in enumerate(levels[:-1]):
        if bounds == "symbol" and min(L.ms) >= 2 * p + 1:
            L.lam = symbol_bound(L.K, d, L.ms, symbol_samples(d))
            L.hi = safety * L.lam
        else:
            L.lam = lanczos_estimate(L, lanczos_steps)
            L.hi = 1.1 * L.lam
        L.lo = L.hi / ratio
        L.nu = nu if l == 0 or nu_coarse is None else nu_coarse
    C = levels[-1]
    C.coarse_factor = sla.cho_factor(C.K.toarray())
    return levels


def symbol_samples(d):
    """Points per axis of the theta grid of the symbol bound."""
    return 129 if d == 2 else 33


def start_vector(d, m):
    """v0 = (-1)^{i_1+...+i_d}, the same in every component (m: points of
    every axis, or one count per axis)."""
    shape = (m,) * d if np.isscalar(m) else tuple(m)
    idx = np.indices(shape).sum(axis=0)
    v = np.where(idx % 2 == 0, 1.0, -1.0).ravel()
    return np.tile(v, d)


def restart_vector(n):
    """r_i = cos(0.7 i + 0.3): a fixed vector with no grid symmetry."""
    return np.cos(0.7 * np.arange(n) + 0.3)


LANCZOS_BREAKDOWN = 1e-10


def lanczos_estimate(L, steps):
    """Largest Ritz value of D^{-1} K on the Krylov space of dimension
    ``steps`` from the start vector.  D^{-1} K is self-adjoint in the inner
    product <u, v>_D = u^T D v, so the Lanczos three-term recurrence in that
    inner product tridiagonalises it: with q_0 = v0 / |v0|_D,
        alpha_j = q_j^T K q_j,
        w = D^{-1} K q_j - alpha_j q_j - beta_j q_{j-1},
        beta_{j+1} = |w|_D,  q_{j+1} = w / beta_{j+1}.
    When beta_{j+1} <= 1e-10 |alpha_j| the Krylov space is invariant (the
    symmetric start vector can span a small invariant subspace on small
    grids): the recurrence restarts from the D-normalised restart vector with
    beta_{j+1} = 0, so the tridiagonal matrix splits into independent runs."""
    v = start_vector(L.d, L.ms)
    q = v / np.sqrt(v @ (L.D * v))
    r = restart_vector(q.size)
    r = r / np.sqrt(r @ (L.D * r))
    qprev = np.zeros_like(q)
    alpha, beta = [], [0.0]
    for _ in range(steps):
        Kq = L.K @ q
        a = q @ Kq
        w = Kq / L.D - a * q - beta[-1] * qprev
        alpha.append(a)
        b = np.sqrt(w @ (L.D * w))
        if b <= LANCZOS_BREAKDOWN * abs(a):
            beta.append(0.0)
            qprev, q = q, r
        else:
            beta.append(b)
            qprev, q = q, w / b
    k = len(alpha)
    return sla.eigvalsh_tridiagonal(np.array(alpha), np.array(beta[1:k]))[-1]


def chebyshev(L, x, b, nu=None):
    """``nu`` steps of Chebyshev iteration for K x = b preconditioned by D,
    on the interval [L.lo, L.hi] (three-term recurrence on the update)."""
    nu = L.nu if nu is None else nu
    theta = 0.5 * (L.hi + L.lo)
    delta = 0.5 * (L.hi - L.lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = x.copy()
    r = b - L.K @ x
    upd = r / L.D / theta
    x += upd
    for _ in range(nu - 1):
        r = b - L.K @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        upd = rho_new * rho * upd + (2.0 * rho_new / delta) * (r / L.D)
        x += upd
        rho = rho_new
    return x


def t_operator(d, p, m):
    """Sparse T = I_d (x) T_{m_1}(m_{p-1}) (x) ... (x) T_{m_d}(m_{p-1})
    (Sec. 6.1) and a solver for it (sparse LU of the assembled Kronecker
    product); m: points of every axis, or one count per axis."""
    ms = [m] * d if np.isscalar(m) else list(m)
    T = _kron(*([np.eye(d)] + [toeplitz_T(ml, p) for ml in ms]))
    lu = spla.splu(T.tocsc())
    return T, lu.solve


def pcg_T(K, Tsolve, r, steps):
    """``steps`` PCG steps on K e = r from e = 0 with preconditioner T (the
    finest post-smoother of P_WL, Sec. 6.2)."""
    e = np.zeros_like(r)
    res = r.copy()
    z = Tsolve(res)
    dd = z.copy()
    rz = res @ z
    for _ in range(steps):
        q = K @ dd
        dq = dd @ q
        if dq <= 0:
            break
        a = rz / dq
        e += a * dd
        res -= a * q
        z = Tsolve(res)
        rz_new = res @ z
        dd = z + (rz_new / rz) * dd
        rz = rz_new
    return e


def gmres_T(K, Tsolve, r, steps):
    """``steps`` GMRES steps on K e = r from e = 0, right preconditioner T."""
    beta0 = np.linalg.norm(r)
    if beta0 == 0.0:
        return np.zeros_like(r)
    V = [r / beta0]
    H = np.zeros((steps + 1, steps))
    s = steps
    for j in range(steps):
        w = K @ Tsolve(V[j])
        h = np.array([vi @ w for vi in V])  # classical Gram-Schmidt
        w = w - sum(hi * vi for hi, vi in zip(h, V))
        H[: j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            s = j + 1
            break
        V.append(w / H[j + 1, j])
    rhs = np.zeros(s + 1)
    rhs[0] = beta0
    y = np.linalg.lstsq(H[: s + 1, :s], rhs, rcond=None)[0]
    return Tsolve(sum(yi * vi for yi, vi in zip(y, V[:s])))


class Method:
    """Hierarchy plus the finest-level T solver; ``vcycle`` is one application
    of the preconditioner, ``solve`` the outer flexible CG."""

    def __init__(self, d, p, n, alpha, beta, transfer="knot", coarse_max_dofs=1000,
                 nu=3, ratio=30.0, lanczos_steps=20, krylov_steps=None, nu_coarse=None, variant="P_MIM",
                 bounds="lanczos", safety=1.5):
        if variant not in ("P_MIM", "P_WL", "MIM"):
            raise ValueError(variant)
        self.d, self.p, self.n, self.variant = d, p, n, variant
        self.levels = build_hierarchy(d, p, n, alpha, beta, transfer, coarse_max_dofs,
                                      lanczos_steps, nu, ratio, nu_coarse, blockdiag=(variant == "P_WL"),
                                      bounds=bounds, safety=safety)
        self.krylov_steps = p if krylov_steps is None else krylov_steps
        self.T, self.Tsolve = t_operator(d, p, self.levels[0].ms)
        # the system matrix (the V-cycle of P_WL runs on its block-diagonal part)
        self.K = curl_div_matrix(d, p, None, alpha, beta, mats=self.levels[0].mats) if variant == "P_WL" \
            else self.levels[0].K

    def _prolong_block(self, l):
        return _kron(*([np.eye(self.d)] + list(self.levels[l].Ps)))

    def vcycle(self, b, l=0):
        L = self.levels[l]
        if l == len(self.levels) - 1:
            return sla.cho_solve(L.coarse_factor, b)
        x = chebyshev(L, np.zeros_like(b), b)
        r = b - L.K @ x
        Pb = self._prolong_block(l)
        x = x + Pb @ self.vcycle(Pb.T @ r, l + 1)
        if l == 0 and self.krylov_steps > 0:
            post = pcg_T if self.variant == "P_WL" else gmres_T
            x = x + post(L.K, self.Tsolve, b - L.K @ x, self.krylov_steps)
        else:
            x = chebyshev(L, x, b)
        return x

    def solve(self, b, tol, maxiter=10000):
        """FCG(1) preconditioned by the V-cycle (P_MIM, P_WL), or the V-cycle
        as a stationary iteration x += V(b - K x) (MIM).  Returns (x,
        iterations, history of ||r_k||_2)."""
        K = self.K
        x = np.zeros_like(b)
        r = b.copy()
        r0 = np.linalg.norm(r)
        hist = [r0]
        if r0 == 0.0:
            return x, 0, hist
        if self.variant == "MIM":
            k = 0
            while k < maxiter:
                x = x + self.vcycle(r)
                r = b - K @ x
                k += 1
                hist.append(np.linalg.norm(r))
                if hist[-1] < tol * r0:
                    break
            return x, k, hist
        dprev = qprev = dq_prev = None
        k = 0
        while k < maxiter:
            z = self.vcycle(r)
            if dprev is None:
                dk = z
            else:
                dk = z - (z @ qprev) / dq_prev * dprev
            q = K @ dk
            dq = dk @ q
            a = (dk @ r) / dq
            x += a * dk
            r -= a * q
            k += 1
            hist.append(np.linalg.norm(r))
            if hist[-1] < tol * r0:
                break
            dprev, qprev, dq_prev = dk, q, dq
        return x, k, hist
