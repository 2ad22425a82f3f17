// Host-side FP64 setup (see setup.hpp).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace cd {

namespace {

constexpr int kMaxP = 8;

// q-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_q.
void legendre(int q, double x, double& pq, double& dpq) {
    double p0 = 1.0, p1 = x;  // P_0, P_1
    for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    pq = p1;
    dpq = q * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int q, std::vector<double>& t, std::vector<double>& w) {
    t.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < q; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (q + 0.5)), pq, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(q, x, pq, dp);
            const double dx = pq / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        legendre(q, x, pq, dp);
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

// Dense solve helper: banded LU without pivoting of an N x N dense-stored
// matrix (bandwidth bw below and above), applied to `nrhs` right-hand sides
// stored row-major N x nrhs.  Used for B-spline collocation at Greville
// points, which is totally positive (no pivoting needed).
void banded_lu_solve(std::vector<double>& A, int N, int bw, std::vector<double>& B, int nrhs) {
    for (int k = 0; k < N; ++k) {
        double piv = A[size_t(k) * N + k];
        if (piv == 0.0) throw std::runtime_error("singular collocation matrix");
        for (int i = k + 1; i < std::min(N, k + bw + 1); ++i) {
            double l = A[size_t(i) * N + k] / piv;
            if (l == 0.0) continue;
            for (int j = k; j < std::min(N, k + bw + 1); ++j) A[size_t(i) * N + j] -= l * A[size_t(k) * N + j];
            for (int r = 0; r < nrhs; ++r) B[size_t(i) * nrhs + r] -= l * B[size_t(k) * nrhs + r];
        }
    }
    for (int k = N - 1; k >= 0; --k) {
        for (int r = 0; r < nrhs; ++r) {
            double s = B[size_t(k) * nrhs + r];
            for (int j = k + 1; j < std::min(N, k + bw + 1); ++j) s -= A[size_t(k) * N + j] * B[size_t(j) * nrhs + r];
            B[size_t(k) * nrhs + r] = s / A[size_t(k) * N + k];
        }
    }
}

Prolong from_dense(const std::vector<double>& P, int mf, int mc) {
    Prolong R;
    R.mf = mf;
    R.mc = mc;
    R.c0.assign(mf, 0);
    R.r0.assign(mc, 0);
    std::vector<int> c1(mf, 0), r1(mc, 0);
    for (int i = 0; i < mf; ++i) {
        int lo = mc, hi = -1;
        for (int j = 0; j < mc; ++j)
            if (P[size_t(i) * mc + j] != 0.0) { lo = std::min(lo, j); hi = std::max(hi, j); }
        if (hi < 0) { lo = 0; hi = -1; }
        R.c0[i] = lo;
        c1[i] = hi;
        R.w = std::max(R.w, hi - lo + 1);
    }
    for (int j = 0; j < mc; ++j) {
        int lo = mf, hi = -1;
        for (int i = 0; i < mf; ++i)
            if (P[size_t(i) * mc + j] != 0.0) { lo = std::min(lo, i); hi = std::max(hi, i); }
        if (hi < 0) { lo = 0; hi = -1; }
        R.r0[j] = lo;
        r1[j] = hi;
        R.wr = std::max(R.wr, hi - lo + 1);
    }
    R.w = std::max(R.w, 1);
    R.wr = std::max(R.wr, 1);
    // keep every window inside the matrix so kernels never index out of range
    for (int i = 0; i < mf; ++i) R.c0[i] = std::max(0, std::min(R.c0[i], mc - R.w));
    for (int j = 0; j < mc; ++j) R.r0[j] = std::max(0, std::min(R.r0[j], mf - R.wr));
    R.v.assign(size_t(mf) * R.w, 0.0);
    R.vt.assign(size_t(mc) * R.wr, 0.0);
    for (int i = 0; i < mf; ++i)
        for (int k = 0; k < R.w; ++k) {
            int j = R.c0[i] + k;
            if (j < mc) R.v[size_t(i) * R.w + k] = P[size_t(i) * mc + j];
        }
    for (int j = 0; j < mc; ++j)
        for (int k = 0; k < R.wr; ++k) {
            int i = R.r0[j] + k;
            if (i < mf) R.vt[size_t(j) * R.wr + k] = P[size_t(i) * mc + j];
        }
    return R;
}

}  // namespace

Band Band::widened(int hb_new) const {
    if (hb_new < hb) throw std::runtime_error("cannot narrow a band");
    Band B(m, hb_new);
    for (int i = 0; i < m; ++i)
        for (int j = std::max(0, i - hb); j <= std::min(m - 1, i + hb); ++j) B.set(i, j, get(i, j));
    return B;
}

double Prolong::get(int i, int j) const {
    int k = j - c0[i];
    return (k < 0 || k >= w) ? 0.0 : v[size_t(i) * w + k];
}

std::vector<double> knots(int n, int p) {
    std::vector<double> xi(n + 2 * p + 1);
    for (int i = 0; i <= p; ++i) xi[i] = 0.0;
    for (int i = 0; i <= n; ++i) xi[p + i] = double(i) / n;
    for (int i = 0; i <= p; ++i) xi[p + n + i] = 1.0;
    return xi;
}

int bspline_local(const std::vector<double>& xi, int p, double x, double* val, double* der) {
    const int nfun = int(xi.size()) - p - 1;
    int k = p;  // span: xi[k] <= x < xi[k+1], clamped to the last nonempty span
    while (k < nfun - 1 && x >= xi[k + 1]) ++k;
    double tbl[kMaxP + 1][kMaxP + 1];
    tbl[0][0] = 1.0;
    for (int q = 1; q <= p; ++q) {
        for (int j = 0; j <= q; ++j) {
            const int i = k - q + j;
            double s = 0.0;
            if (j >= 1) {
                double den = xi[i + q] - xi[i];
                if (den > 0.0) s += (x - xi[i]) / den * tbl[q - 1][j - 1];
            }
            if (j <= q - 1) {
                double den = xi[i + q + 1] - xi[i + 1];
                if (den > 0.0) s += (xi[i + q + 1] - x) / den * tbl[q - 1][j];
            }
            tbl[q][j] = s;
        }
    }
    for (int j = 0; j <= p; ++j) {
        val[j] = tbl[p][j];
        if (der) {
            const int i = k - p + j;
            double s = 0.0;
            if (p >= 1) {
                if (j >= 1) {
                    double den = xi[i + p] - xi[i];
                    if (den > 0.0) s += p * tbl[p - 1][j - 1] / den;
                }
                if (j <= p - 1) {
                    double den = xi[i + p + 1] - xi[i + 1];
                    if (den > 0.0) s -= p * tbl[p - 1][j] / den;
                }
            }
            der[j] = s;
        }
    }
    return k - p;
}

double cardinal(int p, double t) {
    double vals[kMaxP * 2 + 2];
    for (int s = 0; s <= p; ++s) vals[s] = (t - s >= 0.0 && t - s < 1.0) ? 1.0 : 0.0;
    for (int k = 1; k <= p; ++k)
        for (int s = 0; s <= p - k; ++s)
            vals[s] = (t - s) / k * vals[s] + (k + 1 - (t - s)) / k * vals[s + 1];
    return vals[0];
}

void assemble_1d(int n, int p, Band& M, Band& A, Band& S) {
    if (p < 1 || p > kMaxP) throw std::runtime_error("degree out of range");
    const int m = n + p - 2;
    if (m < 1) throw std::runtime_error("n + p - 2 must be >= 1");
    M = Band(m, p);
    A = Band(m, p);
    S = Band(m, p);
    std::vector<double> gt, gw;
    gauss_legendre(p + 1, gt, gw);
    const std::vector<double> xi = knots(n, p);
    double val[kMaxP + 1], der[kMaxP + 1];
    for (int e = 0; e < n; ++e) {
        const double a = double(e) / n, h = 1.0 / n;
        for (int q = 0; q <= p; ++q) {
            const double x = a + 0.5 * h * (gt[q] + 1.0);
            const double w = 0.5 * h * gw[q];
            const int f0 = bspline_local(xi, p, x, val, der);
            for (int r = 0; r <= p; ++r) {
                const int i = f0 + r - 1;  // Dirichlet index (drop the first function)
                if (i < 0 || i >= m) continue;
                for (int c = 0; c <= p; ++c) {
                    const int j = f0 + c - 1;
                    if (j < 0 || j >= m) continue;
                    const size_t off = size_t(i) * (2 * p + 1) + (j - i + p);
                    M.a[off] += w * val[r] * val[c];
                    A.a[off] += w * val[r] * der[c];
                    S.a[off] += w * der[r] * der[c];
                }
            }
        }
    }
}

QuadAxis quad_axis(int n, int p, int q) {
    if (p < 1 || p > kMaxP) throw std::runtime_error("degree out of range");
    QuadAxis Qa;
    Qa.n = n;
    Qa.p = p;
    Qa.q = q;
    Qa.m = n + p - 2;
    Qa.Q = n * q;
    std::vector<double> gt, gw;
    gauss_legendre(q, gt, gw);
    const std::vector<double> xi = knots(n, p);
    Qa.x.resize(Qa.Q);
    Qa.w.resize(Qa.Q);
    Qa.f0.resize(Qa.Q);
    Qa.val.resize(size_t(Qa.Q) * (p + 1));
    Qa.der.resize(size_t(Qa.Q) * (p + 1));
    for (int e = 0; e < n; ++e) {
        const double a = double(e) / n, h = 1.0 / n;
        for (int t = 0; t < q; ++t) {
            const int i = e * q + t;
            Qa.x[i] = a + 0.5 * h * (gt[t] + 1.0);
            Qa.w[i] = 0.5 * h * gw[t];
            Qa.f0[i] = bspline_local(xi, p, Qa.x[i], &Qa.val[size_t(i) * (p + 1)], &Qa.der[size_t(i) * (p + 1)]) - 1;
        }
    }
    return Qa;
}

Prolong knot_insertion(int nf, int p) {
    if (nf % 2) throw std::runtime_error("knot insertion needs an even number of intervals");
    const int nc = nf / 2;
    const std::vector<double> xf = knots(nf, p), xc = knots(nc, p);
    const int Nf = nf + p, Nc = nc + p;
    // Collocation at the Greville abscissae of the fine space: Bf P = Bc
    std::vector<double> Bf(size_t(Nf) * Nf, 0.0), Bc(size_t(Nf) * Nc, 0.0);
    double val[kMaxP + 1];
    for (int i = 0; i < Nf; ++i) {
        double tau = 0.0;
        for (int k = 1; k <= p; ++k) tau += xf[i + k];
        tau /= p;
        int f0 = bspline_local(xf, p, tau, val, nullptr);
        for (int r = 0; r <= p; ++r) Bf[size_t(i) * Nf + f0 + r] = val[r];
        int g0 = bspline_local(xc, p, tau, val, nullptr);
        for (int r = 0; r <= p; ++r) Bc[size_t(i) * Nc + g0 + r] = val[r];
    }
    banded_lu_solve(Bf, Nf, p, Bc, Nc);
    const int mf = Nf - 2, mc = Nc - 2;
    std::vector<double> P(size_t(mf) * mc, 0.0);
    for (int i = 0; i < mf; ++i)
        for (int j = 0; j < mc; ++j) {
            double v = Bc[size_t(i + 1) * Nc + (j + 1)];
            P[size_t(i) * mc + j] = (std::fabs(v) < 1e-13) ? 0.0 : v;
        }
    return from_dense(P, mf, mc);
}

Prolong paper_prolong(int mf) {
    const int mc = mf / 2;
    if (mc < 1) throw std::runtime_error("level too small to coarsen");
    std::vector<double> P(size_t(mf) * mc, 0.0);
    for (int j = 0; j < mc; ++j) {
        const int i = 2 * j + 1;  // fine index of coarse node j (zero-based)
        P[size_t(i - 1) * mc + j] = 0.5;
        P[size_t(i) * mc + j] = 1.0;
        if (i + 1 < mf) P[size_t(i + 1) * mc + j] = 0.5;
    }
    return from_dense(P, mf, mc);
}

Prolong identity_prolong(int m) {
    std::vector<double> P(size_t(m) * m, 0.0);
    for (int i = 0; i < m; ++i) P[size_t(i) * m + i] = 1.0;
    return from_dense(P, m, m);
}

Band galerkin(const Band& X, const Prolong& P) {
    const int mf = P.mf, mc = P.mc;
    std::vector<double> XP(size_t(mf) * mc, 0.0);  // X P
    for (int i = 0; i < mf; ++i)
        for (int k = std::max(0, i - X.hb); k <= std::min(mf - 1, i + X.hb); ++k) {
            const double x = X.get(i, k);
            if (x == 0.0) continue;
            for (int t = 0; t < P.w; ++t) XP[size_t(i) * mc + P.c0[k] + t] += x * P.v[size_t(k) * P.w + t];
        }
    std::vector<double> C(size_t(mc) * mc, 0.0);
    int hb = 0;
    for (int a = 0; a < mc; ++a)
        for (int t = 0; t < P.wr; ++t) {
            const int i = P.r0[a] + t;
            const double pv = P.vt[size_t(a) * P.wr + t];
            if (pv == 0.0) continue;
            for (int b = 0; b < mc; ++b) C[size_t(a) * mc + b] += pv * XP[size_t(i) * mc + b];
        }
    for (int a = 0; a < mc; ++a)
        for (int b = 0; b < mc; ++b)
            if (C[size_t(a) * mc + b] != 0.0) hb = std::max(hb, std::abs(a - b));
    hb = std::max(hb, X.hb);  // keep the fine band width (zero padded)
    Band R(mc, hb);
    for (int a = 0; a < mc; ++a)
        for (int b = std::max(0, a - hb); b <= std::min(mc - 1, a + hb); ++b) R.set(a, b, C[size_t(a) * mc + b]);
    return R;
}

TFactor toeplitz_factor(int m, int p) {
    TFactor F;
    F.m = m;
    F.bw = p - 1;
    F.T = Band(m, std::max(p - 1, 0));
    for (int i = 0; i < m; ++i)
        for (int j = std::max(0, i - p + 1); j <= std::min(m - 1, i + p - 1); ++j)
            F.T.set(i, j, cardinal(2 * p - 1, double(p - i + j)));
    const int bw = F.bw;
    F.l.assign(size_t(m) * std::max(bw, 1), 0.0);
    F.dinv.assign(m, 0.0);
    std::vector<double> D(m, 0.0);
    auto L = [&](int r, int c) -> double& { return F.l[size_t(r) * std::max(bw, 1) + (r - c - 1)]; };
    for (int i = 0; i < m; ++i) {
        double d = F.T.get(i, i);
        for (int k = std::max(0, i - bw); k < i; ++k) d -= L(i, k) * L(i, k) * D[k];
        if (!(d > 0.0)) throw std::runtime_error("T is not positive definite");
        D[i] = d;
        F.dinv[i] = 1.0 / d;
        for (int r = i + 1; r <= std::min(m - 1, i + bw); ++r) {
            double s = F.T.get(r, i);
            for (int k = std::max(0, r - bw); k < i; ++k) s -= L(r, k) * L(i, k) * D[k];
            L(r, i) = s / d;
        }
    }
    return F;
}

int recurrence_warmup(const TFactor& F, double tol) {
    const int bw = F.bw, m = F.m;
    if (bw == 0) return 0;
    const int r = m / 2;  // interior row: coefficients of the asymptotic recurrence
    std::vector<double> c(bw, 0.0);
    for (int k = 1; k <= bw; ++k)
        if (r - k >= 0) c[k - 1] = F.l[size_t(r) * bw + (k - 1)];
    int worst = 0;
    for (int j = 0; j < bw; ++j) {
        std::vector<double> win(bw, 0.0);
        win[j] = 1.0;
        int steps = 0;
        for (; steps < m; ++steps) {
            double mx = 0.0;
            for (double v : win) mx = std::max(mx, std::fabs(v));
            if (mx < tol) break;
            double y = 0.0;
            for (int k = 1; k <= bw; ++k) y -= c[k - 1] * win[k - 1];
            for (int k = bw - 1; k >= 1; --k) win[k] = win[k - 1];
            win[0] = y;
        }
        worst = std::max(worst, steps);
    }
    return std::min(m, worst + bw + 2);
}

namespace {

// Largest eigenvalue of a real symmetric matrix of order 1, 2 or 3 (the
// trigonometric solution of the characteristic cubic for order 3).
double sym_max_eig(int d, const double a[3][3]) {
    if (d == 1) return a[0][0];
    if (d == 2) {
        const double h = 0.5 * (a[0][0] + a[1][1]), g = 0.5 * (a[0][0] - a[1][1]);
        return h + std::sqrt(g * g + a[0][1] * a[0][1]);
    }
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double q = (a[0][0] + a[1][1] + a[2][2]) / 3.0;
    if (off == 0.0) return std::max(a[0][0], std::max(a[1][1], a[2][2]));
    const double b00 = a[0][0] - q, b11 = a[1][1] - q, b22 = a[2][2] - q;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * off;
    const double pp = std::sqrt(p2 / 6.0);
    // det(B / pp) / 2
    const double det = b00 * (b11 * b22 - a[1][2] * a[1][2]) - a[0][1] * (a[0][1] * b22 - a[1][2] * a[0][2]) +
                       a[0][2] * (a[0][1] * a[1][2] - b11 * a[0][2]);
    double r = det / (2.0 * pp * pp * pp);
    r = std::min(1.0, std::max(-1.0, r));
    return q + 2.0 * pp * std::cos(std::acos(r) / 3.0);
}

}  // namespace

double symbol_lambda_max(int d, const Band* M, const Band* A, const Band* S, double alpha, double beta,
                         double offw, int samples) {
    // per axis and sample: Toeplitz symbols of M and S (real: the rows are
    // symmetric) and of A divided by i (A is skew), from the central row
    std::vector<double> mr(size_t(d) * samples), sr(size_t(d) * samples), ai(size_t(d) * samples);
    double m0[3], s0[3];
    for (int l = 0; l < d; ++l) {
        const int m = M[l].m;
        const int hb = std::max(M[l].hb, std::max(A[l].hb, S[l].hb));
        if (m < 2 * hb + 1) return 0.0;
        const int i0 = m / 2;
        m0[l] = M[l].get(i0, i0);
        s0[l] = S[l].get(i0, i0);
        for (int t = 0; t < samples; ++t) {
            const double th = samples > 1 ? M_PI * t / (samples - 1) : 0.0;
            double vm = 0, vs = 0, va = 0;
            for (int k = -hb; k <= hb; ++k) {
                vm += M[l].get(i0, i0 + k) * std::cos(k * th);
                vs += S[l].get(i0, i0 + k) * std::cos(k * th);
                va += A[l].get(i0, i0 + k) * std::sin(k * th);
            }
            mr[size_t(l) * samples + t] = vm;
            sr[size_t(l) * samples + t] = vs;
            ai[size_t(l) * samples + t] = va;
        }
    }
    // constant diagonal of each component block
    double dh[3];
    for (int c = 0; c < d; ++c) {
        dh[c] = 0.0;
        for (int f = 0; f < d; ++f) {
            double t = (f == c) ? beta : alpha;
            for (int l = 0; l < d; ++l) t *= (l == f) ? s0[l] : m0[l];
            dh[c] += t;
        }
        if (!(dh[c] > 0.0)) return 0.0;
    }
    double best = 0.0;
    const int n2 = samples, n3 = d == 3 ? samples : 1;
    for (int t0 = 0; t0 < samples; ++t0)
        for (int t1 = 0; t1 < n2; ++t1)
            for (int t2 = 0; t2 < n3; ++t2) {
                const int ts[3] = {t0, t1, t2};
                double vm[3], vs[3], va[3];
                for (int l = 0; l < d; ++l) {
                    vm[l] = mr[size_t(l) * samples + ts[l]];
                    vs[l] = sr[size_t(l) * samples + ts[l]];
                    va[l] = ai[size_t(l) * samples + ts[l]];
                }
                double F[3][3] = {};
                for (int c = 0; c < d; ++c) {
                    double v = 0.0;
                    for (int f = 0; f < d; ++f) {
                        double t = (f == c) ? beta : alpha;
                        for (int l = 0; l < d; ++l) t *= (l == f) ? vs[l] : vm[l];
                        v += t;
                    }
                    F[c][c] = v / dh[c];
                    for (int e = c + 1; e < d; ++e) {
                        // offw (i a_c)(i a_e) prod of the other axes' M symbols
                        double t = -offw;
                        for (int l = 0; l < d; ++l) t *= (l == c || l == e) ? va[l] : vm[l];
                        F[c][e] = F[e][c] = t / std::sqrt(dh[c] * dh[e]);
                    }
                }
                best = std::max(best, sym_max_eig(d, F));
            }
    return best;
}

}  // namespace cd
