// Load vector of the manufactured solutions of the numerical examples
// (Sec. 6.2) and the L2 error of a discrete solution against them, by
// quadrature with sum factorization (FP64).
//
// Manufactured fields, g = prod_i x_i (1 - x_i):
//   2D  u = (sin(2 pi g), cos(2 pi g) - 1)
//   3D  u = (sin(2 pi g), cos(2 pi g) - 1, u_1 + u_2)
// Both vanish on the boundary, so the load vector of f = L_{alpha,beta} u
// against a test field psi of the Dirichlet space is
//   alpha (curl u, curl psi) + beta (div u, div psi),
// which needs first derivatives of u only.  Quadrature: q points of
// Gauss-Legendre per element and direction (q = p + 3 by default).
//
// Load vector, 3D: (A) for every quadrature point pair (a, b) of axes 1, 2
// and basis function i3 of axis 3, the weighted fields (curl u components,
// div u) are summed against N_{i3} or N'_{i3} over the support of i3 (the
// fields are evaluated on the fly): 7 arrays U; (B) axis 2 against N or N',
// already combined with alpha and beta into the 6 arrays V[c][x-kind] of the
// three components; (C) axis 1.  2D: (A) over axis 2 into 4 arrays, then (C).
// L2 error: u_h is evaluated at the quadrature points axis by axis from the
// coefficients (axis d first), and the last pass evaluates u, squares the
// difference, weights it and reduces.
#include "device_common.hpp"
#include "loadvec.hpp"

namespace cd {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Jac3 {
    double J[3][3];
};

// du_c/dx_j at (x0, x1, x2) (x2 ignored for d = 2).
__device__ inline Jac3 jacobian(int d, double x0, double x1, double x2) {
    const double f[3] = {x0 * (1 - x0), x1 * (1 - x1), d == 3 ? x2 * (1 - x2) : 1.0};
    const double df[3] = {1 - 2 * x0, 1 - 2 * x1, 1 - 2 * x2};
    const double g = f[0] * f[1] * f[2];
    double sg, cg;
    sincos(kTwoPi * g, &sg, &cg);
    const double c1 = kTwoPi * cg, c2 = -kTwoPi * sg;
    Jac3 r{};
    for (int j = 0; j < d; ++j) {
        double dg = df[j];
        for (int l = 0; l < d; ++l)
            if (l != j) dg *= f[l];
        r.J[0][j] = c1 * dg;
        r.J[1][j] = c2 * dg;
        r.J[2][j] = r.J[0][j] + r.J[1][j];
    }
    return r;
}

__device__ inline void field_values(int d, double x0, double x1, double x2, double* u) {
    const double g = x0 * (1 - x0) * x1 * (1 - x1) * (d == 3 ? x2 * (1 - x2) : 1.0);
    double sg, cg;
    sincos(kTwoPi * g, &sg, &cg);
    u[0] = sg;
    u[1] = cg - 1.0;
    u[2] = u[0] + u[1];
}

// Supports: function i (Dirichlet index) of an axis is the full function
// f = i + 1, nonzero on elements f - p .. f; at a quadrature point a its
// local position is i - f0[a].
__device__ inline void support(const QuadDev& A, int i, int& a_lo, int& a_hi) {
    const int f = i + 1;
    const int e0 = max(0, f - A.p), e1 = min(A.n - 1, f);
    a_lo = e0 * A.q;
    a_hi = (e1 + 1) * A.q;
}

// ---- 2D ------------------------------------------------------------------------
// U[k][a * m2 + i2], k: curl N'_{i2}, div N_{i2}, curl N_{i2}, div N'_{i2}
__global__ __launch_bounds__(kThreads) void k_load2_axis2(QuadDev X, QuadDev Y, double* __restrict__ U) {
    const size_t total = size_t(X.Q) * Y.m;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const int a = int(id / Y.m), i2 = int(id % Y.m);
        int b0, b1;
        support(Y, i2, b0, b1);
        double u0 = 0, u1 = 0, u2 = 0, u3 = 0;
        for (int b = b0; b < b1; ++b) {
            const int k = i2 - Y.f0[b];
            if (k < 0 || k > Y.p) continue;
            const Jac3 J = jacobian(2, X.x[a], Y.x[b], 0.0);
            const double W = X.w[a] * Y.w[b];
            const double curl = (J.J[1][0] - J.J[0][1]) * W, dv = (J.J[0][0] + J.J[1][1]) * W;
            const double yb = Y.val[b * (Y.p + 1) + k], yd = Y.der[b * (Y.p + 1) + k];
            u0 += curl * yd;
            u1 += dv * yb;
            u2 += curl * yb;
            u3 += dv * yd;
        }
        U[0 * total + id] = u0;
        U[1 * total + id] = u1;
        U[2 * total + id] = u2;
        U[3 * total + id] = u3;
    }
}

// b1 = sum_a (-alpha N_{i1} curl_D + beta N'_{i1} div_B), b2 = sum_a (alpha N'_{i1} curl_B + beta N_{i1} div_D)
__global__ __launch_bounds__(kThreads) void k_load2_axis1(QuadDev X, QuadDev Y, const double* __restrict__ U,
                                                          double alpha, double beta, double* __restrict__ b) {
    const size_t G = size_t(X.m) * Y.m, tq = size_t(X.Q) * Y.m;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < 2 * G; id += size_t(gridDim.x) * kThreads) {
        const int c = int(id / G);
        const int i1 = int((id % G) / Y.m), i2 = int(id % Y.m);
        int a0, a1;
        support(X, i1, a0, a1);
        double s = 0.0;
        for (int a = a0; a < a1; ++a) {
            const int k = i1 - X.f0[a];
            if (k < 0 || k > X.p) continue;
            const double xb = X.val[a * (X.p + 1) + k], xd = X.der[a * (X.p + 1) + k];
            const size_t u = size_t(a) * Y.m + i2;
            if (c == 0)
                s += -alpha * xb * U[0 * tq + u] + beta * xd * U[1 * tq + u];
            else
                s += alpha * xd * U[2 * tq + u] + beta * xb * U[3 * tq + u];
        }
        b[id] = s;
    }
}

// ---- 3D ------------------------------------------------------------------------
// U[k][(a Q2 + b) m3 + i3], k: cu0 N, cu0 N', cu1 N, cu1 N', cu2 N, div N, div N' (against N_{i3} or N'_{i3})
constexpr int kU3 = 7;
__global__ __launch_bounds__(kThreads) void k_load3_axis3(QuadDev X, QuadDev Y, QuadDev Z, double* __restrict__ U) {
    const size_t total = size_t(X.Q) * Y.Q * Z.m;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const int i3 = int(id % Z.m);
        const size_t ab = id / Z.m;
        const int a = int(ab / Y.Q), bq = int(ab % Y.Q);
        int c0, c1;
        support(Z, i3, c0, c1);
        double acc[kU3] = {0, 0, 0, 0, 0, 0, 0};
        for (int c = c0; c < c1; ++c) {
            const int k = i3 - Z.f0[c];
            if (k < 0 || k > Z.p) continue;
            const Jac3 J = jacobian(3, X.x[a], Y.x[bq], Z.x[c]);
            const double W = X.w[a] * Y.w[bq] * Z.w[c];
            const double cu0 = (J.J[2][1] - J.J[1][2]) * W, cu1 = (J.J[0][2] - J.J[2][0]) * W;
            const double cu2 = (J.J[1][0] - J.J[0][1]) * W, dv = (J.J[0][0] + J.J[1][1] + J.J[2][2]) * W;
            const double zb = Z.val[c * (Z.p + 1) + k], zd = Z.der[c * (Z.p + 1) + k];
            acc[0] += cu0 * zb;
            acc[1] += cu0 * zd;
            acc[2] += cu1 * zb;
            acc[3] += cu1 * zd;
            acc[4] += cu2 * zb;
            acc[5] += dv * zb;
            acc[6] += dv * zd;
        }
        for (int k = 0; k < kU3; ++k) U[k * total + id] = acc[k];
    }
}

// V[c][xk][(a m2 + i2) m3 + i3], xk = 0: against N_{i1}, 1: against N'_{i1}
__global__ __launch_bounds__(kThreads) void k_load3_axis2(QuadDev X, QuadDev Y, QuadDev Z, const double* __restrict__ U,
                                                          double alpha, double beta, double* __restrict__ V) {
    const size_t total = size_t(X.Q) * Y.m * Z.m, tu = size_t(X.Q) * Y.Q * Z.m;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const int i3 = int(id % Z.m);
        const int i2 = int((id / Z.m) % Y.m);
        const int a = int(id / (size_t(Y.m) * Z.m));
        int b0, b1;
        support(Y, i2, b0, b1);
        double v[6] = {0, 0, 0, 0, 0, 0};
        for (int bq = b0; bq < b1; ++bq) {
            const int k = i2 - Y.f0[bq];
            if (k < 0 || k > Y.p) continue;
            const double yb = Y.val[bq * (Y.p + 1) + k], yd = Y.der[bq * (Y.p + 1) + k];
            const size_t u = (size_t(a) * Y.Q + bq) * Z.m + i3;
            const double cu0B = U[0 * tu + u], cu0D = U[1 * tu + u], cu1B = U[2 * tu + u], cu1D = U[3 * tu + u];
            const double cu2B = U[4 * tu + u], dvB = U[5 * tu + u], dvD = U[6 * tu + u];
            v[0] += alpha * cu1D * yb - alpha * cu2B * yd;  // b1 against N_{i1}
            v[1] += beta * dvB * yb;                        // b1 against N'_{i1}
            v[2] += -alpha * cu0D * yb + beta * dvB * yd;   // b2 against N_{i1}
            v[3] += alpha * cu2B * yb;                      // b2 against N'_{i1}
            v[4] += alpha * cu0B * yd + beta * dvD * yb;    // b3 against N_{i1}
            v[5] += -alpha * cu1B * yb;                     // b3 against N'_{i1}
        }
        for (int k = 0; k < 6; ++k) V[k * total + id] = v[k];
    }
}

__global__ __launch_bounds__(kThreads) void k_load3_axis1(QuadDev X, QuadDev Y, QuadDev Z, const double* __restrict__ V,
                                                          double* __restrict__ b) {
    const size_t P = size_t(Y.m) * Z.m, G = size_t(X.m) * P, tv = size_t(X.Q) * P;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < 3 * G; id += size_t(gridDim.x) * kThreads) {
        const int c = int(id / G);
        const int i1 = int((id % G) / P);
        const size_t rest = id % P;
        int a0, a1;
        support(X, i1, a0, a1);
        double s = 0.0;
        for (int a = a0; a < a1; ++a) {
            const int k = i1 - X.f0[a];
            if (k < 0 || k > X.p) continue;
            const double xb = X.val[a * (X.p + 1) + k], xd = X.der[a * (X.p + 1) + k];
            s += xb * V[(2 * c) * tv + size_t(a) * P + rest] + xd * V[(2 * c + 1) * tv + size_t(a) * P + rest];
        }
        b[id] = s;
    }
}

// ---- L2 error ------------------------------------------------------------------
// out[((c n_1 + i_1) ...)]: contract the last axis of the d-component array
// `in` (leading dims `lead`, last axis m -> Q) with the basis values.
__global__ __launch_bounds__(kThreads) void k_eval_last(QuadDev A, const double* __restrict__ in, size_t lead,
                                                        double* __restrict__ out) {
    const size_t total = lead * A.Q;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const size_t r = id / A.Q;
        const int qa = int(id % A.Q);
        double s = 0.0;
        for (int k = 0; k <= A.p; ++k) {
            const int i = A.f0[qa] + k;
            if (i >= 0 && i < A.m) s += A.val[qa * (A.p + 1) + k] * in[r * A.m + i];
        }
        out[id] = s;
    }
}

// the same along a middle axis: in[(r, i, s)] (i over m, s over inner) -> out[(r, qa, s)]
__global__ __launch_bounds__(kThreads) void k_eval_mid(QuadDev A, const double* __restrict__ in, size_t lead,
                                                       size_t inner, double* __restrict__ out) {
    const size_t total = lead * A.Q * inner;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const size_t sI = id % inner;
        const int qa = int((id / inner) % A.Q);
        const size_t r = id / (inner * A.Q);
        double s = 0.0;
        for (int k = 0; k <= A.p; ++k) {
            const int i = A.f0[qa] + k;
            if (i >= 0 && i < A.m) s += A.val[qa * (A.p + 1) + k] * in[(r * A.m + i) * inner + sI];
        }
        out[id] = s;
    }
}

// u_h on the first axis from T[c][i1][rest] (rest = quadrature points of the
// other axes), then sum W (u - u_h)^2 over the points; part[block]
__global__ __launch_bounds__(kThreads) void k_l2_last(int d, QuadDev X, QuadDev Y, QuadDev Z, const double* __restrict__ T,
                                                      double* __restrict__ part) {
    const size_t rest = size_t(Y.Q) * (d == 3 ? Z.Q : 1), total = size_t(X.Q) * rest;
    const size_t tc = size_t(X.m) * rest;
    double acc = 0.0;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const int qa = int(id / rest);
        const size_t r = id % rest;
        const int qb = int(d == 3 ? r / Z.Q : r), qc = int(d == 3 ? r % Z.Q : 0);
        double u[3];
        field_values(d, X.x[qa], Y.x[qb], d == 3 ? Z.x[qc] : 0.0, u);
        const double W = X.w[qa] * Y.w[qb] * (d == 3 ? Z.w[qc] : 1.0);
        for (int c = 0; c < d; ++c) {
            double uh = 0.0;
            for (int k = 0; k <= X.p; ++k) {
                const int i = X.f0[qa] + k;
                if (i >= 0 && i < X.m) uh += X.val[qa * (X.p + 1) + k] * T[c * tc + size_t(i) * rest + r];
            }
            const double e = u[c] - uh;
            acc += W * e * e;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

int grid(size_t n) {
    const size_t nb = (n + kThreads - 1) / kThreads;
    return int(std::max<size_t>(1, std::min<size_t>(nb, 65536)));
}

}  // namespace

void launch_load_vector(int d, const QuadDev* ax, double alpha, double beta, double* b, double* work, hipStream_t s) {
    if (d == 2) {
        const QuadDev &X = ax[0], &Y = ax[1];
        double* U = work;  // 4 Q1 m2
        hipLaunchKernelGGL(k_load2_axis2, dim3(grid(size_t(X.Q) * Y.m)), dim3(kThreads), 0, s, X, Y, U);
        hipLaunchKernelGGL(k_load2_axis1, dim3(grid(2 * size_t(X.m) * Y.m)), dim3(kThreads), 0, s, X, Y, U, alpha,
                           beta, b);
    } else {
        const QuadDev &X = ax[0], &Y = ax[1], &Z = ax[2];
        double* U = work;                                          // 7 Q1 Q2 m3
        double* V = work + size_t(kU3) * X.Q * Y.Q * Z.m;          // 6 Q1 m2 m3
        hipLaunchKernelGGL(k_load3_axis3, dim3(grid(size_t(X.Q) * Y.Q * Z.m)), dim3(kThreads), 0, s, X, Y, Z, U);
        hipLaunchKernelGGL(k_load3_axis2, dim3(grid(size_t(X.Q) * Y.m * Z.m)), dim3(kThreads), 0, s, X, Y, Z, U,
                           alpha, beta, V);
        hipLaunchKernelGGL(k_load3_axis1, dim3(grid(3 * size_t(X.m) * Y.m * Z.m)), dim3(kThreads), 0, s, X, Y, Z, V,
                           b);
    }
    check_launch("load_vector");
}

size_t load_vector_work(int d, const QuadDev* ax) {
    if (d == 2) return 4 * size_t(ax[0].Q) * ax[1].m;
    return size_t(kU3) * ax[0].Q * ax[1].Q * ax[2].m + 6 * size_t(ax[0].Q) * ax[1].m * ax[2].m;
}

void launch_l2_error(int d, const QuadDev* ax, const double* x, double* work, double* part, int nparts, hipStream_t s) {
    const QuadDev &X = ax[0], &Y = ax[1], &Z = ax[2];
    if (d == 2) {
        double* T = work;  // 2 m1 Q2
        hipLaunchKernelGGL(k_eval_last, dim3(grid(size_t(2) * X.m * Y.Q)), dim3(kThreads), 0, s, Y, x,
                           size_t(2) * X.m, T);
        hipLaunchKernelGGL(k_l2_last, dim3(nparts), dim3(kThreads), 0, s, 2, X, Y, Z, T, part);
    } else {
        double* T1 = work;                                // 3 m1 m2 Q3
        double* T2 = work + size_t(3) * X.m * Y.m * Z.Q;  // 3 m1 Q2 Q3
        hipLaunchKernelGGL(k_eval_last, dim3(grid(size_t(3) * X.m * Y.m * Z.Q)), dim3(kThreads), 0, s, Z, x,
                           size_t(3) * X.m * Y.m, T1);
        hipLaunchKernelGGL(k_eval_mid, dim3(grid(size_t(3) * X.m * Y.Q * Z.Q)), dim3(kThreads), 0, s, Y, T1,
                           size_t(3) * X.m, size_t(Z.Q), T2);
        hipLaunchKernelGGL(k_l2_last, dim3(nparts), dim3(kThreads), 0, s, 3, X, Y, Z, T2, part);
    }
    check_launch("l2_error");
}

size_t l2_error_work(int d, const QuadDev* ax) {
    if (d == 2) return 2 * size_t(ax[0].m) * ax[1].Q;
    return 3 * size_t(ax[0].m) * ax[1].m * ax[2].Q + 3 * size_t(ax[0].m) * ax[1].Q * ax[2].Q;
}

}  // namespace cd
