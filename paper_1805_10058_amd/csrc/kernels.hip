// HIP kernels for gfx950: grid transfers, banded Toeplitz line solves,
// reductions and the small Krylov helpers; the dispatch of the operator
// kernels (apply2d.hip, apply3d.hip).
//
// Every reduction accumulates in FP64 and combines partial sums in a fixed
// order, so results are bitwise reproducible run to run.
#include "apply_common.hpp"

namespace cd {

namespace {

// ------------------------------------------------------------------------------
// Grid transfers: Kronecker products of 1D prolongators, one thread per
// output entry (coarse entry for the restriction P^T r, fine entry for x += P e).
// ------------------------------------------------------------------------------
constexpr int kMaxWin = 8;  // widest prolongator window (p + 2 for p <= 6)

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(XferDev<T> X, int ncomp, const T* __restrict__ rf,
                                                       T* __restrict__ rc) {
    const XferAxisDev<T>& a0 = X.ax[0];
    const XferAxisDev<T>& a1 = X.ax[1];
    const XferAxisDev<T>& a2 = X.ax[2];
    const size_t Gc = size_t(a0.mc) * a1.mc * a2.mc;
    const size_t Gf = size_t(a0.mf) * a1.mf * a2.mf;
    const size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x;
    if (id >= Gc * ncomp) return;
    const int c = int(id / Gc);
    size_t rem = id % Gc;
    const int J2 = int(rem % a2.mc);
    rem /= a2.mc;
    const int J1 = int(rem % a1.mc);
    const int J0 = int(rem / a1.mc);
    T p2[kMaxWin];
#pragma unroll
    for (int k2 = 0; k2 < kMaxWin; ++k2) p2[k2] = (k2 < a2.wr) ? a2.vt[J2 * a2.wr + k2] : T(0);
    T acc = T(0);
    for (int k0 = 0; k0 < a0.wr; ++k0) {
        const T p0 = a0.vt[J0 * a0.wr + k0];
        const int i0 = a0.r0[J0] + k0;
        for (int k1 = 0; k1 < a1.wr; ++k1) {
            const T p1 = a1.vt[J1 * a1.wr + k1];
            const int i1 = a1.r0[J1] + k1;
            const T* row = rf + size_t(c) * Gf + (size_t(i0) * a1.mf + i1) * a2.mf + a2.r0[J2];
            T s2 = T(0);
#pragma unroll
            for (int k2 = 0; k2 < kMaxWin; ++k2)
                if (k2 < a2.wr) s2 += p2[k2] * row[k2];
            acc += p0 * p1 * s2;
        }
    }
    rc[id] = acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong_add(XferDev<T> X, int ncomp, const T* __restrict__ ec,
                                                          T* __restrict__ xf) {
    const XferAxisDev<T>& a0 = X.ax[0];
    const XferAxisDev<T>& a1 = X.ax[1];
    const XferAxisDev<T>& a2 = X.ax[2];
    const size_t Gc = size_t(a0.mc) * a1.mc * a2.mc;
    const size_t Gf = size_t(a0.mf) * a1.mf * a2.mf;
    const size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x;
    if (id >= Gf * ncomp) return;
    const int c = int(id / Gf);
    size_t rem = id % Gf;
    const int i2 = int(rem % a2.mf);
    rem /= a2.mf;
    const int i1 = int(rem % a1.mf);
    const int i0 = int(rem / a1.mf);
    T p2[kMaxWin];
#pragma unroll
    for (int k2 = 0; k2 < kMaxWin; ++k2) p2[k2] = (k2 < a2.w) ? a2.v[i2 * a2.w + k2] : T(0);
    T acc = T(0);
    for (int k0 = 0; k0 < a0.w; ++k0) {
        const T p0 = a0.v[i0 * a0.w + k0];
        const int J0 = a0.c0[i0] + k0;
        for (int k1 = 0; k1 < a1.w; ++k1) {
            const T p1 = a1.v[i1 * a1.w + k1];
            const int J1 = a1.c0[i1] + k1;
            const T* row = ec + size_t(c) * Gc + (size_t(J0) * a1.mc + J1) * a2.mc + a2.c0[i2];
            T s2 = T(0);
#pragma unroll
            for (int k2 = 0; k2 < kMaxWin; ++k2)
                if (k2 < a2.w) s2 += p2[k2] * row[k2];
            acc += p0 * p1 * s2;
        }
    }
    xf[id] += acc;
}

// The same transfers with every window width a compile-time constant, so all
// loads of a thread are independent and issue together (2D: the third axis
// has width 1).  Windows are stored clamped inside the matrix, so the fixed
// widths never read outside the vectors.
// CHEB: also the first Chebyshev step of the coarse level from zero,
// u = x = inv_theta D_c^{-1} rc, with D_c the diagonal of the coarse operator.
template <typename T, int W0, int W1, int W2, bool CHEB>
__global__ __launch_bounds__(kThreads) void k_restrict_w(XferDev<T> X, int ncomp, const T* __restrict__ rf,
                                                         T* __restrict__ rc, OpDev<T> opc, T inv_theta,
                                                         T* __restrict__ xo) {
    const XferAxisDev<T>& a0 = X.ax[0];
    const XferAxisDev<T>& a1 = X.ax[1];
    const XferAxisDev<T>& a2 = X.ax[2];
    const size_t Gc = size_t(a0.mc) * a1.mc * a2.mc;
    const size_t Gf = size_t(a0.mf) * a1.mf * a2.mf;
    const size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x;
    if (id >= Gc * ncomp) return;
    const int c = int(id / Gc);
    size_t rem = id % Gc;
    const int J2 = int(rem % a2.mc);
    rem /= a2.mc;
    const int J1 = int(rem % a1.mc);
    const int J0 = int(rem / a1.mc);
    const T* base = rf + size_t(c) * Gf + (size_t(a0.r0[J0]) * a1.mf + a1.r0[J1]) * a2.mf + a2.r0[J2];
    T acc = T(0);
#pragma unroll
    for (int k0 = 0; k0 < W0; ++k0) {
        const T p0 = a0.vt[J0 * W0 + k0];
#pragma unroll
        for (int k1 = 0; k1 < W1; ++k1) {
            const T p1 = a1.vt[J1 * W1 + k1];
            const T* row = base + (size_t(k0) * a1.mf + k1) * a2.mf;
            T s2 = T(0);
#pragma unroll
            for (int k2 = 0; k2 < W2; ++k2) s2 += a2.vt[J2 * W2 + k2] * row[k2];
            acc += p0 * p1 * s2;
        }
    }
    rc[id] = acc;
    if (CHEB) xo[id] = inv_theta * acc / diag_entry(opc, c, J0, J1, J2);
}

template <typename T, int W0, int W1, int W2>
__global__ __launch_bounds__(kThreads) void k_prolong_add_w(XferDev<T> X, int ncomp, const T* __restrict__ ec,
                                                            T* __restrict__ xf) {
    const XferAxisDev<T>& a0 = X.ax[0];
    const XferAxisDev<T>& a1 = X.ax[1];
    const XferAxisDev<T>& a2 = X.ax[2];
    const size_t Gc = size_t(a0.mc) * a1.mc * a2.mc;
    const size_t Gf = size_t(a0.mf) * a1.mf * a2.mf;
    const size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x;
    if (id >= Gf * ncomp) return;
    const int c = int(id / Gf);
    size_t rem = id % Gf;
    const int i2 = int(rem % a2.mf);
    rem /= a2.mf;
    const int i1 = int(rem % a1.mf);
    const int i0 = int(rem / a1.mf);
    const T* base = ec + size_t(c) * Gc + (size_t(a0.c0[i0]) * a1.mc + a1.c0[i1]) * a2.mc + a2.c0[i2];
    T acc = T(0);
#pragma unroll
    for (int k0 = 0; k0 < W0; ++k0) {
        const T p0 = a0.v[i0 * W0 + k0];
#pragma unroll
        for (int k1 = 0; k1 < W1; ++k1) {
            const T p1 = a1.v[i1 * W1 + k1];
            const T* row = base + (size_t(k0) * a1.mc + k1) * a2.mc;
            T s2 = T(0);
#pragma unroll
            for (int k2 = 0; k2 < W2; ++k2) s2 += a2.v[i2 * W2 + k2] * row[k2];
            acc += p0 * p1 * s2;
        }
    }
    xf[id] += acc;
}

// ------------------------------------------------------------------------------
// T^{-1}: banded LDL^T solves along every grid line of one axis, in two
// out-of-place passes (forward L y = v with y scaled by D^{-1}, then backward
// L^T z = y).  Each line is cut into chunks of `chunk` rows processed in
// parallel; a chunk's recurrence starts `warm` rows before (forward) or after
// (backward) the chunk from a zero state, which the recurrence forgets to
// below rounding within `warm` rows (the factor of T_m(m_{p-1}) is well
// conditioned), so every chunk reproduces the sequential solve.
// Consecutive threads take consecutive lines of the same chunk.
// ------------------------------------------------------------------------------
struct LineGeom {
    size_t G, lines_per_comp;
    int ma, axis, m1, m2, nchunk, chunk, ncomp;
};

constexpr int kLineThreads = 64;  // one wave per block in the line solves
constexpr int kRowGroup = 16;     // rows per group: staging loads and recurrence LDS reads

// First element of grid line `line` of component c along axis g.axis, and
// the stride between its rows.
__device__ inline size_t base_of(const LineGeom& g, size_t line, int c) {
    size_t b;
    if (g.axis == 0)
        b = line;
    else if (g.axis == 1)
        b = (line / g.m2) * size_t(g.m1) * g.m2 + line % g.m2;
    else
        b = line * g.m2;
    return b + size_t(c) * g.G;
}

__device__ inline size_t stride_of(const LineGeom& g) {
    return g.axis == 0 ? size_t(g.m1) * g.m2 : (g.axis == 1 ? size_t(g.m2) : size_t(1));
}

// Rows of the staged span, padded to a whole number of row groups.
__host__ __device__ inline int padded_span(int span) { return (span + kRowGroup - 1) / kRowGroup * kRowGroup; }

// One chunk of one grid line per lane; the 64 lanes of a block take 64
// consecutive lines of the same chunk (the line index is padded to a
// multiple of 64), so they share the row span [rs, re) = [r0-warm, r1+warm)
// clipped to the line.  LDS holds the lanes' values [row][lane] (conflict
// free), the factor rows of the span and 1/D, all padded to whole groups of
// 16 rows with zero factor entries, so no loop below branches per row:
//  1. staging: every lane issues the loads of two row groups (clamped to the
//     last row of the span) before it stores them, factor rows likewise;
//  2. forward L y = v over the padded span (padded rows carry 1/D = 0 and
//     store 0), keeping D^{-1} y in LDS;
//  3. backward L^T z = D^{-1} y from the top of the padded span down to the
//     chunk (zero padded rows keep the recurrence state at zero);
//  4. the chunk's rows [r0, r1) are written out.
// Out of place: in != out.
template <typename T, int BW>
__global__ __launch_bounds__(kLineThreads) void k_tsolve_line(const T* __restrict__ in, T* __restrict__ out,
                                                              LineGeom g, size_t lines_padded,
                                                              const T* __restrict__ L,
                                                              const T* __restrict__ dinv, int warm,
                                                              unsigned long long* stamp) {
    stamp_begin(stamp);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sp = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x;
    const size_t first = size_t(blockIdx.x) * kLineThreads;  // block-uniform
    const size_t grp = first / lines_padded;                  // (component, chunk) of the block
    const size_t line = first % lines_padded + lane;
    const int ch = int(grp % g.nchunk);
    const int c = int(grp / g.nchunk);
    const int r0 = ch * g.chunk, r1 = min(g.ma, r0 + g.chunk);
    const int rs = max(0, r0 - warm), re = min(g.ma, r1 + warm);
    const int span = re - rs;
    const int spanP = padded_span(span);
    T* cf = sp + size_t(spanP) * kLineThreads;  // [spanP + BW][BW] factor rows, zero past the span
    T* dv = cf + size_t(spanP + BW) * BW;       // [spanP] 1 / D, zero past the span
    const bool active = line < g.lines_per_comp;
    const size_t base = base_of(g, min(line, g.lines_per_comp - 1), c);
    // 1. staging: factor rows first, then the lane's values, two row groups of
    //    loads issued before they are stored.  Inactive lanes (line padding)
    //    load a valid line and are not used.
    const size_t stride = stride_of(g);
    {
        const int ncf = span * BW, ncfP = (spanP + BW) * BW;
        const T* Ls = L + size_t(rs) * BW;
        for (int e0 = 0; e0 < ncfP; e0 += 4 * kLineThreads) {
            T t[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * kLineThreads + lane;
                const T val = Ls[min(e, ncf - 1)];
                t[q] = (e < ncf) ? val : T(0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * kLineThreads + lane;
                if (e < ncfP) cf[e] = t[q];
            }
        }
        for (int e = lane; e < spanP; e += kLineThreads) {
            const T val = dinv[rs + min(e, span - 1)];
            dv[e] = (e < span) ? val : T(0);
        }
    }
    {
        const T* src = in + base;
        const int last = re - 1;
        for (int rb = 0; rb < spanP; rb += 2 * kRowGroup) {
            T v[2 * kRowGroup];
#pragma unroll
            for (int q = 0; q < 2 * kRowGroup; ++q) v[q] = src[size_t(min(rs + rb + q, last)) * stride];
#pragma unroll
            for (int q = 0; q < kRowGroup; ++q) sp[(rb + q) * kLineThreads + lane] = v[q];
            if (rb + kRowGroup < spanP) {
#pragma unroll
                for (int q = 0; q < kRowGroup; ++q) sp[(rb + kRowGroup + q) * kLineThreads + lane] = v[kRowGroup + q];
            }
        }
    }
    __syncthreads();
    if (active) {
        // 2. forward recurrence
        T win[BW];
    #pragma unroll
        for (int k = 0; k < BW; ++k) win[k] = T(0);
        for (int rb = 0; rb < spanP; rb += kRowGroup) {
            T v[kRowGroup];
    #pragma unroll
            for (int q = 0; q < kRowGroup; ++q) v[q] = sp[(rb + q) * kLineThreads + lane];
    #pragma unroll
            for (int q = 0; q < kRowGroup; ++q) {
                T x = v[q];
    #pragma unroll
                for (int k = 1; k <= BW; ++k) x -= cf[(rb + q) * BW + k - 1] * win[k - 1];
    #pragma unroll
                for (int k = BW - 1; k >= 1; --k) win[k] = win[k - 1];
                win[0] = x;
                v[q] = x * dv[rb + q];
            }
    #pragma unroll
            for (int q = 0; q < kRowGroup; ++q) sp[(rb + q) * kLineThreads + lane] = v[q];
        }
        // 3. backward recurrence, rows spanP-1 down to the chunk start (rows below
        //    it, clamped to row 0, only rewrite LDS rows that are not output)
        const int rlo = r0 - rs;
    #pragma unroll
        for (int k = 0; k < BW; ++k) win[k] = T(0);
        for (int rb = spanP - 1; rb >= rlo; rb -= kRowGroup) {
            T v[kRowGroup];
    #pragma unroll
            for (int q = 0; q < kRowGroup; ++q) v[q] = sp[max(rb - q, 0) * kLineThreads + lane];
    #pragma unroll
            for (int q = 0; q < kRowGroup; ++q) {
                const int r = max(rb - q, 0);
                T x = v[q];
    #pragma unroll
                for (int k = 1; k <= BW; ++k) x -= cf[(r + k) * BW + k - 1] * win[k - 1];
    #pragma unroll
                for (int k = BW - 1; k >= 1; --k) win[k] = win[k - 1];
                win[0] = x;
                v[q] = x;
            }
    #pragma unroll
            for (int q = 0; q < kRowGroup; ++q) sp[max(rb - q, 0) * kLineThreads + lane] = v[q];
        }
        // 4. output rows [r0, r1)
        T* dst = out + base;
        for (int r = r0; r < r1; ++r) dst[size_t(r) * stride] = sp[(r - rs) * kLineThreads + lane];
    }
    stamp_end(stamp);
}

// ------------------------------------------------------------------------------
// Vector kernels
// ------------------------------------------------------------------------------
template <typename TA, typename TB>
__global__ __launch_bounds__(kThreads) void k_dot_partial(const TA* __restrict__ a, const TB* __restrict__ b, size_t n,
                                                          double* __restrict__ part) {
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads)
        s += double(a[i]) * double(b[i]);
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_finalize(const double* __restrict__ part, int np, double* out) {
    const double s = sum_partials(part, np);
    if (threadIdx.x == 0) out[0] = s;
}

template <typename TO, typename TI>
__global__ __launch_bounds__(kThreads) void k_cast(const TI* __restrict__ x, TO* __restrict__ y, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads)
        y[i] = TO(x[i]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill(T* __restrict__ x, T v, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) x[i] = v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpby(T a, const T* __restrict__ x, T b, T* __restrict__ y, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads)
        y[i] = a * x[i] + b * y[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_normalize(const double* __restrict__ part, int np, const T* __restrict__ x,
                                                        T* __restrict__ y, size_t n) {
    const double ss = sum_partials(part, np);
    const T sc = ss > 0.0 ? T(1.0 / sqrt(ss)) : T(0);
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads)
        y[i] = x[i] * sc;
}

template <typename T>
__device__ inline void unflatten(const OpDev<T>& op, size_t id, int& c, int& i0, int& i1, int& i2) {
    const size_t G = size_t(op.m[0]) * op.m[1] * op.m[2];
    c = int(id / G);
    size_t rem = id % G;
    i2 = int(rem % op.m[2]);
    rem /= op.m[2];
    i1 = int(rem % op.m[1]);
    i0 = int(rem / op.m[1]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_diag_scale(OpDev<T> op, bool inv, const T* __restrict__ x,
                                                         T* __restrict__ y, size_t n) {
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        const T d = diag_entry(op, c, i0, i1, i2);
        y[id] = inv ? x[id] / d : x[id] * d;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_diag_dot(OpDev<T> op, const T* __restrict__ x, size_t n,
                                                       double* __restrict__ part) {
    double s = 0.0;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        const double d = double(diag_entry(op, c, i0, i1, i2));
        s += d * double(x[id]) * double(x[id]);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Dense form of a level operator, padded to ld x ld with an identity tail.
// Entry ((c, i), (e, j)) of the block operator: on the diagonal blocks
// beta * (S on axis c, M elsewhere) + alpha * sum over the other axes f of
// (S on f, M elsewhere); off the diagonal (alpha - beta) * (A on axes c and
// e, M elsewhere), each a product of 1D entries X(i_l, j_l).
__global__ __launch_bounds__(kThreads) void k_dense_operator(OpDev<double> op, double* __restrict__ out, int ld,
                                                             size_t N) {
    const size_t G = size_t(op.m[0]) * op.m[1] * op.m[2];
    const size_t total = size_t(ld) * ld;
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < total; id += size_t(gridDim.x) * kThreads) {
        const size_t row = id / ld, col = id % ld;
        double v = (row == col) ? 1.0 : 0.0;
        if (row < N && col < N) {
            int c, i[3], e, j[3];
            unflatten(op, row, c, i[0], i[1], i[2]);
            unflatten(op, col, e, j[0], j[1], j[2]);
            bool near = true;
            double Mv[3], Av[3], Sv[3];
            for (int l = 0; l < op.dim; ++l) {
                const int k = j[l] - i[l] + op.hb;
                if (k < 0 || k > 2 * op.hb) {
                    near = false;
                    break;
                }
                Mv[l] = band_at(op, l, 0, k, i[l]);
                Av[l] = band_at(op, l, 1, k, i[l]);
                Sv[l] = band_at(op, l, 2, k, i[l]);
            }
            v = 0.0;
            if (near) {
                if (c == e) {
                    for (int f = 0; f < op.dim; ++f) {
                        double t = (f == c) ? op.beta : op.alpha;
                        for (int l = 0; l < op.dim; ++l) t *= (l == f) ? Sv[l] : Mv[l];
                        v += t;
                    }
                } else {
                    v = offdiag_weight(op);
                    for (int l = 0; l < op.dim; ++l) v *= (l == c || l == e) ? Av[l] : Mv[l];
                }
            }
        }
        out[id] = v;
    }
}

// Breakdown test of the Lanczos recurrence: beta <= kLanczosBreakdown |alpha|
// (in squares, beta2 <= tol^2 alpha^2) means the Krylov space is invariant.
constexpr double kLanczosBreakdown = 1e-10;

__device__ inline bool lanczos_broke(double beta2, double alpha) {
    return beta2 <= kLanczosBreakdown * kLanczosBreakdown * alpha * alpha;
}

// One Lanczos step on D^{-1} A in the D inner product: w holds A q on entry
// and w = D^{-1} A q - alpha q - beta qp on exit, beta = sqrt(beta2), or 0
// when the previous step broke down (q is then the restart vector).
__global__ __launch_bounds__(kThreads) void k_lanczos_step(OpDev<double> op, const double* __restrict__ alpha,
                                                           const double* __restrict__ alpha_prev,
                                                           const double* __restrict__ beta2,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ qp, double* __restrict__ w,
                                                           size_t n) {
    const double a = alpha[0], b = lanczos_broke(beta2[0], alpha_prev[0]) ? 0.0 : sqrt(beta2[0]);
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        w[id] = w[id] / diag_entry(op, c, i0, i1, i2) - a * q[id] - b * qp[id];
    }
}

// Next Lanczos vector: w / beta (beta2 = |w|_D^2), or the D-normalised
// restart vector r when the step broke down.
__global__ __launch_bounds__(kThreads) void k_lanczos_next(const double* __restrict__ alpha,
                                                           const double* __restrict__ beta2,
                                                           const double* __restrict__ w,
                                                           const double* __restrict__ r, double* __restrict__ q,
                                                           size_t n) {
    const bool broke = lanczos_broke(beta2[0], alpha[0]);
    const double sc = broke ? 0.0 : 1.0 / sqrt(beta2[0]);
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads)
        q[i] = broke ? r[i] : w[i] * sc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cheb_first(OpDev<T> op, const T* __restrict__ b, T* __restrict__ x,
                                                         T inv_theta, size_t n) {
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        x[id] = inv_theta * b[id] / diag_entry(op, c, i0, i1, i2);
    }
}

// y = x (converted) and the first Chebyshev step from zero on y.
template <typename TO, typename TI>
__global__ __launch_bounds__(kThreads) void k_cast_cheb(const TI* __restrict__ x, TO* __restrict__ y, size_t n,
                                                        OpDev<TO> op, TO inv_theta, TO* __restrict__ xo) {
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        const TO b = TO(x[id]);
        y[id] = b;
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        xo[id] = inv_theta * b / diag_entry(op, c, i0, i1, i2);
    }
}

// y = x (converted) and part[block] = partial sums of y . q (FP64).
template <typename TO, typename TI>
__global__ __launch_bounds__(kThreads) void k_cast_dot(const TI* __restrict__ x, TO* __restrict__ y, size_t n,
                                                       const double* __restrict__ q, double* __restrict__ part) {
    double acc = 0.0;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        const TO v = TO(x[i]);
        y[i] = v;
        acc += double(v) * q[i];
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// z = Kinv r, one block per row, FP64 accumulation
template <typename T>
__global__ __launch_bounds__(kThreads) void k_coarse_gemv(const double* __restrict__ Kinv, int N, int ld,
                                                          const T* __restrict__ r, T* __restrict__ z) {
    const int row = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < N; j += kThreads) s += Kinv[size_t(row) * ld + j] * double(r[j]);
    s = block_sum(s);
    if (threadIdx.x == 0) z[row] = T(s);
}

// ---- flexible CG ----------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fcg_direction(int first, const T* __restrict__ z,
                                                            const double* __restrict__ pzq, int npzq,
                                                            const double* __restrict__ dq_prev, T* __restrict__ d,
                                                            const T* __restrict__ r, double* __restrict__ pdr,
                                                            double* __restrict__ beta_out, size_t n) {
    double beta = 0.0;
    if (!first) {
        const double zq = sum_partials(pzq, npzq);
        const double dq = dq_prev[0];
        beta = (dq != 0.0) ? zq / dq : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) beta_out[0] = beta;
    const T bt = T(beta);
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        const T dn = first ? z[i] : z[i] - bt * d[i];
        d[i] = dn;
        s += double(dn) * double(r[i]);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) pdr[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fcg_update(const double* __restrict__ pdr, int npdr,
                                                         const double* __restrict__ pdq, int npdq,
                                                         double* __restrict__ dq_out, T* __restrict__ x,
                                                         T* __restrict__ r, const T* __restrict__ d,
                                                         const T* __restrict__ q, double* __restrict__ prr,
                                                         double* __restrict__ a_out, size_t n) {
    const double dr = sum_partials(pdr, npdr);
    const double dq = sum_partials(pdq, npdq);
    const double a = (dq != 0.0) ? dr / dq : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        dq_out[0] = dq;
        a_out[0] = a;
    }
    const T at = T(a);
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        x[i] += at * d[i];
        const T rn = r[i] - at * q[i];
        r[i] = rn;
        s += double(rn) * double(rn);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) prr[blockIdx.x] = s;
}

// ---- GMRES helpers -----------------------------------------------------------------

// Least squares min || beta0 e1 - H y || for the (k+1) x k Hessenberg H
// (column-major, leading dimension ld) by Givens rotations, one thread.
__device__ inline void hessenberg_lsq(const double* __restrict__ H, int ld, int k, double beta0, double* y) {
    double R[kMaxBasis + 1][kMaxBasis];
    double g[kMaxBasis + 1];
#pragma unroll
    for (int i = 0; i <= kMaxBasis; ++i) {
        g[i] = 0.0;
#pragma unroll
        for (int j = 0; j < kMaxBasis; ++j) R[i][j] = (i <= k && j < k) ? H[size_t(j) * ld + i] : 0.0;
    }
    g[0] = beta0;
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j) {
        if (j < k) {
            const double a = R[j][j], b = R[j + 1][j];
            const double rr = sqrt(a * a + b * b);
            const double c = (rr > 0.0) ? a / rr : 1.0, sn = (rr > 0.0) ? b / rr : 0.0;
#pragma unroll
            for (int col = 0; col < kMaxBasis; ++col) {
                if (col >= j) {
                    const double t0 = R[j][col], t1 = R[j + 1][col];
                    R[j][col] = c * t0 + sn * t1;
                    R[j + 1][col] = -sn * t0 + c * t1;
                }
            }
            const double g0 = g[j], g1 = g[j + 1];
            g[j] = c * g0 + sn * g1;
            g[j + 1] = -sn * g0 + c * g1;
        }
    }
#pragma unroll
    for (int i = kMaxBasis - 1; i >= 0; --i) {
        if (i < k) {
            double sum = g[i];
#pragma unroll
            for (int col = 0; col < kMaxBasis; ++col)
                if (col > i && col < k) sum -= R[i][col] * y[col];
            y[i] = (fabs(R[i][i]) > 0.0) ? sum / R[i][i] : 0.0;
        }
    }
}

// Classical Gram-Schmidt step with the Pythagorean norm, one pass: every
// block sums the partials of the k dots V_i . w and of w . w (written by the
// operator kernel, the same order in every block): h_i = V_i . w,
// ||w'||^2 = w . w - sum h_i^2 for w' = w - sum h_i V_i.  Block 0 stores
// H(0..k-1, j) = h and H(k, j) = ||w'||; with v given, v = w' / ||w'||
// (zero if ||w'|| = 0).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gs_normscale(const double* __restrict__ pdot, int k, int nbp,
                                                           double* __restrict__ Hcol, const T* __restrict__ V,
                                                           const T* __restrict__ w, T* __restrict__ v, size_t n) {
    __shared__ double hs[kMaxBasis + 1];
    for (int i = 0; i <= k; ++i) {
        const double t = sum_partials(pdot + size_t(i) * nbp, nbp);
        if (threadIdx.x == 0) hs[i] = t;
    }
    __syncthreads();
    double h2 = 0.0;
    for (int i = 0; i < k; ++i) h2 += hs[i] * hs[i];
    const double nrm = sqrt(fmax(hs[k] - h2, 0.0));
    if (blockIdx.x == 0 && threadIdx.x < k) Hcol[threadIdx.x] = hs[threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) Hcol[k] = nrm;
    if (v == nullptr) return;
    T h[kMaxBasis];
#pragma unroll
    for (int i = 0; i < kMaxBasis; ++i) h[i] = (i < k) ? T(hs[i]) : T(0);
    const T sc = (nrm != 0.0) ? T(1.0 / nrm) : T(0);
    for (size_t e = size_t(blockIdx.x) * kThreads + threadIdx.x; e < n; e += size_t(gridDim.x) * kThreads) {
        T a = w[e];
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i)
            if (i < k) a -= h[i] * V[size_t(i) * n + e];
        v[e] = a * sc;
    }
}

// The smoother's update: y = argmin || beta0 e1 - H y || (every block solves
// the small problem itself), then x += sum_j y_j Z_j.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsq_combine_add(const double* __restrict__ H, int ld, int k,
                                                              const double* __restrict__ beta0sq,
                                                              const T* __restrict__ Z, T* __restrict__ x,
                                                              size_t n) {
    __shared__ double ys[kMaxBasis];
    if (threadIdx.x == 0) {
        double y[kMaxBasis];
        hessenberg_lsq(H, ld, k, sqrt(beta0sq[0]), y);
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i) ys[i] = (i < k) ? y[i] : 0.0;
    }
    __syncthreads();
    T yv[kMaxBasis];
#pragma unroll
    for (int i = 0; i < kMaxBasis; ++i) yv[i] = T(ys[i]);
    for (size_t e = size_t(blockIdx.x) * kThreads + threadIdx.x; e < n; e += size_t(gridDim.x) * kThreads) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < kMaxBasis; ++j)
            if (j < k) acc += yv[j] * Z[size_t(j) * n + e];
        x[e] += acc;
    }
}

// ss = sum of the partials (every block); block 0 stores ss or sqrt(ss);
// v = w / sqrt(ss) when v is given.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_normscale(const double* __restrict__ pnorm, int np,
                                                        double* __restrict__ out, int square,
                                                        const T* __restrict__ w, T* __restrict__ v, size_t n) {
    const double ss = sum_partials(pnorm, np);
    const double nrm = sqrt(ss);
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = square ? ss : nrm;
    if (v == nullptr) return;
    const T sc = (nrm != 0.0) ? T(1.0 / nrm) : T(0);
    for (size_t e = size_t(blockIdx.x) * kThreads + threadIdx.x; e < n; e += size_t(gridDim.x) * kThreads)
        v[e] = w[e] * sc;
}

// pairs[2 s] = start, pairs[2 s + 1] = latest end of slot s (one block per
// slot); the slot's words are cleared for its next use (start to max: a slot
// no kernel wrote reads as (max, 0)).
__global__ __launch_bounds__(kThreads) void k_stamp_reduce(unsigned long long* __restrict__ st, int slot0,
                                                           unsigned long long* __restrict__ pairs) {
    __shared__ unsigned long long red[kThreads];
    const int sl = slot0 + blockIdx.x;
    unsigned long long* p = st + size_t(sl) * kStampWords;
    unsigned long long mx = 0;
    for (int i = threadIdx.x; i < kStampEnds; i += kThreads) {
        mx = max(mx, p[1 + i]);
        p[1 + i] = 0;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pairs[2 * sl] = p[0];
        pairs[2 * sl + 1] = red[0];
        p[0] = ~0ull;
    }
}

int grid_for(size_t n) {
    const size_t nb = (n + kThreads - 1) / kThreads;
    return int(std::max<size_t>(1, std::min<size_t>(nb, 8192)));
}

}  // namespace

// ================================ launch wrappers =================================

int reduce_blocks(size_t n) {
    const size_t nb = (n + size_t(kThreads) * 2 - 1) / (size_t(kThreads) * 2);
    return int(std::max<size_t>(1, std::min<size_t>(nb, 1024)));
}

template <typename T>
int apply_blocks(const OpDev<T>& op) {
    if (op.dim == 3) return apply3d_geom(op.m, op.hb, sizeof(T), op.x1chunk).nblocks;
    return ((op.m[0] + kT1 - 1) / kT1) * ((op.m[1] + kT2 - 1) / kT2);
}

template <typename T>
void launch_apply(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part,
                  hipStream_t s, int nv, unsigned long long* stamp) {
    if (mode == kApplyYMulti && (nv < 1 || nv > kMaxBasis)) throw std::runtime_error("bad number of dot vectors");
    if (mode < kApplyY || mode > kApplyYMulti) throw std::runtime_error("bad apply mode");
#define CD_APPLY_CASE(H)                                                                      \
    case H:                                                                                   \
        if (op.dim == 3)                                                                      \
            apply3d_run<T, H>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s);        \
        else                                                                                  \
            apply2d_run<T, H>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s);        \
        break;
    switch (op.hb) {
        CD_APPLY_CASE(1)
        CD_APPLY_CASE(2)
        CD_APPLY_CASE(3)
        CD_APPLY_CASE(4)
        CD_APPLY_CASE(5)
        CD_APPLY_CASE(6)
        default: throw std::runtime_error("degree out of range (1..6)");
    }
#undef CD_APPLY_CASE
}

// Fixed-width kernel when every real axis has the same window width w
// (2D: <w, w, 1>, 3D: <w, w, w>); the generic kernel otherwise.
template <typename T, bool Restrict, int W>
bool launch_xfer_w(const XferDev<T>& X, int ncomp, const T* in, T* out, size_t n, const ChebFirst<T>* cf,
                   hipStream_t s) {
    const dim3 grid((n + kThreads - 1) / kThreads);
    const ChebFirst<T> c0{};
    const ChebFirst<T>& c = cf ? *cf : c0;
    if (X.dim == 2) {
        if (Restrict && cf)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, 1, true>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.x);
        else if (Restrict)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, 1, false>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.x);
        else
            hipLaunchKernelGGL((k_prolong_add_w<T, W, W, 1>), grid, dim3(kThreads), 0, s, X, ncomp, in, out);
    } else {
        if (Restrict && cf)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, W, true>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.x);
        else if (Restrict)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, W, false>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.x);
        else
            hipLaunchKernelGGL((k_prolong_add_w<T, W, W, W>), grid, dim3(kThreads), 0, s, X, ncomp, in, out);
    }
    return true;
}

template <typename T, bool Restrict>
bool launch_xfer_fixed(const XferDev<T>& X, int ncomp, const T* in, T* out, size_t n, const ChebFirst<T>* cf,
                       hipStream_t s) {
    auto width = [&](int a) { return Restrict ? X.ax[a].wr : X.ax[a].w; };
    const int w = width(0);
    for (int a = 1; a < X.dim; ++a)
        if (width(a) != w) return false;
    for (int a = X.dim; a < 3; ++a)
        if (width(a) != 1) return false;
    switch (w) {
        case 2: return launch_xfer_w<T, Restrict, 2>(X, ncomp, in, out, n, cf, s);
        case 3: return launch_xfer_w<T, Restrict, 3>(X, ncomp, in, out, n, cf, s);
        case 4: return launch_xfer_w<T, Restrict, 4>(X, ncomp, in, out, n, cf, s);
        case 5: return launch_xfer_w<T, Restrict, 5>(X, ncomp, in, out, n, cf, s);
        case 6: return launch_xfer_w<T, Restrict, 6>(X, ncomp, in, out, n, cf, s);
        case 7: return launch_xfer_w<T, Restrict, 7>(X, ncomp, in, out, n, cf, s);
        case 8: return launch_xfer_w<T, Restrict, 8>(X, ncomp, in, out, n, cf, s);
        default: return false;
    }
}

template <typename T>
void launch_restrict(const XferDev<T>& X, int ncomp, const T* rf, T* rc, hipStream_t s, const ChebFirst<T>* cf) {
    const size_t n = size_t(ncomp) * X.ax[0].mc * X.ax[1].mc * X.ax[2].mc;
    if (!launch_xfer_fixed<T, true>(X, ncomp, rf, rc, n, cf, s)) {
        hipLaunchKernelGGL(k_restrict<T>, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, X, ncomp, rf,
                           rc);
        if (cf) launch_cheb_first<T>(cf->op, rc, cf->x, cf->inv_theta, s);
    }
    check_launch("restrict");
}

template <typename T>
void launch_prolong_add(const XferDev<T>& X, int ncomp, const T* ec, T* xf, hipStream_t s) {
    const size_t n = size_t(ncomp) * X.ax[0].mf * X.ax[1].mf * X.ax[2].mf;
    if (!launch_xfer_fixed<T, false>(X, ncomp, ec, xf, n, nullptr, s))
        hipLaunchKernelGGL(k_prolong_add<T>, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, X, ncomp,
                           ec, xf);
    check_launch("prolong");
}

template <typename T, int BW>
void tsolve_axis(const T* v, T* z, const LineGeom& g, const TFacDev<T>& F, size_t lines_padded, size_t lds,
                 unsigned long long* stamp, hipStream_t s) {
    const size_t items = lines_padded * g.nchunk * size_t(g.ncomp);
    const dim3 grid(items / kLineThreads);
    auto kern = k_tsolve_line<T, BW>;
    allow_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, grid, dim3(kLineThreads), lds, s, v, z, g, lines_padded, F.l, F.dinv, F.warm, stamp);
}

template <typename T>
void launch_tsolve(int dim, const int* m, const TFacDev<T>* fac, const T* v, T* tmp, T* z, hipStream_t s,
                   unsigned long long* stamps) {
    if (v == z || v == tmp || tmp == z) throw std::runtime_error("tsolve needs three distinct buffers");
    const int m0 = m[0], m1 = m[1], m2 = (dim == 3) ? m[2] : 1;
    const size_t G = size_t(m0) * m1 * m2;
    if (fac[0].bw == 0) {  // p = 1: T is the identity
        launch_copy<T>(v, z, size_t(dim) * G, s);
        return;
    }
    const T* src = v;
    for (int a = 0; a < dim; ++a) {
        // alternate destinations so that the last pass lands in z
        T* dst = ((dim - 1 - a) % 2 == 0) ? z : tmp;
        unsigned long long* st = stamps ? stamps + size_t(a) * kStampWords : nullptr;
        const TFacDev<T>& F = fac[a];
        LineGeom g;
        g.G = G;
        g.ma = F.m;
        g.axis = a;
        g.m1 = m1;
        g.m2 = m2;
        g.lines_per_comp = G / F.m;
        const size_t lines = size_t(dim) * g.lines_per_comp;
        // enough independent chunks to fill the device; a chunk is then grown
        // to fill the padding of its staged span (chunk + 2 warm rows,
        // rounded up to whole row groups), which costs nothing extra
        const size_t want = (size_t(1) << 17) / std::max<size_t>(lines, 1) + 1;
        const int nc0 = int(std::max<size_t>(1, std::min<size_t>(want, size_t((F.m + 15) / 16))));
        int chunk = (F.m + nc0 - 1) / nc0;
        if (chunk < F.m) chunk = std::max(chunk, padded_span(chunk + 2 * F.warm) - 2 * F.warm);
        g.chunk = std::min(chunk, F.m);
        g.nchunk = (F.m + g.chunk - 1) / g.chunk;
        const int spanP = padded_span(std::min(F.m, g.chunk + 2 * F.warm));
        const size_t lds = (size_t(spanP) * (kLineThreads + F.bw + 1) + size_t(F.bw) * F.bw) * sizeof(T);
        if (lds > 160 * 1024) throw std::runtime_error("T-solve span does not fit in LDS");
        g.ncomp = dim;
        const size_t lp = (g.lines_per_comp + kLineThreads - 1) / kLineThreads * kLineThreads;
        switch (F.bw) {
            case 1: tsolve_axis<T, 1>(src, dst, g, F, lp, lds, st, s); break;
            case 2: tsolve_axis<T, 2>(src, dst, g, F, lp, lds, st, s); break;
            case 3: tsolve_axis<T, 3>(src, dst, g, F, lp, lds, st, s); break;
            case 4: tsolve_axis<T, 4>(src, dst, g, F, lp, lds, st, s); break;
            case 5: tsolve_axis<T, 5>(src, dst, g, F, lp, lds, st, s); break;
            default: throw std::runtime_error("degree out of range (1..6)");
        }
        check_launch("tsolve");
        src = dst;
    }
}

template <typename TA, typename TB>
void launch_dot_partial(const TA* a, const TB* b, size_t n, double* part, hipStream_t s) {
    hipLaunchKernelGGL((k_dot_partial<TA, TB>), dim3(reduce_blocks(n)), dim3(kThreads), 0, s, a, b, n, part);
    check_launch("dot");
}

void launch_finalize(const double* part, int np, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, part, np, out);
    check_launch("finalize");
}

template <typename TO, typename TI>
void launch_cast_cheb(const TI* x, TO* y, size_t n, const ChebFirst<TO>& cf, hipStream_t s) {
    hipLaunchKernelGGL((k_cast_cheb<TO, TI>), dim3(grid_for(n)), dim3(kThreads), 0, s, x, y, n, cf.op, cf.inv_theta,
                       cf.x);
    check_launch("cast_cheb");
}

template <typename TO, typename TI>
void launch_cast_dot(const TI* x, TO* y, size_t n, const double* q, double* part, hipStream_t s) {
    hipLaunchKernelGGL((k_cast_dot<TO, TI>), dim3(reduce_blocks(n)), dim3(kThreads), 0, s, x, y, n, q, part);
    check_launch("cast_dot");
}

template <typename TO, typename TI>
void launch_cast(const TI* x, TO* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_cast<TO, TI>), dim3(grid_for(n)), dim3(kThreads), 0, s, x, y, n);
    check_launch("cast");
}

template <typename T>
void launch_fill(T* x, T v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, x, v, n);
    check_launch("fill");
}

template <typename T>
void launch_copy(const T* x, T* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_cast<T, T>), dim3(grid_for(n)), dim3(kThreads), 0, s, x, y, n);
    check_launch("copy");
}

template <typename T>
void launch_axpby(T a, const T* x, T b, T* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, a, x, b, y, n);
    check_launch("axpby");
}

template <typename T>
void launch_normalize(const double* part, int np, const T* x, T* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_normalize<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, part, np, x, y, n);
    check_launch("normalize");
}

template <typename T>
static size_t op_len(const OpDev<T>& op) {
    return size_t(op.dim) * op.m[0] * op.m[1] * op.m[2];
}

template <typename T>
void launch_diag_scale(const OpDev<T>& op, bool inv, const T* x, T* y, hipStream_t s) {
    const size_t n = op_len(op);
    hipLaunchKernelGGL(k_diag_scale<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, op, inv, x, y, n);
    check_launch("diag_scale");
}

template <typename T>
void launch_diag_dot(const OpDev<T>& op, const T* x, double* part, hipStream_t s) {
    const size_t n = op_len(op);
    hipLaunchKernelGGL(k_diag_dot<T>, dim3(reduce_blocks(n)), dim3(kThreads), 0, s, op, x, n, part);
    check_launch("diag_dot");
}

void launch_dense_operator(const OpDev<double>& op, double* out, int ld, hipStream_t s) {
    const size_t N = op_len(op);
    if (size_t(ld) < N) throw std::runtime_error("dense_operator: padded order below the operator's");
    hipLaunchKernelGGL(k_dense_operator, dim3(grid_for(size_t(ld) * ld)), dim3(kThreads), 0, s, op, out, ld, N);
    check_launch("dense_operator");
}

void launch_lanczos_step(const OpDev<double>& op, const double* alpha, const double* alpha_prev, const double* beta2,
                         const double* q, const double* qp, double* w, hipStream_t s) {
    const size_t n = op_len(op);
    hipLaunchKernelGGL(k_lanczos_step, dim3(grid_for(n)), dim3(kThreads), 0, s, op, alpha, alpha_prev, beta2, q, qp,
                       w, n);
    check_launch("lanczos_step");
}

void launch_lanczos_next(const double* alpha, const double* beta2, const double* w, const double* r, double* q,
                         size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos_next, dim3(grid_for(n)), dim3(kThreads), 0, s, alpha, beta2, w, r, q, n);
    check_launch("lanczos_next");
}

template <typename T>
void launch_cheb_first(const OpDev<T>& op, const T* b, T* x, T inv_theta, hipStream_t s) {
    const size_t n = op_len(op);
    hipLaunchKernelGGL(k_cheb_first<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, op, b, x, inv_theta, n);
    check_launch("cheb_first");
}

template <typename T>
void launch_coarse_gemv(const double* Kinv, int N, int ld, const T* r, T* z, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_gemv<T>, dim3(N), dim3(kThreads), 0, s, Kinv, N, ld, r, z);
    check_launch("coarse_gemv");
}

template <typename T>
void launch_fcg_direction(bool first, const T* z, const double* pzq, int npzq, const double* dq_prev, T* d,
                          const T* r, double* pdr, double* beta_out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_direction<T>, dim3(reduce_blocks(n)), dim3(kThreads), 0, s, first ? 1 : 0, z, pzq, npzq,
                       dq_prev, d, r, pdr, beta_out, n);
    check_launch("fcg_direction");
}

template <typename T>
void launch_fcg_update(const double* pdr, int npdr, const double* pdq, int npdq, double* dq_out, T* x, T* r,
                       const T* d, const T* q, double* prr, double* a_out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_update<T>, dim3(reduce_blocks(n)), dim3(kThreads), 0, s, pdr, npdr, pdq, npdq, dq_out, x,
                       r, d, q, prr, a_out, n);
    check_launch("fcg_update");
}






void launch_stamp_reduce(unsigned long long* st, int slot0, int nslots, unsigned long long* pairs, hipStream_t s) {
    if (nslots <= 0) return;
    hipLaunchKernelGGL(k_stamp_reduce, dim3(nslots), dim3(kThreads), 0, s, st, slot0, pairs);
    check_launch("stamp_reduce");
}



template <typename T>
void launch_normscale(const double* pnorm, int np, double* out, bool square, const T* w, T* v, size_t n,
                      hipStream_t s) {
    const int grid = (v == nullptr) ? 1 : grid_for(n);
    hipLaunchKernelGGL(k_normscale<T>, dim3(grid), dim3(kThreads), 0, s, pnorm, np, out, square ? 1 : 0, w, v, n);
    check_launch("normscale");
}

template <typename T>
void launch_gs_normscale(const double* pdot, int k, int nbp, double* Hcol, const T* V, const T* w, T* v, size_t n,
                         hipStream_t s) {
    if (k < 1 || k > kMaxBasis) throw std::runtime_error("bad number of Krylov vectors");
    const int grid = (v == nullptr) ? 1 : grid_for(n);
    hipLaunchKernelGGL(k_gs_normscale<T>, dim3(grid), dim3(kThreads), 0, s, pdot, k, nbp, Hcol, V, w, v, n);
    check_launch("gs_normscale");
}

template <typename T>
void launch_lsq_combine_add(const double* H, int ld, int k, const double* beta0sq, const T* Z, T* x, size_t n,
                            hipStream_t s) {
    if (k < 1 || k > kMaxBasis) throw std::runtime_error("bad number of Krylov vectors");
    hipLaunchKernelGGL(k_lsq_combine_add<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, H, ld, k, beta0sq, Z, x, n);
    check_launch("lsq_combine_add");
}

// ---- explicit instantiations ----
#define CD_INST(T)                                                                                                   \
    template int apply_blocks<T>(const OpDev<T>&);                                                                   \
    template void launch_apply<T>(const OpDev<T>&, int, const T*, T*, const T*, T*, T*, T, T, double*, hipStream_t,  \
                                  int, unsigned long long*);                                                         \
    template void launch_restrict<T>(const XferDev<T>&, int, const T*, T*, hipStream_t, const ChebFirst<T>*);        \
    template void launch_prolong_add<T>(const XferDev<T>&, int, const T*, T*, hipStream_t);                          \
    template void launch_tsolve<T>(int, const int*, const TFacDev<T>*, const T*, T*, T*, hipStream_t,                \
                                   unsigned long long*);                            \
    template void launch_fcg_direction<T>(bool, const T*, const double*, int, const double*, T*, const T*, double*,   \
                                          double*, size_t, hipStream_t);                                             \
    template void launch_fcg_update<T>(const double*, int, const double*, int, double*, T*, T*, const T*, const T*,   \
                                       double*, double*, size_t, hipStream_t);                                       \
    template void launch_fill<T>(T*, T, size_t, hipStream_t);                                                        \
    template void launch_copy<T>(const T*, T*, size_t, hipStream_t);                                                 \
    template void launch_axpby<T>(T, const T*, T, T*, size_t, hipStream_t);                                          \
    template void launch_normalize<T>(const double*, int, const T*, T*, size_t, hipStream_t);                        \
    template void launch_diag_scale<T>(const OpDev<T>&, bool, const T*, T*, hipStream_t);                            \
    template void launch_diag_dot<T>(const OpDev<T>&, const T*, double*, hipStream_t);                               \
    template void launch_cheb_first<T>(const OpDev<T>&, const T*, T*, T, hipStream_t);                           \
    template void launch_coarse_gemv<T>(const double*, int, int, const T*, T*, hipStream_t);                              \
    template void launch_gs_normscale<T>(const double*, int, int, double*, const T*, const T*, T*, size_t,            \
                                         hipStream_t);                                                               \
    template void launch_lsq_combine_add<T>(const double*, int, int, const double*, const T*, T*, size_t,            \
                                            hipStream_t);                                                            \
    template void launch_normscale<T>(const double*, int, double*, bool, const T*, T*, size_t, hipStream_t);

CD_INST(double)
CD_INST(float)

template void launch_dot_partial<double, double>(const double*, const double*, size_t, double*, hipStream_t);
template void launch_dot_partial<float, float>(const float*, const float*, size_t, double*, hipStream_t);
template void launch_cast<float, double>(const double*, float*, size_t, hipStream_t);
template void launch_cast<double, float>(const float*, double*, size_t, hipStream_t);
template void launch_cast_cheb<float, double>(const double*, float*, size_t, const ChebFirst<float>&, hipStream_t);
template void launch_cast_cheb<double, double>(const double*, double*, size_t, const ChebFirst<double>&,
                                               hipStream_t);
template void launch_cast_dot<double, float>(const float*, double*, size_t, const double*, double*, hipStream_t);
template void launch_cast_dot<double, double>(const double*, double*, size_t, const double*, double*, hipStream_t);

}  // namespace cd
