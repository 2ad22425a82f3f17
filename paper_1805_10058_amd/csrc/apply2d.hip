// 2D curl-div operator apply (sum factorization), one object per (precision,
// half bandwidth): compiled with -DCD_T=<float|double> -DCD_HB=<1..6>.
#include "apply_common.hpp"

namespace cd {
namespace {

// ------------------------------------------------------------------------------
// 2D operator apply on tiles of kT1 x kT2 output points (x1 rows, x2 columns;
// x2 contiguous).  The block issues the loads of its input tile (both
// components, +-HB halo on both axes, zero outside the grid) before storing
// any of them to LDS, then
//   (A) contracts axis 1: S1 x, M1 x, A1 x of both components at the kT1
//       output rows and all kT2 + 2HB tile columns;
//   (B) contracts axis 2 at the output point:
//   y1 = beta M2(S1 x1) + alpha S2(M1 x1) + (alpha-beta) A2(A1 x2)
//   y2 = alpha M2(S1 x2) + beta S2(M1 x2) + (alpha-beta) A2(A1 x1)
// 12 band contractions per point.
// ------------------------------------------------------------------------------

template <typename T, int HB, int MODE>
__global__ __launch_bounds__(kThreads) void k_apply2d(OpDev<T> op, const T* __restrict__ x, T* __restrict__ y,
                                                      const T* __restrict__ b, T* u,
                                                      T* xout, T c1, T c2, double* __restrict__ part,
                                                      int nv, unsigned long long* stamp) {
    stamp_begin(stamp);
    constexpr int R = 2 * HB + 1;
    constexpr int E1 = kT1 + 2 * HB, E2 = kT2 + 2 * HB;  // input tile rows, columns
    constexpr int NIN = E1 * E2;                         // input tile size per component
    constexpr int NLD = (2 * NIN + kThreads - 1) / kThreads;
    constexpr int NA = kT1 * E2;                         // stage-A positions
    __shared__ T xs[2 * NIN];
    __shared__ T st[6 * NA];  // S1x1 M1x1 A1x1 S1x2 M1x2 A1x2, each [kT1][E2]
    const int m1 = op.m[0], m2 = op.m[1];
    const int G = m1 * m2;
    const int nt2 = (m2 + kT2 - 1) / kT2;
    // blocks go to the XCDs round robin; each XCD takes a contiguous run of
    // row-major tiles, so most of a tile's input was written through the same
    // L2 by the previous launch
    const int xcd = int(blockIdx.x % kXcds), slot = int(blockIdx.x / kXcds);
    const int per = int(gridDim.x) / kXcds, rem = int(gridDim.x) % kXcds;
    const int tile = xcd * per + min(xcd, rem) + slot;
    const int o1 = (tile / nt2) * kT1, o2 = (tile % nt2) * kT2;
    const int tid = threadIdx.x;
    // the thread's output point and its epilogue operands, loaded first
    const int i = tid / kT2, j = tid % kT2;
    const int i1 = o1 + i, i2 = o2 + j;
    const bool own = (i1 < m1 && i2 < m2);
    const int f = own ? i1 * m2 + i2 : 0;
    EpiIn<T> ep[2];
    if (own) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
            epilogue_load<T, MODE>(ep[c], size_t(c) * G + f, x, b, u, c1, nv, size_t(2) * G);
    }
    {
        T v[NLD];
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = min(tid + q * kThreads, 2 * NIN - 1);
            const int c = e / NIN, r = (e % NIN) / E2, cc = e % E2;
            const int g1 = o1 - HB + r, g2 = o2 - HB + cc;
            const bool in = g1 >= 0 && g1 < m1 && g2 >= 0 && g2 < m2;
            const T val = x[size_t(c) * G + size_t(in ? g1 : 0) * m2 + (in ? g2 : 0)];
            v[q] = in ? val : T(0);
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * kThreads;
            if (e < 2 * NIN) xs[e] = v[q];
        }
    }
    __syncthreads();
    for (int p = tid; p < NA; p += kThreads) {
        const int i = p / E2, j = p % E2;
        const int r1 = min(o1 + i, m1 - 1);  // rows past the grid produce unused values
        T v[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T cS = op.band[0][2][k * m1 + r1];
            const T cM = op.band[0][0][k * m1 + r1];
            const T cA = op.band[0][1][k * m1 + r1];
            const T x1 = xs[(i + k) * E2 + j], x2 = xs[NIN + (i + k) * E2 + j];
            v[0] += cS * x1;
            v[1] += cM * x1;
            v[2] += cA * x1;
            v[3] += cS * x2;
            v[4] += cM * x2;
            v[5] += cA * x2;
        }
#pragma unroll
        for (int w = 0; w < 6; ++w) st[w * NA + p] = v[w];
    }
    __syncthreads();
    double dots[apply_ndots<MODE>()];
#pragma unroll
    for (int q = 0; q < apply_ndots<MODE>(); ++q) dots[q] = 0.0;
    if (own) {
        T mS1 = T(0), sM1 = T(0), aA2 = T(0), mS2 = T(0), sM2 = T(0), aA1 = T(0);
        const int q0 = i * E2 + j;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T cM = op.band[1][0][k * m2 + i2];
            const T cA = op.band[1][1][k * m2 + i2];
            const T cS = op.band[1][2][k * m2 + i2];
            mS1 += cM * st[0 * NA + q0 + k];
            sM1 += cS * st[1 * NA + q0 + k];
            aA1 += cA * st[2 * NA + q0 + k];
            mS2 += cM * st[3 * NA + q0 + k];
            sM2 += cS * st[4 * NA + q0 + k];
            aA2 += cA * st[5 * NA + q0 + k];
        }
        const T al = op.alpha, be = op.beta, ab = offdiag_weight(op);
        const T kx[2] = {be * mS1 + al * sM1 + ab * aA2, al * mS2 + be * sM2 + ab * aA1};
#pragma unroll
        for (int c = 0; c < 2; ++c)
            epilogue_store<T, MODE>(op, c, size_t(c) * G + f, kx[c], i1, i2, 0, ep[c], y, u, xout, c1, c2, nv, dots);
    }
    apply_write_dots<MODE>(dots, nv, part);
    stamp_end(stamp);
}

template <typename T, int HB, int MODE>
void launch2d(const OpDev<T>& op, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part, int nv,
              unsigned long long* stamp, hipStream_t s) {
    static_assert(kT1 * kT2 == kThreads, "2D tile must match the block size");
    const int tiles = ((op.m[0] + kT1 - 1) / kT1) * ((op.m[1] + kT2 - 1) / kT2);
    hipLaunchKernelGGL((k_apply2d<T, HB, MODE>), dim3(tiles), dim3(kThreads), 0, s, op, x, y, b, u, xout, c1, c2,
                       part, nv, stamp);
}

}  // namespace

template <typename T, int HB>
void apply2d_run(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2,
                 double* part, int nv, unsigned long long* stamp, hipStream_t s) {
    switch (mode) {
        case kApplyY: launch2d<T, HB, kApplyY>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyRes: launch2d<T, HB, kApplyRes>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyCheb: launch2d<T, HB, kApplyCheb>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyYDot: launch2d<T, HB, kApplyYDot>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyResDot: launch2d<T, HB, kApplyResDot>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyYMulti: launch2d<T, HB, kApplyYMulti>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        default: throw std::runtime_error("bad apply mode");
    }
    check_launch("apply2d");
}

template void apply2d_run<CD_T, CD_HB>(const OpDev<CD_T>&, int, const CD_T*, CD_T*, const CD_T*, CD_T*, CD_T*, CD_T,
                                       CD_T, double*, int, unsigned long long*, hipStream_t);

}  // namespace cd
