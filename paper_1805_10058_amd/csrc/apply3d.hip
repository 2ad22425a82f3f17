// 3D curl-div operator apply (sum factorization), one object per (precision,
// half bandwidth): compiled with -DCD_T=<float|double> -DCD_HB=<1..6>.
#include "apply_common.hpp"

namespace cd {
namespace {

// ------------------------------------------------------------------------------
// 3D operator apply.
//
// A block owns an output tile of k3T2 x (32 - 2HB) columns of the (x2, x3)
// plane (one per thread; the other threads only help with loads and stage A)
// and the output planes x1 in [o0, o1); it marches over the input planes
// t = 0, 1, ... (x1 = o0 - HB + t) up to o1 + HB.  Per input plane:
//   (A) contract axis 2 (stride m3): M2 x, A2 x, S2 x of the three components
//       at one position per thread: the tile rows times all 32 tile columns
//       (LDS tile of the plane with a +-HB halo on both in-plane axes);
//   (B) contract axis 3 at the thread's column and combine the raw products
//       with alpha, beta, alpha-beta into W[c][{S,M,A}], the inputs of the
//       axis-1 contraction of output component c;
//   (C) scatter W into a ring of 2HB+1 per-plane accumulators in registers:
//       acc(i) += X1(i, j) W for i in [j-HB, j+HB].
// After plane j the accumulator of output plane j-HB is complete and goes
// through the epilogue.  33 band contractions per point.
//
// Software pipeline, one barrier per plane: phase t runs stage A of plane
// t+1 and stage B of plane t (independent work for the scheduler), stores the
// prefetched plane t+2 into the input buffer plane t has vacated, and issues
// the loads of plane t+3.  Input tiles and stage-A results are double
// buffered in LDS.
//
// Tiles are numbered with x2 fastest, then x3, then the x1 range, and block b
// takes tile (b mod 8) * ceil-share + b / 8: consecutive blocks land on
// different XCDs, so this keeps spatially adjacent tiles, whose halos overlap,
// on the same XCD and its L2.
// ------------------------------------------------------------------------------
template <typename T, int HB>
constexpr size_t apply3d_lds_words() {
    return 2 * 3 * size_t(k3T2 + 2 * HB) * k3E3 + 2 * 9 * size_t(k3T2) * k3E3 + 3 * size_t(2 * HB + 1) * k3T2;
}

template <typename T, int HB, int MODE>
__global__ __launch_bounds__(kThreads) void k_apply3d(OpDev<T> op, const T* __restrict__ x, T* __restrict__ y,
                                                      const T* __restrict__ b, T* u,
                                                      T* xout, T c1, T c2, double* __restrict__ part,
                                                      int nv, Apply3dGeom g, unsigned long long* stamp) {
    stamp_begin(stamp);
    constexpr int R = 2 * HB + 1;
    constexpr int T3 = k3T3(HB);
    constexpr int E2 = k3T2 + 2 * HB, E3 = k3E3;
    constexpr int NIN = E2 * E3;  // input tile per component and plane
    constexpr int NLD = (3 * NIN + kThreads - 1) / kThreads;
    constexpr int NA = k3T2 * E3;  // stage-A positions
    static_assert(NA == kThreads, "one stage-A position per thread");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);  // [2][3][E2][E3] input tiles
    T* st = xs + 2 * 3 * NIN;                // [2][9][k3T2][E3]: M2x A2x S2x of components 0, 1, 2
    T* ca = st + 2 * 9 * NA;                 // [3][R][k3T2] axis-2 band rows of the tile
    const int m1 = op.m[0], m2 = op.m[1], m3 = op.m[2];
    const size_t PL = size_t(m2) * m3, G = size_t(m1) * PL;
    const int xcd = int(blockIdx.x % kXcds), slot = int(blockIdx.x / kXcds);
    const int per = g.nblocks / kXcds, rem = g.nblocks % kXcds;
    const int tile = xcd * per + min(xcd, rem) + slot;
    const int o2 = (tile % g.nt2) * k3T2;
    const int o3 = ((tile / g.nt2) % g.nt3) * T3;
    const int o0 = (tile / (g.nt2 * g.nt3)) * g.c1len;
    const int o1 = min(o0 + g.c1len, m1);
    const int tid = threadIdx.x;
    for (int e = tid; e < 3 * R * k3T2; e += kThreads) {
        const int i = e % k3T2, k = (e / k3T2) % R, w = e / (k3T2 * R);
        ca[e] = op.band[1][w][k * m2 + min(o2 + i, m2 - 1)];  // rows past the grid feed unused outputs
    }
    // stage-A position of this thread
    const int ai = tid / E3, aq = tid % E3;
    // output column of this thread and its axis-3 band row
    const int ty = tid / E3, tx = tid % E3;
    const int i2 = o2 + ty, i3 = o3 + tx;
    const bool active = (tx < T3) && (i2 < m2) && (i3 < m3);
    T cb[3][R];
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int k = 0; k < R; ++k) cb[w][k] = active ? op.band[2][w][k * m3 + i3] : T(0);
    T acc[3][R];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[c][r] = T(0);
    double dots[apply_ndots<MODE>()];
#pragma unroll
    for (int i = 0; i < apply_ndots<MODE>(); ++i) dots[i] = 0.0;
    const T al = op.alpha, be = op.beta, ab = op.alpha - op.beta;
    const T* __restrict__ colM = op.col0[0];
    const T* __restrict__ colA = op.col0[1];
    const T* __restrict__ colS = op.col0[2];

    // the thread's loads of the input tile: offsets within a plane of the
    // component stack (the same for every plane), -1 outside the grid
    long long loff[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        const int e = min(tid + q * kThreads, 3 * NIN - 1);
        const int c = e / NIN, rr = e % NIN;
        const int g2 = o2 - HB + rr / E3, g3 = o3 - HB + rr % E3;
        const bool in = g2 >= 0 && g2 < m2 && g3 >= 0 && g3 < m3;
        loff[q] = in ? (long long)(size_t(c) * G + size_t(g2) * m3 + g3) : -1;
    }
    T v[NLD];
    auto load_plane = [&](int t) {
        const int j = o0 - HB + t;
        const bool jin = (j >= 0 && j < m1);  // block-uniform
        const size_t jo = size_t(jin ? j : 0) * PL;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const bool in = jin && loff[q] >= 0;
            const T val = x[in ? jo + size_t(loff[q]) : 0];
            v[q] = in ? val : T(0);
        }
    };
    auto store_plane = [&](int t) {
        T* dst = xs + (t & 1) * 3 * NIN;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * kThreads;
            if (e < 3 * NIN) dst[e] = v[q];
        }
    };
    auto live = [&](int t) {
        const int j = o0 - HB + t;
        return j >= 0 && j < m1;
    };
    auto stage_a = [&](int t) {
        const T* src = xs + (t & 1) * 3 * NIN;
        T* dst = st + (t & 1) * 9 * NA;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T aM = T(0), aA = T(0), aS = T(0);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T xv = src[c * NIN + (ai + k) * E3 + aq];
                aM += ca[(0 * R + k) * k3T2 + ai] * xv;
                aA += ca[(1 * R + k) * k3T2 + ai] * xv;
                aS += ca[(2 * R + k) * k3T2 + ai] * xv;
            }
            dst[(3 * c + 0) * NA + tid] = aM;
            dst[(3 * c + 1) * NA + tid] = aA;
            dst[(3 * c + 2) * NA + tid] = aS;
        }
    };

    const int TI = (o1 - o0) + 2 * HB;  // input planes of the block
    load_plane(0);
    store_plane(0);
    if (TI > 1) {
        load_plane(1);
        store_plane(1);
    }
    if (TI > 2) load_plane(2);
    __syncthreads();
    if (live(0)) stage_a(0);
    __syncthreads();
    for (int t0 = 0; t0 < TI; t0 += R) {
#pragma unroll
        for (int uu = 0; uu < R; ++uu) {
            const int t = t0 + uu;
            if (t < TI) {  // block-uniform
                const int j = o0 - HB + t;
                const int io = j - HB;  // output plane completed in this phase
                const bool emit = (io >= o0 && io < o1);
                // operands of this phase's epilogue, loaded before the contractions
                // (not for the Krylov-dot mode: its basis rows would cost too many registers)
                constexpr bool kPre = (MODE != kApplyYMulti);
                EpiIn<T> ep[3];
                if (kPre && emit && active) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        epilogue_load<T, MODE>(ep[c], size_t(c) * G + size_t(io) * PL + size_t(i2) * m3 + i3, x, b, u,
                                               c1, nv, 3 * G);
                }
                if (t + 1 < TI && live(t + 1)) stage_a(t + 1);
                if (live(t)) {
                    const T* sb = st + (t & 1) * 9 * NA;
                    T W[3][3];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int w = 0; w < 3; ++w) W[c][w] = T(0);
                    if (active) {
                        // raw products per input component c: M3(M2x), S3(M2x), A3(M2x), M3(S2x), M3(A2x), A3(A2x)
                        T mm[3], sm[3], am[3], ms[3], ma[3], aa[3];
                        const int q0 = ty * E3 + tx;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            mm[c] = sm[c] = am[c] = ms[c] = ma[c] = aa[c] = T(0);
#pragma unroll
                            for (int k = 0; k < R; ++k) {
                                const T vM = sb[(3 * c + 0) * NA + q0 + k];
                                const T vA = sb[(3 * c + 1) * NA + q0 + k];
                                const T vS = sb[(3 * c + 2) * NA + q0 + k];
                                mm[c] += cb[0][k] * vM;
                                sm[c] += cb[2][k] * vM;
                                if (c != 1) am[c] += cb[1][k] * vM;
                                ms[c] += cb[0][k] * vS;
                                if (c != 2) ma[c] += cb[0][k] * vA;
                                if (c != 0) aa[c] += cb[1][k] * vA;
                            }
                        }
                        W[0][0] = be * mm[0];
                        W[0][1] = al * (sm[0] + ms[0]);
                        W[0][2] = ab * (ma[1] + am[2]);
                        W[1][0] = al * mm[1];
                        W[1][1] = al * sm[1] + be * ms[1] + ab * aa[2];
                        W[1][2] = ab * ma[0];
                        W[2][0] = al * mm[2];
                        W[2][1] = be * sm[2] + al * ms[2] + ab * aa[1];
                        W[2][2] = ab * am[0];
                    }
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const int i = j - HB + k;
                        if (i >= o0 && i < o1) {
                            const T cS = colS[j * R + k];  // X1(i, j)
                            const T cM = colM[j * R + k];
                            const T cA = colA[j * R + k];
                            const int sl = (uu + k + 1) % R;
#pragma unroll
                            for (int c = 0; c < 3; ++c)
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    if (r == sl) acc[c][r] += cS * W[c][0] + cM * W[c][1] + cA * W[c][2];
                        }
                    }
                }
                if (emit) {
                    const int sl = (uu + 1) % R;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        T kx = T(0);
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if (r == sl) {
                                kx = acc[c][r];
                                acc[c][r] = T(0);
                            }
                        if (active) {
                            const size_t idx = size_t(c) * G + size_t(io) * PL + size_t(i2) * m3 + i3;
                            if (kPre)
                                epilogue_store<T, MODE>(op, c, idx, kx, io, i2, i3, ep[c], y, u, xout, c1, c2, nv,
                                                        dots);
                            else
                                apply_epilogue<T, MODE>(op, c, idx, kx, io, i2, i3, x, y, b, u, xout, c1, c2, nv,
                                                        3 * G, dots);
                        }
                    }
                }
                if (t + 2 < TI) store_plane(t + 2);  // into the buffer plane t vacated
                if (t + 3 < TI) load_plane(t + 3);
                __syncthreads();
            }
        }
    }
    apply_write_dots<MODE>(dots, nv, part);
    stamp_end(stamp);
}

template <typename T, int HB, int MODE>
void launch3d(const OpDev<T>& op, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part, int nv,
              unsigned long long* stamp, hipStream_t s) {
    const Apply3dGeom g = apply3d_geom(op.m, HB, sizeof(T), op.x1chunk);
    const size_t lds = apply3d_lds_words<T, HB>() * sizeof(T);
    auto kern = k_apply3d<T, HB, MODE>;
    allow_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, dim3(g.nblocks), dim3(kThreads), lds, s, op, x, y, b, u, xout, c1, c2, part, nv, g,
                       stamp);
}

}  // namespace

template <typename T, int HB>
void apply3d_run(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2,
                 double* part, int nv, unsigned long long* stamp, hipStream_t s) {
    switch (mode) {
        case kApplyY: launch3d<T, HB, kApplyY>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyRes: launch3d<T, HB, kApplyRes>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyCheb: launch3d<T, HB, kApplyCheb>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyYDot: launch3d<T, HB, kApplyYDot>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyResDot: launch3d<T, HB, kApplyResDot>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyYMulti: launch3d<T, HB, kApplyYMulti>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        default: throw std::runtime_error("bad apply mode");
    }
    check_launch("apply3d");
}

template void apply3d_run<CD_T, CD_HB>(const OpDev<CD_T>&, int, const CD_T*, CD_T*, const CD_T*, CD_T*, CD_T*, CD_T,
                                       CD_T, double*, int, unsigned long long*, hipStream_t);

}  // namespace cd
