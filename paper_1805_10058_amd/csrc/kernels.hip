// HIP kernels for gfx950: sum-factorized curl-div operator, grid transfers,
// banded Toeplitz line solves, reductions and the small Krylov helpers.
//
// Every reduction accumulates in FP64 and combines partial sums in a fixed
// order, so results are bitwise reproducible run to run.
#include <algorithm>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>

#include "kernels.hpp"

namespace cd {

namespace {

constexpr int kThreads = 256;  // block size of every kernel in this file

void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block; the result is returned to every thread.
__device__ inline double block_sum(double v) {
    __shared__ double red[kThreads / 64];
    __shared__ double total;
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < int(blockDim.x) / 64; ++i) s += red[i];
        total = s;
    }
    __syncthreads();
    const double r = total;
    __syncthreads();
    return r;
}

__device__ inline double sum_partials(const double* part, int np) {
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
    return block_sum(v);
}

// Kernel-side timing on the constant-rate wall clock.  A timing slot is
// kStampWords words: [0] = start of block 0 (the first block dispatched),
// [1 + b % kStampEnds] = latest end of the blocks b mapped there, taken after
// the block's memory operations completed.  The end words start at zero
// (k_stamp_reduce clears them after use).  stamp == nullptr: no timing.
// stamp_end must be reached by every thread of the block.
__device__ inline void stamp_begin(unsigned long long* stamp) {
    if (stamp != nullptr && blockIdx.x == 0 && threadIdx.x == 0) stamp[0] = (unsigned long long)wall_clock64();
}

__device__ inline void stamp_end(unsigned long long* stamp) {
    if (stamp != nullptr) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads and stores are done
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(stamp + 1 + blockIdx.x % kStampEnds, (unsigned long long)wall_clock64());
    }
}

template <typename T>
__device__ inline T band_at(const OpDev<T>& op, int axis, int which, int k, int i) {
    return op.band[axis][which][k * op.m[axis] + i];
}

// Diagonal entry of block (c,c) at multi-index (i0,i1,i2):
// beta * prod(S on axis c, M elsewhere) + alpha * sum_{e != c} prod(S on e, M elsewhere).
template <typename T>
__device__ inline T diag_entry(const OpDev<T>& op, int c, int i0, int i1, int i2) {
    const int hb = op.hb;
    const T m0 = band_at(op, 0, 0, hb, i0), s0 = band_at(op, 0, 2, hb, i0);
    const T m1 = band_at(op, 1, 0, hb, i1), s1 = band_at(op, 1, 2, hb, i1);
    if (op.dim == 2) {
        const T t0 = s0 * m1, t1 = m0 * s1;
        return (c == 0) ? op.beta * t0 + op.alpha * t1 : op.alpha * t0 + op.beta * t1;
    }
    const T m2 = band_at(op, 2, 0, hb, i2), s2 = band_at(op, 2, 2, hb, i2);
    const T t0 = s0 * m1 * m2, t1 = m0 * s1 * m2, t2 = m0 * m1 * s2;
    return (c == 0 ? op.beta : op.alpha) * t0 + (c == 1 ? op.beta : op.alpha) * t1 +
           (c == 2 ? op.beta : op.alpha) * t2;
}

// 3D output tile: k3T2 rows (x2) of k3T3(HB) = 32 - 2HB columns (x3), so that
// the stage-A positions (k3T2 rows of 32 tile columns) are exactly one per thread.
constexpr int k3T2 = 8, k3E3 = 32;
__host__ __device__ constexpr int k3T3(int hb) { return k3E3 - 2 * hb; }
constexpr int kXcds = 8;

// Launch geometry of the 3D operator kernel: tiles of the (x2, x3) plane times
// ranges of x1 planes, about as many blocks as fit on the device at once (two
// per compute unit in FP64, four in FP32, set by the register footprint).
struct Apply3dGeom {
    int nt2, nt3, c1len, nblocks;
};

Apply3dGeom apply3d_geom(const int* m, int hb, size_t elem) {
    const int kTargetBlocks = elem == 4 ? 1024 : 512;
    Apply3dGeom g;
    g.nt2 = (m[1] + k3T2 - 1) / k3T2;
    g.nt3 = (m[2] + k3T3(hb) - 1) / k3T3(hb);
    const int planar = g.nt2 * g.nt3;
    const int nx1 = std::max(1, std::min(m[0], kTargetBlocks / planar));
    g.c1len = (m[0] + nx1 - 1) / nx1;
    g.nblocks = planar * ((m[0] + g.c1len - 1) / g.c1len);
    return g;
}

// Partial dot products an operator kernel accumulates per thread.
template <int MODE>
constexpr int apply_ndots() {
    return MODE == kApplyYMulti ? kMaxBasis + 1 : 1;
}

// Operands the epilogue of an operator kernel reads at one output entry,
// loaded as early as the kernel knows the entry (the 2D kernel: before its
// input tile), so their latency hides behind the contractions.
template <typename T>
struct EpiIn {
    T b, u, x;
    T v[kMaxBasis];
};

template <typename T, int MODE>
__device__ inline void epilogue_load(EpiIn<T>& e, size_t idx, const T* __restrict__ x, const T* __restrict__ b,
                                     const T* __restrict__ u, T c1, int nv, size_t ntot) {
    if (MODE == kApplyRes || MODE == kApplyResDot || MODE == kApplyCheb) e.b = b[idx];
    if (MODE == kApplyCheb) {
        e.u = (c1 != T(0)) ? u[idx] : T(0);  // u is not read on a first step
        e.x = x[idx];
    }
    if (MODE == kApplyYDot) e.x = x[idx];
    if (MODE == kApplyYMulti) {
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i) e.v[i] = (i < nv) ? b[size_t(i) * ntot + idx] : T(0);
    }
}

// Epilogue at one output entry idx (component c, grid point (i1, i2, i3))
// with kx = (A x)[idx] and the entry's operands e.
template <typename T, int MODE>
__device__ inline void epilogue_store(const OpDev<T>& op, int c, size_t idx, T kx, int i1, int i2, int i3,
                                      const EpiIn<T>& e, T* __restrict__ y, T* __restrict__ u,
                                      T* __restrict__ xout, T c1, T c2, int nv, double* dots) {
    if (MODE == kApplyY) {
        y[idx] = kx;
    } else if (MODE == kApplyRes) {
        y[idx] = e.b - kx;
    } else if (MODE == kApplyResDot) {
        const T r = e.b - kx;
        y[idx] = r;
        dots[0] += double(r) * double(r);
    } else if (MODE == kApplyYMulti) {
        y[idx] = kx;
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i)
            if (i < nv) dots[i] += double(e.v[i]) * double(kx);
        dots[kMaxBasis] += double(kx) * double(kx);
    } else if (MODE == kApplyCheb) {
        const T r = e.b - kx;
        const T dg = diag_entry(op, c, i1, i2, i3);
        const T un = c1 * e.u + c2 * r / dg;
        u[idx] = un;
        xout[idx] = e.x + un;
    } else {
        y[idx] = kx;
        dots[0] += double(e.x) * double(kx);
    }
}

// Both at once (the 3D kernel, whose output entries change plane by plane).
template <typename T, int MODE>
__device__ inline void apply_epilogue(const OpDev<T>& op, int c, size_t idx, T kx, int i1, int i2, int i3,
                                      const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ b,
                                      T* __restrict__ u, T* __restrict__ xout, T c1, T c2, int nv, size_t ntot,
                                      double* dots) {
    EpiIn<T> e;
    epilogue_load<T, MODE>(e, idx, x, b, u, c1, nv, ntot);
    epilogue_store<T, MODE>(op, c, idx, kx, i1, i2, i3, e, y, u, xout, c1, c2, nv, dots);
}

// Block sums of the per-thread partial dots: part[i * gridDim.x + block].
template <int MODE>
__device__ inline void apply_write_dots(const double* dots, int nv, double* __restrict__ part) {
    if (MODE == kApplyYDot || MODE == kApplyResDot) {
        const double tot = block_sum(dots[0]);
        if (threadIdx.x == 0) part[blockIdx.x] = tot;
    } else if (MODE == kApplyYMulti) {
#pragma unroll
        for (int i = 0; i < kMaxBasis; ++i) {
            if (i < nv) {  // block-uniform
                const double tot = block_sum(dots[i]);
                if (threadIdx.x == 0) part[size_t(i) * gridDim.x + blockIdx.x] = tot;
            }
        }
        const double ww = block_sum(dots[kMaxBasis]);
        if (threadIdx.x == 0) part[size_t(nv) * gridDim.x + blockIdx.x] = ww;
    }
}

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
                                                      const T* __restrict__ b, T* __restrict__ u,
                                                      T* __restrict__ xout, T c1, T c2, double* __restrict__ part,
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
constexpr int kT1 = 8, kT2 = 32;  // 2D output tile: kT1 * kT2 = kThreads points

template <typename T, int HB, int MODE>
__global__ __launch_bounds__(kThreads) void k_apply2d(OpDev<T> op, const T* __restrict__ x, T* __restrict__ y,
                                                      const T* __restrict__ b, T* __restrict__ u,
                                                      T* __restrict__ xout, T c1, T c2, double* __restrict__ part,
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
        const T al = op.alpha, be = op.beta, ab = op.alpha - op.beta;
        const T kx[2] = {be * mS1 + al * sM1 + ab * aA2, al * mS2 + be * sM2 + ab * aA1};
#pragma unroll
        for (int c = 0; c < 2; ++c)
            epilogue_store<T, MODE>(op, c, size_t(c) * G + f, kx[c], i1, i2, 0, ep[c], y, u, xout, c1, c2, nv, dots);
    }
    apply_write_dots<MODE>(dots, nv, part);
    stamp_end(stamp);
}

// Raise a kernel's dynamic-LDS limit (default 64 KiB) to what a launch needs,
// once per kernel and size.  The first launch of every kernel with a given
// problem happens in setup or in the first, uncaptured outer iteration, so
// this never runs inside a stream capture.
void allow_lds(const void* kern, size_t lds) {
    if (lds <= 64 * 1024) return;
    static std::mutex mu;
    static std::map<const void*, size_t> done;
    std::lock_guard<std::mutex> g(mu);
    auto it = done.find(kern);
    if (it != done.end() && it->second >= lds) return;
    const hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::runtime_error(std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
    done[kern] = lds;
}

template <typename T, int HB, int MODE>
void apply_dispatch(const OpDev<T>& op, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part,
                    int nv, unsigned long long* stamp, hipStream_t s) {
    if (op.dim == 3) {
        const Apply3dGeom g = apply3d_geom(op.m, HB, sizeof(T));
        const size_t lds = apply3d_lds_words<T, HB>() * sizeof(T);
        auto kern = k_apply3d<T, HB, MODE>;
        allow_lds(reinterpret_cast<const void*>(kern), lds);
        hipLaunchKernelGGL(kern, dim3(g.nblocks), dim3(kThreads), lds, s, op, x, y, b, u, xout, c1, c2, part, nv, g,
                           stamp);
    } else {
        static_assert(kT1 * kT2 == kThreads, "2D tile must match the block size");
        const int tiles = ((op.m[0] + kT1 - 1) / kT1) * ((op.m[1] + kT2 - 1) / kT2);
        hipLaunchKernelGGL((k_apply2d<T, HB, MODE>), dim3(tiles), dim3(kThreads), 0, s, op, x, y, b, u, xout, c1,
                           c2, part, nv, stamp);
    }
    check_launch("apply");
}

template <typename T, int HB>
void apply_mode(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part,
                int nv, unsigned long long* stamp, hipStream_t s) {
    switch (mode) {
        case kApplyY: apply_dispatch<T, HB, kApplyY>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyRes: apply_dispatch<T, HB, kApplyRes>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyCheb: apply_dispatch<T, HB, kApplyCheb>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyYDot: apply_dispatch<T, HB, kApplyYDot>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyResDot: apply_dispatch<T, HB, kApplyResDot>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case kApplyYMulti: apply_dispatch<T, HB, kApplyYMulti>(op, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        default: throw std::runtime_error("bad apply mode");
    }
}

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
                                                         T* __restrict__ u, T* __restrict__ xo) {
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
    if (CHEB) {
        const T v = inv_theta * acc / diag_entry(opc, c, J0, J1, J2);
        u[id] = v;
        xo[id] = v;
    }
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
                    v = op.alpha - op.beta;
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
__global__ __launch_bounds__(kThreads) void k_cheb_first(OpDev<T> op, const T* __restrict__ b, T* __restrict__ u,
                                                         T* __restrict__ x, T inv_theta, size_t n) {
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        const T v = inv_theta * b[id] / diag_entry(op, c, i0, i1, i2);
        u[id] = v;
        x[id] = v;
    }
}

// y = x (converted) and the first Chebyshev step from zero on y.
template <typename TO, typename TI>
__global__ __launch_bounds__(kThreads) void k_cast_cheb(const TI* __restrict__ x, TO* __restrict__ y, size_t n,
                                                        OpDev<TO> op, TO inv_theta, TO* __restrict__ u,
                                                        TO* __restrict__ xo) {
    for (size_t id = size_t(blockIdx.x) * kThreads + threadIdx.x; id < n; id += size_t(gridDim.x) * kThreads) {
        const TO b = TO(x[id]);
        y[id] = b;
        int c, i0, i1, i2;
        unflatten(op, id, c, i0, i1, i2);
        const TO v = inv_theta * b / diag_entry(op, c, i0, i1, i2);
        u[id] = v;
        xo[id] = v;
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
__global__ __launch_bounds__(kThreads) void k_fcg_direction(int first, const double* __restrict__ z,
                                                            const double* __restrict__ pzq, int npzq,
                                                            const double* __restrict__ dq_prev, double* __restrict__ d,
                                                            const double* __restrict__ r, double* __restrict__ pdr,
                                                            size_t n) {
    double beta = 0.0;
    if (!first) {
        const double zq = sum_partials(pzq, npzq);
        const double dq = dq_prev[0];
        beta = (dq != 0.0) ? zq / dq : 0.0;
    }
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        const double dn = first ? z[i] : z[i] - beta * d[i];
        d[i] = dn;
        s += dn * r[i];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) pdr[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_fcg_update(const double* __restrict__ pdr, int npdr,
                                                         const double* __restrict__ pdq, int npdq,
                                                         double* __restrict__ dq_out, double* __restrict__ x,
                                                         double* __restrict__ r, const double* __restrict__ d,
                                                         const double* __restrict__ q, double* __restrict__ prr,
                                                         size_t n) {
    const double dr = sum_partials(pdr, npdr);
    const double dq = sum_partials(pdq, npdq);
    const double a = (dq != 0.0) ? dr / dq : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) dq_out[0] = dq;
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        x[i] += a * d[i];
        const double rn = r[i] - a * q[i];
        r[i] = rn;
        s += rn * rn;
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
    if (op.dim == 3) return apply3d_geom(op.m, op.hb, sizeof(T)).nblocks;
    return ((op.m[0] + kT1 - 1) / kT1) * ((op.m[1] + kT2 - 1) / kT2);
}

template <typename T>
void launch_apply(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part,
                  hipStream_t s, int nv,
                  unsigned long long* stamp) {
    if (mode == kApplyYMulti && (nv < 1 || nv > kMaxBasis)) throw std::runtime_error("bad number of dot vectors");
    switch (op.hb) {
        case 1: apply_mode<T, 1>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case 2: apply_mode<T, 2>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case 3: apply_mode<T, 3>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case 4: apply_mode<T, 4>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case 5: apply_mode<T, 5>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        case 6: apply_mode<T, 6>(op, mode, x, y, b, u, xout, c1, c2, part, nv, stamp, s); break;
        default: throw std::runtime_error("degree out of range (1..6)");
    }
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
                               c.inv_theta, c.u, c.x);
        else if (Restrict)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, 1, false>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.u, c.x);
        else
            hipLaunchKernelGGL((k_prolong_add_w<T, W, W, 1>), grid, dim3(kThreads), 0, s, X, ncomp, in, out);
    } else {
        if (Restrict && cf)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, W, true>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.u, c.x);
        else if (Restrict)
            hipLaunchKernelGGL((k_restrict_w<T, W, W, W, false>), grid, dim3(kThreads), 0, s, X, ncomp, in, out, c.op,
                               c.inv_theta, c.u, c.x);
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
        if (cf) launch_cheb_first<T>(cf->op, rc, cf->u, cf->x, cf->inv_theta, s);
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
                       cf.u, cf.x);
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
void launch_cheb_first(const OpDev<T>& op, const T* b, T* u, T* x, T inv_theta, hipStream_t s) {
    const size_t n = op_len(op);
    hipLaunchKernelGGL(k_cheb_first<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, op, b, u, x, inv_theta, n);
    check_launch("cheb_first");
}

template <typename T>
void launch_coarse_gemv(const double* Kinv, int N, int ld, const T* r, T* z, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_gemv<T>, dim3(N), dim3(kThreads), 0, s, Kinv, N, ld, r, z);
    check_launch("coarse_gemv");
}

void launch_fcg_direction(bool first, const double* z, const double* pzq, int npzq, const double* dq_prev, double* d,
                          const double* r, double* pdr, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_direction, dim3(reduce_blocks(n)), dim3(kThreads), 0, s, first ? 1 : 0, z, pzq, npzq,
                       dq_prev, d, r, pdr, n);
    check_launch("fcg_direction");
}

void launch_fcg_update(const double* pdr, int npdr, const double* pdq, int npdq, double* dq_out, double* x, double* r,
                       const double* d, const double* q, double* prr, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_update, dim3(reduce_blocks(n)), dim3(kThreads), 0, s, pdr, npdr, pdq, npdq, dq_out, x, r,
                       d, q, prr, n);
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
    template void launch_fill<T>(T*, T, size_t, hipStream_t);                                                        \
    template void launch_copy<T>(const T*, T*, size_t, hipStream_t);                                                 \
    template void launch_axpby<T>(T, const T*, T, T*, size_t, hipStream_t);                                          \
    template void launch_normalize<T>(const double*, int, const T*, T*, size_t, hipStream_t);                        \
    template void launch_diag_scale<T>(const OpDev<T>&, bool, const T*, T*, hipStream_t);                            \
    template void launch_diag_dot<T>(const OpDev<T>&, const T*, double*, hipStream_t);                               \
    template void launch_cheb_first<T>(const OpDev<T>&, const T*, T*, T*, T, hipStream_t);                           \
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
