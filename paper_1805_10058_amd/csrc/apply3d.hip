// 3D curl-div operator apply (sum factorization), one object per (precision,
// half bandwidth): compiled with -DCD_T=<float|double> -DCD_HB=<1..6>.
#include "apply_common.hpp"
#include "curldiv.h"

namespace cd {
namespace {

// ------------------------------------------------------------------------------
// 3D operator apply.
//
// A block of 32 TR threads (TR/2 waves) owns an output tile of TR rows (x2) by
// 32 - 2HB columns (x3) of the (x2, x3) plane and the output planes x1 in
// [o0, o1); it marches over the input planes t = 0, 1, ... (x1 = o0 - HB + t)
// up to o1 + HB.  Thread (ty, tx) sits at grid row o2 + ty and column
// o3 - HB + tx: a wave holds two tile rows of 32 columns, of which the middle
// 32 - 2HB are output columns and the HB on each side their halo.  Per input
// plane j:
//   (A) contract axis 2 (rows) at the thread's point: M2 x, A2 x, S2 x of the
//       three components from the plane's input tile in LDS (rows with a +-HB
//       halo), with the thread's row of the axis-2 bands in registers (FP32;
//       in LDS for FP64, whose registers are scarcer);
//   (B) contract axis 3 (columns): the 2HB + 1 neighbours of a column sit in
//       the neighbouring lanes of the same wave, and whole-wave lane shifts
//       (DPP) bring them in, so this stage touches no memory; lanes whose
//       shifts cross from one tile row into the other are halo lanes, whose
//       results are discarded.  The raw products combine with alpha, beta and
//       alpha - beta into W[c][{S, M, A}], the inputs of the axis-1
//       contraction of output component c;
//   (C) scatter W into a ring of 2HB + 1 per-plane accumulators in registers:
//       acc(i) += X1(i, j) W for i in [j - HB, j + HB], with the axis-1
//       coefficients of plane j (a row of the level's table: X1(j - HB + k, j)
//       for the three 1D matrices and the diagonal entries of plane j - HB)
//       read through block-uniform addresses, i.e. into scalar registers.
// After plane j the accumulator of output plane j - HB is complete and goes
// through the epilogue.  33 band contractions per point.
//
// Memory: every global access goes through a buffer descriptor of one plane of
// one component (base and size in scalar registers, built per plane), with a
// per-thread byte offset fixed for the whole march.  Tile entries outside the
// grid and the output lanes that are not output points carry an offset past
// the descriptor's range: their loads return zero and their stores are
// dropped, with no per-thread address arithmetic or branches.  The loads of
// plane t + 3 are issued while plane t is computed and stored into LDS in the
// phase after (double-buffered input tiles, one barrier per plane); the
// epilogue operands of the next output plane are loaded right after the
// current one is written.  The Chebyshev step's diagonal comes from per-thread
// in-plane factors and the plane's diagonal entries in the table row; FP32
// divides by it through the hardware reciprocal.
//
// Accumulator slots: the accumulator of output plane i lives in slot
// (i - o0 + 2HB + 1) mod (2HB + 1).  Every phase reads and clears the slot of
// the plane it completes, emitted or not, so slots need no range checks: a
// plane's slot is cleared one phase before its first contribution.
//
// Tiles are numbered with x2 fastest, then x3, then the x1 range, and block b
// takes tile (b mod 8) * ceil-share + b / 8: consecutive blocks land on
// different XCDs, so this keeps spatially adjacent tiles, whose halos overlap,
// on the same XCD and its L2.
// ------------------------------------------------------------------------------
constexpr int kDppShl1 = 0x130;         // DPP wave_shl:1, lane l reads lane l + 1
constexpr int kDppShr1 = 0x138;         // DPP wave_shr:1, lane l reads lane l - 1
constexpr unsigned kOob = 0xFFFFFFF0u;  // a byte offset past every plane descriptor's range
constexpr int kRsrcWord3 = 0x00020000;  // descriptor word 3: 32-bit elements, no swizzle

// whole-wave lane shifts; lanes past either end of the wave read zero
template <int CTRL>
__device__ inline float lane_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double lane_shift(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = unsigned(__builtin_amdgcn_mov_dpp(int(unsigned(u)), CTRL, 0xF, 0xF, true));
    const unsigned hi = unsigned(__builtin_amdgcn_mov_dpp(int(unsigned(u >> 32)), CTRL, 0xF, 0xF, true));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// raw buffer access: offsets at or past `bytes` read zero and drop stores
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(bytes), kRsrcWord3);
}
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ inline void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    using u2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
}

// W[c][{S, M, A}] from the axis-2/axis-3 products of one plane, shared by
// every variant.  The three-term sums are written as explicit fused
// multiply-adds: left to the compiler, their contraction was seen to differ
// between kernels (FP64, p = 6), and every variant must round alike.
template <typename T>
__device__ inline void combine_w(const T (&mm)[3], const T (&sm)[3], const T (&am)[3], const T (&ms)[3],
                                 const T (&ma)[3], const T (&aa)[3], T al, T be, T ab, T (&W)[9]) {
    W[0] = be * mm[0];
    W[1] = al * (sm[0] + ms[0]);
    W[2] = ab * (ma[1] + am[2]);
    W[3] = al * mm[1];
    W[4] = fma(ab, aa[2], fma(be, ms[1], al * sm[1]));
    W[5] = ab * ma[0];
    W[6] = al * mm[2];
    W[7] = fma(ab, aa[1], fma(al, ms[2], be * sm[2]));
    W[8] = ab * am[0];
}

// The Chebyshev step's diagonal at one point, for the three components:
// diag_c = fd[c] d0s + fe[c] d0m, with d0m and d0s the axis-1 mass and
// stiffness diagonal entries of the point's x1 plane (the diagonal of the
// Kronecker sum, blocks on the diagonal only).  Lanes that are not output
// points get fd = 0, fe = 1, a positive diagonal whose results are dropped.
template <typename T>
struct ChebDiag {
    T fd[3], fe[3];
};
template <typename T, int HB>
__device__ inline void cheb_diag_one(const OpDev<T>& op, int c, int i2c, int i3c, bool active, T& fd, T& fe) {
    const int m2 = op.m[1], m3 = op.m[2];
    const T dm1 = op.band[1][0][HB * m2 + i2c], ds1 = op.band[1][2][HB * m2 + i2c];
    const T dm2 = op.band[2][0][HB * m3 + i3c], ds2 = op.band[2][2][HB * m3 + i3c];
    const T dmm = dm1 * dm2, dsm = ds1 * dm2, dms = dm1 * ds2;
    const T al = op.alpha, be = op.beta;
    fd = active ? (c == 0 ? be : al) * dmm : T(0);
    fe = active ? fma(c == 1 ? be : al, dsm, (c == 2 ? be : al) * dms) : T(1);
}
template <typename T, int HB>
__device__ inline ChebDiag<T> cheb_diag(const OpDev<T>& op, int i2c, int i3c, bool active) {
    ChebDiag<T> d;
#pragma unroll
    for (int c = 0; c < 3; ++c) cheb_diag_one<T, HB>(op, c, i2c, i3c, active, d.fd[c], d.fe[c]);
    return d;
}
// x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 (b - A x_k) / diag at one entry
template <typename T>
__device__ inline T cheb_update(T xk, T xp, T bv, T kx, T fd, T fe, T d0m, T d0s, T c1, T c2) {
    const T dg = fma(fd, d0s, fe * d0m);
    const T r = bv - kx;
    T upd;
    if constexpr (sizeof(T) == 4)
        upd = c2 * r * __builtin_amdgcn_rcpf(dg);
    else
        upd = c2 * r / dg;
    return xk + (c1 * (xk - xp) + upd);
}

template <typename T, int HB>
struct Tile3 {
    static constexpr int TR = k3Rows<T>();          // tile rows (x2)
    static constexpr int NT = TR * k3E3;            // threads: one point of the tile rows each
    static constexpr int R = 2 * HB + 1;
    static constexpr int E2 = TR + 2 * HB;          // input rows with the x2 halo
    static constexpr int NIN = E2 * k3E3;           // input tile of one component
    static constexpr int NX = 3 * NIN;              // input tile of a plane
    static constexpr int NLC = (NIN + NT - 1) / NT; // tile loads per thread and component
    static constexpr int NC = 3 * R + 2;            // axis-1 table row
    static constexpr bool CAREG = sizeof(T) == 4;   // axis-2 band rows in registers
    static constexpr size_t lds_words() { return 2 * size_t(NX) + (CAREG ? 0 : 3 * size_t(R) * TR); }
};

template <typename T, int HB, int MODE>
__global__ __launch_bounds__(k3Rows<T>() * k3E3) void k_apply3d(OpDev<T> op, const T* __restrict__ x,
                                                               T* __restrict__ y, const T* __restrict__ b,
                                                               const T* xprev, T* xout, T c1, T c2,
                                                               double* __restrict__ part, int nv, Apply3dGeom g,
                                                               unsigned long long* stamp, const T* __restrict__ c1g) {
    using Q = Tile3<T, HB>;
    constexpr int TR = Q::TR, NT = Q::NT, R = Q::R, E3 = k3E3, T3 = k3T3(HB);
    constexpr int NIN = Q::NIN, NX = Q::NX, NLC = Q::NLC, NC = Q::NC;
    constexpr unsigned S = sizeof(T);
    stamp_begin(stamp);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);  // [2][3][E2][E3] input tiles
    const int m1 = op.m[0], m2 = op.m[1], m3 = op.m[2];
    const unsigned PL = unsigned(m2) * m3, G = unsigned(m1) * PL;
    const int xcd = int(blockIdx.x % kXcds), slot = int(blockIdx.x / kXcds);
    const int per = g.nblocks / kXcds, rem = g.nblocks % kXcds;
    const int tile = xcd * per + min(xcd, rem) + slot;
    const int o2 = (tile % g.nt2) * TR;
    const int o3 = ((tile / g.nt2) % g.nt3) * T3;
    const int o0 = (tile / (g.nt2 * g.nt3)) * g.c1len;
    const int o1 = min(o0 + g.c1len, m1);
    const int tid = threadIdx.x;
    const int ty = tid / E3, tx = tid % E3;
    const int i2 = o2 + ty, i3 = o3 - HB + tx;
    const bool active = (tx >= HB) && (tx < E3 - HB) && (i2 < m2) && (i3 < m3);
    const int i2c = min(i2, m2 - 1), i3c = min(max(i3, 0), m3 - 1);
    T car[Q::CAREG ? 3 : 1][Q::CAREG ? R : 1];
    T* ca = xs + 2 * NX;  // [3][R][TR] when not in registers
    if constexpr (Q::CAREG) {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int k = 0; k < R; ++k) car[w][k] = op.band[1][w][k * m2 + i2c];
    } else {
        for (int e = tid; e < 3 * R * TR; e += NT) {
            const int i = e % TR, k = (e / TR) % R, w = e / (TR * R);
            ca[e] = op.band[1][w][k * m2 + min(o2 + i, m2 - 1)];
        }
    }
    T cb[3][R];
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int k = 0; k < R; ++k) cb[w][k] = active ? op.band[2][w][k * m3 + i3] : T(0);
    const ChebDiag<T> cd = cheb_diag<T, HB>(op, i2c, i3c, active);
    // byte offset of the output point within a plane; out of range for inactive lanes
    const unsigned ptb = active ? (unsigned(i2c) * m3 + unsigned(i3c)) * S : kOob;
    T acc[3][R];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[c][r] = T(0);
    double dots[apply_ndots<MODE>()];
#pragma unroll
    for (int i = 0; i < apply_ndots<MODE>(); ++i) dots[i] = 0.0;
    const T al = op.alpha, be = op.beta, ab = offdiag_weight(op);

    // tile loads: NLC entries per component; in-plane byte offsets (out of range
    // outside the grid, so those entries read as zero)
    unsigned loffb[NLC];
#pragma unroll
    for (int q = 0; q < NLC; ++q) {
        const int e = min(tid + q * NT, NIN - 1);
        const int g2 = o2 - HB + e / E3, g3 = o3 - HB + e % E3;
        const bool in = g2 >= 0 && g2 < m2 && g3 >= 0 && g3 < m3;
        loffb[q] = in ? (unsigned(g2) * m3 + unsigned(g3)) * S : kOob;
    }
    T v[3][NLC];
    auto plane_rsrc = [&](const T* base, int c, int j) {
        const bool jin = (j >= 0 && j < m1);  // block-uniform
        return make_rsrc(base + (size_t(c) * G + size_t(jin ? j : 0) * PL), jin ? PL * S : 0u);
    };
    auto load_plane = [&](int t) {
        const int j = o0 - HB + t;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const auto r = plane_rsrc(x, c, j);
#pragma unroll
            for (int q = 0; q < NLC; ++q) v[c][q] = buf_load(r, loffb[q], T(0));
        }
    };
    auto store_plane = [&](int t) {
        T* dst = xs + (t & 1) * NX;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < NLC; ++q) {
                const int e = tid + q * NT;
                if ((q + 1) * NT <= NIN || e < NIN) dst[c * NIN + e] = v[c][q];
            }
    };
    auto live = [&](int t) {
        const int j = o0 - HB + t;
        return j >= 0 && j < m1;
    };
    auto stage_a = [&](int t, T (&sa)[9]) {
        const T* src = xs + (t & 1) * NX;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T aM = T(0), aA = T(0), aS = T(0);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T xv = src[c * NIN + (ty + k) * E3 + tx];
                if constexpr (Q::CAREG) {
                    aM = fma(car[0][k], xv, aM);
                    aA = fma(car[1][k], xv, aA);
                    aS = fma(car[2][k], xv, aS);
                } else {
                    aM = fma(ca[(0 * R + k) * TR + ty], xv, aM);
                    aA = fma(ca[(1 * R + k) * TR + ty], xv, aA);
                    aS = fma(ca[(2 * R + k) * TR + ty], xv, aS);
                }
            }
            sa[3 * c + 0] = aM;
            sa[3 * c + 1] = aA;
            sa[3 * c + 2] = aS;
        }
    };
    auto stencil = [&](T val, T (&s)[R]) {
        s[HB] = val;
#pragma unroll
        for (int d = 1; d <= HB; ++d) {
            s[HB - d] = lane_shift<kDppShr1>(s[HB - d + 1]);
            s[HB + d] = lane_shift<kDppShl1>(s[HB + d - 1]);
        }
    };
    // epilogue operands of output plane io, loaded one phase before its emit
    T eb[3], ex[3], ep[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) eb[c] = ex[c] = ep[c] = T(0);
    const bool use_prev = (c1 != T(0) && xprev != nullptr);
    auto epi_load = [&](int io) {
        if (io < o0 || io >= o1) return;  // block-uniform
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (MODE == kApplyRes || MODE == kApplyResDot || MODE == kApplyCheb) eb[c] = buf_load(plane_rsrc(b, c, io), ptb, T(0));
            if (MODE == kApplyCheb || MODE == kApplyYDot) ex[c] = buf_load(plane_rsrc(x, c, io), ptb, T(0));
            if (MODE == kApplyCheb) ep[c] = use_prev ? buf_load(plane_rsrc(xprev, c, io), ptb, T(0)) : T(0);
        }
    };

    const int TI = (o1 - o0) + 2 * HB;
    load_plane(0);
    store_plane(0);
    if (TI > 1) {
        load_plane(1);
        store_plane(1);
    }
    if (TI > 2) load_plane(2);
    __syncthreads();
    T sa[9];
    for (int t0 = 0; t0 < TI; t0 += R) {
#pragma unroll
        for (int uu = 0; uu < R; ++uu) {
            const int t = t0 + uu;
            if (t < TI) {
                const int j = o0 - HB + t;
                const int io = j - HB;
                const bool emit = (io >= o0 && io < o1);
                // Krylov-basis rows of this phase's output plane, loaded before
                // the contractions so that they hide the loads' latency (FP32 up
                // to HB = 4; the others have no registers to spare and load
                // them at the emit)
                constexpr bool kPreBasis = (MODE == kApplyYMulti) && sizeof(T) == 4 && HB <= 4;
                T ev[kPreBasis ? kMaxBasis : 1][3];
                if (kPreBasis && emit) {
#pragma unroll
                    for (int i = 0; i < kMaxBasis; ++i)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            ev[i][c] = (i < nv) ? buf_load(plane_rsrc(b + size_t(i) * (3 * size_t(G)), c, io), ptb, T(0))
                                                : T(0);
                }
                if (live(t)) stage_a(t, sa);
                __syncthreads();  // every wave has read plane t's tile
                const T* row = c1g + unsigned(o0 + t) * NC;  // table row of plane j
                if (live(t)) {
                    T W[3][3];
                    {
                        // each chain starts with a product: a zero start costs a
                        // register per chain (fma(a, b, 0) differs from a * b in
                        // the sign of a zero product), and the first neighbour's
                        // lane shift folds into it; every variant keeps this order
                        T mm[3], sm[3], am[3], ms[3], ma[3], aa[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            T s[R];
                            stencil(sa[3 * c + 0], s);
                            mm[c] = cb[0][0] * s[0];
                            sm[c] = cb[2][0] * s[0];
                            am[c] = c != 1 ? cb[1][0] * s[0] : T(0);
#pragma unroll
                            for (int k = 1; k < R; ++k) {
                                mm[c] = fma(cb[0][k], s[k], mm[c]);
                                sm[c] = fma(cb[2][k], s[k], sm[c]);
                                if (c != 1) am[c] = fma(cb[1][k], s[k], am[c]);
                            }
                            stencil(sa[3 * c + 2], s);
                            ms[c] = cb[0][0] * s[0];
#pragma unroll
                            for (int k = 1; k < R; ++k) ms[c] = fma(cb[0][k], s[k], ms[c]);
                            stencil(sa[3 * c + 1], s);
                            ma[c] = c != 2 ? cb[0][0] * s[0] : T(0);
                            aa[c] = c != 0 ? cb[1][0] * s[0] : T(0);
#pragma unroll
                            for (int k = 1; k < R; ++k) {
                                if (c != 2) ma[c] = fma(cb[0][k], s[k], ma[c]);
                                if (c != 0) aa[c] = fma(cb[1][k], s[k], aa[c]);
                            }
                        }
                        T w9[9];
                        combine_w(mm, sm, am, ms, ma, aa, al, be, ab, w9);
#pragma unroll
                        for (int i = 0; i < 9; ++i) W[i / 3][i % 3] = w9[i];
                    }
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const T cM = row[0 * R + k], cA = row[1 * R + k], cS = row[2 * R + k];
                        const int sl = (uu + k + 1) % R;
#pragma unroll
                        for (int c = 0; c < 3; ++c)
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                if (r == sl) {
                                    acc[c][r] = fma(cS, W[c][0], acc[c][r]);
                                    acc[c][r] = fma(cM, W[c][1], acc[c][r]);
                                    acc[c][r] = fma(cA, W[c][2], acc[c][r]);
                                }
                    }
                }
                {
                    const int sl = (uu + 1) % R;
                    T kx[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        kx[c] = T(0);
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if (r == sl) {
                                kx[c] = acc[c][r];
                                acc[c][r] = T(0);
                            }
                    }
                    if (emit) {
                        const T d0m = row[3 * R], d0s = row[3 * R + 1];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (MODE == kApplyY) {
                                buf_store(kx[c], plane_rsrc(y, c, io), ptb);
                            } else if (MODE == kApplyRes) {
                                buf_store(eb[c] - kx[c], plane_rsrc(y, c, io), ptb);
                            } else if (MODE == kApplyResDot) {
                                const T r = eb[c] - kx[c];
                                buf_store(r, plane_rsrc(y, c, io), ptb);
                                dots[0] += double(r) * double(r);
                            } else if (MODE == kApplyYDot) {
                                buf_store(kx[c], plane_rsrc(y, c, io), ptb);
                                dots[0] += double(ex[c]) * double(kx[c]);
                            } else if (MODE == kApplyCheb) {
                                buf_store(cheb_update(ex[c], ep[c], eb[c], kx[c], cd.fd[c], cd.fe[c], d0m, d0s, c1, c2),
                                          plane_rsrc(xout, c, io), ptb);
                            } else {
                                buf_store(kx[c], plane_rsrc(y, c, io), ptb);
                                if constexpr (kPreBasis) {
#pragma unroll
                                    for (int i = 0; i < kMaxBasis; ++i)
                                        if (i < nv) dots[i] += double(ev[i][c]) * double(kx[c]);
                                } else if (active) {
                                    const size_t idx = size_t(c) * G + size_t(io) * PL + size_t(i2c) * m3 + i3c;
#pragma unroll
                                    for (int i = 0; i < kMaxBasis; ++i)
                                        if (i < nv) dots[i] += double(b[size_t(i) * (3 * size_t(G)) + idx]) * double(kx[c]);
                                }
                                dots[kMaxBasis] += double(kx[c]) * double(kx[c]);
                            }
                        }
                    }
                    epi_load(io + 1);
                }
                if (t + 2 < TI) store_plane(t + 2);  // into the buffer plane t vacated
                if (t + 3 < TI) load_plane(t + 3);
            }
        }
    }
    apply_write_dots<MODE>(dots, nv, part);
    stamp_end(stamp);
}

// ------------------------------------------------------------------------------
// Short marches: when every block would march over a single output plane
// (small coarse levels), its 2 HB + 1 input planes are processed side by side
// instead of one after the other.  A block holds R = 2 HB + 1 groups of
// 32 TRS threads (TRS tile rows); group g computes stages A and B of input
// plane io - HB + g exactly as the marching kernel does and leaves W in LDS;
// then the groups of components 0, 1, 2 sum the axis-1 contributions of the R
// planes in the marching kernel's order, with the same fused multiply-adds, so
// A x is bitwise that of the marching kernel (the FP32 Chebyshev update may
// round its last bit differently), and run the epilogue.  One barrier-separated
// phase instead of 2 HB + 1.
// ------------------------------------------------------------------------------
template <typename T, int HB>
struct TileS {
    static constexpr int TR = k3ShortRows<T>();
    static constexpr int NP = TR * k3E3;            // threads per group
    static constexpr int R = 2 * HB + 1;            // groups (input planes)
    static constexpr int NT = R * NP;
    static constexpr int E2 = TR + 2 * HB;
    static constexpr int NIN = E2 * k3E3;
    static constexpr int NX = 3 * NIN;
    static constexpr int NLC = (NIN + NP - 1) / NP;
    static constexpr int NC = 3 * R + 2;
    static constexpr bool CAREG = sizeof(T) == 4;
    static constexpr size_t lds_words() {
        return size_t(R) * NX + size_t(R) * 9 * NP + (CAREG ? 0 : 3 * size_t(R) * TR);
    }
};

template <typename T, int HB, int MODE>
__global__ __launch_bounds__((2 * HB + 1) * k3ShortRows<T>() * k3E3) void k_apply3d_short(
    OpDev<T> op, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ b, const T* xprev, T* xout, T c1,
    T c2, Apply3dGeom g, unsigned long long* stamp, const T* __restrict__ c1r) {
    using Q = TileS<T, HB>;
    constexpr int TR = Q::TR, NP = Q::NP, R = Q::R, E3 = k3E3, T3 = k3T3(HB);
    constexpr int NIN = Q::NIN, NX = Q::NX, NLC = Q::NLC, NC = Q::NC;
    constexpr unsigned S = sizeof(T);
    stamp_begin(stamp);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);  // [R][3][E2][E3] input tiles
    T* ws = xs + size_t(R) * NX;             // [R][9][NP] W of each plane
    T* ca = ws + size_t(R) * 9 * NP;         // [3][R][TR] when not in registers
    const int m1 = op.m[0], m2 = op.m[1], m3 = op.m[2];
    const unsigned PL = unsigned(m2) * m3, G = unsigned(m1) * PL;
    const int xcd = int(blockIdx.x % kXcds), slot = int(blockIdx.x / kXcds);
    const int per = g.nblocks / kXcds, rem = g.nblocks % kXcds;
    const int tile = xcd * per + min(xcd, rem) + slot;
    const int o2 = (tile % g.nt2) * TR;
    const int o3 = ((tile / g.nt2) % g.nt3) * T3;
    const int io = tile / (g.nt2 * g.nt3);  // the block's output plane
    // a group is whole waves (NP is a multiple of 64): its index is wave-uniform,
    // and read into a scalar register so that plane descriptors and table rows
    // built from it stay scalar
    const int grp = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / NP), tid = threadIdx.x % NP;
    const int j = io - HB + grp;                 // this group's input plane
    const bool jlive = (j >= 0 && j < m1);       // uniform within the group
    const int ty = tid / E3, tx = tid % E3;
    const int i2 = o2 + ty, i3 = o3 - HB + tx;
    const bool active = (tx >= HB) && (tx < E3 - HB) && (i2 < m2) && (i3 < m3);
    const int i2c = min(i2, m2 - 1), i3c = min(max(i3, 0), m3 - 1);
    const unsigned ptb = active ? (unsigned(i2c) * m3 + unsigned(i3c)) * S : kOob;
    auto plane_rsrc = [&](const T* base, int c, int jj) {
        const bool jin = (jj >= 0 && jj < m1);
        return make_rsrc(base + (size_t(c) * G + size_t(jin ? jj : 0) * PL), jin ? PL * S : 0u);
    };
    // epilogue operands (groups 0..2: component grp of the output point)
    T eb = T(0), ex = T(0), ep = T(0);
    if (grp < 3) {
        if (MODE == kApplyRes || MODE == kApplyCheb) eb = buf_load(plane_rsrc(b, grp, io), ptb, T(0));
        if (MODE == kApplyCheb) {
            ex = buf_load(plane_rsrc(x, grp, io), ptb, T(0));
            ep = (c1 != T(0) && xprev != nullptr) ? buf_load(plane_rsrc(xprev, grp, io), ptb, T(0)) : T(0);
        }
    }
    // this group's input tile
    {
        T v[3][NLC];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const auto r = plane_rsrc(x, c, j);
#pragma unroll
            for (int q = 0; q < NLC; ++q) {
                const int e = min(tid + q * NP, NIN - 1);
                const int g2 = o2 - HB + e / E3, g3 = o3 - HB + e % E3;
                const bool in = g2 >= 0 && g2 < m2 && g3 >= 0 && g3 < m3;
                v[c][q] = buf_load(r, in ? (unsigned(g2) * m3 + unsigned(g3)) * S : kOob, T(0));
            }
        }
        T* dst = xs + size_t(grp) * NX;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < NLC; ++q) {
                const int e = tid + q * NP;
                if ((q + 1) * NP <= NIN || e < NIN) dst[c * NIN + e] = v[c][q];
            }
    }
    T car[Q::CAREG ? 3 : 1][Q::CAREG ? R : 1];
    if constexpr (Q::CAREG) {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int k = 0; k < R; ++k) car[w][k] = op.band[1][w][k * m2 + i2c];
    } else {
        for (int e = threadIdx.x; e < 3 * R * TR; e += Q::NT) {
            const int i = e % TR, k = (e / TR) % R, w = e / (TR * R);
            ca[e] = op.band[1][w][k * m2 + min(o2 + i, m2 - 1)];
        }
    }
    T cb[3][R];
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int k = 0; k < R; ++k) cb[w][k] = active ? op.band[2][w][k * m3 + i3] : T(0);
    const T al = op.alpha, be = op.beta, ab = offdiag_weight(op);
    __syncthreads();
    if (jlive) {
        // stage A (axis 2) and stage B (axis 3) of plane j, as in k_apply3d
        const T* src = xs + size_t(grp) * NX;
        T sa[9];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T aM = T(0), aA = T(0), aS = T(0);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T xv = src[c * NIN + (ty + k) * E3 + tx];
                if constexpr (Q::CAREG) {
                    aM = fma(car[0][k], xv, aM);
                    aA = fma(car[1][k], xv, aA);
                    aS = fma(car[2][k], xv, aS);
                } else {
                    aM = fma(ca[(0 * R + k) * TR + ty], xv, aM);
                    aA = fma(ca[(1 * R + k) * TR + ty], xv, aA);
                    aS = fma(ca[(2 * R + k) * TR + ty], xv, aS);
                }
            }
            sa[3 * c + 0] = aM;
            sa[3 * c + 1] = aA;
            sa[3 * c + 2] = aS;
        }
        auto stencil = [&](T val, T (&st)[R]) {
            st[HB] = val;
#pragma unroll
            for (int d = 1; d <= HB; ++d) {
                st[HB - d] = lane_shift<kDppShr1>(st[HB - d + 1]);
                st[HB + d] = lane_shift<kDppShl1>(st[HB + d - 1]);
            }
        };
        T mm[3], sm[3], am[3], ms[3], ma[3], aa[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T st[R];
            stencil(sa[3 * c + 0], st);
            mm[c] = cb[0][0] * st[0];
            sm[c] = cb[2][0] * st[0];
            am[c] = c != 1 ? cb[1][0] * st[0] : T(0);
#pragma unroll
            for (int k = 1; k < R; ++k) {
                mm[c] = fma(cb[0][k], st[k], mm[c]);
                sm[c] = fma(cb[2][k], st[k], sm[c]);
                if (c != 1) am[c] = fma(cb[1][k], st[k], am[c]);
            }
            stencil(sa[3 * c + 2], st);
            ms[c] = cb[0][0] * st[0];
#pragma unroll
            for (int k = 1; k < R; ++k) ms[c] = fma(cb[0][k], st[k], ms[c]);
            stencil(sa[3 * c + 1], st);
            ma[c] = c != 2 ? cb[0][0] * st[0] : T(0);
            aa[c] = c != 0 ? cb[1][0] * st[0] : T(0);
#pragma unroll
            for (int k = 1; k < R; ++k) {
                if (c != 2) ma[c] = fma(cb[0][k], st[k], ma[c]);
                if (c != 0) aa[c] = fma(cb[1][k], st[k], aa[c]);
            }
        }
        T W[9];
        combine_w(mm, sm, am, ms, ma, aa, al, be, ab, W);
        T* wd = ws + size_t(grp) * 9 * NP;
#pragma unroll
        for (int i = 0; i < 9; ++i) wd[i * NP + tid] = W[i];
    }
    __syncthreads();
    if (grp < 3) {
        const int c = grp;
        const T* orow = c1r + unsigned(io) * NC;  // axis-1 row of output plane io
        T kx = T(0);
#pragma unroll
        for (int gg = 0; gg < R; ++gg) {
            const int jj = io - HB + gg;
            if (jj >= 0 && jj < m1) {  // block-uniform; X1(io, jj) = orow[w R + gg]
                const T* wsrc = ws + size_t(gg) * 9 * NP + size_t(3 * c) * NP + tid;
                kx = fma(orow[2 * R + gg], wsrc[0 * NP], kx);
                kx = fma(orow[0 * R + gg], wsrc[1 * NP], kx);
                kx = fma(orow[1 * R + gg], wsrc[2 * NP], kx);
            }
        }
        const auto rs = (MODE == kApplyCheb) ? plane_rsrc(xout, c, io) : plane_rsrc(y, c, io);
        if (MODE == kApplyY) {
            buf_store(kx, rs, ptb);
        } else if (MODE == kApplyRes) {
            buf_store(eb - kx, rs, ptb);
        } else {  // Chebyshev step
            const T d0m = orow[3 * R], d0s = orow[3 * R + 1];  // diagonal entries of plane io
            T fd, fe;
            cheb_diag_one<T, HB>(op, c, i2c, i3c, active, fd, fe);
            buf_store(cheb_update(ex, ep, eb, kx, fd, fe, d0m, d0s, c1, c2), rs, ptb);
        }
    }
    stamp_end(stamp);
}

// ------------------------------------------------------------------------------
// Grouped marches: a block of G groups of 32 TRS threads (TRS tile rows) owns
// an output tile and a range [o0, o1) of x1 planes, like the marching kernel,
// but takes its input planes G at a time.  In phase p, group g computes
// stages A and B of input plane o0 - HB + G p + g and leaves its W in a ring
// of W planes in LDS; after a barrier, group g sums the axis-1 contributions
// of output plane o0 - 2 HB + G p + g from the ring, in the marching kernel's
// order and with the same fused multiply-adds (A x is bitwise that of the
// marching kernel), and runs the epilogue.  A range of L planes costs L + 2 HB
// planes of in-plane work and L sums, where the marching kernel pays L + 2 HB
// of both; G groups per block let the ranges be G times longer at the same
// number of waves, so the halo planes weigh less.
//
// One barrier per phase: every lane loads the 2 HB + 1 input rows of stage A
// at its own column straight from the caches (no shared input tile), one
// phase ahead, and the ring holds 2 G + 2 HB planes, so that the W a group
// writes in phase p + 1 never lands on a plane another group may still read
// for phase p (phases p and p + 1 touch 2 G + 2 HB consecutive planes;
// phase p + 2 starts after the barrier of p + 1, which every wave reaches only
// after its phase-p sums).
// ------------------------------------------------------------------------------
template <typename T, int HB>
struct TileG {
    static constexpr int TR = k3ShortRows<T>();
    static constexpr int NP = TR * k3E3;              // threads per group
    static constexpr int GR = k3Groups;               // groups: input planes per phase
    static constexpr int NT = GR * NP;
    static constexpr int R = 2 * HB + 1;
    static constexpr int RING = 2 * GR + 2 * HB;      // W planes held
    static constexpr int NC = 3 * R + 2;
    // axis-2 band rows in registers in FP32 up to HB = 3; above, they would
    // push the kernel past 128 VGPRs (3 waves per SIMD instead of 4)
    static constexpr bool CAREG = sizeof(T) == 4 && HB <= 3;
    static constexpr size_t lds_words() { return size_t(RING) * 9 * NP + (CAREG ? 0 : 3 * size_t(R) * TR); }
};

template <typename T, int HB, int MODE>
__global__ __launch_bounds__(k3Groups * k3ShortRows<T>() * k3E3) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && HB <= 4 ? 4 : 1))) void k_apply3d_group(
    OpDev<T> op, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ b, const T* xprev, T* xout, T c1,
    T c2, Apply3dGeom g, unsigned long long* stamp, const T* __restrict__ c1r) {
    using Q = TileG<T, HB>;
    constexpr int TR = Q::TR, NP = Q::NP, GR = Q::GR, R = Q::R, RING = Q::RING, E3 = k3E3, T3 = k3T3(HB);
    constexpr int NC = Q::NC;
    constexpr unsigned S = sizeof(T);
    stamp_begin(stamp);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* ws = reinterpret_cast<T*>(smem_raw);  // [RING][9][NP] W of the ring's planes
    T* ca = ws + size_t(RING) * 9 * NP;      // [3][R][TR] when not in registers
    const int m1 = op.m[0], m2 = op.m[1], m3 = op.m[2];
    const unsigned PL = unsigned(m2) * m3, G = unsigned(m1) * PL;
    const int xcd = int(blockIdx.x % kXcds), slot = int(blockIdx.x / kXcds);
    const int per = g.nblocks / kXcds, rem = g.nblocks % kXcds;
    const int tile = xcd * per + min(xcd, rem) + slot;
    const int o2 = (tile % g.nt2) * TR;
    const int o3 = ((tile / g.nt2) % g.nt3) * T3;
    const int o0 = (tile / (g.nt2 * g.nt3)) * g.c1len;
    const int o1 = min(o0 + g.c1len, m1);
    // a group is whole waves (NP is a multiple of 64): its index is wave-uniform,
    // and read into a scalar register so that plane descriptors, table rows and
    // ring slots built from it stay scalar
    const int grp = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / NP), tid = threadIdx.x % NP;
    const int ty = tid / E3, tx = tid % E3;
    const int i2 = o2 + ty, i3 = o3 - HB + tx;
    const bool active = (tx >= HB) && (tx < E3 - HB) && (i2 < m2) && (i3 < m3);
    const int i2c = min(i2, m2 - 1), i3c = min(max(i3, 0), m3 - 1);
    const unsigned ptb = active ? (unsigned(i2c) * m3 + unsigned(i3c)) * S : kOob;
    auto plane_rsrc = [&](const T* base, int c, int jj) {
        const bool jin = (jj >= 0 && jj < m1);
        return make_rsrc(base + (size_t(c) * G + size_t(jin ? jj : 0) * PL), jin ? PL * S : 0u);
    };
    T car[Q::CAREG ? 3 : 1][Q::CAREG ? R : 1];
    if constexpr (Q::CAREG) {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int k = 0; k < R; ++k) car[w][k] = op.band[1][w][k * m2 + i2c];
    } else {
        for (int e = threadIdx.x; e < 3 * R * TR; e += Q::NT) {
            const int i = e % TR, k = (e / TR) % R, w = e / (TR * R);
            ca[e] = op.band[1][w][k * m2 + min(o2 + i, m2 - 1)];
        }
    }
    T cb[3][R];
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int k = 0; k < R; ++k) cb[w][k] = active ? op.band[2][w][k * m3 + i3] : T(0);
    const ChebDiag<T> cd = cheb_diag<T, HB>(op, i2c, i3c, active);
    const T al = op.alpha, be = op.beta, ab = offdiag_weight(op);

    // the 2 HB + 1 input rows of stage A at this lane's column (offsets out of
    // range outside the grid, so those entries read as zero)
    unsigned roff[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = i2 - HB + k;
        const bool in = r >= 0 && r < m2 && i3 >= 0 && i3 < m3;
        roff[k] = in ? (unsigned(r) * m3 + unsigned(i3)) * S : kOob;
    }
    T xin[3][R];
    auto load_in = [&](int jj) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const auto r = plane_rsrc(x, c, jj);
#pragma unroll
            for (int k = 0; k < R; ++k) xin[c][k] = buf_load(r, roff[k], T(0));
        }
    };
    T eb[3], ex[3], ep[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) eb[c] = ex[c] = ep[c] = T(0);
    const bool use_prev = (c1 != T(0) && xprev != nullptr);
    auto epi_load = [&](int io) {
        if (io < o0 || io >= o1) return;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (MODE == kApplyRes || MODE == kApplyCheb) eb[c] = buf_load(plane_rsrc(b, c, io), ptb, T(0));
            if (MODE == kApplyCheb) {
                ex[c] = buf_load(plane_rsrc(x, c, io), ptb, T(0));
                ep[c] = use_prev ? buf_load(plane_rsrc(xprev, c, io), ptb, T(0)) : T(0);
            }
        }
    };
    auto stencil = [&](T val, T (&st)[R]) {
        st[HB] = val;
#pragma unroll
        for (int d = 1; d <= HB; ++d) {
            st[HB - d] = lane_shift<kDppShr1>(st[HB - d + 1]);
            st[HB + d] = lane_shift<kDppShl1>(st[HB + d - 1]);
        }
    };

    const int TI = (o1 - o0) + 2 * HB;  // input planes of the range
    const int NPH = (TI + GR - 1) / GR;  // phases
    load_in(o0 - HB + grp);
    epi_load(o0 - 2 * HB + grp);
    if constexpr (!Q::CAREG) __syncthreads();  // the axis-2 band rows are in LDS
    for (int ph = 0; ph < NPH; ++ph) {
        const int t = ph * GR + grp;  // this group's input plane index in the range
        const int j = o0 - HB + t;
        const bool jlive = t < TI && j >= 0 && j < m1;
        const int io = o0 - 2 * HB + t;  // this group's output plane
        const bool emit = io >= o0 && io < o1;
        // the axis-1 row of the output plane, read early so that its scalar
        // loads are in flight during stages A and B
        T oc[NC];
        if (emit) {
            const T* orow = c1r + unsigned(io) * NC;
#pragma unroll
            for (int i = 0; i < NC; ++i) oc[i] = orow[i];
        }
        T sa[9];
        if (jlive) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T aM = T(0), aA = T(0), aS = T(0);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T xv = xin[c][k];
                    if constexpr (Q::CAREG) {
                        aM = fma(car[0][k], xv, aM);
                        aA = fma(car[1][k], xv, aA);
                        aS = fma(car[2][k], xv, aS);
                    } else {
                        aM = fma(ca[(0 * R + k) * TR + ty], xv, aM);
                        aA = fma(ca[(1 * R + k) * TR + ty], xv, aA);
                        aS = fma(ca[(2 * R + k) * TR + ty], xv, aS);
                    }
                }
                sa[3 * c + 0] = aM;
                sa[3 * c + 1] = aA;
                sa[3 * c + 2] = aS;
            }
        }
        if (t + GR < TI) load_in(j + GR);  // the next phase's rows, into the registers stage A freed
        if (jlive) {
            T mm[3], sm[3], am[3], ms[3], ma[3], aa[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T st[R];
                stencil(sa[3 * c + 0], st);
                mm[c] = cb[0][0] * st[0];
                sm[c] = cb[2][0] * st[0];
                am[c] = c != 1 ? cb[1][0] * st[0] : T(0);
#pragma unroll
                for (int k = 1; k < R; ++k) {
                    mm[c] = fma(cb[0][k], st[k], mm[c]);
                    sm[c] = fma(cb[2][k], st[k], sm[c]);
                    if (c != 1) am[c] = fma(cb[1][k], st[k], am[c]);
                }
                stencil(sa[3 * c + 2], st);
                ms[c] = cb[0][0] * st[0];
#pragma unroll
                for (int k = 1; k < R; ++k) ms[c] = fma(cb[0][k], st[k], ms[c]);
                stencil(sa[3 * c + 1], st);
                ma[c] = c != 2 ? cb[0][0] * st[0] : T(0);
                aa[c] = c != 0 ? cb[1][0] * st[0] : T(0);
#pragma unroll
                for (int k = 1; k < R; ++k) {
                    if (c != 2) ma[c] = fma(cb[0][k], st[k], ma[c]);
                    if (c != 0) aa[c] = fma(cb[1][k], st[k], aa[c]);
                }
            }
            T W[9];
            combine_w(mm, sm, am, ms, ma, aa, al, be, ab, W);
            T* wd = ws + size_t(t % RING) * 9 * NP + tid;
#pragma unroll
            for (int i = 0; i < 9; ++i) wd[i * NP] = W[i];
        }
        __syncthreads();  // W of the phase's planes in the ring
        if (emit) {
            T kx[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int gg = 0; gg < R; ++gg) {
                const int jj = io - HB + gg;
                if (jj >= 0 && jj < m1) {  // X1(io, jj) = oc[w R + gg]
                    const T cM = oc[0 * R + gg], cA = oc[1 * R + gg], cS = oc[2 * R + gg];
                    const T* wsrc = ws + size_t((t - 2 * HB + gg) % RING) * 9 * NP + tid;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        kx[c] = fma(cS, wsrc[(3 * c + 0) * NP], kx[c]);
                        kx[c] = fma(cM, wsrc[(3 * c + 1) * NP], kx[c]);
                        kx[c] = fma(cA, wsrc[(3 * c + 2) * NP], kx[c]);
                    }
                }
            }
            const T d0m = oc[3 * R], d0s = oc[3 * R + 1];  // diagonal entries of plane io
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (MODE == kApplyY) {
                    buf_store(kx[c], plane_rsrc(y, c, io), ptb);
                } else if (MODE == kApplyRes) {
                    buf_store(eb[c] - kx[c], plane_rsrc(y, c, io), ptb);
                } else {  // Chebyshev step
                    buf_store(cheb_update(ex[c], ep[c], eb[c], kx[c], cd.fd[c], cd.fe[c], d0m, d0s, c1, c2),
                              plane_rsrc(xout, c, io), ptb);
                }
            }
        }
        epi_load(io + GR);  // the next phase's output plane
    }
    stamp_end(stamp);
}

// The variant for one launch: the caller's choice, else the short-march
// variant on small grids (apply3d_geom_short), the grouped march where the
// marching kernel's ranges would be short (apply3d_prefer_group) and the
// marching kernel otherwise.  Kernels with fused dot products always march.
template <typename T, int HB, int MODE>
int apply3d_variant(const OpDev<T>& op) {
    constexpr bool kPlain = (MODE == kApplyY || MODE == kApplyRes || MODE == kApplyCheb);
    if (!kPlain) return CD_APPLY3D_MARCH;
    int v = op.variant;
    if (v == CD_APPLY3D_AUTO) {
        if (op.x1chunk != 0) return CD_APPLY3D_MARCH;
        if (apply3d_geom_short(op.m, HB, sizeof(T), 0).nblocks > 0)
            v = CD_APPLY3D_SHORT;
        else if (apply3d_prefer_group(op.m, HB, sizeof(T)))
            v = CD_APPLY3D_GROUP;
        else
            v = CD_APPLY3D_MARCH;
    }
    if (v == CD_APPLY3D_SHORT && HB > 3) v = CD_APPLY3D_MARCH;
    return v;
}

template <typename T, int HB, int MODE>
void launch3d(const OpDev<T>& op, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2, double* part, int nv,
              unsigned long long* stamp, hipStream_t s) {
    if (size_t(3) * op.m[0] * op.m[1] * op.m[2] >= (size_t(1) << 31))
        throw std::runtime_error("3D operator kernel: too many unknowns for 32-bit offsets");
    if (size_t(op.m[1]) * op.m[2] * sizeof(T) >= (size_t(1) << 31))
        throw std::runtime_error("3D operator kernel: a grid plane exceeds the 2 GiB of a buffer descriptor");
    const int variant = apply3d_variant<T, HB, MODE>(op);
    if constexpr (MODE == kApplyY || MODE == kApplyRes || MODE == kApplyCheb) {
        if constexpr (HB <= 3) {
            if (variant == CD_APPLY3D_SHORT) {
                using QS = TileS<T, HB>;
                const Apply3dGeom gs = apply3d_geom_short(op.m, HB, sizeof(T), 0, true);
                const size_t lds = QS::lds_words() * sizeof(T);
                auto kern = k_apply3d_short<T, HB, MODE>;
                allow_lds(reinterpret_cast<const void*>(kern), lds);
                hipLaunchKernelGGL(kern, dim3(gs.nblocks), dim3(QS::NT), lds, s, op, x, y, b, u, xout, c1, c2, gs,
                                   stamp, op.c1r);
                return;
            }
        }
        if (variant == CD_APPLY3D_GROUP) {
            using QG = TileG<T, HB>;
            const Apply3dGeom gg = apply3d_geom_group(op.m, HB, sizeof(T), op.x1chunk);
            const size_t lds = QG::lds_words() * sizeof(T);
            auto kern = k_apply3d_group<T, HB, MODE>;
            allow_lds(reinterpret_cast<const void*>(kern), lds);
            hipLaunchKernelGGL(kern, dim3(gg.nblocks), dim3(QG::NT), lds, s, op, x, y, b, u, xout, c1, c2, gg, stamp,
                               op.c1r);
            return;
        }
    }
    using Q = Tile3<T, HB>;
    const Apply3dGeom g = apply3d_geom(op.m, HB, sizeof(T), op.x1chunk);
    const size_t lds = Q::lds_words() * sizeof(T);
    auto kern = k_apply3d<T, HB, MODE>;
    allow_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, dim3(g.nblocks), dim3(Q::NT), lds, s, op, x, y, b, u, xout, c1, c2, part, nv, g, stamp,
                       op.c1p);
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
