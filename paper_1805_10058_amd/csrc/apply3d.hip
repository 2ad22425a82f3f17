// 3D curl-div operator apply (sum factorization), one object per (precision,
// half bandwidth): compiled with -DCD_T=<float|double> -DCD_HB=<1..6>.
#include "apply_common.hpp"

namespace cd {
namespace {

// ------------------------------------------------------------------------------
// 3D operator apply.
//
// A block of 32 TR threads owns an output tile of TR x (32 - 2HB) columns of
// the (x2, x3) plane (one output column per thread; the other threads only
// help with loads and stage A) and the output planes x1 in [o0, o1); it
// marches over the input planes t = 0, 1, ... (x1 = o0 - HB + t) up to
// o1 + HB.  Per input plane j:
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
// buffered in LDS.  The axis-1 coefficients of plane j (the row of the
// level's table: X1(j-HB+k, j) and the diagonal of plane j-HB) travel with
// the plane's loads into a ring of 4 rows, so the row a phase reads is never
// the one a faster wave overwrites in the same phase.  In FP32 the operands
// of the epilogue (b, x, the previous iterate) are loaded one phase before
// their plane is emitted; in FP64, whose registers allow fewer waves, at the
// start of that phase.  The Chebyshev step's diagonal comes from per-thread
// in-plane factors and the plane's diagonal entries in the table row.
//
// Accumulator slots: the accumulator of output plane i lives in slot
// (i - o0 + 2HB + 1) mod (2HB+1).  Every phase reads and clears the slot of
// the plane it completes, emitted or not, so slots need no range checks: a
// plane's slot is cleared one phase before its first contribution.
//
// Tiles are numbered with x2 fastest, then x3, then the x1 range, and block b
// takes tile (b mod 8) * ceil-share + b / 8: consecutive blocks land on
// different XCDs, so this keeps spatially adjacent tiles, whose halos overlap,
// on the same XCD and its L2.
// ------------------------------------------------------------------------------
template <typename T, int HB>
struct Tile3 {
    static constexpr int TR = k3Rows<T>();  // tile rows (x2)
    static constexpr int NT = TR * k3E3;    // threads: one stage-A position each
    static constexpr int R = 2 * HB + 1;
    static constexpr int E2 = TR + 2 * HB;  // input rows with the x2 halo
    static constexpr int NIN = E2 * k3E3;   // input tile of one component
    static constexpr int NX = 3 * NIN;      // input tile of a plane
    static constexpr int NLX = (NX + NT - 1) / NT;
    static constexpr int NC = 3 * R + 2;    // axis-1 table row
    static constexpr size_t lds_words() {
        return 2 * size_t(NX) + 2 * 9 * size_t(NT) + 3 * size_t(R) * TR + 4 * size_t(NC);
    }
};

template <typename T>
struct Epi3 {
    T b[3], x[3], xp[3];
};

template <typename T, int HB, int MODE>
__global__ __launch_bounds__(k3Rows<T>() * k3E3) void k_apply3d(OpDev<T> op, const T* __restrict__ x,
                                                               T* __restrict__ y, const T* __restrict__ b,
                                                               const T* xprev, T* xout, T c1, T c2,
                                                               double* __restrict__ part, int nv, Apply3dGeom g,
                                                               unsigned long long* stamp) {
    using Q = Tile3<T, HB>;
    constexpr int TR = Q::TR, NT = Q::NT, R = Q::R, E3 = k3E3, T3 = k3T3(HB);
    constexpr int NIN = Q::NIN, NX = Q::NX, NLX = Q::NLX, NC = Q::NC, NA = NT;
    stamp_begin(stamp);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);  // [2][3][E2][E3] input tiles
    T* st = xs + 2 * NX;                     // [2][9][TR][E3]: M2x A2x S2x of components 0, 1, 2
    T* ca = st + 2 * 9 * NA;                 // [3][R][TR] axis-2 band rows of the tile
    T* rows = ca + 3 * R * TR;               // [4][NC] ring of axis-1 table rows
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
    for (int e = tid; e < 3 * R * TR; e += NT) {
        const int i = e % TR, k = (e / TR) % R, w = e / (TR * R);
        ca[e] = op.band[1][w][k * m2 + min(o2 + i, m2 - 1)];  // rows past the grid feed unused outputs
    }
    // stage-A position of this thread; output column of this thread
    const int ai = tid / E3, aq = tid % E3;
    const int ty = tid / E3, tx = tid % E3;
    const int i2 = o2 + ty, i3 = o3 + tx;
    const bool active = (tx < T3) && (i2 < m2) && (i3 < m3);
    const int i2c = min(i2, m2 - 1), i3c = min(i3, m3 - 1);
    T cb[3][R];  // axis-3 band row of the thread's column (zero when inactive)
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int k = 0; k < R; ++k) cb[w][k] = active ? op.band[2][w][k * m3 + i3] : T(0);
    // in-plane factors of the diagonal at the thread's output column
    const T dm1 = op.band[1][0][HB * m2 + i2c], ds1 = op.band[1][2][HB * m2 + i2c];
    const T dm2 = op.band[2][0][HB * m3 + i3c], ds2 = op.band[2][2][HB * m3 + i3c];
    const T dmm = dm1 * dm2, dsm = ds1 * dm2, dms = dm1 * ds2;
    const unsigned pt = unsigned(i2c) * m3 + unsigned(i3c);  // in-plane offset of the output point
    T acc[3][R];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[c][r] = T(0);
    double dots[apply_ndots<MODE>()];
#pragma unroll
    for (int i = 0; i < apply_ndots<MODE>(); ++i) dots[i] = 0.0;
    const T al = op.alpha, be = op.beta, ab = offdiag_weight(op);

    // loads of one plane: NLX entries of the 3 component tiles per thread
    // (offsets within a plane of the component stack, the same for every
    // plane; ~0u outside the grid) and the plane's table row (threads < NC)
    unsigned loff[NLX];
#pragma unroll
    for (int q = 0; q < NLX; ++q) {
        const int e = min(tid + q * NT, NX - 1);
        const int c = e / NIN, rr = e % NIN;
        const int g2 = o2 - HB + rr / E3, g3 = o3 - HB + rr % E3;
        const bool in = g2 >= 0 && g2 < m2 && g3 >= 0 && g3 < m3;
        loff[q] = in ? unsigned(c) * G + unsigned(g2) * m3 + unsigned(g3) : ~0u;
    }
    T v[NLX];
    T vt = T(0);
    const T* __restrict__ c1p = op.c1p;
    auto load_plane = [&](int t) {
        const int j = o0 - HB + t;
        const bool jin = (j >= 0 && j < m1);  // block-uniform
        const unsigned jo = unsigned(jin ? j : 0) * PL;
#pragma unroll
        for (int q = 0; q < NLX; ++q) {
            const bool in = jin && loff[q] != ~0u;
            const T val = x[in ? jo + loff[q] : 0u];
            v[q] = in ? val : T(0);
        }
        if (tid < NC) vt = c1p[unsigned(j + HB) * NC + tid];  // rows of planes -HB .. m1+HB-1
    };
    auto store_plane = [&](int t) {
        T* dst = xs + (t & 1) * NX;
#pragma unroll
        for (int q = 0; q < NLX; ++q) {
            const int e = tid + q * NT;
            if (q + 1 < NLX || e < NX) dst[e] = v[q];
        }
        if (tid < NC) rows[(t & 3) * NC + tid] = vt;
    };
    auto live = [&](int t) {
        const int j = o0 - HB + t;
        return j >= 0 && j < m1;
    };
    auto stage_a = [&](int t) {
        const T* src = xs + (t & 1) * NX;
        T* dst = st + (t & 1) * 9 * NA;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T aM = T(0), aA = T(0), aS = T(0);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T xv = src[c * NIN + (ai + k) * E3 + aq];
                aM += ca[(0 * R + k) * TR + ai] * xv;
                aA += ca[(1 * R + k) * TR + ai] * xv;
                aS += ca[(2 * R + k) * TR + ai] * xv;
            }
            dst[(3 * c + 0) * NA + tid] = aM;
            dst[(3 * c + 1) * NA + tid] = aA;
            dst[(3 * c + 2) * NA + tid] = aS;
        }
    };
    // epilogue operands at the thread's output point of plane io
    constexpr bool kPre = (MODE != kApplyYMulti);  // the Krylov basis rows are loaded at the store
    constexpr bool kAhead = (sizeof(T) == 4);
    Epi3<T> en{};
    auto epi_load = [&](int io) {
        if (!kPre || io < o0 || io >= o1 || !active) return;
        const unsigned base = unsigned(io) * PL + pt;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const unsigned idx = unsigned(c) * G + base;
            if (MODE == kApplyRes || MODE == kApplyResDot || MODE == kApplyCheb) en.b[c] = b[idx];
            if (MODE == kApplyCheb) {
                en.x[c] = x[idx];
                en.xp[c] = (c1 != T(0) && xprev != nullptr) ? xprev[idx] : T(0);
            }
            if (MODE == kApplyYDot) en.x[c] = x[idx];
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
                Epi3<T> ec;
                if (kAhead) {
                    ec = en;
                    epi_load(io + 1);
                } else {
                    epi_load(io);
                    ec = en;
                }
                if (t + 1 < TI && live(t + 1)) stage_a(t + 1);
                const T* row = rows + (t & 3) * NC;
                if (live(t)) {
                    const T* sb = st + (t & 1) * 9 * NA;
                    T W[3][3];
                    {
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
                        const T cM = row[0 * R + k], cA = row[1 * R + k], cS = row[2 * R + k];  // X1(j-HB+k, j)
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
                    if (emit && active) {
                        const unsigned base = unsigned(io) * PL + pt;
                        const T d0m = row[3 * R], d0s = row[3 * R + 1];  // M1, S1 at (io, io)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const unsigned idx = unsigned(c) * G + base;
                            if (MODE == kApplyY) {
                                y[idx] = kx[c];
                            } else if (MODE == kApplyRes) {
                                y[idx] = ec.b[c] - kx[c];
                            } else if (MODE == kApplyResDot) {
                                const T r = ec.b[c] - kx[c];
                                y[idx] = r;
                                dots[0] += double(r) * double(r);
                            } else if (MODE == kApplyYDot) {
                                y[idx] = kx[c];
                                dots[0] += double(ec.x[c]) * double(kx[c]);
                            } else if (MODE == kApplyCheb) {
                                // diagonal: beta prod(S on axis c, M elsewhere) + alpha sum over the other axes
                                const T dg = (c == 0 ? be : al) * d0s * dmm + (c == 1 ? be : al) * d0m * dsm +
                                             (c == 2 ? be : al) * d0m * dms;
                                const T r = ec.b[c] - kx[c];
                                xout[idx] = ec.x[c] + (c1 * (ec.x[c] - ec.xp[c]) + c2 * r / dg);
                            } else {  // y = A x with the Krylov-basis dots
                                y[idx] = kx[c];
#pragma unroll
                                for (int i = 0; i < kMaxBasis; ++i)
                                    if (i < nv) dots[i] += double(b[size_t(i) * (3 * size_t(G)) + idx]) * double(kx[c]);
                                dots[kMaxBasis] += double(kx[c]) * double(kx[c]);
                            }
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
    using Q = Tile3<T, HB>;
    const Apply3dGeom g = apply3d_geom(op.m, HB, sizeof(T), op.x1chunk);
    if (size_t(3) * op.m[0] * op.m[1] * op.m[2] >= (size_t(1) << 31))
        throw std::runtime_error("3D operator kernel: too many unknowns for 32-bit offsets");
    const size_t lds = Q::lds_words() * sizeof(T);
    auto kern = k_apply3d<T, HB, MODE>;
    allow_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, dim3(g.nblocks), dim3(Q::NT), lds, s, op, x, y, b, u, xout, c1, c2, part, nv, g, stamp);
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
