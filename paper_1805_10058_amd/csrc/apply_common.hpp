// Operator-apply helpers shared by the 2D and 3D kernels (internal header):
// launch geometry, the fused epilogue modes and the per-block dot products.
#pragma once

#include "device_common.hpp"

namespace cd {

// Launch entry points of the operator kernels, one explicit instantiation per
// (precision, half bandwidth) in its own object (apply2d.hip, apply3d.hip).
template <typename T, int HB>
void apply3d_run(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2,
                 double* part, int nv, unsigned long long* stamp, hipStream_t s);
template <typename T, int HB>
void apply2d_run(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2,
                 double* part, int nv, unsigned long long* stamp, hipStream_t s);

constexpr int kT1 = 8, kT2 = 32;  // 2D output tile: kT1 * kT2 = kThreads points

namespace {

// 3D output tile: k3Rows(T) rows (x2) of k3T3(HB) = 32 - 2HB columns (x3);
// a thread per point of the tile rows times 32 columns (the output columns
// and their x3 halo): 256-thread blocks of 8 rows in FP32, 128-thread blocks
// of 4 rows in FP64.
constexpr int k3E3 = 32;
__host__ __device__ constexpr int k3T3(int hb) { return k3E3 - 2 * hb; }
template <typename T>
__host__ __device__ constexpr int k3Rows() { return sizeof(T) == 4 ? 8 : 4; }
// tile rows of the short-march variant (one wave per group in FP64)
template <typename T>
__host__ __device__ constexpr int k3ShortRows() { return sizeof(T) == 4 ? 4 : 2; }

// Launch geometry of the 3D operator kernel: tiles of the (x2, x3) plane times
// ranges of x1 planes.  Blocks march along x1, and each of their input planes
// costs the in-plane contractions whether or not it is a halo plane, so the x1
// range is made as long as the device's resident blocks allow: about as many
// blocks as fit at once (4 per compute unit in both precisions, from the
// register footprint of the kernels: 4 waves per SIMD in FP32, 2 in FP64).
// Where that leaves ranges of HB planes or fewer (2 HB halo planes each), the
// ranges are doubled for HB >= 3: measured in the solves at m = 65 (ranges of
// 4 instead of 2: 17 instead of 22 us per Chebyshev step) and m = 33 (2
// instead of 1: 11 instead of 12 us), while at m = 129 halving the blocks to
// 22-plane ranges costs 10%.
struct Apply3dGeom {
    int nt2, nt3, c1len, nblocks;
};

// x1chunk > 0 fixes the number of x1 planes per block (the last block of a
// column takes the remainder).
inline Apply3dGeom apply3d_geom(const int* m, int hb, size_t elem, int x1chunk = 0) {
    const int kTargetBlocks = 1024;
    const int rows = elem == 4 ? k3Rows<float>() : k3Rows<double>();
    Apply3dGeom g;
    g.nt2 = (m[1] + rows - 1) / rows;
    g.nt3 = (m[2] + k3T3(hb) - 1) / k3T3(hb);
    const int planar = g.nt2 * g.nt3;
    if (x1chunk > 0) {
        g.c1len = std::min(x1chunk, m[0]);
    } else {
        const int nx1 = std::max(1, std::min(m[0], kTargetBlocks / planar));
        g.c1len = (m[0] + nx1 - 1) / nx1;
        if (hb >= 3 && g.c1len <= hb) {
            if (g.c1len > 1)
                g.c1len = std::min(2 * g.c1len, m[0]);
            else if (m[0] >= 10 * hb)
                g.c1len = 2;
        }
    }
    g.nblocks = planar * ((m[0] + g.c1len - 1) / g.c1len);
    return g;
}

// Geometry of the short-march variant of the 3D kernel (tiles of
// k3ShortRows rows, one output plane per block, 2 HB + 1 groups of threads):
// nblocks = 0 when the marching kernel is used instead.  The variant does
// 2 HB + 1 planes of in-plane work per output plane, the marching kernel with
// one-plane ranges as much but one plane after another, so it pays where the
// grid is small enough that latency, not work, sets the time: automatic
// geometry (x1chunk = 0), HB <= 3, one-plane ranges under the marching rule,
// and at most 3072 waves in all (measured: 17^3 8.0 against 10.4 us per
// Chebyshev step in FP32, 7.0 against 12.5 us in FP64; at 33^3 and above the
// marching kernel is faster).
// With force, the geometry regardless of the rule (for HB <= 3).
inline Apply3dGeom apply3d_geom_short(const int* m, int hb, size_t elem, int x1chunk, bool force = false) {
    Apply3dGeom g{0, 0, 1, 0};
    if (x1chunk != 0 || hb > 3) return g;
    const int rows = elem == 4 ? k3Rows<float>() : k3Rows<double>();
    const int planar = ((m[1] + rows - 1) / rows) * ((m[2] + k3T3(hb) - 1) / k3T3(hb));
    if (!force && std::max(1, std::min(m[0], 1024 / planar)) < m[0]) return g;  // ranges of more than one plane
    const int srows = elem == 4 ? k3ShortRows<float>() : k3ShortRows<double>();
    const int nt2 = (m[1] + srows - 1) / srows, nt3 = (m[2] + k3T3(hb) - 1) / k3T3(hb);
    const long waves = long(nt2) * nt3 * m[0] * (2 * hb + 1) * srows / 2;  // 32 srows threads per group
    if (!force && waves > 3072) return g;
    g.nt2 = nt2;
    g.nt3 = nt3;
    g.nblocks = nt2 * nt3 * m[0];
    return g;
}

// Grouped-march variant of the 3D kernel: k3Groups groups of 32 k3ShortRows
// threads per block, each taking one input plane per phase.  Ranges are set
// from a target number of waves in all (what fits at once: 4 per SIMD in
// FP32, 2 in FP64), then lengthened so that the range and its 2 HB halo
// planes fill whole phases.
constexpr int k3Groups = 4;
// x1chunk > 0 fixes the range length instead.
inline Apply3dGeom apply3d_geom_group(const int* m, int hb, size_t elem, int x1chunk) {
    const int waves = elem == 4 ? 4096 : 2048;  // FP64: 2 waves per SIMD fit (registers)
    Apply3dGeom g{0, 0, 1, 0};
    const int srows = elem == 4 ? k3ShortRows<float>() : k3ShortRows<double>();
    const int wpb = k3Groups * srows / 2;  // waves per block
    g.nt2 = (m[1] + srows - 1) / srows;
    g.nt3 = (m[2] + k3T3(hb) - 1) / k3T3(hb);
    const int planar = g.nt2 * g.nt3;
    const int nx1 = std::max(1, std::min(m[0], waves / wpb / planar));
    const int len = (m[0] + nx1 - 1) / nx1;
    const int phases = (len + 2 * hb + k3Groups - 1) / k3Groups;
    g.c1len = x1chunk > 0 ? std::min(x1chunk, m[0]) : std::min(m[0], phases * k3Groups - 2 * hb);
    g.nblocks = planar * ((m[0] + g.c1len - 1) / g.c1len);
    return g;
}

// Whether the grouped march beats the marching kernel on a grid: where the
// marching kernel's ranges are short, its halo planes dominate and the
// grouped march's longer ranges pay for its LDS exchange of W.  Measured per
// FP32 Chebyshev step (grouped against marching): p=3, m = 33 (marching
// ranges of 2) 11.1 against 13.4 us, m = 65 (ranges of 4) 19.9 against
// 20.7, m = 129 (ranges of 11) 56.5 against 55.3 at best; p=2, m = 64, 48 and
// 32: 13.5 / 10.9 / 8.3 against 14.8 / 13.0 / 10.2, m = 96 (ranges of 5) a
// tie; p=4, m = 66 and 34: 22.8 / 14.1 against 27.5 / 20.6, m = 98 (ranges
// of 6) a tie.  FP64, p=3, m = 65: 23.8 against 28.1 us.
inline bool apply3d_prefer_group(const int* m, int hb, size_t elem) {
    const int len = apply3d_geom(m, hb, elem, 0).c1len;
    return len < m[0] && len <= hb + 1;
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
                                     const T* u, T c1, int nv, size_t ntot) {
    if (MODE == kApplyRes || MODE == kApplyResDot || MODE == kApplyCheb) e.b = b[idx];
    if (MODE == kApplyCheb) {
        // the previous iterate (u holds it; nullptr: zero, the step after a start from zero);
        // not read on a first step (c1 = 0)
        e.u = (c1 != T(0) && u != nullptr) ? u[idx] : T(0);
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
                                      const EpiIn<T>& e, T* __restrict__ y, T* u,
                                      T* xout, T c1, T c2, int nv, double* dots) {
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
        xout[idx] = e.x + (c1 * (e.x - e.u) + c2 * r / dg);
    } else {
        y[idx] = kx;
        dots[0] += double(e.x) * double(kx);
    }
}

// Both at once (the 3D kernel, whose output entries change plane by plane).
template <typename T, int MODE>
__device__ inline void apply_epilogue(const OpDev<T>& op, int c, size_t idx, T kx, int i1, int i2, int i3,
                                      const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ b,
                                      T* u, T* xout, T c1, T c2, int nv, size_t ntot,
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

}  // namespace
}  // namespace cd
