// Device helpers shared by the kernel sources (internal header): block size,
// FP64 wave/block reductions, kernel-side timing stamps, band access and the
// diagonal of a level operator.
#pragma once

#include <hip/hip_runtime.h>

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

// Weight of the off-diagonal blocks (alpha - beta) A (x) A (x) M, zero for the
// block-diagonal part D (Sec. 6.1, eq. diag).
template <typename T>
__device__ inline T offdiag_weight(const OpDev<T>& op) {
    return op.blockdiag ? T(0) : op.alpha - op.beta;
}

constexpr int kXcds = 8;  // XCDs of the device; blocks are dispatched to them round robin

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

}  // namespace
}  // namespace cd
