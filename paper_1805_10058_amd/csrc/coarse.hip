// Coarsest-level solve: dense FP64 Cholesky factorization K = L L^T of the
// coarse operator on the GPU, then its inverse K^{-1} = L^{-T} L^{-1} by
// blocked forward / backward substitution on the identity.  The O(N^3)
// parts (trailing updates of the factorization, block updates of the
// substitutions) run on the FP64 matrix cores: v_mfma_f64_16x16x4f64.
//
// The matrix comes padded to Np = 32 * ceil(N / 32) with an identity tail,
// so every tile is a full 32 x 32 block.  Row-major storage, leading dimension Np.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "coarse.hpp"

namespace cd {

namespace {

constexpr int NB = 32;  // tile size

typedef double double4_t __attribute__((ext_vector_type(4)));

void check(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// Lane layout of v_mfma_f64_16x16x4f64 (D = A B + C, A 16x4, B 4x16):
// lane l holds A[l%16][l/16], B[l/16][l%16] and D[4q+l/16][l%16] in its q-th
// register, q = 0..3 (checked against a host product on gfx950).
__device__ inline double4_t mfma16(double a, double b, double4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---- factorization ----------------------------------------------------------
// Unblocked Cholesky of diagonal tile (k,k) in LDS; zeros above the diagonal.
__global__ __launch_bounds__(256) void k_potrf_tile(double* A, int ld, int k, int* notspd) {
    __shared__ double t[NB][NB + 1];
    const int tid = threadIdx.x;
    double* T = A + size_t(k) * NB * ld + size_t(k) * NB;
    for (int e = tid; e < NB * NB; e += 256) t[e / NB][e % NB] = T[size_t(e / NB) * ld + e % NB];
    __syncthreads();
    for (int j = 0; j < NB; ++j) {
        if (tid == 0) {
            const double d = t[j][j];
            if (!(d > 0.0)) notspd[0] = 1;
            t[j][j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        if (tid > j && tid < NB) t[tid][j] /= t[j][j];
        __syncthreads();
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e / NB, c = e % NB;
            if (c > j && r >= c) t[r][c] -= t[r][j] * t[c][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += 256) {
        const int r = e / NB, c = e % NB;
        T[size_t(r) * ld + c] = (c <= r) ? t[r][c] : 0.0;
    }
}

// Panel: tile (i,k) <- A_ik L_kk^{-T} for i = k+1+blockIdx.x; row r of the
// tile solves x L_kk^T = a by forward substitution.
__global__ __launch_bounds__(64) void k_trsm_panel(double* A, int ld, int k) {
    __shared__ double L[NB][NB + 1];
    const int i = k + 1 + blockIdx.x;
    const int tid = threadIdx.x;
    const double* Lk = A + size_t(k) * NB * ld + size_t(k) * NB;
    for (int e = tid; e < NB * NB; e += 64) L[e / NB][e % NB] = Lk[size_t(e / NB) * ld + e % NB];
    __syncthreads();
    if (tid >= NB) return;
    double* row = A + (size_t(i) * NB + tid) * ld + size_t(k) * NB;
    double x[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = row[j];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double s = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) s -= L[j][l] * x[l];
        x[j] = s / L[j][j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) row[j] = x[j];
}

// Trailing update A_ij -= L_ik L_jk^T for k < j <= i, on MFMA: each of the
// 4 waves owns one 16 x 16 quarter of the 32 x 32 tile.
__global__ __launch_bounds__(256) void k_syrk_tiles(double* A, int ld, int k, int nrem) {
    // lower-triangle tile index t -> (i, j) with 0 <= j <= i < nrem, offset k+1
    const int t = blockIdx.x;
    int ii = int((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
    while (ii * (ii + 1) / 2 > t) --ii;
    const int jj = t - ii * (ii + 1) / 2;
    const int i = k + 1 + ii, j = k + 1 + jj;
    const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
    const int si = wave / 2, sj = wave % 2;
    const double* Li = A + (size_t(i) * NB + si * 16) * ld + size_t(k) * NB;
    const double* Lj = A + (size_t(j) * NB + sj * 16) * ld + size_t(k) * NB;
    double* C = A + (size_t(i) * NB + si * 16) * ld + size_t(j) * NB + sj * 16;
    double4_t acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = C[size_t(4 * q + l / 16) * ld + l % 16];
#pragma unroll
    for (int kc = 0; kc < NB; kc += 4) {
        const double a = -Li[size_t(l % 16) * ld + kc + l / 16];
        const double b = Lj[size_t(l % 16) * ld + kc + l / 16];
        acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) C[size_t(4 * q + l / 16) * ld + l % 16] = acc[q];
}

// ---- inverse by substitution on B = I -----------------------------------------
// Block row k of B: B_k <- L_kk^{-1} B_k (lower, forward) or L_kk^{-T} B_k
// (upper, backward); one thread per column.
__global__ __launch_bounds__(256) void k_trsm_rows(const double* A, double* B, int ld, int k, int upper) {
    __shared__ double L[NB][NB + 1];
    const int tid = threadIdx.x;
    const double* Lk = A + size_t(k) * NB * ld + size_t(k) * NB;
    for (int e = tid; e < NB * NB; e += 256) L[e / NB][e % NB] = Lk[size_t(e / NB) * ld + e % NB];
    __syncthreads();
    const int col = blockIdx.x * 256 + tid;
    if (col >= ld) return;
    double* bc = B + size_t(k) * NB * ld + col;
    double x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) x[r] = bc[size_t(r) * ld];
    if (!upper) {
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            double s = x[r];
#pragma unroll
            for (int c = 0; c < r; ++c) s -= L[r][c] * x[c];
            x[r] = s / L[r][r];
        }
    } else {
#pragma unroll
        for (int r = NB - 1; r >= 0; --r) {
            double s = x[r];
#pragma unroll
            for (int c = r + 1; c < NB; ++c) s -= L[c][r] * x[c];
            x[r] = s / L[r][r];
        }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) bc[size_t(r) * ld] = x[r];
}

// B_i -= L_ik B_k (forward, i > k) or B_i -= L_ki^T B_k (backward, i < k),
// over column tiles; MFMA, 4 waves per 32 x 32 tile.
__global__ __launch_bounds__(256) void k_gemm_rows(const double* A, double* B, int ld, int k, int backward,
                                                   int ncoltiles) {
    const int ct = blockIdx.x % ncoltiles;
    const int rt = blockIdx.x / ncoltiles;
    const int i = backward ? rt : k + 1 + rt;
    const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
    const int si = wave / 2, sj = wave % 2;
    const double* Bk = B + size_t(k) * NB * ld + size_t(ct) * NB + sj * 16;
    double* C = B + (size_t(i) * NB + si * 16) * ld + size_t(ct) * NB + sj * 16;
    double4_t acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = C[size_t(4 * q + l / 16) * ld + l % 16];
#pragma unroll
    for (int kc = 0; kc < NB; kc += 4) {
        const int kk = kc + l / 16;
        double a;
        if (!backward) {
            a = -A[(size_t(i) * NB + si * 16 + l % 16) * ld + size_t(k) * NB + kk];  // L_ik[m][kk]
        } else {
            a = -A[(size_t(k) * NB + kk) * ld + size_t(i) * NB + si * 16 + l % 16];  // L_ki[kk][m]
        }
        const double b = Bk[size_t(kk) * ld + l % 16];
        acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) C[size_t(4 * q + l / 16) * ld + l % 16] = acc[q];
}

__global__ __launch_bounds__(256) void k_identity(double* B, int ld) {
    const size_t id = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (id >= size_t(ld) * ld) return;
    B[id] = (id / ld == id % ld) ? 1.0 : 0.0;
}

}  // namespace

int coarse_padded(int N) { return NB * ((N + NB - 1) / NB); }

void coarse_inverse(double* A, int N, double* Kinv, int* flag, hipStream_t s) {
    const int ld = coarse_padded(N);
    const int nblk = ld / NB;
    const size_t tot = size_t(ld) * ld;
    const dim3 gfill((tot + 255) / 256);
    for (int k = 0; k < nblk; ++k) {
        hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, s, A, ld, k, flag);
        const int nrem = nblk - 1 - k;
        if (nrem > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3(nrem), dim3(64), 0, s, A, ld, k);
            hipLaunchKernelGGL(k_syrk_tiles, dim3(nrem * (nrem + 1) / 2), dim3(256), 0, s, A, ld, k, nrem);
        }
        check("coarse cholesky");
    }
    hipLaunchKernelGGL(k_identity, gfill, dim3(256), 0, s, Kinv, ld);
    const int ncol = (ld + 255) / 256;
    for (int k = 0; k < nblk; ++k) {  // L Y = I
        hipLaunchKernelGGL(k_trsm_rows, dim3(ncol), dim3(256), 0, s, A, Kinv, ld, k, 0);
        if (k + 1 < nblk)
            hipLaunchKernelGGL(k_gemm_rows, dim3((nblk - 1 - k) * nblk), dim3(256), 0, s, A, Kinv, ld, k, 0, nblk);
        check("coarse forward");
    }
    for (int k = nblk - 1; k >= 0; --k) {  // L^T X = Y
        hipLaunchKernelGGL(k_trsm_rows, dim3(ncol), dim3(256), 0, s, A, Kinv, ld, k, 1);
        if (k > 0) hipLaunchKernelGGL(k_gemm_rows, dim3(k * nblk), dim3(256), 0, s, A, Kinv, ld, k, 1, nblk);
        check("coarse backward");
    }
}

}  // namespace cd
