// Coarsest-level dense FP64 Cholesky and inverse on the GPU (MFMA).
#pragma once

#include <hip/hip_runtime.h>

namespace cd {

// Padded order Np (multiple of 32) used for the coarse matrices.
int coarse_padded(int N);

// K: N x N row-major SPD matrix (device).  A: Np x Np workspace (device),
// receives the Cholesky factor L (lower, zeros above).  Kinv: Np x Np
// (device), receives K^{-1} in its leading N x N block (identity tail).
// flag: device int set to 1 if a non-positive pivot appeared (must be 0 on
// entry).  Asynchronous on stream s.
void coarse_inverse(const double* K, int N, double* A, double* Kinv, int* flag, hipStream_t s);

}  // namespace cd
