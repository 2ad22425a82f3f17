// Coarsest-level dense FP64 Cholesky and inverse on the GPU (MFMA).
#pragma once

#include <hip/hip_runtime.h>

namespace cd {

// Padded order Np (multiple of 32) used for the coarse matrices.
int coarse_padded(int N);

// A: Np x Np row-major (device), holds the SPD matrix K in its leading
// N x N block and the identity in the tail on entry, and the Cholesky factor
// L (lower, zeros above) on exit.  Kinv: Np x Np (device), receives K^{-1}
// in its leading N x N block (identity tail).  flag: device int set to 1 if
// a non-positive pivot appeared (must be 0 on entry).  Asynchronous on
// stream s.
void coarse_inverse(double* A, int N, double* Kinv, int* flag, hipStream_t s);

}  // namespace cd
