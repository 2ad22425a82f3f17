// Device data structures and launch wrappers of the curl-div kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace cd {

// Operator of one level: 1D banded matrices per axis, stored k-major on the
// device: for axis a and matrix w (0 = M, 1 = A, 2 = S) the entry (i, i+k-hb)
// is at band[a][w][k * m[a] + i]; columns outside [0, m) hold zeros.
template <typename T>
struct OpDev {
    const T* band[3][3];
    // axis-0 columns, row-window form: col0[w][j * (2hb+1) + k] = X(j - hb + k, j)
    // (zero outside the matrix), so one plane's coefficients are contiguous
    const T* col0[3];
    // axis-0 table of the 3D kernel, one row of 3(2hb+1)+2 entries per plane j
    // in [-hb, m[0]+hb): X(j-hb+k, j) for X = M, A, S and k < 2hb+1, then
    // M(j-hb, j-hb) and S(j-hb, j-hb); zero where an index leaves [0, m[0])
    const T* c1p;
    // the same entries by output plane, one row of 3(2hb+1)+2 per plane i in
    // [0, m[0]): X(i, i-hb+g) for X = M, A, S and g < 2hb+1, then M(i, i) and
    // S(i, i) (the variants of the 3D kernel that sum one output plane at a time)
    const T* c1r;
    int m[3];   // unknowns per axis (m[2] = 1 in 2D)
    int hb;     // half bandwidth (= p on every level)
    int x1chunk;  // 3D kernel: x1 planes per block (0: chosen from the grid size)
    int variant;  // 3D kernel: CD_APPLY3D_* (0: chosen from the grid size)
    int blockdiag;  // 1: the block-diagonal part D of the operator (off-diagonal blocks dropped)
    int dim;
    T alpha, beta;
};

// Prolongator tables of one axis (see setup.hpp, Prolong), device copies.
template <typename T>
struct XferAxisDev {
    const int* c0;
    const T* v;
    const int* r0;
    const T* vt;
    int mf, mc, w, wr;
};

template <typename T>
struct XferDev {
    XferAxisDev<T> ax[3];  // axis 2 of a 2D problem is the identity on 1 point
    int dim;
};

// Banded LDL^T factor of T_m(m_{p-1}) for one axis.
template <typename T>
struct TFacDev {
    const T* l;     // l[i*bw + k-1] = L(i, i-k)
    const T* dinv;  // 1 / D(i)
    int m, bw;
    int warm;       // rows a chunk's recurrence starts early (see recurrence_warmup)
};

enum ApplyMode : int {
    kApplyY = 0,     // y = A x
    kApplyRes = 1,   // y = b - A x
    kApplyCheb = 2,  // xout = x + c1 (x - xprev) + c2 D^{-1}(b - A x), xprev passed as u (nullptr:
                     // zero); xout may alias xprev (each entry is read before it is written)
    kApplyYDot = 3,  // y = A x; part[block] = sum x.y (FP64)
    kApplyResDot = 4,  // y = b - A x; part[block] = sum y.y (FP64)
    kApplyYMulti = 5,  // y = A x; part[i*nblocks + block] = sum V_i.y, i < nv, V_i = b + i*n, and
                       // part[nv*nblocks + block] = sum y.y (FP64)
};

constexpr int kMaxBasis = 8;  // most Krylov vectors of the GMRES post-smoother

// Partial-sum count used by every reduction of a vector of length n.
int reduce_blocks(size_t n);
// Number of blocks of the apply kernel: partial sums per dot in the dot modes.
template <typename T>
int apply_blocks(const OpDev<T>& op);

// Kernel-side timing: a slot of kStampWords words per timed launch (see
// stamp_begin / stamp_end in kernels.hip).
constexpr int kStampEnds = 2048;
constexpr int kStampWords = 1 + kStampEnds;
// stamp: nullptr, or the timing slot of this launch.
template <typename T>
void launch_apply(const OpDev<T>& op, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2,
                  double* part, hipStream_t s, int nv = 0, unsigned long long* stamp = nullptr);
// pairs[2 i], pairs[2 i + 1] = start and end of slots i in [slot0, slot0 +
// nslots); clears those slots for reuse.
void launch_stamp_reduce(unsigned long long* st, int slot0, int nslots, unsigned long long* pairs, hipStream_t s);

// First Chebyshev step from zero on a level: x = inv_theta D^{-1} b.
template <typename T>
struct ChebFirst {
    OpDev<T> op;
    T inv_theta;
    T* x;
};

// rc = P^T rf; with cf also the first Chebyshev step of the coarse level on rc.
template <typename T>
void launch_restrict(const XferDev<T>& X, int ncomp, const T* rf, T* rc, hipStream_t s,
                     const ChebFirst<T>* cf = nullptr);
template <typename T>
void launch_prolong_add(const XferDev<T>& X, int ncomp, const T* ec, T* xf, hipStream_t s);

// z = T^{-1} v, T = I_d (x) T_1 (x) ... (x) T_d; v, tmp, z distinct, tmp: n
// scratch.  stamps: nullptr or dim consecutive timing slots, one per axis pass.
template <typename T>
void launch_tsolve(int dim, const int* m, const TFacDev<T>* fac, const T* v, T* tmp, T* z, hipStream_t s,
                   unsigned long long* stamps = nullptr);

// ---- vector kernels ---------------------------------------------------------
template <typename TA, typename TB>
void launch_dot_partial(const TA* a, const TB* b, size_t n, double* part, hipStream_t s);
// out[0] = sum of part[0..np)
void launch_finalize(const double* part, int np, double* out, hipStream_t s);
template <typename TO, typename TI>
void launch_cast(const TI* x, TO* y, size_t n, hipStream_t s);
// y = x converted, then the first Chebyshev step on y (cf.op is y's level)
template <typename TO, typename TI>
void launch_cast_cheb(const TI* x, TO* y, size_t n, const ChebFirst<TO>& cf, hipStream_t s);
// y = x converted; part[block] = partial sums of y . q, reduce_blocks(n) of them
template <typename TO, typename TI>
void launch_cast_dot(const TI* x, TO* y, size_t n, const double* q, double* part, hipStream_t s);
template <typename T>
void launch_fill(T* x, T v, size_t n, hipStream_t s);
template <typename T>
void launch_copy(const T* x, T* y, size_t n, hipStream_t s);
// y = a x + b y with host scalars
template <typename T>
void launch_axpby(T a, const T* x, T b, T* y, size_t n, hipStream_t s);
// y = x * (1/sqrt(sum part)) (zero if the sum is zero); FP64 partials
template <typename T>
void launch_normalize(const double* part, int np, const T* x, T* y, size_t n, hipStream_t s);
// Diagonal of a level operator: y = x / D (inv = true) or y = x * D.
template <typename T>
void launch_diag_scale(const OpDev<T>& op, bool inv, const T* x, T* y, hipStream_t s);
// part[block] = sum D x^2 (FP64)
template <typename T>
void launch_diag_dot(const OpDev<T>& op, const T* x, double* part, hipStream_t s);
// out (ld x ld, row-major) = the level operator as a dense matrix in its
// leading block, identity in the tail; ld >= the operator's order
void launch_dense_operator(const OpDev<double>& op, double* out, int ld, hipStream_t s);
// Lanczos step on D^{-1} A (D inner product): w = D^{-1} w - alpha q - beta qp,
// beta = sqrt(beta2), or 0 when beta2 <= (1e-10 alpha_prev)^2 (breakdown);
// scalars read from device memory
void launch_lanczos_step(const OpDev<double>& op, const double* alpha, const double* alpha_prev, const double* beta2,
                         const double* q, const double* qp, double* w, hipStream_t s);
// q = w / sqrt(beta2), or q = r (restart) when beta2 <= (1e-10 alpha)^2
void launch_lanczos_next(const double* alpha, const double* beta2, const double* w, const double* r, double* q,
                         size_t n, hipStream_t s);
// First Chebyshev step from x = 0: u = D^{-1} b / theta; x = u
template <typename T>
void launch_cheb_first(const OpDev<T>& op, const T* b, T* x, T inv_theta, hipStream_t s);

// ---- coarse level -------------------------------------------------------------
// z = Kinv r, Kinv N x N inside an ld x ld row-major array
template <typename T>
void launch_coarse_gemv(const double* Kinv, int N, int ld, const T* r, T* z, hipStream_t s);

// ---- flexible CG: the outer iteration (FP64) and the PCG post-smoother of the
// block-diagonal cycle (vectors T, inner products FP64) -----------------------
// d = z - (sum pzq / *dq_prev) d   (first = true: d = z); pdr[block] = d.r
// (*beta_out = the coefficient b of d = z - b d_prev, 0 on the first step)
template <typename T>
void launch_fcg_direction(bool first, const T* z, const double* pzq, int npzq, const double* dq_prev,
                          T* d, const T* r, double* pdr, double* beta_out, size_t n, hipStream_t s);
// a = sum pdr / sum pdq; x += a d; r -= a q; prr[block] = r.r; *dq_out = sum pdq; *a_out = a
template <typename T>
void launch_fcg_update(const double* pdr, int npdr, const double* pdq, int npdq, double* dq_out,
                       T* x, T* r, const T* d, const T* q, double* prr, double* a_out,
                       size_t n, hipStream_t s);

// ---- GMRES helpers (vectors of type T, scalars FP64) ----------------------------
// Classical Gram-Schmidt step with the Pythagorean norm: h_i = sum of the
// nbp partials pdot[i*nbp ..] (V_i . w, i < k), ww = those of pdot[k*nbp ..]
// (w . w); block 0 stores Hcol[0..k) = h and Hcol[k] = sqrt(ww - |h|^2);
// unless v == nullptr, v = (w - sum_i h_i V_i) / Hcol[k] (zero if that is 0).
template <typename T>
void launch_gs_normscale(const double* pdot, int k, int nbp, double* Hcol, const T* V, const T* w, T* v, size_t n,
                         hipStream_t s);
// ss = sum of the np partials; *out = square ? ss : sqrt(ss) (block 0);
// v = w / sqrt(ss) (zero if ss == 0) unless v == nullptr.
template <typename T>
void launch_normscale(const double* pnorm, int np, double* out, bool square, const T* w, T* v, size_t n,
                      hipStream_t s);
// x += sum_j y_j Z_j with y = argmin || sqrt(*beta0sq) e1 - H y || for the
// (k+1) x k Hessenberg H (column-major, leading dimension ld), solved by
// Givens rotations in every block.
template <typename T>
void launch_lsq_combine_add(const double* H, int ld, int k, const double* beta0sq, const T* Z, T* x, size_t n,
                            hipStream_t s);

}  // namespace cd
