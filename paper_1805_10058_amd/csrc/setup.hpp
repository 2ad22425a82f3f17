// Host-side FP64 setup of the curl-div solver: 1D B-spline matrices, grid
// transfers, Galerkin coarse matrices, the Toeplitz preconditioner factor and
// the dense coarse-level matrix.  Everything here is O(m p^2) per axis except
// the dense coarse matrix, whose size is bounded by coarse_max_dofs.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

namespace cd {

// Square banded matrix, row-major band storage: a[i*(2*hb+1) + k] holds
// entry (i, i+k-hb); entries whose column falls outside [0, m) are zero.
struct Band {
    int m = 0;
    int hb = 0;
    std::vector<double> a;
    Band() = default;
    Band(int m_, int hb_) : m(m_), hb(hb_), a(size_t(m_) * (2 * hb_ + 1), 0.0) {}
    double get(int i, int j) const {
        int k = j - i + hb;
        return (k < 0 || k > 2 * hb || j < 0 || j >= m) ? 0.0 : a[size_t(i) * (2 * hb + 1) + k];
    }
    void set(int i, int j, double v) { a[size_t(i) * (2 * hb + 1) + (j - i + hb)] = v; }
    Band widened(int hb_new) const;  // same matrix stored with a larger half-bandwidth
};

// Sparse 1D prolongator P (mf x mc): row i has entries in columns
// [c0[i], c0[i]+w); the transpose Pt (mc x mf) row j has entries in fine
// rows [r0[j], r0[j]+wr).
struct Prolong {
    int mf = 0, mc = 0, w = 0, wr = 0;
    std::vector<int> c0, r0;
    std::vector<double> v, vt;  // v[i*w + k] = P(i, c0[i]+k); vt[j*wr + k] = P(r0[j]+k, j)
    double get(int i, int j) const;
};

// Knot sequence of Sec. 3.1 (p+1 zeros, i/n, p+1 ones).
std::vector<double> knots(int n, int p);
// Values and first derivatives of the p+1 B-splines that are nonzero at x,
// returned with the index of the first one (zero-based).  Cox-de Boor.
int bspline_local(const std::vector<double>& xi, int p, double x, double* val, double* der);
// Cardinal B-spline phi_p(t) (Sec. 3.1 recursion).
double cardinal(int p, double t);

// 1D mass, advection and stiffness matrices of the Dirichlet B-splines
// N_2..N_{n+p-1} (Sec. 3.2), (p+1)-point Gauss-Legendre per element.
void assemble_1d(int n, int p, Band& M, Band& A, Band& S);

// Knot-insertion prolongator n -> n/2 restricted to the Dirichlet space.
Prolong knot_insertion(int nf, int p);
// The (1/2)[1 2 1] prolongator of Sec. 6.1 with m_c = floor(m_f/2).
Prolong paper_prolong(int mf);
// The identity on m points (an axis that a level does not coarsen).
Prolong identity_prolong(int m);
// Galerkin product P^T X P.
Band galerkin(const Band& X, const Prolong& P);

// Largest eigenvalue of the symbol of diag(K)^{-1} K for a level operator K
// built from per-axis 1D matrices M[l], A[l], S[l] (l < d) with the block
// structure of Sec. 4 (diagonal blocks beta S x M x .. + alpha sum of the
// other S terms; off-diagonal blocks offw times A on the two axes of the pair
// and M elsewhere): the Toeplitz part of each 1D matrix is read off its
// central row, the d x d symbol F(theta) of Sec. 5 is formed from the 1D
// symbols, scaled by its constant diagonal Dh, and the largest eigenvalue of
// Dh^{-1/2} F Dh^{-1/2} is maximised over theta in {pi k / (s - 1)}^d,
// k = 0..s-1, s = samples.  Returns 0 when an axis has fewer than 2 hb + 1
// points (no interior row).
double symbol_lambda_max(int d, const Band* M, const Band* A, const Band* S, double alpha, double beta,
                         double offw, int samples);

// Quadrature tables of one axis: q-point Gauss-Legendre on each of the n
// elements (Q = n q points in element order), and at every point the values
// and first derivatives of the p+1 B-splines nonzero there; f0[a] is the
// Dirichlet index (full index - 1, so -1 for the dropped first function) of
// the first of them.
struct QuadAxis {
    int n = 0, p = 0, q = 0, m = 0, Q = 0;
    std::vector<double> x, w, val, der;  // val[a*(p+1) + k], der[a*(p+1) + k]
    std::vector<int> f0;
};
QuadAxis quad_axis(int n, int p, int q);

// Banded LDL^T of T_m(m_{p-1}) (Sec. 6.1): L unit lower with half-bandwidth
// p-1 stored as l[i*(p-1) + (k-1)] = L(i, i-k), and dinv[i] = 1/D(i).
struct TFactor {
    int m = 0, bw = 0;  // bw = p-1
    std::vector<double> l, dinv;
    Band T;  // the matrix itself (for export)
};
TFactor toeplitz_factor(int m, int p);
// Number of steps after which the homogeneous part of the factor's line
// recurrence (forward L y = v, or backward L^T z = w) has decayed below
// `tol` relative to its start, measured on the interior coefficients; m if
// it does not within m steps.  A line solve that starts this many rows
// early from a zero state agrees with the exact solve to `tol`.
int recurrence_warmup(const TFactor& F, double tol);

}  // namespace cd
