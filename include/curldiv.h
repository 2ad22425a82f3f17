/*
 * curldiv.h - C ABI of the MI355X solver for the B-spline (isogeometric)
 * discretization of the parameter-dependent curl-div problem
 *
 *     alpha (curl u, curl v) + beta (div u, div v) = (f, v)
 *
 * on (0,1)^d, d = 2 or 3, homogeneous Dirichlet conditions, tensor-product
 * B-splines of degree p with maximal smoothness on n uniform intervals per
 * direction (Mazza, Manni, Ratnani, Serra-Capizzano, Speleers,
 * "Isogeometric analysis for 2D and 3D curl-div problems: spectral symbols
 * and fast iterative solvers", Sec. 1 (problem), Sec. 3.1 (spline space),
 * Sec. 4.1 / 4.2 (the 2x2 and 3x3 block system matrix A^{p,alpha,beta}_n)).
 *
 * The solver is the paper's multi-iterative method (Sec. 6.1) used as the
 * preconditioner of a conjugate-gradient iteration (Remark 6.1, "P_MIM" in
 * Sec. 6.2): a V-cycle with Kronecker-product grid transfers, a parallel
 * (Chebyshev-Jacobi) smoother in place of the sequential Gauss-Seidel
 * sweeps, p steps of GMRES preconditioned by the banded Toeplitz matrix
 * T = I_d (x) T_m(m_{p-1})^{(x) d} as finest-level post-smoother, and an
 * exact dense solve on the coarsest level; the outer iteration is flexible
 * CG.  Every step runs in HIP kernels on the GPU.
 *
 * Vector layout (Sec. 4.1): a vector of the system has d * prod_l m_l
 * entries, m_l = n_l + p - 2.  It is component-major; inside a component the
 * coefficient u_{i_1,...,i_d} (i_l = 2..n_l+p-1 in the paper's numbering) is
 * stored at offset ((i_1-2) m_2 + (i_2-2)) m_3 + (i_3-2) (3D) or
 * (i_1-2) m_2 + (i_2-2) (2D): i_1 slowest, i_d fastest.
 *
 * Memory: "dev" pointers are device (HBM) pointers owned by the caller; they
 * must stay valid until the call returns and the stream given at creation
 * has finished the work.  The library owns its handles and all workspace.
 * Functions return a status code (CD_OK = 0, CD_NOT_CONVERGED = 1, negative
 * codes for errors); cd_last_error() gives the message of the last error on
 * the calling thread.  A handle must not be used by two threads at once;
 * distinct handles are independent.
 */
#ifndef CURLDIV_H
#define CURLDIV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CD_OK 0
#define CD_NOT_CONVERGED 1   /* max_iter reached; x holds the last iterate   */
#define CD_EINVAL (-1)       /* invalid argument (see cd_last_error)          */
#define CD_ENOMEM (-2)       /* device allocation failed                      */
#define CD_EBREAKDOWN (-3)   /* Krylov breakdown: d^T A d <= 0 or non-finite  */
#define CD_EHIP (-4)         /* HIP runtime error                             */
#define CD_EAGAIN (-5)       /* server: request queued, not yet admitted      */
#define CD_ENOTFOUND (-6)    /* server: unknown ticket                        */

/* ---- problem and options ----------------------------------------------- */
/* The discrete problem of Sec. 4: dimension d, degree p >= 1, n[l] >= 1
 * intervals along axis l (n[2] ignored for d = 2; needs n[l]+p-2 >= 1), and
 * the weights alpha, beta > 0 of the curl and div terms (the matrix is SPD
 * only when both are positive, Corollaries 5.4 and 5.8). */
typedef struct {
    int dim;
    int degree;
    int n[3];
    double alpha;
    double beta;
} cd_problem;

#define CD_METHOD_PMIM 0   /* flexible CG preconditioned by one V-cycle (Sec. 6.2, P_MIM) */
#define CD_METHOD_PWL 1    /* flexible CG preconditioned by one V-cycle on the block-diagonal
                              part D (Sec. 6.1 eq. diag, P_WL in Sec. 6.2), with p steps of CG
                              preconditioned by T as finest post-smoother                     */
#define CD_METHOD_MIM 2    /* the V-cycle as a stand-alone iteration x += V(b - A x) (MIM)    */
#define CD_METHOD_CG 3     /* unpreconditioned CG (the CG columns of Tables 1-4)          */

#define CD_XFER_KNOT 0     /* knot-insertion prolongator, n -> n/2 (exact subspace embedding) */
#define CD_XFER_PAPER 1    /* (1/2)[1 2 1] stencil, m -> floor(m/2) (Sec. 6.1)                 */

#define CD_BOUNDS_LANCZOS 0 /* smoother bound: Lanczos on diag(A_l)^{-1} A_l (lanczos_steps steps), hi = 1.1 x
                              its largest Ritz value                                        */
#define CD_BOUNDS_SYMBOL 1  /* smoother bound from the spectral symbol (Sec. 5) of each level's Toeplitz part:
                              hi = bound_safety x the symbol's maximum of diag^{-1} A_l (levels with an
                              axis shorter than 2p+1 points fall back to Lanczos)               */

#define CD_APPLY3D_AUTO 0   /* 3D operator kernel variant chosen from the level's grid size      */
#define CD_APPLY3D_MARCH 1  /* blocks march over their x1 range one input plane at a time      */
#define CD_APPLY3D_SHORT 2  /* one output plane per block, its 2p+1 input planes side by side
                              (p <= 3; the marching kernel otherwise)                       */
#define CD_APPLY3D_GROUP 3  /* four thread groups per block take four input planes at a time  */

#define CD_FP64 0          /* every step in FP64                                              */
#define CD_MIXED_FP32 1    /* V-cycle (smoother, transfers, level operators, T-solves, GMRES
                              vectors) in FP32; outer residual, Krylov inner products and the
                              coarse solve in FP64                                             */

typedef struct {
    int method;           /* CD_METHOD_*                                     */
    int transfer;         /* CD_XFER_*                                       */
    int precision;        /* CD_FP64 or CD_MIXED_FP32                        */
    double rtol;          /* stop when ||r_k||_2 / ||r_0||_2 < rtol (Sec. 6.2) */
    int max_iter;
    int coarse_max_dofs;  /* coarsen while a level has more unknowns          */
    int cheb_degree;      /* Chebyshev smoother degree per application (>=1)  */
    double cheb_ratio;    /* smoothing interval [hi/ratio, hi]               */
    int lanczos_steps;    /* Lanczos steps for the smoother's eigenvalue bound (1..200) */
    int krylov_steps;     /* finest post-smoothing GMRES steps; < 0 means p  */
    int graphs;           /* 1: replay outer iterations from a captured HIP graph
                             (identical arithmetic); 0: launch every kernel eagerly */
    int cheb_degree_coarse; /* Chebyshev degree on levels >= 1; 0 means cheb_degree; < 0 (the
                             default) chooses from beta / alpha: 8 at 1e-2 and above, 16
                             from 1e-5 to 1e-2, 32 below (small beta leaves the smoother a
                             branch of the spectrum it damps slowly, and the cheap coarse
                             levels are where more steps pay; at large beta the outer
                             iteration count does not move and fewer steps are faster).
                             Measured, mixed precision, solve times with 8 / 16 / 32:
                             3D p=3 n=128 beta = 1e-6 379 iterations with 16, 238 with 32
                             (1.84 against 1.47 s); beta = 1e-4 51 / 32 iterations with
                             8 / 16 (210 / 150 ms); 2D p=3 n=256 beta = 1 2.4 / 3.0 ms,
                             3D p=2 n=64 beta = 1 and 1e-2 4.1 / 4.8 and 6.1 / 7.2 ms */
    int apply_x1_chunk;   /* 3D operator kernel: x1 planes each block covers (the launch
                             geometry only; results depend on it only through the rounding
                             of the per-block partial dot products and, in FP32, the last
                             bit of a Chebyshev update); 0 = chosen from the grid size.
                             Applies to the marching and grouped-march variants            */
    int eig_bounds;       /* CD_BOUNDS_LANCZOS (default) or CD_BOUNDS_SYMBOL                 */
    double bound_safety;  /* CD_BOUNDS_SYMBOL: hi = bound_safety x symbol maximum; 0 = 1.5
                             (the symbol describes the interior of the spectrum; the boundary
                             rows of diag^{-1} A put outliers up to 1.42x above it in 3D,
                             1.23x in 2D, on the operators measured)                        */
    int apply3d_kernel;   /* CD_APPLY3D_*: variant of the 3D operator kernel for y = A x, the
                             residual and the Chebyshev step (the kernels with fused dot
                             products always march); every variant sums each output entry's
                             terms in the same order, so A x does not depend on it.  A fixed
                             apply_x1_chunk implies CD_APPLY3D_MARCH under AUTO.  Default
                             AUTO.                                                          */
} cd_options;

/* Fill *opt with the defaults: P_MIM, knot insertion, FP64, rtol 1e-8,
 * max_iter 10000, coarse_max_dofs 2500, cheb_degree 48, cheb_ratio 1000,
 * lanczos_steps 20, krylov_steps = p, graphs 1, cheb_degree_coarse -1 (8, 16
 * or 32 from beta / alpha), apply_x1_chunk 0, eig_bounds Lanczos,
 * apply3d_kernel AUTO.  The
 * smoother settings were chosen by measured solve rate on 2D and 3D
 * problems; a wide interval needs the eigenvalue bound to cover the top of
 * the spectrum, which the Lanczos estimate times 1.1 does on every tested
 * operator.  Light smoothing (cheb_degree 3, cheb_ratio 30,
 * cheb_degree_coarse 0) is the classical setting. */
void cd_default_options(cd_options* opt);

/* Result of a solve.  kappa_estimate is the ratio of the extreme Ritz values
 * of the Lanczos matrix that the outer iteration's step lengths a_j and
 * direction coefficients b_j define (diagonal 1/a_j + b_j/a_{j-1},
 * off-diagonal sqrt(b_{j+1})/a_j): an estimate from below of the condition
 * number of the preconditioned operator B A (of A itself for CD_METHOD_CG),
 * exact in the limit for a linear SPD preconditioner; 0 when the solve ran no
 * iteration.  With x* the exact solution and r = b - A x, the forward error
 * obeys ||x - x*||_2 / ||x*||_2 <= kappa_2(A) ||r||_2 / ||b||_2, and in the
 * energy norm ||x - x*||_A / ||x*||_A <= sqrt(kappa(B A)) ||r||_B / ||b||_B
 * for an SPD B; kappa_estimate estimates kappa(B A) (kappa_2(A) for CG). */
typedef struct {
    int status;                 /* CD_OK, CD_NOT_CONVERGED or an error code  */
    int iterations;             /* outer iterations performed                 */
    double rel_residual;        /* recursive ||r_k|| / ||r_0|| at exit        */
    double true_rel_residual;   /* ||b - A x||_2 / ||b||_2 recomputed in FP64 */
    double kappa_estimate;      /* Lanczos estimate of the condition number (see above) */
} cd_result;

/* Number of unknowns of the system: d components (Sec. 4.1 for d = 2,
 * Sec. 4.2 for d = 3), each the tensor-product spline space with homogeneous
 * Dirichlet conditions of Sec. 3.1, n_l + p - 2 functions along axis l:
 * d * prod_l (n_l + p - 2).  0 for an invalid problem (no error code). */
size_t cd_num_dofs(const cd_problem* prob);

/* CD_OK if (prob, opt) is a valid combination, else CD_EINVAL. */
int cd_validate(const cd_problem* prob, const cd_options* opt);

/* The symbol-based smoother bound of `level` of the hierarchy (prob, opt)
 * would build, computed on the host without a device: the maximum over a
 * uniform grid of theta in [0, pi]^d (129 points per axis in 2D, 33 in 3D)
 * of the largest eigenvalue of Dh^{-1/2} F(theta) Dh^{-1/2}, F the d x d
 * symbol (Sec. 5: f^{p,alpha,beta} of Sec. 5.1 / 5.2, from the central rows
 * of the level's 1D matrices) and Dh its constant diagonal.  *lam = 0 when an
 * axis of the level has fewer than 2p+1 points.  CD_EINVAL for an invalid
 * problem or a level the hierarchy does not have (the coarsest level has no
 * smoother). */
int cd_symbol_bound(const cd_problem* prob, const cd_options* opt, int level, double* lam);

/* Device bytes a solver for (prob, opt) needs at its peak (hierarchy,
 * coarse inverse, workspace, and the set-up's temporary factor and Lanczos
 * vectors); the server's unit of admission. */
size_t cd_footprint_bytes(const cd_problem* prob, const cd_options* opt);

/* ---- solver handle ----------------------------------------------------- */
typedef struct cd_solver cd_solver;

/* Set up the hierarchy on the host in FP64 (1D matrices M, A, S of
 * Sec. 3.2 by Gauss quadrature, the prolongators of Sec. 6.1, Galerkin coarse
 * 1D matrices, banded LDL^T of T_m(m_{p-1}) of Sec. 6.1) and on the device
 * (dense coarse matrix, its Cholesky factor and inverse, eigenvalue bounds of
 * the smoother).  *out receives the handle (owned by the caller, released by
 * cd_solver_destroy); on error *out is NULL and the code is CD_EINVAL (an
 * invalid problem or option, see cd_validate), CD_ENOMEM (device memory) or
 * CD_EHIP (another HIP error).  `stream` is a hipStream_t;
 * all later work of the handle is queued on it.  With NULL the handle
 * creates its own non-blocking stream and orders it after the null stream at
 * every entry point (outer iterations are replayed from HIP graphs, which
 * cannot be captured on the null stream). */
int cd_solver_create(const cd_problem* prob, const cd_options* opt, void* stream, cd_solver** out);
void cd_solver_destroy(cd_solver* s);

/* Solve A x = b (Sec. 6, the linear system of the problem) from x_0 = 0.
 * b_dev, x_dev: device arrays of cd_num_dofs() doubles.  Blocks until done. */
int cd_solve(cd_solver* s, const double* b_dev, double* x_dev, cd_result* out);

/* Device bytes the handle holds (its allocations after setup; the setup's
 * temporary workspace is released before cd_solver_create returns).  The
 * server admits by cd_footprint_bytes, which is at least this. */
size_t cd_solver_device_bytes(const cd_solver* s);

/* ---- hooks for parity tests and measurement ----------------------------- */
int cd_num_levels(const cd_solver* s);
/* m_l per axis of a level (3 ints; m[2] = 1 in 2D) and its unknown count. */
int cd_level_shape(const cd_solver* s, int level, int* m3, size_t* ndofs);
/* Host copy of a 1D setup matrix of `level` along `axis` as a dense
 * row-major m x m array: which = 'M', 'A', 'S' (Sec. 3.2 matrices or their
 * Galerkin coarse versions), 'T' (T_m(m_{p-1}), level 0 only) or 'P' (the
 * prolongator from level+1 to level, m_level x m_{level+1}). */
int cd_get_matrix(const cd_solver* s, int level, int axis, char which, double* host_out);
/* The smoother's eigenvalue estimate of `level`: the largest Ritz value of
 * lanczos_steps Lanczos steps on diag(A_l)^{-1} A_l, or with CD_BOUNDS_SYMBOL
 * the symbol maximum of cd_symbol_bound where the level has one. */
int cd_get_lambda(const cd_solver* s, int level, double* lam);

/* Launches of one outer iteration (a measurement hook): the kernel nodes
 * (*kernels) and all nodes (*nodes, kernels plus copies) of the HIP graph the
 * handle captured to replay outer iterations k >= 1; both 0 before a solve
 * has reached its second iteration or with graphs = 0.  Either pointer may be
 * NULL. */
int cd_graph_launches(const cd_solver* s, size_t* kernels, size_t* nodes);

/* The smoother of `level` (a level above the coarsest): Chebyshev degree and
 * interval [lo, hi] on diag(A_l)^{-1} A_l, as the handle resolved them from
 * its options and the eigenvalue bound.  Any output pointer may be NULL. */
int cd_get_smoother(const cd_solver* s, int level, int* degree, double* lo, double* hi);

/* y = A_level x in FP64.  Level 0 is the system matrix of Sec. 4.1 (2D) /
 * Sec. 4.2 (3D), the block matrix of Kronecker products of the 1D matrices
 * (for CD_METHOD_PWL the V-cycle's operator, the block-diagonal part D of
 * Sec. 6.1 eq. diag, on every level; the outer iteration of that method
 * still multiplies by the full matrix); level l > 0 is the Galerkin operator
 * P^T A_{l-1} P of the same form.  x_dev, y_dev: device arrays of the level's
 * unknown count (cd_level_shape), component-major, each component row-major
 * with the last axis fastest; they must not overlap.  CD_EINVAL for a level
 * out of range.  Ordered on the handle's stream; blocks until done. */
int cd_apply(cd_solver* s, int level, const double* x_dev, double* y_dev);
/* y = A_level x in FP32 with FP32 coefficients. */
int cd_apply_f32(cd_solver* s, int level, const float* x_dev, float* y_dev);
/* One smoother application (cheb_degree Chebyshev steps) on level `level`
 * for A_l x = b starting from x_in; writes x_out (FP64). */
int cd_smooth(cd_solver* s, int level, const double* b_dev, const double* x_in_dev, double* x_out_dev);
/* r_c = P^T r (level -> level+1) and x += P e (level+1 -> level), FP64
 * (Sec. 6.1: the block prolongator I_d (x) P (x) ... (x) P, P the
 * knot-insertion or the (1/2)[1 2 1] prolongator of the handle). */
int cd_restrict(cd_solver* s, int level, const double* r_fine_dev, double* r_coarse_dev);
int cd_prolong_add(cd_solver* s, int level, const double* e_coarse_dev, double* x_fine_dev);
/* z = T^{-1} v on the finest level (Sec. 6.1, the preconditioner of the
 * Krylov post-smoother), FP64. */
int cd_tsolve(cd_solver* s, const double* v_dev, double* z_dev);
/* The same steps in FP32 with FP32 coefficients (the kernels the mixed
 * precision V-cycle runs): smoother, transfers and T-solve on FP32 device
 * vectors.  On an FP64 handle the first call allocates an FP32 workspace. */
int cd_smooth_f32(cd_solver* s, int level, const float* b_dev, const float* x_in_dev, float* x_out_dev);
int cd_restrict_f32(cd_solver* s, int level, const float* r_fine_dev, float* r_coarse_dev);
int cd_prolong_add_f32(cd_solver* s, int level, const float* e_coarse_dev, float* x_fine_dev);
int cd_tsolve_f32(cd_solver* s, const float* v_dev, float* z_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * z = T^{-1} v as cd_tsolve, with the same kernels and bitwise the same
 * result, but its intermediate vectors live in a static device workspace of
 * the library instead of the handle's buffers, and the call allocates
 * nothing.  The workspace holds two vectors of 2^20 doubles (16 MiB per GPU,
 * kept until the process ends), so the handle's problem must have at most
 * 1,048,576 unknowns; larger problems return CD_EINVAL.  v_dev may equal
 * z_dev.  Every call on one GPU shares that GPU's workspace: calls that
 * overlap in time on one GPU (from two threads, or on two handles whose
 * streams run concurrently) race and give undefined results.  The current
 * device must be the handle's device.  Blocks until done. */
int cd_tsolve_noalloc(cd_solver* s, const double* v_dev, double* z_dev);
/* The numerical examples of Sec. 6.2 (manufactured solutions):
 * u = (sin(2 pi g), cos(2 pi g) - 1) in 2D and (sin(2 pi g), cos(2 pi g) - 1,
 * u_1 + u_2) in 3D, g = prod_i x_i (1 - x_i).  cd_load_vector writes the
 * Galerkin load vector of f = L_{alpha,beta} u for the handle's problem,
 * alpha (curl u, curl psi_i) + beta (div u, div psi_i) (the fields vanish on
 * the boundary), into b_dev (cd_num_dofs doubles, the layout of the system);
 * cd_l2_error writes ||u - u_h||_{L2((0,1)^d)} for the discrete field u_h
 * with coefficients x_dev.  Both use (p+3)-point Gauss-Legendre quadrature
 * per element and direction, run on the GPU in FP64 and allocate their
 * workspace for the call (3D load vector: about 7 Q^2 m + 6 Q m^2 doubles,
 * Q = n (p+3), m = n + p - 2). */
int cd_load_vector(cd_solver* s, double* b_dev);
int cd_l2_error(cd_solver* s, const double* x_dev, double* err);
/* z = A_L^{-1} r on the coarsest level, FP64. */
int cd_coarse_solve(cd_solver* s, const double* r_dev, double* z_dev);
/* z = one application of the preconditioner to r: one V-cycle of the
 * multi-iterative method of Sec. 6.1 (Chebyshev pre- and post-smoothing on
 * every level, the Krylov post-smoother with the T preconditioner on the
 * finest level, the exact coarse solve), in the handle's precision, from a
 * zero start.  r_dev, z_dev: device arrays of cd_num_dofs doubles; they may
 * not overlap.  Blocks until done. */
int cd_precondition(cd_solver* s, const double* r_dev, double* z_dev);

/* ---- live kernel timing ------------------------------------------------- */
/* When enabled, the operator-apply kernels and the T-solve line kernels of
 * the handle time themselves: each launch writes the wall-clock time of its
 * earliest block start and latest block end (after its stores) into a
 * device slot; slots are cleared before and copied to pinned host memory
 * after each timed outer iteration (inside the replayed HIP graph as well),
 * and folded into per-(kernel, level, precision) totals at the next
 * synchronisation point.  Hooks (cd_apply, cd_tsolve, cd_precondition, ...)
 * are always timed; during cd_solve every `on`-th outer iteration is (on = 1:
 * all of them).  `bytes` accumulates the algorithmic traffic of those
 * launches: the vectors each launch must read and write once (2 N s for
 * y = A x, 3 N s for the residual, 4 N s for a Chebyshev step (3 N s on its
 * first step), (2 + k) N s
 * for y = A x fused with k Krylov-basis dot products, 2 N s per T-solve axis
 * pass; s = 8 or 4 bytes). */
typedef struct {
    long long launches;
    double total_ms;
    double bytes;
} cd_kernel_stats;
/* Enable (on > 0, the sampling period of outer iterations) or disable
 * (on <= 0) timing; enabling resets the totals. */
int cd_profile_enable(cd_solver* s, int on);
/* Totals of level `level` applies in FP64 (fp32 = 0) or FP32 (fp32 = 1). */
int cd_profile_read(const cd_solver* s, int level, int fp32, cd_kernel_stats* out);
/* Totals of the Chebyshev-step applies of level `level` alone (a subset of
 * what cd_profile_read counts): each reads x_k, b and (after the first step)
 * x_{k-1} and writes x_{k+1}, so its bytes are 4 N s (3 N s on a first
 * step). */
int cd_profile_read_smoother(const cd_solver* s, int level, int fp32, cd_kernel_stats* out);
/* Totals of the finest-level T-solve axis passes (Sec. 6.1 preconditioner
 * T of the Krylov post-smoother), one launch per axis pass. */
int cd_profile_read_tsolve(const cd_solver* s, int fp32, cd_kernel_stats* out);

/* ---- serving: continuous batching of independent solves ----------------- */
/* A server keeps a FIFO of submitted solves and a set of active ones.  Each
 * cd_server_step() admits queued requests while the sum of their footprints
 * (cd_footprint_bytes) stays within the HBM budget and fewer than max_active
 * are in flight, handing their set-up (cd_solver_create and the first
 * residual) to a worker thread of the server, and advances every active
 * solve whose last outer iteration has finished: stopping test, then the
 * next iteration is enqueued or the solve retires.  Each solve runs on its
 * own stream, so the kernels of different solves overlap on the device and
 * a short solve never waits for a long one.  The call returns as soon as
 * something progressed (or after about a millisecond without progress).
 * A request's arithmetic never depends on the others: its result is
 * bitwise the same alone or in a mix.  A request whose set-up runs out of
 * device memory while other solves hold it goes back to the head of the
 * queue.  Callers keep b_dev and x_dev valid until the request's completion
 * has been polled. */
typedef struct cd_server cd_server;
typedef struct {
    size_t hbm_budget_bytes;  /* admission budget; 0 = 80% of the free HBM at creation */
    int max_active;           /* solves in flight at once; 0 = 64 */
    int num_streams;          /* 0 (default): one stream per active solve; k in 1..64: a pool
                                 of k streams shared round robin (solves on one stream
                                 run one after the other) */
} cd_server_options;
typedef struct {
    uint64_t ticket;
    cd_result result;
    double t_submit, t_admit, t_done;  /* seconds since server creation (host monotonic clock) */
    size_t footprint_bytes;            /* device bytes the solve held */
} cd_completion;
void cd_server_default_options(cd_server_options* opt);
int cd_server_create(const cd_server_options* opt, cd_server** out);
/* Queue a solve of A x = b; CD_EINVAL for an invalid problem, CD_ENOMEM if
 * its footprint exceeds the whole budget.  *ticket identifies it. */
int cd_server_submit(cd_server* srv, const cd_problem* prob, const cd_options* opt, const double* b_dev,
                     double* x_dev, uint64_t* ticket);
/* One scheduling pass (see above); *n_active counts solves in set-up or
 * iterating, *n_queued those not admitted yet. */
int cd_server_step(cd_server* srv, int* n_active, int* n_queued);
/* Move up to `max` finished solves into out[]; *n_out = how many. */
int cd_server_poll(cd_server* srv, cd_completion* out, int max, int* n_out);
void cd_server_destroy(cd_server* srv);

const char* cd_status_string(int status);
const char* cd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CURLDIV_H */
