// Solver orchestration and the C ABI (include/curldiv.h).
//
// One handle = one problem: an FP64 host setup, device copies of the 1D
// operators of every level (FP64 and FP32), transfer tables, the banded
// factor of T, the inverse of the coarsest operator, and the device
// workspace of the V-cycle and of the outer flexible CG.  All device work
// is queued on the handle's stream; the only host synchronisation in a solve
// is one 16-byte read per outer iteration (the residual norm and the
// curvature d^T A d, for the stopping test and breakdown detection).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <cstring>
#include <condition_variable>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/curldiv.h"
#include "coarse.hpp"
#include "kernels.hpp"
#include "loadvec.hpp"
#include "setup.hpp"

// Static device workspace of cd_tsolve_noalloc, the entry point for callers
// that cannot allocate device memory: two vectors of kNoAllocMaxDofs doubles
// (16 MiB), one copy per GPU for the life of the process.  Host code must use
// the address hipGetSymbolAddress returns for the current device (taken once
// per device, see noalloc_workspace), never the symbol itself.
constexpr size_t kNoAllocMaxDofs = size_t(1) << 20;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxDofs];

namespace {

thread_local std::string g_last_error;

struct CdError : std::runtime_error {
    int code;
    CdError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the caller's next HIP call
        if (e == hipErrorOutOfMemory) throw CdError(CD_ENOMEM, std::string(what) + ": out of device memory");
        throw CdError(CD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current; later calls reuse the stored address.
double* noalloc_workspace() {
    static std::mutex mu;
    static std::map<int, double*> addr;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) throw CdError(CD_EHIP, "hipGetSymbolAddress(scratch) returned null");
    addr[dev] = static_cast<double*>(ptr);
    return static_cast<double*>(ptr);
}

// Owning list of device allocations.
struct DevArena {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    template <typename T>
    T* alloc(size_t n) {
        void* p = nullptr;
        const size_t nb = std::max<size_t>(n, 1) * sizeof(T);
        hip_check(hipMalloc(&p, nb), "hipMalloc");
        ptrs.push_back(p);
        bytes += nb;
        return static_cast<T*>(p);
    }
    template <typename T>
    T* upload(const std::vector<T>& h, hipStream_t s) {
        T* d = alloc<T>(h.size());
        if (!h.empty()) hip_check(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
        return d;
    }
    ~DevArena() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

template <typename T>
std::vector<T> convert(const std::vector<double>& v) {
    return std::vector<T>(v.begin(), v.end());
}

// k-major band layout of the device: entry (i, i+k-hb) at k*m + i
std::vector<double> kmajor(const cd::Band& B) {
    const int w = 2 * B.hb + 1;
    std::vector<double> out(size_t(w) * B.m);
    for (int i = 0; i < B.m; ++i)
        for (int k = 0; k < w; ++k) out[size_t(k) * B.m + i] = B.a[size_t(i) * w + k];
    return out;
}

struct LevelHost {
    int n = 0;       // intervals per axis (knot insertion); 0 for the paper transfer below level 0
    int m[3] = {1, 1, 1};
    size_t N = 0;    // unknowns
    cd::Band M[3], A[3], S[3];
    cd::Prolong P[3];  // prolongator from the next level (valid if not coarsest)
    double lam = 0, lo = 0, hi = 0;
};

template <typename T>
struct LevelDev {
    cd::OpDev<T> op{};
    cd::XferDev<T> xf{};  // from level+1 to this level
};

// Workspace of a V-cycle in precision T.
template <typename T>
struct VWork {
    struct L {
        T* b = nullptr;
        T* xa = nullptr;
        T* xb = nullptr;
        T* r = nullptr;
        T* xcur = nullptr;
    };
    std::vector<L> lv;
    T* V = nullptr;  // finest GMRES basis, (s+1) x N
    T* Z = nullptr;  // T^{-1} V_j, s x N
    T* w = nullptr;
    T* z = nullptr;
    T* io_in = nullptr;   // precision-converted input (mixed mode)
    T* tmp = nullptr;     // scratch of the T-solve
    double* H = nullptr;  // (s+1) x s column-major
    double* pdot = nullptr;   // partial dot products of the apply kernel: ks x nba
    double* pnorm = nullptr;  // partial sums of squares: max(nba, nb)
    double* scal = nullptr;   // [0] beta0^2 (GMRES); [1..3] d.q, direction and step coefficients (PCG)
    double* ppcg = nullptr;   // partial sums of the PCG post-smoother: z.q, d.r, r.r (nb each), d.q (nba)
    int nb = 0;               // reduce_blocks(N)
    int nba = 0;              // blocks of the level-0 apply kernel
};

}  // namespace

struct SolveState {
    const double* b = nullptr;
    double* x = nullptr;
    double r0 = 0.0, rel = 1.0;
    int k = 0, status = CD_NOT_CONVERGED;
    bool done = true;
    std::vector<double> alpha, beta;  // step lengths and direction coefficients, one per outer iteration
};

struct cd_solver {
    cd_problem prob{};
    cd_options opt{};
    hipStream_t stream = nullptr;  // all work of the handle
    bool own_stream = false;       // created here because the caller passed the null stream
    hipEvent_t entry_event = nullptr;
    int d = 0, p = 0, ksteps = 0;
    size_t N = 0;
    std::vector<LevelHost> lv;
    cd::TFactor tf[3];
    int Nc = 0;

    DevArena arena;
    std::vector<LevelDev<double>> ld64;
    std::vector<LevelDev<float>> ld32;
    cd::TFacDev<double> tfd64[3]{};
    cd::TFacDev<float> tfd32[3]{};
    cd::OpDev<double> outer_op{};  // the system operator A of the outer iteration (level 0, never block-diagonal)
    double* Kinv = nullptr;  // inverse of the coarsest operator, leading dimension ldK
    int ldK = 0;

    std::unique_ptr<VWork<double>> w64;
    std::unique_ptr<VWork<float>> w32;
    std::unique_ptr<DevArena> hook_arena;    // FP64 V-cycle workspace created on demand in mixed mode
    std::unique_ptr<DevArena> hook_arena32;  // FP32 workspace created on demand by the FP32 hooks (FP64 mode)

    // outer FCG (FP64)
    double *r = nullptr, *z = nullptr, *dd = nullptr, *q = nullptr;
    double* bw = nullptr;  // MIM: copy of the right-hand side (graph replays read solver-owned buffers only)
    double *pzq = nullptr, *pdr = nullptr, *pdq = nullptr, *prr = nullptr, *scal = nullptr;
    // device and pinned host scalars of the outer iteration: [0] r.r, [1] d.q,
    // [2] step length a, [3] direction coefficient b (d = z - b d_prev), [4] ||b - A x||^2
    double* host_scal = nullptr;
    int nbr = 0, nba = 0;

    // live kernel timing (cd_profile_enable): every timed launch gets a slot,
    // a pair of wall-clock stamps the kernel itself writes (earliest block
    // start, latest block end).  A timed unit (one outer iteration, or one
    // hook call) clears its slots first and copies them to pinned host memory
    // last; the captured timed iteration uses slots [0, kGraphSlots) and does
    // both inside the graph.
    struct ProfRec {
        int slot;
        int cls;  // kind * 2L + 2 level + fp32; kind 0 = operator apply, 1 = T-solve pass
        double bytes;
    };
    static constexpr int kGraphSlots = 256, kStampSlots = 1024, kUnitSlots = 256;
    unsigned long long* stamps = nullptr;       // device, kStampSlots slots of cd::kStampWords words
    unsigned long long* pairs = nullptr;        // device, 2 kStampSlots: (start, end) per slot
    unsigned long long* stamps_host = nullptr;  // pinned copy of pairs
    double wall_khz = 0.0;                      // wall-clock rate
    bool unit_open = false;
    int unit_base = 0, unit_next = 0, eager_next = kGraphSlots;
    SolveState state;
    hipEvent_t iter_event = nullptr;
    double* xw = nullptr;                 // iterate of the outer iteration (copied to the caller's x)
    hipGraphExec_t iter_graph = nullptr;  // captured outer iteration k >= 1
    // the same iteration captured with live timing (stamp slots [0, kGraphSlots))
    hipGraphExec_t iter_graph_prof = nullptr;
    size_t graph_kernels = 0, graph_nodes = 0;  // of iter_graph
    std::vector<ProfRec> prof_graph;
    bool capturing = false, graph_prof_ran = false;
    int prof_period = 1;        // time every prof_period-th outer iteration
    long long prof_iter = 0;    // outer iterations run while timing was on
    bool prof_sample = true;    // the current iteration is timed

    bool prof = false;
    std::vector<ProfRec> prof_pending;
    std::vector<cd_kernel_stats> prof_stats;  // index cls
    ~cd_solver() {
        if (iter_event) (void)hipEventDestroy(iter_event);
        if (entry_event) (void)hipEventDestroy(entry_event);
        if (iter_graph) (void)hipGraphExecDestroy(iter_graph);
        if (iter_graph_prof) (void)hipGraphExecDestroy(iter_graph_prof);
        if (stamps) (void)hipFree(stamps);
        if (pairs) (void)hipFree(pairs);
        if (stamps_host) (void)hipHostFree(stamps_host);
    }
};

namespace {

void need(const cd_solver* s) {
    if (!s) throw CdError(CD_EINVAL, "null solver handle");
}
void need_level(const cd_solver* s, int l) {
    need(s);
    if (l < 0 || l >= int(s->lv.size())) throw CdError(CD_EINVAL, "level out of range");
}

using cd::kApplyCheb;
using cd::kApplyRes;
using cd::kApplyY;
using cd::kApplyYDot;

void validate(const cd_problem* pr, const cd_options* op) {
    if (!pr || !op) throw CdError(CD_EINVAL, "null problem or options");
    if (pr->dim != 2 && pr->dim != 3) throw CdError(CD_EINVAL, "dim must be 2 or 3");
    if (pr->degree < 1 || pr->degree > 6) throw CdError(CD_EINVAL, "degree must be in 1..6");
    for (int l = 0; l < pr->dim; ++l)
        if (pr->n[l] < 1 || pr->n[l] + pr->degree - 2 < 1) throw CdError(CD_EINVAL, "need n >= 1 and n + p - 2 >= 1");
    if (!(pr->alpha > 0.0) || !(pr->beta > 0.0) || !std::isfinite(pr->alpha) || !std::isfinite(pr->beta))
        throw CdError(CD_EINVAL, "alpha and beta must be positive and finite");
    if (op->method != CD_METHOD_PMIM && op->method != CD_METHOD_PWL && op->method != CD_METHOD_MIM &&
        op->method != CD_METHOD_CG)
        throw CdError(CD_EINVAL, "unknown method");
    if (op->transfer != CD_XFER_KNOT && op->transfer != CD_XFER_PAPER) throw CdError(CD_EINVAL, "unknown transfer");
    if (op->precision != CD_FP64 && op->precision != CD_MIXED_FP32) throw CdError(CD_EINVAL, "unknown precision");
    if (!(op->rtol > 0.0)) throw CdError(CD_EINVAL, "rtol must be positive");
    if (op->max_iter < 1) throw CdError(CD_EINVAL, "max_iter must be >= 1");
    if (op->cheb_degree < 1 || op->cheb_degree > 128) throw CdError(CD_EINVAL, "cheb_degree must be in 1..128");
    if (op->cheb_degree_coarse > 128) throw CdError(CD_EINVAL, "cheb_degree_coarse must be at most 128");
    if (!(op->cheb_ratio > 1.0)) throw CdError(CD_EINVAL, "cheb_ratio must be > 1");
    if (op->lanczos_steps < 1 || op->lanczos_steps > 200) throw CdError(CD_EINVAL, "lanczos_steps must be in 1..200");
    if (op->krylov_steps > 7) throw CdError(CD_EINVAL, "krylov_steps must be <= 7");
    if (op->graphs != 0 && op->graphs != 1) throw CdError(CD_EINVAL, "graphs must be 0 or 1");
    if (op->apply_x1_chunk < 0) throw CdError(CD_EINVAL, "apply_x1_chunk must be >= 0");
    if (op->eig_bounds != CD_BOUNDS_LANCZOS && op->eig_bounds != CD_BOUNDS_SYMBOL)
        throw CdError(CD_EINVAL, "unknown eig_bounds");
    if (!(op->bound_safety == 0.0 || (op->bound_safety >= 1.0 && op->bound_safety <= 10.0)))
        throw CdError(CD_EINVAL, "bound_safety must be 0 or in [1, 10]");
    if (op->apply3d_kernel < CD_APPLY3D_AUTO || op->apply3d_kernel > CD_APPLY3D_GROUP)
        throw CdError(CD_EINVAL, "unknown apply3d_kernel");
    if (op->coarse_max_dofs < 1 || op->coarse_max_dofs > 8192)
        throw CdError(CD_EINVAL, "coarse_max_dofs must be in 1..8192");
    // the operator kernels use fixed-size LDS tiles (no limit on the grid) and
    // 32-bit offsets within the 3D vectors
    size_t N = size_t(pr->dim);
    for (int l = 0; l < pr->dim; ++l) N *= size_t(pr->n[l] + pr->degree - 2);
    if (pr->dim == 3 && N >= (size_t(1) << 31)) throw CdError(CD_EINVAL, "3D problem too large (2^31 unknowns)");
}

size_t level_dofs(int d, const int* m) {
    size_t G = 1;
    for (int l = 0; l < d; ++l) G *= size_t(m[l]);
    return size_t(d) * G;
}

// Build the host hierarchy (Sec. 6.1: Galerkin coarse operators of the
// Kronecker form, coarsened until coarse_max_dofs).
void build_host(cd_solver* s) {
    const int d = s->d, p = s->p;
    LevelHost L0;
    for (int l = 0; l < 3; ++l) L0.m[l] = 1;
    for (int l = 0; l < d; ++l) {
        cd::assemble_1d(s->prob.n[l], p, L0.M[l], L0.A[l], L0.S[l]);
        L0.m[l] = L0.M[l].m;
    }
    L0.n = s->prob.n[0];
    L0.N = level_dofs(d, L0.m);
    s->lv.clear();
    s->lv.push_back(std::move(L0));
    // Per axis: knot insertion (n -> n/2) while the axis's n is even and the
    // handle asks for it, else the (1/2)[1 2 1] prolongator (m -> floor(m/2),
    // Sec. 6.1) from then on, else (m = 1) no coarsening of that axis.
    int nl[3] = {s->prob.n[0], s->prob.n[1], d == 3 ? s->prob.n[2] : 1};
    bool knot[3] = {s->opt.transfer == CD_XFER_KNOT, s->opt.transfer == CD_XFER_KNOT, s->opt.transfer == CD_XFER_KNOT};
    while (true) {
        LevelHost& F = s->lv.back();
        if (F.N <= size_t(s->opt.coarse_max_dofs)) break;
        int kind[3] = {0, 0, 0};  // 0 none, 1 knot insertion, 2 paper prolongator
        bool any = false;
        for (int l = 0; l < d; ++l) {
            if (knot[l] && nl[l] % 2 == 0 && nl[l] / 2 + p - 2 >= 1) {
                kind[l] = 1;
            } else if (F.m[l] / 2 >= 1) {
                kind[l] = 2;
                knot[l] = false;
            }
            any = any || kind[l] != 0;
        }
        if (!any) break;
        LevelHost C;
        for (int l = 0; l < 3; ++l) C.m[l] = 1;
        for (int l = 0; l < d; ++l) {
            F.P[l] = kind[l] == 1 ? cd::knot_insertion(nl[l], p)
                     : kind[l] == 2 ? cd::paper_prolong(F.m[l])
                                    : cd::identity_prolong(F.m[l]);
            if (F.P[l].w > 8 || F.P[l].wr > 8) throw CdError(CD_EINVAL, "prolongator window wider than 8");
            C.M[l] = cd::galerkin(F.M[l], F.P[l]);
            C.A[l] = cd::galerkin(F.A[l], F.P[l]);
            C.S[l] = cd::galerkin(F.S[l], F.P[l]);
            // every level is stored with half bandwidth p (zero padded)
            if (C.M[l].hb > p || C.A[l].hb > p || C.S[l].hb > p) throw CdError(CD_EINVAL, "coarse band wider than p");
            C.M[l] = C.M[l].widened(p);
            C.A[l] = C.A[l].widened(p);
            C.S[l] = C.S[l].widened(p);
            C.m[l] = C.M[l].m;
            if (kind[l] == 1) nl[l] /= 2;
        }
        C.n = nl[0];
        C.N = level_dofs(d, C.m);
        s->lv.push_back(std::move(C));
    }
    // every axis can be coarsened down to one point, so only a cap below d is left over
    if (s->lv.back().N > size_t(s->opt.coarse_max_dofs) && s->lv.back().N > size_t(d))
        throw CdError(CD_EINVAL, "the coarsest level has " + std::to_string(s->lv.back().N) +
                                     " unknowns, more than coarse_max_dofs = " +
                                     std::to_string(s->opt.coarse_max_dofs));
    for (int l = 0; l < d; ++l) s->tf[l] = cd::toeplitz_factor(s->lv[0].m[l], p);
    const LevelHost& Lc = s->lv.back();
    s->Nc = int(Lc.N);
}

template <typename T>
cd::OpDev<T> make_op(cd_solver* s, const LevelHost& L, hipStream_t st) {
    cd::OpDev<T> op{};
    op.dim = s->d;
    op.hb = s->p;
    op.x1chunk = s->opt.apply_x1_chunk;
    op.variant = s->opt.apply3d_kernel;
    op.blockdiag = (s->opt.method == CD_METHOD_PWL) ? 1 : 0;  // P_WL cycles on D (Sec. 6.1, eq. diag)
    op.alpha = T(s->prob.alpha);
    op.beta = T(s->prob.beta);
    for (int l = 0; l < 3; ++l) op.m[l] = L.m[l];
    for (int l = 0; l < 3; ++l)
        for (int w = 0; w < 3; ++w) op.band[l][w] = nullptr;
    for (int l = 0; l < s->d; ++l) {
        const cd::Band* mats[3] = {&L.M[l], &L.A[l], &L.S[l]};
        for (int w = 0; w < 3; ++w) op.band[l][w] = s->arena.upload(convert<T>(kmajor(*mats[w])), st);
    }
    {
        const cd::Band* mats[3] = {&L.M[0], &L.A[0], &L.S[0]};
        const int hb = s->p, R = 2 * hb + 1, m0 = L.m[0];
        for (int w = 0; w < 3; ++w) {
            std::vector<double> col(size_t(m0) * R, 0.0);
            for (int j = 0; j < m0; ++j)
                for (int k = 0; k < R; ++k) {
                    const int i = j - hb + k;
                    if (i >= 0 && i < m0) col[size_t(j) * R + k] = mats[w]->get(i, j);
                }
            op.col0[w] = s->arena.upload(convert<T>(col), st);
        }
        // the same columns as one row per plane j in [-hb, m0 + hb), with the
        // diagonal entries of M and S at plane j - hb (the 3D kernel's table)
        const int NC = 3 * R + 2;
        std::vector<double> tab(size_t(m0 + 2 * hb) * NC, 0.0);
        auto at = [&](int w, int i, int j) { return (i >= 0 && i < m0 && j >= 0 && j < m0) ? mats[w]->get(i, j) : 0.0; };
        for (int j = -hb; j < m0 + hb; ++j) {
            double* row = tab.data() + size_t(j + hb) * NC;
            for (int w = 0; w < 3; ++w)
                for (int k = 0; k < R; ++k) row[w * R + k] = at(w, j - hb + k, j);
            row[3 * R] = at(0, j - hb, j - hb);
            row[3 * R + 1] = at(2, j - hb, j - hb);
        }
        op.c1p = s->arena.upload(convert<T>(tab), st);
        std::vector<double> rows(size_t(m0) * NC, 0.0);
        for (int i = 0; i < m0; ++i) {
            double* row = rows.data() + size_t(i) * NC;
            for (int w = 0; w < 3; ++w)
                for (int g = 0; g < R; ++g) row[w * R + g] = at(w, i, i - hb + g);
            row[3 * R] = at(0, i, i);
            row[3 * R + 1] = at(2, i, i);
        }
        op.c1r = s->arena.upload(convert<T>(rows), st);
    }
    if (s->d == 2) {  // unused third axis: a 1x1 identity band keeps pointers valid
        std::vector<double> id(2 * s->p + 1, 0.0);
        id[s->p] = 1.0;
        for (int w = 0; w < 3; ++w) op.band[2][w] = s->arena.upload(convert<T>(id), st);
    }
    return op;
}

template <typename T>
cd::XferDev<T> make_xfer(cd_solver* s, const LevelHost& L, hipStream_t st) {
    cd::XferDev<T> X{};
    X.dim = s->d;
    for (int l = 0; l < 3; ++l) {
        cd::XferAxisDev<T>& a = X.ax[l];
        if (l < s->d) {
            const cd::Prolong& P = L.P[l];
            a.mf = P.mf;
            a.mc = P.mc;
            a.w = P.w;
            a.wr = P.wr;
            a.c0 = s->arena.upload(P.c0, st);
            a.r0 = s->arena.upload(P.r0, st);
            a.v = s->arena.upload(convert<T>(P.v), st);
            a.vt = s->arena.upload(convert<T>(P.vt), st);
        } else {
            a.mf = a.mc = a.w = a.wr = 1;
            a.c0 = s->arena.upload(std::vector<int>{0}, st);
            a.r0 = s->arena.upload(std::vector<int>{0}, st);
            a.v = s->arena.upload(std::vector<T>{T(1)}, st);
            a.vt = s->arena.upload(std::vector<T>{T(1)}, st);
        }
    }
    return X;
}

template <typename T>
cd::TFacDev<T> make_tfac(cd_solver* s, const cd::TFactor& F, hipStream_t st) {
    cd::TFacDev<T> t{};
    t.m = F.m;
    t.bw = F.bw;
    t.l = s->arena.upload(convert<T>(F.l), st);
    t.dinv = s->arena.upload(convert<T>(F.dinv), st);
    // start each chunk's recurrence early enough that the zero start state has
    // decayed below the unit roundoff of T
    t.warm = cd::recurrence_warmup(F, sizeof(T) == 8 ? 0x1p-53 : 0x1p-24);
    return t;
}

template <typename T>
const std::vector<LevelDev<T>>& devlevels(cd_solver* s);
template <>
const std::vector<LevelDev<double>>& devlevels<double>(cd_solver* s) { return s->ld64; }
template <>
const std::vector<LevelDev<float>>& devlevels<float>(cd_solver* s) { return s->ld32; }

template <typename T>
std::unique_ptr<VWork<T>> make_work(cd_solver* s, DevArena& ar) {
    auto w = std::make_unique<VWork<T>>();
    const int L = int(s->lv.size());
    w->lv.resize(L);
    for (int l = 0; l < L; ++l) {
        const size_t n = s->lv[l].N;
        auto& W = w->lv[l];
        W.b = ar.alloc<T>(n);
        W.xa = ar.alloc<T>(n);
        if (l < L - 1) {
            W.xb = ar.alloc<T>(n);
            W.r = ar.alloc<T>(n);
        }
    }
    const int ks = std::max(s->ksteps, 1);
    w->V = ar.alloc<T>(size_t(ks + 1) * s->N);
    w->Z = ar.alloc<T>(size_t(ks) * s->N);
    w->w = ar.alloc<T>(s->N);
    w->z = ar.alloc<T>(s->N);
    w->io_in = ar.alloc<T>(s->N);
    w->tmp = ar.alloc<T>(s->N);
    w->H = ar.alloc<double>(size_t(ks + 1) * ks);
    w->nb = cd::reduce_blocks(s->N);
    w->nba = cd::apply_blocks<T>(devlevels<T>(s)[0].op);
    w->pdot = ar.alloc<double>(size_t(w->nba) * (ks + 1));
    w->pnorm = ar.alloc<double>(size_t(std::max(w->nba, w->nb)));
    w->scal = ar.alloc<double>(4);
    w->ppcg = ar.alloc<double>(size_t(3) * w->nb + size_t(w->nba));
    return w;
}

template <typename T>
const cd::TFacDev<T>* tfacs(cd_solver* s);
template <>
const cd::TFacDev<double>* tfacs<double>(cd_solver* s) { return s->tfd64; }
template <>
const cd::TFacDev<float>* tfacs<float>(cd_solver* s) { return s->tfd32; }

// ---- live kernel timing ----------------------------------------------------------------
// Classes of timed launches: kind 0 = operator applies other than Chebyshev
// steps, 1 = T-solve axis passes (level 0), 2 = Chebyshev-step applies; per
// level and precision.
constexpr int kProfKinds = 3;
int prof_class(const cd_solver* s, int kind, int level, bool fp32) {
    return kind * 2 * int(s->lv.size()) + 2 * level + (fp32 ? 1 : 0);
}

// Fold the stamps of the records into the totals (host copies complete).
void prof_add(cd_solver* s, const std::vector<cd_solver::ProfRec>& recs) {
    for (const auto& r : recs) {
        const unsigned long long t0 = s->stamps_host[2 * r.slot], t1 = s->stamps_host[2 * r.slot + 1];
        if (t0 == ~0ull || t1 == 0 || t1 < t0) continue;  // slot not written (no kernel ran)
        cd_kernel_stats& st = s->prof_stats[r.cls];
        st.launches += 1;
        st.total_ms += double(t1 - t0) / s->wall_khz;
        st.bytes += r.bytes;
    }
}

// Call after a stream sync.
void prof_flush(cd_solver* s) {
    if (s->prof_stats.size() < kProfKinds * 2 * s->lv.size())
        s->prof_stats.resize(kProfKinds * 2 * s->lv.size(), cd_kernel_stats{0, 0.0, 0.0});
    prof_add(s, s->prof_pending);
    s->prof_pending.clear();
    s->eager_next = cd_solver::kGraphSlots;
    if (s->graph_prof_ran) {  // stamps of the last replay of the timed graph
        prof_add(s, s->prof_graph);
        s->graph_prof_ran = false;
    }
}

void prof_unit_begin(cd_solver* s) {
    if (s->capturing) {
        s->unit_base = 0;
        s->prof_graph.clear();
    } else {
        if (s->eager_next + cd_solver::kUnitSlots > cd_solver::kStampSlots) {
            hip_check(hipStreamSynchronize(s->stream), "sync");
            prof_flush(s);
        }
        s->unit_base = s->eager_next;
    }
    s->unit_next = s->unit_base;
    s->unit_open = true;
}

// n consecutive slots of class cls, bytes each.
unsigned long long* prof_slots(cd_solver* s, int n, int cls, double bytes) {
    if (s->unit_next + n > s->unit_base + cd_solver::kUnitSlots)
        throw CdError(CD_EHIP, "too many timed launches in one outer iteration");
    unsigned long long* p = s->stamps + size_t(s->unit_next) * cd::kStampWords;
    for (int i = 0; i < n; ++i) {
        const cd_solver::ProfRec rec{s->unit_next + i, cls, bytes};
        (s->capturing ? s->prof_graph : s->prof_pending).push_back(rec);
    }
    s->unit_next += n;
    return p;
}

void prof_unit_end(cd_solver* s) {
    const int n = s->unit_next - s->unit_base;
    if (n > 0) {
        cd::launch_stamp_reduce(s->stamps, s->unit_base, n, s->pairs, s->stream);
        hip_check(hipMemcpyAsync(s->stamps_host + 2 * s->unit_base, s->pairs + 2 * s->unit_base,
                                 size_t(2 * n) * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream),
                  "read stamps");
    }
    if (!s->capturing) s->eager_next = s->unit_next;
    s->unit_open = false;
}

bool timing(const cd_solver* s) { return s->prof && s->prof_sample; }

// ---- operator apply and T-solve with optional live timing ------------------------------
template <typename T>
void apply_with(cd_solver* s, const cd::OpDev<T>& op, int level, int mode, const T* x, T* y, const T* b, T* u,
                T* xout, T c1, T c2, double* part, int nv = 0) {
    if (!timing(s)) {
        cd::launch_apply<T>(op, mode, x, y, b, u, xout, c1, c2, part, s->stream, nv);
        return;
    }
    const bool own = !s->unit_open;
    if (own) prof_unit_begin(s);
    // vectors read and written once: the residual reads b; a Chebyshev step
    // reads b and the previous iterate (not on a first step, c1 = 0)
    const double nvec = (mode == kApplyRes || mode == cd::kApplyResDot) ? 3.0
                        : (mode == kApplyCheb)                         ? ((c1 != T(0) && u) ? 4.0 : 3.0)
                        : (mode == cd::kApplyYMulti)                   ? 2.0 + nv
                                                                       : 2.0;
    unsigned long long* st = prof_slots(s, 1, prof_class(s, mode == kApplyCheb ? 2 : 0, level, sizeof(T) == 4),
                                        nvec * double(s->lv[level].N) * sizeof(T));
    cd::launch_apply<T>(op, mode, x, y, b, u, xout, c1, c2, part, s->stream, nv, st);
    if (own) prof_unit_end(s);
}

// Apply the V-cycle's operator of `level` (A_l, or its block-diagonal part D_l for P_WL).
template <typename T>
void apply_op(cd_solver* s, int level, int mode, const T* x, T* y, const T* b, T* u, T* xout, T c1, T c2,
              double* part, int nv = 0) {
    apply_with<T>(s, devlevels<T>(s)[level].op, level, mode, x, y, b, u, xout, c1, c2, part, nv);
}

// z = T^{-1} v on the finest level.
template <typename T>
void tsolve_op(cd_solver* s, const T* v, T* tmp, T* z) {
    const int d = s->d;
    if (!timing(s) || s->tf[0].bw == 0) {
        cd::launch_tsolve<T>(d, s->lv[0].m, tfacs<T>(s), v, tmp, z, s->stream);
        return;
    }
    const bool own = !s->unit_open;
    if (own) prof_unit_begin(s);
    // one pass per axis, each reads its input and writes its output once
    unsigned long long* st = prof_slots(s, d, prof_class(s, 1, 0, sizeof(T) == 4), 2.0 * double(s->N) * sizeof(T));
    cd::launch_tsolve<T>(d, s->lv[0].m, tfacs<T>(s), v, tmp, z, s->stream, st);
    if (own) prof_unit_end(s);
}

// ---- V-cycle pieces ------------------------------------------------------------

// Chebyshev smoothing on level l (Sec. 6.1 smoother reading): cheb_degree
// steps on D^{-1} A_l on the finest level, cheb_degree_coarse (when set) on
// the others, interval [lo, hi], in the three-term form
//   x_{k+1} = x_k + c1_k (x_k - x_{k-1}) + c2_k D^{-1} (b - A_l x_k),
// so a step reads x_k, x_{k-1} and b and writes x_{k+1} over x_{k-1}.
// Starts from zero when from_zero (the first step needs no operator apply:
// x_1 = D^{-1} b / theta; first_done: the producer of b already wrote it into
// x), else from *x; the result pointer is returned (x or other).
template <typename T>
T* chebyshev(cd_solver* s, int l, const T* b, T* x, T* other, bool from_zero, bool first_done = false) {
    const LevelHost& L = s->lv[l];
    const cd::OpDev<T>& op = devlevels<T>(s)[l].op;
    const double theta = 0.5 * (L.hi + L.lo), delta = 0.5 * (L.hi - L.lo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    const int nu = (l > 0) ? s->opt.cheb_degree_coarse : s->opt.cheb_degree;  // resolved in create
    T* cur = x;
    T* nxt = other;
    const T* prev = nullptr;  // x_{k-1}; nullptr: zero
    if (from_zero) {
        if (!first_done) cd::launch_cheb_first<T>(op, b, cur, T(1.0 / theta), s->stream);
    } else {
        apply_op<T>(s, l, kApplyCheb, cur, nullptr, b, nullptr, nxt, T(0), T(1.0 / theta), nullptr);
        std::swap(cur, nxt);
        prev = nxt;
    }
    for (int k = 1; k < nu; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        apply_op<T>(s, l, kApplyCheb, cur, nullptr, b, const_cast<T*>(prev), nxt, T(rn * rho), T(2.0 * rn / delta),
                    nullptr);
        std::swap(cur, nxt);
        prev = nxt;
        rho = rn;
    }
    return cur;
}

// The first Chebyshev step from zero on level l, to be fused into the kernel
// that produces the level's right-hand side; result in the level's xa.
template <typename T>
cd::ChebFirst<T> cheb_first_of(cd_solver* s, VWork<T>& W, int l) {
    const LevelHost& L = s->lv[l];
    return cd::ChebFirst<T>{devlevels<T>(s)[l].op, T(1.0 / (0.5 * (L.hi + L.lo))), W.lv[l].xa};
}

// p steps of GMRES on A_0 e = b - A_0 x from e = 0, right preconditioner T
// (Sec. 6.1 post-smoother), classical Gram-Schmidt; x += T^{-1} V y.
template <typename T>
void gmres_post(cd_solver* s, VWork<T>& W, const T* b, T* x) {
    const size_t N = s->N;
    const int ks = s->ksteps, ld = ks + 1, nba = W.nba;
    hipStream_t st = s->stream;
    T* V = W.V;
    // r = b - A x and its norm: V_0 = r / ||r||, beta0^2 kept for the least squares
    apply_op<T>(s, 0, cd::kApplyResDot, x, W.w, b, nullptr, nullptr, T(0), T(0), W.pnorm);
    cd::launch_normscale<T>(W.pnorm, nba, W.scal, true, W.w, V, N, st);
    for (int j = 0; j < ks; ++j) {
        double* Hcol = W.H + size_t(j) * ld;
        T* Zj = W.Z + size_t(j) * N;
        tsolve_op<T>(s, V + size_t(j) * N, W.tmp, Zj);
        // w = A T^{-1} V_j together with the dots V_i . w (i <= j) and w . w
        apply_op<T>(s, 0, cd::kApplyYMulti, Zj, W.w, V, nullptr, nullptr, T(0), T(0), W.pdot, j + 1);
        // H(0..j, j) = V_i . w, H(j+1, j) = ||w - sum_i H(i, j) V_i|| (Pythagoras),
        // V_{j+1} = that vector normalised (not needed after the last step)
        cd::launch_gs_normscale<T>(W.pdot, j + 1, nba, Hcol, V, W.w, (j + 1 < ks) ? V + size_t(j + 1) * N : nullptr,
                                   N, st);
    }
    // x += T^{-1} (V y) = sum_j y_j T^{-1} V_j  (T is linear), y from the least squares
    cd::launch_lsq_combine_add<T>(W.H, ld, ks, W.scal, W.Z, x, N, st);
}

// p steps of CG on D_0 e = b - D_0 x from e = 0, preconditioned by T (the
// finest post-smoother of P_WL, Sec. 6.1-6.2), written in the flexible form
// d_j = z_j - ((z_j . q_{j-1}) / (d_{j-1} . q_{j-1})) d_{j-1}, step
// (d_j . r_j) / (d_j . q_j), which equals PCG for the fixed SPD T; the steps
// accumulate into x directly (x + e).
template <typename T>
void pcg_post(cd_solver* s, VWork<T>& W, const T* b, T* x) {
    const size_t N = s->N;
    const int nb = W.nb, nba = W.nba;
    hipStream_t st = s->stream;
    T* r = W.w;
    T* z = W.z;
    T* d = W.V;
    T* q = W.V + N;
    double* pzq = W.ppcg;
    double* pdr = W.ppcg + nb;
    double* prr = W.ppcg + 2 * nb;
    double* pdq = W.ppcg + 3 * nb;
    apply_op<T>(s, 0, kApplyRes, x, r, b, nullptr, nullptr, T(0), T(0), nullptr);
    for (int j = 0; j < s->ksteps; ++j) {
        tsolve_op<T>(s, r, W.tmp, z);
        if (j > 0) cd::launch_dot_partial<T, T>(z, q, N, pzq, st);
        cd::launch_fcg_direction<T>(j == 0, z, pzq, nb, W.scal + 1, d, r, pdr, W.scal + 2, N, st);
        apply_op<T>(s, 0, kApplyYDot, d, q, nullptr, nullptr, nullptr, T(0), T(0), pdq);
        cd::launch_fcg_update<T>(pdr, nb, pdq, nba, W.scal + 1, x, r, d, q, prr, W.scal + 3, N, st);
    }
}

// One V-cycle on level l for A_l x = W.lv[l].b; result in W.lv[l].xcur.
// first_done: the first pre-smoothing step was fused into the producer of b.
template <typename T>
void vcycle(cd_solver* s, VWork<T>& W, int l, bool first_done = false) {
    const int L = int(s->lv.size());
    auto& Wl = W.lv[l];
    hipStream_t st = s->stream;
    if (l == L - 1) {
        cd::launch_coarse_gemv<T>(s->Kinv, s->Nc, s->ldK, Wl.b, Wl.xa, st);
        Wl.xcur = Wl.xa;
        return;
    }
    const auto& D = devlevels<T>(s)[l];
    T* x = chebyshev<T>(s, l, Wl.b, Wl.xa, Wl.xb, true, first_done);
    T* other = (x == Wl.xa) ? Wl.xb : Wl.xa;
    apply_op<T>(s, l, kApplyRes, x, Wl.r, Wl.b, nullptr, nullptr, T(0), T(0), nullptr);
    const bool fuse = (l + 1 < L - 1);  // the next level smooths (it is not the coarsest)
    const cd::ChebFirst<T> cf = fuse ? cheb_first_of<T>(s, W, l + 1) : cd::ChebFirst<T>{};
    cd::launch_restrict<T>(D.xf, s->d, Wl.r, W.lv[l + 1].b, st, fuse ? &cf : nullptr);
    vcycle<T>(s, W, l + 1, fuse);
    cd::launch_prolong_add<T>(D.xf, s->d, W.lv[l + 1].xcur, x, st);
    if (l == 0 && s->ksteps > 0) {
        if (s->opt.method == CD_METHOD_PWL)
            pcg_post<T>(s, W, Wl.b, x);
        else
            gmres_post<T>(s, W, Wl.b, x);
    } else {
        x = chebyshev<T>(s, l, Wl.b, x, other, false);
    }
    Wl.xcur = x;
}

// Work given the legacy null stream goes to a stream owned by the handle
// (stream capture is not permitted on the null stream); every entry point
// first orders it after the work already queued on the null stream.
void enter(cd_solver* s) {
    if (!s->own_stream) return;
    hip_check(hipEventRecord(s->entry_event, nullptr), "hipEventRecord");
    hip_check(hipStreamWaitEvent(s->stream, s->entry_event, 0), "hipStreamWaitEvent");
}

VWork<double>& work64(cd_solver* s) {
    if (!s->w64) {
        s->hook_arena = std::make_unique<DevArena>();
        s->w64 = make_work<double>(s, *s->hook_arena);
    }
    return *s->w64;
}

VWork<float>& work32(cd_solver* s) {
    if (!s->w32) {
        s->hook_arena32 = std::make_unique<DevArena>();
        s->w32 = make_work<float>(s, *s->hook_arena32);
    }
    return *s->w32;
}

template <typename T>
VWork<T>& work_of(cd_solver* s);
template <>
VWork<double>& work_of<double>(cd_solver* s) { return work64(s); }
template <>
VWork<float>& work_of<float>(cd_solver* s) { return work32(s); }

// Test hooks in precision T (see cd_smooth, cd_restrict, cd_prolong_add, cd_tsolve).
template <typename T>
void hook_smooth(cd_solver* s, int level, const T* b, const T* x_in, T* x_out) {
    need_level(s, level);
    enter(s);
    if (level == int(s->lv.size()) - 1) throw CdError(CD_EINVAL, "coarsest level has no smoother");
    if (s->opt.method == CD_METHOD_CG) throw CdError(CD_EINVAL, "no smoother for plain CG");
    VWork<T>& W = work_of<T>(s);
    auto& Wl = W.lv[level];
    const size_t n = s->lv[level].N;
    cd::launch_copy<T>(b, Wl.b, n, s->stream);
    cd::launch_copy<T>(x_in, Wl.xa, n, s->stream);
    T* r = chebyshev<T>(s, level, Wl.b, Wl.xa, Wl.xb, false);
    cd::launch_copy<T>(r, x_out, n, s->stream);
    hip_check(hipStreamSynchronize(s->stream), "sync");
}

template <typename T>
void hook_transfer(cd_solver* s, int level, bool restrict_, const T* in, T* out) {
    need_level(s, level);
    enter(s);
    if (level == int(s->lv.size()) - 1) throw CdError(CD_EINVAL, "coarsest level");
    const auto& X = devlevels<T>(s)[level].xf;
    if (restrict_)
        cd::launch_restrict<T>(X, s->d, in, out, s->stream);
    else
        cd::launch_prolong_add<T>(X, s->d, in, out, s->stream);
    hip_check(hipStreamSynchronize(s->stream), "sync");
}

template <typename T>
void hook_tsolve(cd_solver* s, const T* v, T* z) {
    need(s);
    enter(s);
    VWork<T>& W = work_of<T>(s);  // its T-solve scratch and spare vector
    const T* src = v;
    if (v == z) {
        cd::launch_copy<T>(v, W.w, s->N, s->stream);
        src = W.w;
    }
    tsolve_op<T>(s, src, W.tmp, z);
    hip_check(hipStreamSynchronize(s->stream), "sync");
    if (s->prof) prof_flush(s);
}

// z = V(r) in the handle's precision; r, z FP64 device vectors.
// With q != nullptr also part[block] = partial sums of z . q (reduce_blocks(N)).
void precondition(cd_solver* s, const double* r, double* z, const double* q = nullptr, double* part = nullptr) {
    hipStream_t st = s->stream;
    const bool fuse = s->lv.size() > 1;  // level 0 smooths: its first step is fused into the input conversion
    if (s->opt.precision == CD_FP64) {
        VWork<double>& W = work64(s);
        if (fuse)
            cd::launch_cast_cheb<double, double>(r, W.lv[0].b, s->N, cheb_first_of<double>(s, W, 0), st);
        else
            cd::launch_copy<double>(r, W.lv[0].b, s->N, st);
        vcycle<double>(s, W, 0, fuse);
        if (q)
            cd::launch_cast_dot<double, double>(W.lv[0].xcur, z, s->N, q, part, st);
        else
            cd::launch_copy<double>(W.lv[0].xcur, z, s->N, st);
    } else {
        VWork<float>& W = *s->w32;
        if (fuse)
            cd::launch_cast_cheb<float, double>(r, W.lv[0].b, s->N, cheb_first_of<float>(s, W, 0), st);
        else
            cd::launch_cast<float, double>(r, W.lv[0].b, s->N, st);
        vcycle<float>(s, W, 0, fuse);
        if (q)
            cd::launch_cast_dot<double, float>(W.lv[0].xcur, z, s->N, q, part, st);
        else
            cd::launch_cast<double, float>(W.lv[0].xcur, z, s->N, st);
    }
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..k)
// and off-diagonal b[1..k) (b[i] couples rows i-1 and i), by bisection on the
// Sturm count: the number of negative pivots of T - x I is the number of
// eigenvalues below x.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
    const int k = int(a.size());
    auto below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < k; ++i) {
            d = a[i] - x - (i > 0 ? b[i] * b[i] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < k ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-16 * std::fabs(hi); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) >= k) hi = mid; else lo = mid;
    }
    return hi;
}

// Condition-number estimate from the outer iteration's coefficients: the
// step lengths a_j and direction coefficients b_j (d_j = z_j + b_j d_{j-1})
// of a conjugate-gradient iteration define the Lanczos matrix of the
// (preconditioned) operator, diagonal 1/a_j + b_j/a_{j-1}, off-diagonal
// sqrt(b_{j+1})/a_j; its extreme eigenvalues (Ritz values) approach the
// extreme eigenvalues of the operator from inside.  Returns their ratio, or
// 0 when there is no coefficient to use.  A non-positive b_j (possible with
// a nonlinear preconditioner) splits the matrix there.
double lanczos_kappa(const std::vector<double>& a, const std::vector<double>& b) {
    const int k = int(a.size());
    if (k == 0 || !(a[0] > 0.0)) return 0.0;
    std::vector<double> diag(k), off(k, 0.0);
    for (int j = 0; j < k; ++j) {
        if (!(a[j] > 0.0) || !std::isfinite(a[j])) return 0.0;
        diag[j] = 1.0 / a[j] + (j > 0 ? std::max(b[j], 0.0) / a[j - 1] : 0.0);
        if (j > 0) off[j] = std::sqrt(std::max(b[j], 0.0)) / a[j - 1];
    }
    const double hi = tridiag_max_eig(diag, off);
    std::vector<double> neg(k);
    for (int j = 0; j < k; ++j) neg[j] = -diag[j];
    const double lo = -tridiag_max_eig(neg, off);
    return (lo > 0.0) ? hi / lo : 0.0;
}

// Smoother eigenvalue bounds: lanczos_steps steps of Lanczos on D^{-1} A_l in
// the D inner product (no reorthogonalisation) from v0 = (-1)^{i_1+...+i_d}
// in every component; the estimate is the largest Ritz value.  Where
// beta_{j+1} <= 1e-10 |alpha_j| the Krylov space is invariant and the
// recurrence restarts from r_i = cos(0.7 i + 0.3) (D-normalised) with
// beta_{j+1} = 0.  The recurrence coefficients stay on the device until the
// last step.
// Smoother bounds from the spectral symbol (Sec. 5) of each smoothed level's
// Toeplitz part: lam = the symbol maximum of diag^{-1} A_l, hi = safety x lam.
// Levels without an interior row keep lam = 0 and get the Lanczos bound.
constexpr double kDefaultBoundSafety = 1.5;
int symbol_samples(int d) { return d == 2 ? 129 : 33; }

double level_symbol_bound(const cd_solver* s, const LevelHost& H) {
    const double offw = (s->opt.method == CD_METHOD_PWL) ? 0.0 : s->prob.alpha - s->prob.beta;
    return cd::symbol_lambda_max(s->d, H.M, H.A, H.S, s->prob.alpha, s->prob.beta, offw, symbol_samples(s->d));
}

void symbol_bounds(cd_solver* s) {
    const double safety = s->opt.bound_safety > 0.0 ? s->opt.bound_safety : kDefaultBoundSafety;
    for (size_t l = 0; l + 1 < s->lv.size(); ++l) {
        LevelHost& H = s->lv[l];
        const double lam = level_symbol_bound(s, H);
        if (lam > 0.0 && std::isfinite(lam)) {
            H.lam = lam;
            H.hi = safety * lam;
            H.lo = H.hi / s->opt.cheb_ratio;
        }
    }
}

void estimate_bounds(cd_solver* s) {
    hipStream_t st = s->stream;
    const int L = int(s->lv.size());
    bool any = false;  // a smoothed level without a bound from the symbol
    for (int l = 0; l < L - 1; ++l) any = any || !(s->lv[l].lam > 0.0);
    if (!any) return;
    const int ks = s->opt.lanczos_steps;
    DevArena tmp;
    double* qa = tmp.alloc<double>(s->N);
    double* qb = tmp.alloc<double>(s->N);
    double* w = tmp.alloc<double>(s->N);
    double* rr = tmp.alloc<double>(s->N);
    const int nbmax = std::max(cd::reduce_blocks(s->N), cd::apply_blocks<double>(s->ld64[0].op));
    double* part = tmp.alloc<double>(nbmax);
    double* coef = tmp.alloc<double>(2 * size_t(ks) + 1);  // alpha[0..ks), beta2[0..ks]
    for (int l = 0; l < L - 1; ++l) {
        LevelHost& H = s->lv[l];
        if (H.lam > 0.0) continue;  // bound already set from the symbol
        const cd::OpDev<double>& op = s->ld64[l].op;
        const size_t n = H.N;
        std::vector<double> v0(n);
        const int m0 = H.m[0], m1 = H.m[1], m2 = H.m[2];
        const size_t G = size_t(m0) * m1 * m2;
        for (size_t id = 0; id < n; ++id) {
            size_t rem = id % G;
            const int i2 = int(rem % m2);
            rem /= m2;
            const int i1 = int(rem % m1);
            const int i0 = int(rem / m1);
            v0[id] = ((i0 + i1 + i2) % 2 == 0) ? 1.0 : -1.0;
        }
        std::vector<double> r0(n);
        for (size_t id = 0; id < n; ++id) r0[id] = std::cos(0.7 * double(id) + 0.3);
        hip_check(hipMemcpyAsync(w, v0.data(), n * sizeof(double), hipMemcpyHostToDevice, st), "upload v0");
        hip_check(hipMemcpyAsync(rr, r0.data(), n * sizeof(double), hipMemcpyHostToDevice, st), "upload r");
        const int nbr = cd::reduce_blocks(n);
        const int nba = cd::apply_blocks<double>(op);
        double* alpha = coef;
        double* beta2 = coef + ks;
        cd::launch_fill<double>(qa, 0.0, n, st);
        cd::launch_fill<double>(beta2, 0.0, 1, st);
        cd::launch_diag_dot<double>(op, rr, part, st);
        cd::launch_normalize<double>(part, nbr, rr, rr, n, st);
        cd::launch_diag_dot<double>(op, w, part, st);
        cd::launch_normalize<double>(part, nbr, w, qb, n, st);
        // qa = q_{j-1}, qb = q_j
        for (int j = 0; j < ks; ++j) {
            cd::launch_apply<double>(op, kApplyYDot, qb, w, nullptr, nullptr, nullptr, 0.0, 0.0, part, st);
            cd::launch_finalize(part, nba, alpha + j, st);
            cd::launch_lanczos_step(op, alpha + j, alpha + (j > 0 ? j - 1 : 0), beta2 + j, qb, qa, w, st);
            cd::launch_diag_dot<double>(op, w, part, st);
            cd::launch_finalize(part, nbr, beta2 + j + 1, st);
            cd::launch_lanczos_next(alpha + j, beta2 + j + 1, w, rr, qa, n, st);
            std::swap(qa, qb);
        }
        std::vector<double> h(2 * size_t(ks) + 1);
        hip_check(hipMemcpyAsync(h.data(), coef, h.size() * sizeof(double), hipMemcpyDeviceToHost, st),
                  "read lanczos coefficients");
        hip_check(hipStreamSynchronize(st), "sync");
        std::vector<double> a(h.begin(), h.begin() + ks), b(ks, 0.0);
        const double tol = 1e-10;  // breakdown test, as in the kernels
        for (int j = 1; j < ks; ++j)
            b[j] = (h[ks + j] <= tol * tol * a[j - 1] * a[j - 1]) ? 0.0 : std::sqrt(std::max(h[ks + j], 0.0));
        if (!(a[0] > 0.0)) throw CdError(CD_EINVAL, "operator is not positive definite");
        H.lam = tridiag_max_eig(a, b);
        if (!(H.lam > 0.0) || !std::isfinite(H.lam)) throw CdError(CD_EINVAL, "operator is not positive definite");
        H.hi = 1.1 * H.lam;
        H.lo = H.hi / s->opt.cheb_ratio;
    }
}

// Chebyshev degree on the levels below the finest: > 0 as given, 0 = the
// finest level's, < 0 = from beta / alpha: the smaller beta, the more of the
// spectrum the smoother damps slowly and the more the cheap coarse levels'
// extra steps pay (measured solve times in the options' documentation).
constexpr double kSmallBeta = 1e-5, kLargeBeta = 1e-2;
int resolve_coarse_degree(const cd_problem& pr, const cd_options& o) {
    if (o.cheb_degree_coarse > 0) return o.cheb_degree_coarse;
    if (o.cheb_degree_coarse == 0) return o.cheb_degree;
    if (pr.beta < kSmallBeta * pr.alpha) return 32;
    return (pr.beta < kLargeBeta * pr.alpha) ? 16 : 8;
}

void create(cd_solver* s, const cd_problem* pr, const cd_options* op, void* stream) {
    validate(pr, op);
    s->prob = *pr;
    s->opt = *op;
    s->opt.cheb_degree_coarse = resolve_coarse_degree(*pr, *op);
    if (s->prob.dim == 2) s->prob.n[2] = 1;
    s->stream = static_cast<hipStream_t>(stream);
    if (!s->stream) {
        hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
        s->own_stream = true;
        hip_check(hipEventCreateWithFlags(&s->entry_event, hipEventDisableTiming), "hipEventCreate");
        enter(s);
    }
    s->d = pr->dim;
    s->p = pr->degree;
    s->ksteps = (op->krylov_steps < 0) ? pr->degree : op->krylov_steps;
    build_host(s);
    s->N = s->lv[0].N;
    hipStream_t st = s->stream;
    const int L = int(s->lv.size());
    for (int l = 0; l < L; ++l) {
        LevelDev<double> a;
        LevelDev<float> b;
        a.op = make_op<double>(s, s->lv[l], st);
        b.op = make_op<float>(s, s->lv[l], st);
        if (l < L - 1) {
            a.xf = make_xfer<double>(s, s->lv[l], st);
            b.xf = make_xfer<float>(s, s->lv[l], st);
        }
        s->ld64.push_back(a);
        s->ld32.push_back(b);
    }
    s->outer_op = s->ld64[0].op;
    s->outer_op.blockdiag = 0;  // the outer iteration always applies the system matrix
    for (int l = 0; l < s->d; ++l) {
        s->tfd64[l] = make_tfac<double>(s, s->tf[l], st);
        s->tfd32[l] = make_tfac<float>(s, s->tf[l], st);
    }
    // coarse level: dense operator, Cholesky factorization and inverse, all
    // on the GPU (FP64 MFMA); the factor workspace is released after setup
    {
        const int ld = cd::coarse_padded(s->Nc);
        s->ldK = ld;
        s->Kinv = s->arena.alloc<double>(size_t(ld) * ld);
        DevArena tmp;
        double* fac = tmp.alloc<double>(size_t(ld) * ld);
        int* flag = tmp.alloc<int>(1);
        hip_check(hipMemsetAsync(flag, 0, sizeof(int), st), "hipMemsetAsync");
        cd::launch_dense_operator(s->ld64.back().op, fac, ld, st);
        cd::coarse_inverse(fac, s->Nc, s->Kinv, flag, st);
        int hflag = 0;
        hip_check(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st), "read");
        hip_check(hipStreamSynchronize(st), "sync");
        if (hflag) throw CdError(CD_EINVAL, "coarse operator is not positive definite");
    }
    // outer vectors
    const size_t N = s->N;
    s->r = s->arena.alloc<double>(N);
    s->xw = s->arena.alloc<double>(N);
    s->z = s->arena.alloc<double>(N);
    s->dd = s->arena.alloc<double>(N);
    s->q = s->arena.alloc<double>(N);
    if (op->method == CD_METHOD_MIM) s->bw = s->arena.alloc<double>(N);
    s->nbr = cd::reduce_blocks(N);
    s->nba = cd::apply_blocks<double>(s->ld64[0].op);
    s->pzq = s->arena.alloc<double>(s->nbr);
    s->pdr = s->arena.alloc<double>(s->nbr);
    s->prr = s->arena.alloc<double>(s->nbr);
    s->pdq = s->arena.alloc<double>(std::max(s->nba, s->nbr));
    s->scal = s->arena.alloc<double>(6);
    void* hp = nullptr;
    hip_check(hipHostMalloc(&hp, 6 * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
    s->host_scal = static_cast<double*>(hp);
    if (L > 1 && op->method != CD_METHOD_CG) {
        if (op->eig_bounds == CD_BOUNDS_SYMBOL) symbol_bounds(s);
        estimate_bounds(s);
    }
    if (op->method != CD_METHOD_CG) {
        if (op->precision == CD_FP64) {
            s->w64 = make_work<double>(s, s->arena);
        } else {
            s->w32 = make_work<float>(s, s->arena);
        }
    }
    hip_check(hipStreamSynchronize(st), "sync");
}

// ---- the outer flexible CG as a resumable state machine ---------------------------
// begin: x = 0, r = b, ||r_0|| (one synchronisation); iterate: enqueue one
// outer iteration (preconditioner, direction, A d, updates) and an
// asynchronous read of (r.r, d.q) into pinned memory followed by an event;
// check: after the event completed, apply the stopping rule ||r_k||/||r_0|| <
// rtol of Sec. 6.2 and the breakdown test; finish: FP64 true residual.
void solve_begin(cd_solver* s, const double* b, double* x) {
    hipStream_t st = s->stream;
    const size_t N = s->N;
    SolveState& S = s->state;
    S = SolveState{};
    S.b = b;
    S.x = x;
    cd::launch_fill<double>(s->xw, 0.0, N, st);
    cd::launch_copy<double>(b, s->r, N, st);
    if (s->bw) cd::launch_copy<double>(b, s->bw, N, st);
    cd::launch_dot_partial<double, double>(s->r, s->r, N, s->prr, st);
    cd::launch_finalize(s->prr, s->nbr, s->scal, st);
    hip_check(hipMemcpyAsync(s->host_scal, s->scal, sizeof(double), hipMemcpyDeviceToHost, st), "read");
    hip_check(hipStreamSynchronize(st), "sync");
    const double rr0 = s->host_scal[0];
    if (!std::isfinite(rr0)) throw CdError(CD_EINVAL, "right-hand side is not finite");
    S.r0 = std::sqrt(rr0);
    S.rel = 1.0;
    S.status = (rr0 == 0.0) ? CD_OK : CD_NOT_CONVERGED;
    S.done = (rr0 == 0.0);
    if (!s->iter_event) hip_check(hipEventCreateWithFlags(&s->iter_event, hipEventDisableTiming), "hipEventCreate");
}

void enqueue_iteration(cd_solver* s, bool first) {
    hipStream_t st = s->stream;
    const size_t N = s->N;
    // z = B r, with the partial sums of z . q for the direction update fused in
    if (s->opt.method == CD_METHOD_CG) {
        if (first)
            cd::launch_copy<double>(s->r, s->z, N, st);
        else
            cd::launch_cast_dot<double, double>(s->r, s->z, N, s->q, s->pzq, st);
    } else {
        const bool dot = !first && s->opt.method != CD_METHOD_MIM;
        precondition(s, s->r, s->z, dot ? s->q : nullptr, s->pzq);
    }
    if (s->opt.method == CD_METHOD_MIM) {
        // stand-alone V-cycle: x += V(r), r = b - A x with its norm (scal[1] = 1: no curvature to test)
        cd::launch_axpby<double>(1.0, s->z, 1.0, s->xw, N, st);
        apply_with<double>(s, s->outer_op, 0, cd::kApplyResDot, s->xw, s->r, s->bw, nullptr, nullptr, 0.0, 0.0,
                           s->pdq);
        cd::launch_finalize(s->pdq, s->nba, s->scal, st);
        cd::launch_fill<double>(s->scal + 1, 1.0, 3, st);
        hip_check(hipMemcpyAsync(s->host_scal, s->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st), "read");
        return;
    }
    cd::launch_fcg_direction<double>(first, s->z, s->pzq, s->nbr, s->scal + 1, s->dd, s->r, s->pdr, s->scal + 3, N,
                                     st);
    apply_with<double>(s, s->outer_op, 0, kApplyYDot, s->dd, s->q, nullptr, nullptr, nullptr, 0.0, 0.0, s->pdq);
    cd::launch_fcg_update<double>(s->pdr, s->nbr, s->pdq, s->nba, s->scal + 1, s->xw, s->r, s->dd, s->q, s->prr,
                                  s->scal + 2, N, st);
    cd::launch_finalize(s->prr, s->nbr, s->scal, st);
    hip_check(hipMemcpyAsync(s->host_scal, s->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st), "read");
}

// Enqueue one outer iteration.  Every iteration after the first reads and
// writes the same solver-owned buffers with the same coefficients, so it is
// captured once into a HIP graph and replayed (no memset nodes: buffers are
// cleared by kernels).  With live timing enabled a second graph is captured
// whose operator applies are bracketed by external event-record nodes.
void solve_iterate(cd_solver* s) {
    hipStream_t st = s->stream;
    SolveState& S = s->state;
    const bool first = (S.k == 0);
    const bool timed = s->prof && (s->prof_iter++ % s->prof_period == 0);
    s->prof_sample = timed;
    auto enqueue = [&](bool f) {
        if (timed) prof_unit_begin(s);
        enqueue_iteration(s, f);
        if (timed) prof_unit_end(s);
    };
    if (first || !s->opt.graphs) {
        enqueue(first);
    } else {
        hipGraphExec_t& exec = timed ? s->iter_graph_prof : s->iter_graph;
        if (!exec) {
            hipGraph_t g = nullptr;
            hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            s->capturing = timed;
            try {
                enqueue(false);
            } catch (...) {
                s->capturing = false;
                s->unit_open = false;
                (void)hipStreamEndCapture(st, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            s->capturing = false;
            hip_check(hipStreamEndCapture(st, &g), "hipStreamEndCapture");
            if (!timed) {
                size_t nn = 0;
                if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess && nn > 0) {
                    std::vector<hipGraphNode_t> nodes(nn);
                    size_t nk = 0;
                    if (hipGraphGetNodes(g, nodes.data(), &nn) == hipSuccess) {
                        for (size_t i = 0; i < nn; ++i) {
                            hipGraphNodeType ty;
                            if (hipGraphNodeGetType(nodes[i], &ty) == hipSuccess && ty == hipGraphNodeTypeKernel) ++nk;
                        }
                        s->graph_nodes = nn;
                        s->graph_kernels = nk;
                    }
                }
            }
            const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            hip_check(e, "hipGraphInstantiate");
        }
        hip_check(hipGraphLaunch(exec, st), "hipGraphLaunch");
        if (timed) s->graph_prof_ran = true;
    }
    s->prof_sample = true;
    hip_check(hipEventRecord(s->iter_event, st), "hipEventRecord");
}

// Call after s->iter_event completed; returns true when the solve has ended.
bool solve_check(cd_solver* s) {
    SolveState& S = s->state;
    if (s->prof) prof_flush(s);
    ++S.k;
    const double rr = s->host_scal[0], dq = s->host_scal[1];
    if (s->opt.method != CD_METHOD_MIM) {
        S.alpha.push_back(s->host_scal[2]);
        S.beta.push_back(-s->host_scal[3]);  // d = z + beta_cg d_prev
    }
    S.rel = std::sqrt(rr) / S.r0;
    if (!std::isfinite(rr) || !std::isfinite(dq) || !(dq > 0.0)) {
        S.status = CD_EBREAKDOWN;
        S.done = true;
    } else if (S.rel < s->opt.rtol) {
        S.status = CD_OK;
        S.done = true;
    } else if (S.k >= s->opt.max_iter) {
        S.status = CD_NOT_CONVERGED;
        S.done = true;
    }
    return S.done;
}

cd_result solve_finish(cd_solver* s) {
    hipStream_t st = s->stream;
    const size_t N = s->N;
    SolveState& S = s->state;
    cd_result out{};
    out.status = S.status;
    out.iterations = S.k;
    out.rel_residual = (S.r0 > 0.0) ? S.rel : 0.0;
    cd::launch_copy<double>(s->xw, S.x, N, st);
    if (S.r0 > 0.0) {
        cd::launch_apply<double>(s->outer_op, kApplyRes, S.x, s->z, S.b, nullptr, nullptr, 0.0, 0.0, nullptr, st);
        cd::launch_dot_partial<double, double>(s->z, s->z, N, s->prr, st);
        cd::launch_finalize(s->prr, s->nbr, s->scal + 4, st);
        hip_check(hipMemcpyAsync(s->host_scal + 4, s->scal + 4, sizeof(double), hipMemcpyDeviceToHost, st), "read");
        hip_check(hipStreamSynchronize(st), "sync");
        out.true_rel_residual = std::sqrt(s->host_scal[4]) / S.r0;
        out.kappa_estimate = lanczos_kappa(S.alpha, S.beta);
    }
    return out;
}

void solve(cd_solver* s, const double* b, double* x, cd_result* res) {
    solve_begin(s, b, x);
    while (!s->state.done) {
        solve_iterate(s);
        hip_check(hipEventSynchronize(s->iter_event), "hipEventSynchronize");
        solve_check(s);
    }
    const cd_result out = solve_finish(s);
    if (res) *res = out;
    if (out.status == CD_EBREAKDOWN) throw CdError(CD_EBREAKDOWN, "Krylov breakdown (d^T A d <= 0 or non-finite)");
}

}  // namespace

// ================================== C ABI ==================================

namespace {
int run(const std::function<void()>& f) {
    try {
        f();
        return CD_OK;
    } catch (const CdError& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return CD_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return CD_EHIP;
    }
}

}  // namespace

extern "C" {

void cd_default_options(cd_options* o) {
    if (!o) return;
    o->method = CD_METHOD_PMIM;
    o->transfer = CD_XFER_KNOT;
    o->precision = CD_FP64;
    o->rtol = 1e-8;
    o->max_iter = 10000;
    o->coarse_max_dofs = 2500;
    o->cheb_degree = 48;
    o->cheb_ratio = 1000.0;
    o->lanczos_steps = 20;
    o->krylov_steps = -1;
    o->graphs = 1;
    o->cheb_degree_coarse = -1;
    o->apply_x1_chunk = 0;
    o->eig_bounds = CD_BOUNDS_LANCZOS;
    o->bound_safety = 0.0;
    o->apply3d_kernel = CD_APPLY3D_AUTO;
}

size_t cd_num_dofs(const cd_problem* pr) {
    if (!pr || (pr->dim != 2 && pr->dim != 3) || pr->degree < 1) return 0;
    size_t G = 1;
    for (int l = 0; l < pr->dim; ++l) {
        const int m = pr->n[l] + pr->degree - 2;
        if (pr->n[l] < 1 || m < 1) return 0;
        G *= size_t(m);
    }
    return size_t(pr->dim) * G;
}

int cd_validate(const cd_problem* pr, const cd_options* op) {
    return run([&] { validate(pr, op); });
}

size_t cd_footprint_bytes(const cd_problem* pr, const cd_options* op) {
    size_t total = 0;
    int rc = run([&] {
        validate(pr, op);
        cd_solver tmp;
        tmp.prob = *pr;
        tmp.opt = *op;
        tmp.d = pr->dim;
        tmp.p = pr->degree;
        tmp.ksteps = (op->krylov_steps < 0) ? pr->degree : op->krylov_steps;
        if (tmp.prob.dim == 2) tmp.prob.n[2] = 1;
        build_host(&tmp);
        const size_t N = tmp.lv[0].N;
        const size_t es = (op->precision == CD_FP64) ? 8 : 4;
        size_t vw = 0;
        for (size_t l = 0; l < tmp.lv.size(); ++l) vw += tmp.lv[l].N * ((l + 1 < tmp.lv.size()) ? 4 : 2);
        const size_t ks = size_t(std::max(tmp.ksteps, 1));
        vw += N * (2 * ks + 5);                             // V (ks+1), Z (ks), w, z, io_in, tmp
        total = (op->method == CD_METHOD_MIM ? 6 : 5) * N * 8  // outer r, z, d, q, iterate (MIM: and b)
                + (op->method != CD_METHOD_CG ? vw * es : 0)  // V-cycle workspace
                + 2 * size_t(cd::coarse_padded(tmp.Nc)) * cd::coarse_padded(tmp.Nc) * 8  // coarse inverse and,
                                                                       // during set-up, its factor
                + (op->method != CD_METHOD_CG ? 4 * N * 8 : 0)      // set-up: Lanczos vectors
                + (1 << 20);                                 // 1D tables and partial sums
    });
    return rc == CD_OK ? total : 0;
}

int cd_symbol_bound(const cd_problem* pr, const cd_options* op, int level, double* lam) {
    return run([&] {
        validate(pr, op);
        if (!lam) throw CdError(CD_EINVAL, "null output pointer");
        cd_solver tmp;
        tmp.prob = *pr;
        tmp.opt = *op;
        tmp.d = pr->dim;
        tmp.p = pr->degree;
        tmp.ksteps = (op->krylov_steps < 0) ? pr->degree : op->krylov_steps;
        if (tmp.prob.dim == 2) tmp.prob.n[2] = 1;
        build_host(&tmp);
        if (level < 0 || level + 1 >= int(tmp.lv.size())) throw CdError(CD_EINVAL, "level has no smoother");
        *lam = level_symbol_bound(&tmp, tmp.lv[level]);
    });
}

int cd_solver_create(const cd_problem* prob, const cd_options* opt, void* stream, cd_solver** out) {
    if (!out) {
        g_last_error = "null output pointer";
        return CD_EINVAL;
    }
    *out = nullptr;
    cd_solver* s = new (std::nothrow) cd_solver();
    if (!s) return CD_ENOMEM;
    const int rc = run([&] { create(s, prob, opt, stream); });
    if (rc != CD_OK) {
        cd_solver_destroy(s);
        return rc;
    }
    *out = s;
    return CD_OK;
}

void cd_solver_destroy(cd_solver* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->host_scal) (void)hipHostFree(s->host_scal);
    const bool own = s->own_stream;
    hipStream_t st = s->stream;
    delete s;
    if (own) (void)hipStreamDestroy(st);
}

int cd_solve(cd_solver* s, const double* b, double* x, cd_result* res) {
    if (res) std::memset(res, 0, sizeof(*res));
    int st = CD_OK;
    const int rc = run([&] {
        need(s);
        enter(s);
        if (!b || !x) throw CdError(CD_EINVAL, "null vector");
        cd_result r{};
        solve(s, b, x, &r);
        st = r.status;
        if (res) *res = r;
    });
    if (rc != CD_OK) {
        if (res) res->status = rc;
        return rc;
    }
    return st;
}

size_t cd_solver_device_bytes(const cd_solver* s) {
    if (!s) return 0;
    size_t b = s->arena.bytes + (s->hook_arena ? s->hook_arena->bytes : 0) + (s->hook_arena32 ? s->hook_arena32->bytes : 0);
    if (s->stamps) b += size_t(cd_solver::kStampSlots) * (cd::kStampWords + 2) * sizeof(unsigned long long);
    return b;
}

int cd_num_levels(const cd_solver* s) { return s ? int(s->lv.size()) : 0; }

int cd_level_shape(const cd_solver* s, int level, int* m3, size_t* ndofs) {
    return run([&] {
        need_level(s, level);
        if (m3)
            for (int l = 0; l < 3; ++l) m3[l] = s->lv[level].m[l];
        if (ndofs) *ndofs = s->lv[level].N;
    });
}

int cd_get_matrix(const cd_solver* s, int level, int axis, char which, double* out) {
    return run([&] {
        need_level(s, level);
        if (axis < 0 || axis >= s->d) throw CdError(CD_EINVAL, "axis out of range");
        if (!out) throw CdError(CD_EINVAL, "null output");
        const LevelHost& L = s->lv[level];
        const int m = L.m[axis];
        if (which == 'M' || which == 'A' || which == 'S') {
            const cd::Band& B = (which == 'M') ? L.M[axis] : (which == 'A') ? L.A[axis] : L.S[axis];
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) out[size_t(i) * m + j] = B.get(i, j);
        } else if (which == 'T') {
            if (level != 0) throw CdError(CD_EINVAL, "T exists on level 0 only");
            const cd::Band& B = s->tf[axis].T;
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) out[size_t(i) * m + j] = B.get(i, j);
        } else if (which == 'P') {
            if (level + 1 >= int(s->lv.size())) throw CdError(CD_EINVAL, "coarsest level has no prolongator");
            const cd::Prolong& P = L.P[axis];
            for (int i = 0; i < P.mf; ++i)
                for (int j = 0; j < P.mc; ++j) out[size_t(i) * P.mc + j] = P.get(i, j);
        } else {
            throw CdError(CD_EINVAL, "which must be one of M, A, S, T, P");
        }
    });
}

int cd_get_smoother(const cd_solver* s, int level, int* degree, double* lo, double* hi) {
    return run([&] {
        if (!s) throw CdError(CD_EINVAL, "null solver");
        if (level < 0 || level + 1 >= int(s->lv.size())) throw CdError(CD_EINVAL, "level has no smoother");
        if (degree) *degree = (level == 0) ? s->opt.cheb_degree : s->opt.cheb_degree_coarse;
        if (lo) *lo = s->lv[level].lo;
        if (hi) *hi = s->lv[level].hi;
    });
}

int cd_graph_launches(const cd_solver* s, size_t* kernels, size_t* nodes) {
    return run([&] {
        if (!s) throw CdError(CD_EINVAL, "null solver");
        if (kernels) *kernels = s->graph_kernels;
        if (nodes) *nodes = s->graph_nodes;
    });
}

int cd_get_lambda(const cd_solver* s, int level, double* lam) {
    return run([&] {
        need_level(s, level);
        if (level == int(s->lv.size()) - 1) throw CdError(CD_EINVAL, "coarsest level has no smoother");
        if (lam) *lam = s->lv[level].lam;
    });
}

int cd_apply(cd_solver* s, int level, const double* x, double* y) {
    return run([&] {
        need_level(s, level);
        enter(s);
        apply_op<double>(s, level, kApplyY, x, y, nullptr, nullptr, nullptr, 0.0, 0.0, nullptr);
        hip_check(hipStreamSynchronize(s->stream), "sync");
        if (s->prof) prof_flush(s);
    });
}

int cd_apply_f32(cd_solver* s, int level, const float* x, float* y) {
    return run([&] {
        need_level(s, level);
        enter(s);
        apply_op<float>(s, level, kApplyY, x, y, nullptr, nullptr, nullptr, 0.f, 0.f, nullptr);
        hip_check(hipStreamSynchronize(s->stream), "sync");
        if (s->prof) prof_flush(s);
    });
}

int cd_smooth(cd_solver* s, int level, const double* b, const double* x_in, double* x_out) {
    return run([&] { hook_smooth<double>(s, level, b, x_in, x_out); });
}
int cd_smooth_f32(cd_solver* s, int level, const float* b, const float* x_in, float* x_out) {
    return run([&] { hook_smooth<float>(s, level, b, x_in, x_out); });
}

int cd_restrict(cd_solver* s, int level, const double* rf, double* rc) {
    return run([&] { hook_transfer<double>(s, level, true, rf, rc); });
}
int cd_restrict_f32(cd_solver* s, int level, const float* rf, float* rc) {
    return run([&] { hook_transfer<float>(s, level, true, rf, rc); });
}

int cd_prolong_add(cd_solver* s, int level, const double* ec, double* xf) {
    return run([&] { hook_transfer<double>(s, level, false, ec, xf); });
}
int cd_prolong_add_f32(cd_solver* s, int level, const float* ec, float* xf) {
    return run([&] { hook_transfer<float>(s, level, false, ec, xf); });
}

int cd_tsolve(cd_solver* s, const double* v, double* z) {
    return run([&] {
        need(s);
        enter(s);
        // the outer vectors q and z are free outside a solve and serve as scratch
        const double* src = v;
        if (v == z) {
            cd::launch_copy<double>(v, s->z, s->N, s->stream);
            src = s->z;
        }
        tsolve_op<double>(s, src, s->q, z);
        hip_check(hipStreamSynchronize(s->stream), "sync");
        if (s->prof) prof_flush(s);
    });
}
int cd_tsolve_f32(cd_solver* s, const float* v, float* z) {
    return run([&] { hook_tsolve<float>(s, v, z); });
}

int cd_tsolve_noalloc(cd_solver* s, const double* v, double* z) {
    return run([&] {
        need(s);
        if (!v || !z) throw CdError(CD_EINVAL, "null vector");
        if (s->N > kNoAllocMaxDofs)
            throw CdError(CD_EINVAL, "cd_tsolve_noalloc: problem has " + std::to_string(s->N) +
                                         " unknowns, the static workspace holds at most " +
                                         std::to_string(kNoAllocMaxDofs));
        double* ws = noalloc_workspace();  // two vectors of kNoAllocMaxDofs doubles
        enter(s);
        const double* src = v;
        if (v == z) {  // in place: solve from a copy of v
            cd::launch_copy<double>(v, ws + kNoAllocMaxDofs, s->N, s->stream);
            src = ws + kNoAllocMaxDofs;
        }
        cd::launch_tsolve<double>(s->d, s->lv[0].m, s->tfd64, src, ws, z, s->stream);
        hip_check(hipStreamSynchronize(s->stream), "sync");
    });
}

namespace {
// Quadrature tables of the handle's axes on the device ((p+3)-point Gauss per element).
struct QuadSet {
    DevArena ar;
    cd::QuadDev ax[3]{};
};
void make_quad(cd_solver* s, QuadSet& Q) {
    const int q = s->p + 3;
    for (int l = 0; l < 3; ++l) {
        const int nl = (l < s->d) ? s->prob.n[l] : 1;
        const cd::QuadAxis A = cd::quad_axis(nl, s->p, l < s->d ? q : 1);
        cd::QuadDev& D = Q.ax[l];
        D.x = Q.ar.upload(A.x, s->stream);
        D.w = Q.ar.upload(A.w, s->stream);
        D.val = Q.ar.upload(A.val, s->stream);
        D.der = Q.ar.upload(A.der, s->stream);
        D.f0 = Q.ar.upload(A.f0, s->stream);
        D.n = A.n;
        D.p = A.p;
        D.q = A.q;
        D.m = A.m;
        D.Q = A.Q;
    }
}
}  // namespace

int cd_load_vector(cd_solver* s, double* b) {
    return run([&] {
        need(s);
        if (!b) throw CdError(CD_EINVAL, "null vector");
        enter(s);
        QuadSet Q;
        make_quad(s, Q);
        double* work = Q.ar.alloc<double>(cd::load_vector_work(s->d, Q.ax));
        cd::launch_load_vector(s->d, Q.ax, s->prob.alpha, s->prob.beta, b, work, s->stream);
        hip_check(hipStreamSynchronize(s->stream), "sync");
    });
}

int cd_l2_error(cd_solver* s, const double* x, double* err) {
    return run([&] {
        need(s);
        if (!x || !err) throw CdError(CD_EINVAL, "null argument");
        enter(s);
        QuadSet Q;
        make_quad(s, Q);
        double* work = Q.ar.alloc<double>(cd::l2_error_work(s->d, Q.ax));
        const int np = 1024;
        double* part = Q.ar.alloc<double>(np + 1);
        cd::launch_l2_error(s->d, Q.ax, x, work, part, np, s->stream);
        cd::launch_finalize(part, np, part + np, s->stream);
        double h = 0.0;
        hip_check(hipMemcpyAsync(&h, part + np, sizeof(double), hipMemcpyDeviceToHost, s->stream), "read");
        hip_check(hipStreamSynchronize(s->stream), "sync");
        *err = std::sqrt(h);
    });
}

int cd_coarse_solve(cd_solver* s, const double* r, double* z) {
    return run([&] {
        need(s);
        enter(s);
        cd::launch_coarse_gemv<double>(s->Kinv, s->Nc, s->ldK, r, z, s->stream);
        hip_check(hipStreamSynchronize(s->stream), "sync");
    });
}

int cd_precondition(cd_solver* s, const double* r, double* z) {
    return run([&] {
        need(s);
        enter(s);
        if (s->opt.method == CD_METHOD_CG) throw CdError(CD_EINVAL, "plain CG has no preconditioner");
        if (s->lv.size() == 1) {
            cd::launch_coarse_gemv<double>(s->Kinv, s->Nc, s->ldK, r, z, s->stream);
        } else {
            precondition(s, r, z);
        }
        hip_check(hipStreamSynchronize(s->stream), "sync");
    });
}

int cd_profile_enable(cd_solver* s, int on) {
    return run([&] {
        need(s);
        enter(s);
        hip_check(hipStreamSynchronize(s->stream), "sync");
        if (s->stamps) prof_flush(s);
        if (on > 0 && !s->stamps) {
            int dev = 0, khz = 0;
            hip_check(hipGetDevice(&dev), "hipGetDevice");
            hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
            if (khz <= 0) throw CdError(CD_EHIP, "device reports no wall-clock rate");
            s->wall_khz = double(khz);
            const size_t words = size_t(cd_solver::kStampSlots) * cd::kStampWords;
            const size_t pbytes = size_t(2 * cd_solver::kStampSlots) * sizeof(unsigned long long);
            hip_check(hipMalloc(&s->stamps, words * sizeof(unsigned long long)), "hipMalloc stamps");
            hip_check(hipMemsetAsync(s->stamps, 0, words * sizeof(unsigned long long), s->stream), "clear stamps");
            hip_check(hipMalloc(&s->pairs, pbytes), "hipMalloc stamps");
            hip_check(hipHostMalloc(&s->stamps_host, pbytes, hipHostMallocDefault), "hipHostMalloc stamps");
            hip_check(hipStreamSynchronize(s->stream), "sync");
        }
        s->prof = (on > 0);
        s->prof_period = std::max(on, 1);
        s->prof_iter = 0;
        if (s->prof) s->prof_stats.assign(kProfKinds * 2 * s->lv.size(), cd_kernel_stats{0, 0.0, 0.0});
    });
}

int cd_profile_read(const cd_solver* s, int level, int fp32, cd_kernel_stats* out) {
    return run([&] {
        need_level(s, level);
        if (!out) throw CdError(CD_EINVAL, "null output");
        cd_kernel_stats t{0, 0.0, 0.0};
        for (int kind : {0, 2}) {  // every operator apply of the level: other modes and Chebyshev steps
            const size_t k = size_t(prof_class(s, kind, level, fp32 != 0));
            if (k < s->prof_stats.size()) {
                t.launches += s->prof_stats[k].launches;
                t.total_ms += s->prof_stats[k].total_ms;
                t.bytes += s->prof_stats[k].bytes;
            }
        }
        *out = t;
    });
}
int cd_profile_read_smoother(const cd_solver* s, int level, int fp32, cd_kernel_stats* out) {
    return run([&] {
        need_level(s, level);
        if (!out) throw CdError(CD_EINVAL, "null output");
        const size_t k = size_t(prof_class(s, 2, level, fp32 != 0));
        *out = (k < s->prof_stats.size()) ? s->prof_stats[k] : cd_kernel_stats{0, 0.0, 0.0};
    });
}

int cd_profile_read_tsolve(const cd_solver* s, int fp32, cd_kernel_stats* out) {
    return run([&] {
        need(s);
        if (!out) throw CdError(CD_EINVAL, "null output");
        const size_t k = size_t(prof_class(s, 1, 0, fp32 != 0));
        *out = (k < s->prof_stats.size()) ? s->prof_stats[k] : cd_kernel_stats{0, 0.0, 0.0};
    });
}

// =============================== serving loop ===============================
struct cd_server {
    cd_server_options opt{};
    std::vector<hipStream_t> streams;  // num_streams > 0: a fixed pool shared round robin
    std::vector<hipStream_t> free_streams;  // num_streams == 0: one stream per active solve, reused
    int streams_made = 0;
    struct Req {
        uint64_t ticket = 0;
        cd_problem prob{};
        cd_options opt{};
        const double* b = nullptr;
        double* x = nullptr;
        size_t fp = 0;
        double t_submit = 0, t_admit = 0;
        cd_solver* solver = nullptr;
        hipStream_t stream = nullptr;
        bool own_stream = false;
        int setup_rc = CD_OK;        // result of the set-up on the worker
        cd_result early{};          // the result when the set-up already finished the solve
        bool finished_early = false;
        bool in_flight = false;     // an outer iteration is enqueued
    };
    std::deque<std::unique_ptr<Req>> queue;       // submitted, not admitted
    std::vector<std::unique_ptr<Req>> iterating;  // set up, iterating
    std::deque<cd_completion> done;
    size_t used = 0;  // footprint of the admitted requests
    int in_setup = 0;
    uint64_t next_ticket = 1;
    uint64_t admitted = 0;
    std::chrono::steady_clock::time_point t0;
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    // Set-up worker: creates the solvers of admitted requests (host set-up,
    // uploads, coarse factorisation, eigenvalue bounds, first residual) and
    // destroys retired ones, on its own thread, so that the scheduling thread
    // keeps the running solves fed meanwhile.
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req*> setup_todo;
    std::deque<Req*> setup_done;
    std::deque<cd_solver*> destroy_todo;
    bool stop = false;

    void work() {
        for (;;) {
            Req* r = nullptr;
            cd_solver* dead = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !setup_todo.empty() || !destroy_todo.empty(); });
                if (!destroy_todo.empty()) {
                    dead = destroy_todo.front();
                    destroy_todo.pop_front();
                } else if (!setup_todo.empty()) {
                    r = setup_todo.front();
                    setup_todo.pop_front();
                } else {
                    return;  // stop requested and nothing left
                }
            }
            if (dead) {
                cd_solver_destroy(dead);
                continue;
            }
            cd_solver* h = nullptr;
            r->setup_rc = cd_solver_create(&r->prob, &r->opt, r->stream, &h);
            if (r->setup_rc == CD_OK) {
                r->solver = h;
                r->setup_rc = run([&] {
                    solve_begin(h, r->b, r->x);
                    if (h->state.done) {  // zero right-hand side: x = 0
                        r->early = solve_finish(h);
                        r->finished_early = true;
                    }
                });
            }
            std::lock_guard<std::mutex> lk(mu);
            setup_done.push_back(r);
        }
    }

    ~cd_server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        if (worker.joinable()) worker.join();
        for (auto& r : iterating)
            if (r->solver) cd_solver_destroy(r->solver);
        for (Req* r : setup_done) {  // the worker has drained its queues before it returned
            if (r->solver) cd_solver_destroy(r->solver);
            delete r;
        }
        for (hipStream_t st : streams) (void)hipStreamDestroy(st);
        for (hipStream_t st : free_streams) (void)hipStreamDestroy(st);
    }
};

namespace {
void server_complete(cd_server* srv, const cd_server::Req& r, const cd_result& res) {
    cd_completion c{};
    c.ticket = r.ticket;
    c.result = res;
    c.t_submit = r.t_submit;
    c.t_admit = r.t_admit;
    c.t_done = srv->now();
    c.footprint_bytes = r.fp;
    srv->done.push_back(c);
}

hipStream_t server_take_stream(cd_server* srv, bool* own) {
    if (!srv->streams.empty()) {
        *own = false;
        return srv->streams[srv->admitted % srv->streams.size()];
    }
    *own = true;
    if (!srv->free_streams.empty()) {
        hipStream_t st = srv->free_streams.back();
        srv->free_streams.pop_back();
        return st;
    }
    hipStream_t st = nullptr;
    hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    ++srv->streams_made;
    return st;
}

// Give a request's resources back (its solver goes to the worker for destruction).
void server_release(cd_server* srv, cd_server::Req& r) {
    if (r.solver) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->destroy_todo.push_back(r.solver);
        }
        srv->cv.notify_one();
        r.solver = nullptr;
    }
    if (r.own_stream && r.stream) srv->free_streams.push_back(r.stream);
    r.stream = nullptr;
    srv->used -= r.fp;
}
}  // namespace

void cd_server_default_options(cd_server_options* o) {
    if (!o) return;
    o->hbm_budget_bytes = 0;
    o->max_active = 64;
    o->num_streams = 0;
}

int cd_server_create(const cd_server_options* opt, cd_server** out) {
    if (!out) {
        g_last_error = "null output pointer";
        return CD_EINVAL;
    }
    *out = nullptr;
    cd_server* srv = new (std::nothrow) cd_server();
    if (!srv) return CD_ENOMEM;
    const int rc = run([&] {
        cd_server_options o;
        cd_server_default_options(&o);
        if (opt) o = *opt;
        if (o.max_active <= 0) o.max_active = 64;
        if (o.num_streams < 0 || o.num_streams > 64) throw CdError(CD_EINVAL, "num_streams must be in 0..64");
        if (o.hbm_budget_bytes == 0) {
            size_t fr = 0, tot = 0;
            hip_check(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
            o.hbm_budget_bytes = size_t(0.8 * double(fr));
        }
        srv->opt = o;
        for (int i = 0; i < o.num_streams; ++i) {
            hipStream_t st = nullptr;
            hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
            srv->streams.push_back(st);
        }
        srv->t0 = std::chrono::steady_clock::now();
        srv->worker = std::thread([srv] { srv->work(); });
    });
    if (rc != CD_OK) {
        delete srv;
        return rc;
    }
    *out = srv;
    return CD_OK;
}

int cd_server_submit(cd_server* srv, const cd_problem* prob, const cd_options* opt, const double* b, double* x,
                     uint64_t* ticket) {
    return run([&] {
        if (!srv) throw CdError(CD_EINVAL, "null server");
        if (!b || !x) throw CdError(CD_EINVAL, "null vector");
        validate(prob, opt);
        const size_t fp = cd_footprint_bytes(prob, opt);
        if (fp == 0 || fp > srv->opt.hbm_budget_bytes) throw CdError(CD_ENOMEM, "request larger than the server's HBM budget");
        auto r = std::make_unique<cd_server::Req>();
        r->ticket = srv->next_ticket++;
        r->prob = *prob;
        r->opt = *opt;
        r->b = b;
        r->x = x;
        r->fp = fp;
        r->t_submit = srv->now();
        if (ticket) *ticket = r->ticket;
        srv->queue.push_back(std::move(r));
    });
}

int cd_server_step(cd_server* srv, int* n_active, int* n_queued) {
    return run([&] {
        if (!srv) throw CdError(CD_EINVAL, "null server");
        bool progress = false;
        // 1. solvers the worker has set up: start iterating (or complete)
        std::deque<cd_server::Req*> ready;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            ready.swap(srv->setup_done);
        }
        for (cd_server::Req* rp : ready) {
            std::unique_ptr<cd_server::Req> r(rp);
            --srv->in_setup;
            progress = true;
            if (r->setup_rc == CD_ENOMEM && r->solver == nullptr &&
                (!srv->iterating.empty() || srv->in_setup > 0)) {
                // the device could not hold it next to the running solves: back to
                // the head of the queue, admitted again when they have retired
                server_release(srv, *r);
                srv->queue.push_front(std::move(r));
                continue;
            }
            if (r->setup_rc != CD_OK || r->finished_early) {
                cd_result res = r->early;
                if (r->setup_rc != CD_OK) res.status = r->setup_rc;
                server_complete(srv, *r, res);
                server_release(srv, *r);
                continue;
            }
            solve_iterate(r->solver);
            r->in_flight = true;
            srv->iterating.push_back(std::move(r));
        }
        // 2. admission: FIFO, by footprint and slot count; the set-up runs on the worker
        while (!srv->queue.empty() && int(srv->iterating.size()) + srv->in_setup < srv->opt.max_active &&
               srv->used + srv->queue.front()->fp <= srv->opt.hbm_budget_bytes) {
            std::unique_ptr<cd_server::Req> r = std::move(srv->queue.front());
            srv->queue.pop_front();
            r->t_admit = srv->now();
            r->stream = server_take_stream(srv, &r->own_stream);
            ++srv->admitted;
            srv->used += r->fp;
            ++srv->in_setup;
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->setup_todo.push_back(r.release());
            }
            srv->cv.notify_one();
            progress = true;
        }
        // 3. every solve whose last outer iteration has finished: stopping test,
        //    then retire it or enqueue its next iteration; the others keep running
        auto pass = [&] {
            bool any = false;
            std::vector<std::unique_ptr<cd_server::Req>> keep;
            keep.reserve(srv->iterating.size());
            for (auto& r : srv->iterating) {
                const hipError_t q = hipEventQuery(r->solver->iter_event);
                if (q == hipErrorNotReady) {
                    keep.push_back(std::move(r));
                    continue;
                }
                hip_check(q, "hipEventQuery");
                any = true;
                if (solve_check(r->solver)) {
                    const cd_result res = solve_finish(r->solver);
                    server_complete(srv, *r, res);
                    server_release(srv, *r);
                } else {
                    solve_iterate(r->solver);
                    keep.push_back(std::move(r));
                }
            }
            srv->iterating.swap(keep);
            return any;
        };
        progress = pass() || progress;
        // nothing changed: wait briefly for the next iteration or set-up to finish
        for (int spin = 0; !progress && spin < 200 && (!srv->iterating.empty() || srv->in_setup > 0); ++spin) {
            std::this_thread::sleep_for(std::chrono::microseconds(5));
            progress = pass();
            if (!progress) {
                std::lock_guard<std::mutex> lk(srv->mu);
                progress = !srv->setup_done.empty();
            }
        }
        if (n_active) *n_active = int(srv->iterating.size()) + srv->in_setup;
        if (n_queued) *n_queued = int(srv->queue.size());
    });
}

int cd_server_poll(cd_server* srv, cd_completion* out, int max, int* n_out) {
    return run([&] {
        if (!srv) throw CdError(CD_EINVAL, "null server");
        int n = 0;
        while (n < max && !srv->done.empty()) {
            if (out) out[n] = srv->done.front();
            srv->done.pop_front();
            ++n;
        }
        if (n_out) *n_out = n;
    });
}

void cd_server_destroy(cd_server* srv) { delete srv; }

const char* cd_status_string(int st) {
    switch (st) {
        case CD_OK: return "converged";
        case CD_NOT_CONVERGED: return "maximum number of iterations reached";
        case CD_EINVAL: return "invalid argument";
        case CD_ENOMEM: return "out of memory";
        case CD_EBREAKDOWN: return "Krylov breakdown";
        case CD_EHIP: return "HIP runtime error";
        case CD_EAGAIN: return "request queued";
        case CD_ENOTFOUND: return "unknown ticket";
        default: return "unknown status";
    }
}

const char* cd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
