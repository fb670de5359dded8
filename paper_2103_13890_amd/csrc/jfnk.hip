// libjfnk host side: context and workspace, multigrid setup (projection of
// the Newton iterate, level caches, power method), the V-cycle of
// Algorithm 1, flexible GMRES with two-pass classical Gram-Schmidt, the
// inexact Newton iteration with cubic backtracking (Sec. 3, setup), the
// adjoint solve, and the C entry points declared in include/libjfnk.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "ops.hpp"

using namespace jfnk;

namespace {

// A named range on the profiler's marker trace (rocprofv3 --marker-trace):
// the solve, each Newton step, the multigrid setup, the outer Krylov solve,
// each V-cycle, the line search and the adjoint solve.  Host-side only; a
// push and a pop per range.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

constexpr int NSLOT = 1024;
constexpr size_t PART_CAP = 4096 * 32;    // partial sums (blocks x sums)
constexpr int MAXR = 32;                  // restart cap (Gram-Schmidt slots)

// device scalar slots
enum {
    S_FN2 = 0, S_FT2, S_ENER, S_BU, S_NUM64, S_ZN2, S_XN2, S_W2, S_EPS, S_SLOPE, S_DOT, S_RN2,
    S_COARSE = 16,          // 8 coarse statistics
    S_COEF = 32,            // 96: Gram-Schmidt coefficients of one Krylov step
    S_LEV = 128,            // 16 per level
};
// per-level slots; L_PQ, L_PQB, L_PQC: rotating (Rayleigh quotient, ||q||^2)
// pairs of the power iterations in flight
enum { L_NUM = 0, L_D0, L_D1, L_S, L_B, L_PQ, L_PQ2, L_V, L_T, L_PQB, L_PQB2, L_PQC, L_PQC2 };

struct Level {
    Grid g;
    void *x, *Ax, *kap, *b, *s, *r, *d[2], *t, *eig, *q, *cw;
    double lam;
    int power_iters;
};

struct TimerRec {
    bool on = false;
    std::vector<hipEvent_t> ev;
    size_t used = 0;
};

}  // namespace

struct jfnk_ctx {
    jfnk_problem prob;
    jfnk_options opt;
    Phys ph;
    int nc = 1, L = 0, vprec = JFNK_F64;
    Level lev[JFNK_MAX_LEVELS];
    hipStream_t st = nullptr;
    Exec ex;
    double *scal = nullptr, *part = nullptr;
    double *lazy_part = nullptr;   // partial buffers of the deferred slots
    LazyTable lazy;
    // finest level, FP64
    long long nn = 0, n = 0;
    long long ldv = 0;   // column stride of the Krylov bases V and Z: n rounded up to 64 entries
    double *u = nullptr, *ut = nullptr, *Au = nullptr, *Aut = nullptr, *F = nullptr, *Ft = nullptr;
    double *dx = nullptr, *w = nullptr, *V = nullptr, *bm = nullptr, *kap64 = nullptr;
    double *tmpA = nullptr, *tmpB = nullptr, *lamv = nullptr, *mf = nullptr;
    void *Z = nullptr;
    bool have_eigs = false, setup_done = false;
    double ge[JFNK_MAX_LEVELS];
    std::string err;
    TimerRec timers[JFNK_TIMER_COUNT];
    hipEvent_t t0 = nullptr, t1 = nullptr;
    // coarse L-BFGS preconditioner (CG-QN): recorded steps, kept pairs, state
    void *qn_rec = nullptr, *qn_pairs = nullptr;
    double *qn_state = nullptr;
    int qn_cap = 0;
    // pinned host copies of the power method's slot pairs, one event each
    double *hpin = nullptr;
    hipEvent_t pev[3] = {nullptr, nullptr, nullptr};
};

// Scratch of jfnk_residual_static (below): 128 KB of per-block partial sums.
constexpr long long STATIC_SCRATCH_DOUBLES = 16384;
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

namespace {

thread_local std::string g_err;

jfnk_status fail(jfnk_ctx *c, jfnk_status s, const std::string &msg) {
    if (c) c->err = msg;
    else g_err = msg;
    return s;
}

#define HIPCHK(c, call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return fail((c), JFNK_E_DEVICE, std::string(#call) + ": " + \
                                                              hipGetErrorString(e_));     \
    } while (0)

size_t esize(int prec) { return prec == JFNK_F32 ? 4 : 8; }

Grid level_grid(const jfnk_problem &p, int l) {
    Grid g;
    const int sh = p.nlevels - 1 - l;
    g.dim = p.dim;
    g.nx = p.n[0] >> sh;
    g.ny = p.n[1] >> sh;
    g.nz = p.dim == 3 ? (p.n[2] >> sh) : 0;
    g.NX = g.nx + 1;
    g.NY = g.ny + 1;
    g.NZ = p.dim == 3 ? g.nz + 1 : 1;
    g.nn = (long long)g.NX * g.NY * g.NZ;
    g.h = p.h * (double)(1LL << sh);
    g.dir = p.dirichlet;
    g.rNX = 1.0 / g.NX;
    g.rNY = 1.0 / g.NY;
    return g;
}

long long level_dofs(const Grid &g, int nc) {
    long long nx = g.NX, ny = g.NY, nz = g.NZ;
    if (g.dir & JFNK_FACE_XLO) nx--;
    if (g.dir & JFNK_FACE_XHI) nx--;
    if (g.dir & JFNK_FACE_YLO) ny--;
    if (g.dir & JFNK_FACE_YHI) ny--;
    if (g.dim == 3) {
        if (g.dir & JFNK_FACE_ZLO) nz--;
        if (g.dir & JFNK_FACE_ZHI) nz--;
    }
    return std::max(0LL, nx) * std::max(0LL, ny) * std::max(0LL, nz) * nc;
}

std::string validate_problem(const jfnk_problem *p) {
    if (!p) return "null problem";
    if (p->kind < JFNK_BRATU || p->kind > JFNK_PLAP_GAUSS) return "unknown problem kind";
    if (p->dim != 2 && p->dim != 3) return "dim must be 2 or 3";
    if (p->kind == JFNK_NEOHOOKE && p->dim != 3) return "NEOHOOKE needs dim 3";
    if (p->nlevels < 1 || p->nlevels > JFNK_MAX_LEVELS) return "nlevels out of range";
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return "h must be positive";
    for (int k = 0; k < p->dim; ++k) {
        if (p->n[k] < 1) return "element counts must be >= 1";
        if (p->n[k] % (1 << (p->nlevels - 1))) return "element counts must be divisible by 2^(nlevels-1)";
        if ((p->n[k] >> (p->nlevels - 1)) < 1) return "coarsest grid is empty";
    }
    long long nn = (long long)(p->n[0] + 1) * (p->n[1] + 1) * (p->dim == 3 ? p->n[2] + 1 : 1);
    if (nn > (1LL << 31) - 1) return "grid too large for 32-bit node indices";
    if ((p->kind == JFNK_PLAP || p->kind == JFNK_PLAP_GAUSS) && !(p->param[0] >= 1.0)) return "PLAP needs p >= 1";
    if (p->kind == JFNK_NEOHOOKE && !(p->param[0] > 0.0 && p->param[1] > -1.0 && p->param[1] < 0.5))
        return "NEOHOOKE needs E > 0 and -1 < nu < 0.5";
    return "";
}

std::string validate(const jfnk_problem *p, const jfnk_options *o) {
    if (!p || !o) return "null problem or options";
    const std::string vp = validate_problem(p);
    if (!vp.empty()) return vp;
    if (o->restart < 1 || o->restart > MAXR - 1) return "restart must be in [1, 31]";
    if (o->coarse_qn < 0 || o->coarse_qn > QN_MAX) return "coarse_qn must be in [0, 32]";
    if (o->nu_pre < 0 || o->nu_post < 0) return "smoothing degrees must be >= 0";
    if (o->vcycle_prec != JFNK_F32 && o->vcycle_prec != JFNK_F64) return "vcycle_prec must be F32 or F64";
    if (o->eps_mode != JFNK_EPS_NORM && o->eps_mode != JFNK_EPS_PAPER) return "unknown eps_mode";
    if (!(o->cheb_hi > o->cheb_lo) || !(o->cheb_lo > 0.0)) return "need 0 < cheb_lo < cheb_hi";
    if (o->power_maxit < 1) return "power_maxit must be >= 1";
    if (o->fd_form < 0 || o->fd_form > 2) return "fd_form must be 0, 1 or 2";
    if (o->kernel_path < 0 || o->kernel_path > 2) return "kernel_path must be 0, 1 or 2";
    if (o->outer_krylov != JFNK_OUTER_FGMRES && o->outer_krylov != JFNK_OUTER_CG)
        return "outer_krylov must be FGMRES or CG";
    if (o->newton_maxit < 0 || o->max_cycles < 1 || o->ls_maxit < 1) return "iteration caps must be positive";
    if (!(o->armijo > 0.0 && o->armijo < 1.0)) return "need 0 < armijo < 1";
    Grid g0 = level_grid(*p, 0);
    if (g0.nn > coarse_max_nodes()) return "coarsest grid too large for the coarse solver: add levels";
    return "";
}

// Workspace plan: a bump allocator over the caller's buffer (or a dry run).
struct Carve {
    char *base;
    size_t off = 0;
    void *take(size_t bytes) {
        off = (off + 255) & ~size_t(255);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

void plan(jfnk_ctx *c, Carve &cv) {
    const int nc = c->nc;
    const size_t es = esize(c->vprec);
    c->scal = (double *)cv.take(NSLOT * sizeof(double));
    c->part = (double *)cv.take(PART_CAP * sizeof(double));
    c->lazy_part = (double *)cv.take((size_t)(4 * c->prob.nlevels + 1) * LAZY_CAP * sizeof(double));
    for (int l = 0; l < c->prob.nlevels; ++l) {
        Level &L = c->lev[l];
        L.g = level_grid(c->prob, l);
        const size_t vb = (size_t)L.g.nn * nc * es;
        L.x = cv.take(vb);
        L.Ax = cv.take(vb);
        L.kap = c->prob.kind == JFNK_INVCOEF ? cv.take((size_t)L.g.nn * es) : nullptr;
        L.b = cv.take(vb);
        L.s = cv.take(vb);
        L.r = cv.take(vb);
        L.d[0] = cv.take(vb);
        L.d[1] = cv.take(vb);
        L.t = cv.take(vb);
        L.eig = cv.take(vb);
        L.q = cv.take(vb);
        // coarse solver: r, p, q, z and the per-element contributions
        L.cw = l == 0 ? cv.take(coarse_work_elems(L.g, nc) * es) : nullptr;
    }
    if (c->opt.coarse_qn > 0) {
        const Grid &g0 = c->lev[0].g;
        const size_t vb0 = (size_t)g0.nn * nc * es;
        c->qn_cap = c->opt.coarse_maxit > 0 ? c->opt.coarse_maxit : (int)level_dofs(g0, nc);
        c->qn_rec = cv.take(2 * (size_t)c->qn_cap * vb0);
        c->qn_pairs = cv.take(2 * (size_t)c->opt.coarse_qn * vb0);
        c->qn_state = (double *)cv.take(QN_STATE_LEN * sizeof(double));
    }
    const Grid gf = level_grid(c->prob, c->prob.nlevels - 1);
    c->nn = gf.nn;
    c->n = gf.nn * nc;
    const size_t fb = (size_t)c->n * sizeof(double);
    c->u = (double *)cv.take(fb);
    c->ut = (double *)cv.take(fb);
    c->Au = (double *)cv.take(fb);
    c->Aut = (double *)cv.take(fb);
    c->F = (double *)cv.take(fb);
    c->Ft = (double *)cv.take(fb);
    c->dx = (double *)cv.take(fb);
    c->w = (double *)cv.take(fb);
    c->bm = (double *)cv.take(fb);
    c->lamv = (double *)cv.take(fb);
    c->tmpA = (double *)cv.take(fb);
    c->tmpB = (double *)cv.take(fb);
    c->kap64 = c->prob.kind == JFNK_INVCOEF ? (double *)cv.take((size_t)gf.nn * sizeof(double)) : nullptr;
    c->mf = c->prob.kind == JFNK_INVCOEF ? (double *)cv.take((size_t)gf.nn * sizeof(double)) : nullptr;
    // basis columns start on 512-byte boundaries (the Gram-Schmidt and
    // combine kernels then read two adjacent entries per 16-byte access)
    c->ldv = (c->n + 63) / 64 * 64;
    c->V = (double *)cv.take((size_t)c->ldv * sizeof(double) * (c->opt.restart + 1));
    c->Z = cv.take((size_t)c->ldv * es * c->opt.restart);
}

Phys make_phys(const jfnk_problem &p) {
    Phys ph;
    ph.kind = p.kind;
    ph.ncomp = p.kind == JFNK_NEOHOOKE ? 3 : 1;
    ph.a0 = p.param[0];
    ph.a1 = p.param[1];
    if (p.kind == JFNK_NEOHOOKE) {   // Lame parameters from E, nu (Sec. 3, hyperelasticity)
        const double E = p.param[0], nu = p.param[1];
        ph.a0 = E / (2.0 * (1.0 + nu));
        ph.a1 = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    }
    return ph;
}

double *slot(jfnk_ctx *c, int i) { return c->scal + i; }
double *lslot(jfnk_ctx *c, int l, int k) { return c->scal + S_LEV + 16 * l + k; }

jfnk_status read_slots(jfnk_ctx *c, int first, int count, double *out) {
    for (int i = first; i < first + count; ++i) materialize(c->ex, c->scal + i);
    HIPCHK(c, hipMemcpyAsync(out, c->scal + first, count * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return JFNK_OK;
}

jfnk_status check_launch(jfnk_ctx *c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, JFNK_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return JFNK_OK;
}

#define CHK(expr)                        \
    do {                                 \
        jfnk_status s_ = (expr);         \
        if (s_ != JFNK_OK) return s_;    \
    } while (0)

// event timers around launches of one kernel class
struct TimeScope {
    jfnk_ctx *c;
    TimerRec *t;
    size_t k;
    // main_only: the end event is taken right after the stencil kernel,
    // before its reduction finish (see Exec::mark_main_end); otherwise at
    // the end of the scope
    TimeScope(jfnk_ctx *c_, int which, bool main_only = true) : c(c_), t(nullptr), k(0), main(main_only) {
        if (which >= 0 && which < JFNK_TIMER_COUNT) t = &c_->timers[which];
        if (t && t->on && t->used + 2 <= t->ev.size()) {
            k = t->used;
            t->used += 2;
            (void)hipEventRecord(t->ev[k], c->st);
            if (main) c->ex.ev_main_end = t->ev[k + 1];
        } else {
            t = nullptr;
        }
    }
    ~TimeScope() {
        if (!t) return;
        if (!main) (void)hipEventRecord(t->ev[k + 1], c->st);
        else if (c->ex.ev_main_end == t->ev[k + 1]) c->ex.mark_main_end();   // not consumed by a stencil launch
    }
    bool main;
};

template <typename T> T *P(void *p) { return (T *)p; }
template <typename T> const T *CP(const void *p) { return (const T *)p; }

// FD evaluation forms: the multigrid levels and the outer FP64 operator
int mg_mode(const jfnk_ctx *c) { return c->opt.fd_form == 1 ? M_FD_PLAIN : M_FD_DIFF; }
int outer_mode(const jfnk_ctx *c) { return c->opt.fd_form == 2 ? M_FD_DIFF : M_FD_PLAIN; }

// root of the FD step (Sec. 1: sqrt of the machine precision).  The
// two-evaluation quotient loses about root^2 / root = root of its digits to
// cancellation, so it needs the root of the precision it is evaluated in.
// The difference form cancels nothing, so its step is taken with the FP64
// root on every level: an FP32 level then evaluates the quotient for a step
// small enough to stay in the linear regime of the residual, where a step
// of sqrt(2^-23) (1 + ||x||) / ||v|| can move a localised direction far
// into the nonlinear range of the coefficient.
double root_eps(jfnk_ctx *c, int prec, int mode = M_FD_PLAIN) {
    if (c->opt.fd_root > 0.0) return c->opt.fd_root;
    if (mode == M_FD_DIFF) return Prec<double>::root_eps;
    return prec == JFNK_F32 ? Prec<float>::root_eps : Prec<double>::root_eps;
}

// ---------------------------------------------------------------------------
// multigrid setup (Sec. 2): projection, level caches, power method
// ---------------------------------------------------------------------------
// Iterations of the power method queued before the host has tested the
// previous ones.  On small levels an iteration takes less GPU time than the
// host's round trip, which is then hidden; an iteration queued past the
// stopping point is discarded and changes no result.  On large levels one
// extra evaluation costs more than the round trip saves.
inline int power_lookahead(long long n) { return n >= (1LL << 23) ? 0 : (n >= (1LL << 20) ? 1 : 2); }

template <typename T> jfnk_status power_method(jfnk_ctx *c, int l) {
    Level &L = c->lev[l];
    const Grid &g = L.g;
    const int nc = c->nc;
    // Iteration k reads buf[(k-1) % 4] (k = 1: the start vector, in L.eig),
    // writes its unnormalised image q_k = J(v_{k-1}/||v_{k-1}||) to
    // buf[k % 4] and (v^T q, ||q_k||^2) to the slot pair pq[k % 3].  With at
    // most two iterations queued beyond the one under test, neither its input
    // nor its output is overwritten before the host has decided.
    T *buf[4] = {P<T>(L.eig), P<T>(L.q), P<T>(L.t), P<T>(L.d[0])};
    const int pq[3] = {L_PQ, L_PQB, L_PQC};
    if (!c->have_eigs) vec_random<T>(c->ex, g, nc, c->opt.seed, l, buf[0], lslot(c, l, L_V));
    else vec_dot<T, T>(c->ex, g.nn * nc, buf[0], buf[0], lslot(c, l, L_V));
    const int maxit = c->opt.power_maxit;
    const int ahead = power_lookahead(g.nn * nc);
    int queued = 0;
    auto queue = [&](int k) -> jfnk_status {
        const double *n2 = k == 1 ? lslot(c, l, L_V) : lslot(c, l, pq[(k - 1) % 3] + 1);
        double *out = lslot(c, l, pq[k % 3]);
        op_power<T>(c->ex, mg_mode(c), g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), buf[(k - 1) % 4],
                    lslot(c, l, L_NUM), n2, buf[k % 4], out);
        CHK(check_launch(c));
        HIPCHK(c, hipMemcpyAsync(c->hpin + 2 * (k % 3), out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipEventRecord(c->pev[k % 3], c->st));
        queued = k;
        return JFNK_OK;
    };
    double lam = 0.0, lam_prev = 0.0;
    double n2_in = 0.0, n2_fin = 0.0;   // ||q||^2 of the input of iteration it / of the final image
    int it = 0, fin = 0;                // fin: the iteration whose image is the eigenvector
    bool zero = false;
    for (it = 1; it <= maxit; ++it) {
        while (queued < maxit && queued < it + ahead) CHK(queue(queued + 1));
        HIPCHK(c, hipEventSynchronize(c->pev[it % 3]));
        const double q_dot = c->hpin[2 * (it % 3)], q_n2 = c->hpin[2 * (it % 3) + 1];
        c->ge[l] += 1;
        lam = q_dot;
        if (!(q_n2 > 0.0)) {       // J v = 0: keep v
            zero = true;
            break;
        }
        fin = it;
        n2_fin = q_n2;
        if (!c->opt.power_fixed && it > 1 && std::fabs(lam - lam_prev) < c->opt.power_rtol * std::fabs(lam)) break;
        lam_prev = lam;
        n2_in = q_n2;
    }
    // the eigenvector estimate, normalised, into L.eig
    if (zero && it == 1) vec_scale<T>(c->ex, g, nc, buf[0], buf[0], 1.0, lslot(c, l, L_V), nullptr);
    else if (zero) vec_scale<T>(c->ex, g, nc, buf[(it - 1) % 4], buf[0], 1.0 / std::sqrt(n2_in), nullptr, nullptr);
    else vec_scale<T>(c->ex, g, nc, buf[fin % 4], buf[0], 1.0 / std::sqrt(n2_fin), nullptr, nullptr);
    L.lam = lam;
    L.power_iters = std::min(it, maxit);
    if (!std::isfinite(lam)) return fail(c, JFNK_E_NONFINITE, "power method: non-finite eigenvalue estimate");
    return JFNK_OK;
}

template <typename T> jfnk_status setup_t(jfnk_ctx *c, const double *u, const double *m) {
    const int nc = c->nc, Lf = c->L;
    // iterate on every level: finest by conversion, then P = 2^-d I^T downwards
    vec_cast<double, T>(c->ex, c->lev[Lf].g, nc, u, P<T>(c->lev[Lf].x), nullptr);
    // keep the Dirichlet data of u (the cast zeroes Dirichlet nodes): project
    // fills them by injection, and the finest level copies them below
    if (Lf >= 1) tr_project<double, T>(c->ex, c->lev[Lf].g, c->lev[Lf - 1].g, nc, u, P<T>(c->lev[Lf - 1].x));
    for (int l = Lf - 1; l >= 1; --l)
        tr_project<T, T>(c->ex, c->lev[l].g, c->lev[l - 1].g, nc, CP<T>(c->lev[l].x), P<T>(c->lev[l - 1].x));
    if (c->prob.kind == JFNK_INVCOEF) {
        // coefficient: project m in FP64, then e^m per level
        const double *mf = m;
        double *bufs[2] = {c->tmpA, c->tmpB};
        vec_exp<T>(c->ex, c->lev[Lf].g.nn, mf, P<T>(c->lev[Lf].kap));
        for (int l = Lf - 1, k = 0; l >= 0; --l, k ^= 1) {
            tr_project<double, double>(c->ex, c->lev[l + 1].g, c->lev[l].g, 1, mf, bufs[k]);
            vec_exp<T>(c->ex, c->lev[l].g.nn, bufs[k], P<T>(c->lev[l].kap));
            mf = bufs[k];
        }
    }
    CHK(check_launch(c));
    return JFNK_OK;
}

// Dirichlet data of the finest iterate: the cast above zeroes Dirichlet
// nodes, so copy u there (all BJ configurations have zero data, but the
// library honours nonzero data).
template <typename T> __global__ void k_copy_dirichlet(Grid g, int nc, const double *u, T *x) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.nn;
         i += (long long)gridDim.x * blockDim.x) {
        int X, Y, Z;
        node_coords(g, i, X, Y, Z);
        if (is_dirichlet(g, X, Y, Z))
            for (int k = 0; k < nc; ++k) x[k * g.nn + i] = (T)u[k * g.nn + i];
    }
}

template <typename T> jfnk_status setup_levels(jfnk_ctx *c, const double *u, const double *m) {
    CHK(setup_t<T>(c, u, m));
    const int Lf = c->L, nc = c->nc;
    {
        const Grid &g = c->lev[Lf].g;
        int nb = (int)std::min<long long>((g.nn + 255) / 256, 2048);
        k_copy_dirichlet<T><<<nb, 256, 0, c->st>>>(g, nc, u, P<T>(c->lev[Lf].x));
    }
    for (int l = 0; l <= Lf; ++l) {
        Level &L = c->lev[l];
        // T* scratch for F: use t
        op_residual<T>(c->ex, L.g, c->ph, CP<T>(L.kap), CP<T>(L.x), nullptr, P<T>(L.t), P<T>(L.Ax), nullptr);
        c->ge[l] += 1;
        vec_eps_num<T>(c->ex, L.g, nc, CP<T>(L.x), root_eps(c, c->vprec, mg_mode(c)), c->opt.eps_mode,
                       lslot(c, l, L_NUM));
    }
    CHK(check_launch(c));
    for (int l = 1; l <= Lf; ++l) CHK(power_method<T>(c, l));
    c->have_eigs = true;
    c->setup_done = true;
    return JFNK_OK;
}

jfnk_status do_setup(jfnk_ctx *c, const double *u, const double *m) {
    Range range("mg_setup");
    if (c->vprec == JFNK_F32) return setup_levels<float>(c, u, m);
    return setup_levels<double>(c, u, m);
}

// ---------------------------------------------------------------------------
// V-cycle (Algorithm 1)
// ---------------------------------------------------------------------------
struct ChebCoef {
    double theta, delta, sigma;
};
ChebCoef cheb_coef(jfnk_ctx *c, int l) {
    const double lam = c->lev[l].lam;
    const double a = c->opt.cheb_lo * lam, b = c->opt.cheb_hi * lam;
    ChebCoef k;
    k.theta = 0.5 * (b + a);
    k.delta = 0.5 * (b - a);
    k.sigma = k.theta / k.delta;
    return k;
}

// nu Chebyshev steps on J_l s = b; the result goes to out (||out||^2 -> out_n2).
// zero: start from s = 0.  Otherwise ||s||^2 must be in the level's L_S slot.
template <typename T>
void chebyshev(jfnk_ctx *c, int l, const T *b, T *s, int nu, bool zero, T *out, double *out_n2,
               const double *b_n2 = nullptr) {
    Level &L = c->lev[l];
    const Grid &g = L.g;
    const int nc = c->nc;
    if (nu <= 0) {
        if (zero) {
            vec_fill<T>(c->ex, s, g.nn * nc, T(0));
            if (out != s) vec_fill<T>(c->ex, out, g.nn * nc, T(0));
        } else if (out != s) {
            vec_cast<T, T>(c->ex, g, nc, s, out, nullptr);
        }
        if (out_n2) vec_dot<T, T>(c->ex, g.nn * nc, out, out, out_n2);
        return;
    }
    const ChebCoef k = cheb_coef(c, l);
    double rho = 1.0 / k.sigma;
    const bool fine = (l == c->L);
    // the steps k = 0 .. nu-2 each cost one J d_k; the last update s += d_{nu-1}
    // none.  From s = 0 the first step runs on the direction b itself (||b||^2
    // in b_n2, or computed here); the last step with a J d writes s + d + d'.
    const bool fuse_first = zero && nu >= 3;
    int first_it = 0;
    if (fuse_first) {
        if (!b_n2) {
            vec_dot<T, T>(c->ex, g.nn * nc, b, b, lslot(c, l, L_B));
            b_n2 = lslot(c, l, L_B);
        }
        const double rn = 1.0 / (2.0 * k.sigma - rho);
        op_cheb_first<T>(c->ex, mg_mode(c), g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), b, lslot(c, l, L_NUM),
                         b_n2, P<T>(L.r), s, P<T>(L.d[1]), 1.0 / k.theta, rn * rho, 2.0 * rn / k.delta,
                         lslot(c, l, L_D1));
        c->ge[l] += 1;
        rho = rn;
        first_it = 1;
    } else if (zero) {
        vec_cheb_zero<T>(c->ex, g, nc, b, P<T>(L.r), P<T>(L.d[0]), s, 1.0 / k.theta, lslot(c, l, L_D0));
    } else {
        op_cheb_init<T>(c->ex, mg_mode(c), g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), s, lslot(c, l, L_NUM),
                        lslot(c, l, L_S), b, P<T>(L.r), P<T>(L.d[0]), 1.0 / k.theta, lslot(c, l, L_D0));
        c->ge[l] += 1;
    }
    int cur = first_it;
    for (int it = first_it; it < nu - 1; ++it) {
        const double rn = 1.0 / (2.0 * k.sigma - rho);
        const double c1 = rn * rho, c2 = 2.0 * rn / k.delta;
        if (it == nu - 2) {
            op_cheb_last<T>(c->ex, mg_mode(c), g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), CP<T>(L.d[cur]),
                            lslot(c, l, L_NUM), lslot(c, l, cur ? L_D1 : L_D0), CP<T>(L.r), s, out, c1, c2, out_n2);
            c->ge[l] += 1;
            return;
        }
        {
            // the timer brackets the interior steps only (28 B/node each)
            TimeScope ts(c, fine ? JFNK_TIMER_CHEB_FINE : JFNK_TIMER_COUNT);
            op_cheb_step<T>(c->ex, mg_mode(c), g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), CP<T>(L.d[cur]),
                            lslot(c, l, L_NUM), lslot(c, l, cur ? L_D1 : L_D0), P<T>(L.r), s, P<T>(L.d[1 - cur]),
                            c1, c2, lslot(c, l, cur ? L_D0 : L_D1));
        }
        c->ge[l] += 1;
        rho = rn;
        cur = 1 - cur;
    }
    vec_add<T>(c->ex, g, nc, s, CP<T>(L.d[cur]), out, out_n2);
}

// b_n2: device slot holding ||b||^2, or nullptr (then computed where needed)
template <typename T>
void vcycle(jfnk_ctx *c, int l, const T *b, T *s_out, double *s_out_n2, const double *b_n2 = nullptr) {
    Level &L = c->lev[l];
    const int nc = c->nc;
    if (l == 0) {
        CoarseArgs ca;
        ca.maxit = c->opt.coarse_maxit > 0 ? c->opt.coarse_maxit : (int)level_dofs(L.g, nc);
        ca.shift_max = c->opt.shift_max;
        ca.atol = c->opt.coarse_atol;
        ca.rtol = c->opt.coarse_rtol;
        ca.gamma = c->opt.shift_gamma;
        ca.stats = slot(c, S_COARSE);
        if (c->opt.coarse_qn > 0) {
            ca.qn_m = c->opt.coarse_qn;
            ca.qn_cap = c->qn_cap;
            ca.qn_rec = c->qn_rec;
            ca.qn_pairs = c->qn_pairs;
            ca.qn_state = c->qn_state;
        }
        coarse_solve<T>(c->ex, mg_mode(c), L.g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), lslot(c, 0, L_NUM), b, s_out,
                        P<T>(L.cw), ca);
        if (s_out_n2) vec_dot<T, T>(c->ex, L.g.nn * nc, s_out, s_out, s_out_n2);
        return;
    }
    T *s = P<T>(L.s);
    // pre-smoothing from s = 0; s and ||s||^2 (L_S) materialised
    chebyshev<T>(c, l, b, s, c->opt.nu_pre, true, s, lslot(c, l, L_S), b_n2);
    // r_{l-1} = R (b - J s)
    op_resid_jv<T>(c->ex, mg_mode(c), L.g, c->ph, CP<T>(L.kap), CP<T>(L.x), CP<T>(L.Ax), s, lslot(c, l, L_NUM),
                   lslot(c, l, L_S), b, P<T>(L.t));
    c->ge[l] += 1;
    Level &C = c->lev[l - 1];
    tr_restrict<T>(c->ex, L.g, C.g, nc, CP<T>(L.t), P<T>(C.b), lslot(c, l - 1, L_B));
    vcycle<T>(c, l - 1, CP<T>(C.b), P<T>(C.s), nullptr, lslot(c, l - 1, L_B));
    // s += I c, ||s||^2 for the post-smoother's first FD step
    tr_prolong_add<T>(c->ex, L.g, C.g, nc, CP<T>(C.s), s, lslot(c, l, L_S));
    chebyshev<T>(c, l, b, s, c->opt.nu_post, false, s_out, s_out_n2);
}

// precondition: z = MG(a v) with v FP64 on the finest level and
// a = 1/sqrt(*rs) (rs null: a = 1); ||z||^2 -> S_ZN2
template <typename T> void precondition(jfnk_ctx *c, const double *v, const double *rs, T *z) {
    Range range("vcycle");
    Level &L = c->lev[c->L];
    if (std::is_same<T, double>::value && rs == nullptr) {
        vcycle<T>(c, c->L, (const T *)v, z, slot(c, S_ZN2));
        return;
    }
    vec_scale_cast<double, T>(c->ex, L.g, c->nc, v, P<T>(L.b), 1.0, rs, lslot(c, c->L, L_B));
    vcycle<T>(c, c->L, CP<T>(L.b), z, slot(c, S_ZN2), lslot(c, c->L, L_B));
}

// ---------------------------------------------------------------------------
// flexible GMRES(m), right-preconditioned, CGS2 (FP64)
// ---------------------------------------------------------------------------
enum OpKind { OP_FD = 0, OP_VJP = 1 };

template <typename T> jfnk_status apply_op(jfnk_ctx *c, OpKind op, const T *z, const double *zn2, double *w) {
    const Grid &g = c->lev[c->L].g;
    if (op == OP_FD) {
        TimeScope ts(c, JFNK_TIMER_JV_OUTER);
        op_jv<double, T>(c->ex, outer_mode(c), g, c->ph, c->kap64, c->u, c->Au, z, slot(c, S_NUM64), zn2, 0.0, w);
        c->ge[c->L] += 1;
    } else {
        if (!std::is_same<T, double>::value) {
            vec_cast<T, double>(c->ex, g, c->nc, z, c->tmpA, nullptr);
            op_vjp(c->ex, g, c->ph, c->kap64, c->u, c->tmpA, 0, w);
        } else {
            op_vjp(c->ex, g, c->ph, c->kap64, c->u, (const double *)z, 0, w);
        }
    }
    return check_launch(c);
}

template <typename T>
jfnk_status fgmres(jfnk_ctx *c, OpKind op, const double *rhs, double sign, double rhs_norm, double tol, double *x,
                   int *iters, double *est_out) {
    const Grid &g = c->lev[c->L].g;
    const int nc = c->nc;
    const long long n = c->n;
    const int m = c->opt.restart;
    double *V = c->V;
    T *Z = (T *)c->Z;
    vec_fill<double>(c->ex, x, n, 0.0);
    int total = 0;
    double est = rhs_norm;
    // Hr: the Hessenberg matrix as the Gram-Schmidt passes deliver it (column
    // j is completed by the delayed reorthogonalisation of step j + 1); R, gv:
    // its Givens QR and the rotated right-hand side, rebuilt every step
    std::vector<double> Hr((m + 1) * m), R((m + 1) * m), gv(m + 1), y(m);
    auto Hij = [&](int i, int j) -> double & { return Hr[i * m + j]; };
    auto Rij = [&](int i, int j) -> double & { return R[i * m + j]; };
    auto givens = [&](int ncol, double g0) {
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = g0;
        std::vector<double> cs(ncol), sn(ncol);
        for (int j = 0; j < ncol; ++j) {
            for (int i = 0; i <= j + 1; ++i) Rij(i, j) = Hij(i, j);
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Rij(i, j) + sn[i] * Rij(i + 1, j);
                Rij(i + 1, j) = -sn[i] * Rij(i, j) + cs[i] * Rij(i + 1, j);
                Rij(i, j) = t;
            }
            const double rad = std::hypot(Rij(j, j), Rij(j + 1, j));
            cs[j] = Rij(j, j) / rad;
            sn[j] = Rij(j + 1, j) / rad;
            Rij(j, j) = rad;
            Rij(j + 1, j) = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
        }
    };
    bool converged = false;
    for (int cycle = 0; cycle < c->opt.max_cycles && !converged; ++cycle) {
        // the first candidate u_0 = the residual, unnormalised; its squared
        // norm scales the first preconditioner input
        double beta;
        const double *u0n2;
        if (cycle == 0) {
            beta = rhs_norm;
            if (beta <= tol) { converged = true; est = beta; break; }
            vec_scale<double>(c->ex, g, nc, rhs, V, sign, nullptr, slot(c, S_RN2));
        } else {
            // r = sign*rhs - A x
            vec_dot<double, double>(c->ex, n, x, x, slot(c, S_XN2));
            CHK(apply_op<double>(c, op, x, slot(c, S_XN2), c->w));
            vec_axpy(c->ex, n, c->w, -sign, rhs, c->w);          // w = A x - sign rhs
            vec_scale<double>(c->ex, g, nc, c->w, V, -1.0, nullptr, slot(c, S_RN2));
            double rn2;
            CHK(read_slots(c, S_RN2, 1, &rn2));
            beta = std::sqrt(rn2);
            est = beta;
            if (!std::isfinite(beta)) return fail(c, JFNK_E_NONFINITE, "FGMRES: non-finite residual");
            if (beta <= tol) { converged = true; break; }
        }
        u0n2 = slot(c, S_RN2);
        std::fill(Hr.begin(), Hr.end(), 0.0);
        double g0 = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            // z_j = M^-1 (u_j / ||u_j||), w = A z_j
            T *zj = Z + (size_t)j * c->ldv;
            precondition<T>(c, V + (size_t)j * c->ldv, j == 0 ? u0n2 : slot(c, S_W2), zj);
            CHK(apply_op<T>(c, op, zj, slot(c, S_ZN2), c->w));
            {
                TimeScope ts(c, JFNK_TIMER_ARNOLDI, false);
                dcgs_dots(c->ex, n, V, c->ldv, j, c->w, slot(c, S_COEF));
                dcgs_update(c->ex, n, V, c->ldv, j, slot(c, S_COEF), c->w, slot(c, S_W2));
            }
            CHK(check_launch(c));
            double hh[2 * MAXR + 4];
            HIPCHK(c, hipMemcpyAsync(hh, c->scal + S_COEF, sizeof(double) * (2 * j + 3), hipMemcpyDeviceToHost, c->st));
            HIPCHK(c, hipMemcpyAsync(hh + 2 * j + 3, c->scal + S_W2, sizeof(double), hipMemcpyDeviceToHost, c->st));
            HIPCHK(c, hipStreamSynchronize(c->st));
            const double *sj = hh, *bj = hh + j;
            const double hjj = hh[2 * j + 1], rj = hh[2 * j + 2], un = std::sqrt(hh[2 * j + 3]);
            if (!std::isfinite(rj) || !std::isfinite(un) || !std::isfinite(hjj))
                return fail(c, JFNK_E_NONFINITE, "FGMRES: non-finite Arnoldi coefficients");
            if (j == 0) {
                g0 = rj;                                  // u_0 = r v_0
            } else {
                for (int i = 0; i < j; ++i) Hij(i, j - 1) += sj[i];   // delayed second projection
                Hij(j, j - 1) = rj;
                if (rj == 0.0) {                          // u_j lay in the span: column j - 1 ends the basis
                    givens(j, g0);
                    k = j;
                    est = std::fabs(gv[j]);
                    break;
                }
            }
            // column j from the first projection of w; its last two entries
            // are corrected by the next step, and are exact to rounding
            // level (the once-projected norm) if the solve stops here
            for (int i = 0; i < j; ++i) Hij(i, j) = bj[i];
            Hij(j, j) = hjj;
            Hij(j + 1, j) = un;
            givens(j + 1, g0);
            k = j + 1;
            ++total;
            est = std::fabs(gv[j + 1]);
            if (est <= tol || un == 0.0) break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double acc = gv[i];
            for (int j = i + 1; j < k; ++j) acc -= Rij(i, j) * y[j];
            y[i] = acc / Rij(i, i);
        }
        if (k > 0) arn_combine<T>(c->ex, n, Z, c->ldv, k, y.data(), x);
        CHK(check_launch(c));
        if (est <= tol) converged = true;
    }
    *iters = total;
    *est_out = est;
    return converged ? JFNK_OK : JFNK_E_NOCONV;
}

jfnk_status run_fgmres(jfnk_ctx *c, OpKind op, const double *rhs, double sign, double rhs_norm, double tol,
                       double *x, int *iters, double *est) {
    if (c->vprec == JFNK_F32) return fgmres<float>(c, op, rhs, sign, rhs_norm, tol, x, iters, est);
    return fgmres<double>(c, op, rhs, sign, rhs_norm, tol, x, iters, est);
}

// ---------------------------------------------------------------------------
// preconditioned CG, the paper's CG-MG (Sec. 3, setup): z = M r by one
// V-cycle, at most restart * max_cycles steps; a direction with p.Ap <= 0
// ends the solve unconverged with x as it stands.  Vectors: r and p in the
// first two basis columns, q = A p in w, z in the first preconditioned
// column.  One host read per step (p.Ap and ||r||^2 after the update).
// Non-positive curvature on the first direction returns that direction.
// ---------------------------------------------------------------------------
template <typename T>
jfnk_status pcg(jfnk_ctx *c, OpKind op, const double *rhs, double sign, double rhs_norm, double tol, double *x,
                int *iters, double *est_out) {
    const Grid &g = c->lev[c->L].g;
    const long long n = c->n;
    double *r = c->V, *p = c->V + c->ldv;
    T *z = (T *)c->Z;
    // slots: p.Ap, ||r||^2 (read together), r.z of this and the previous step, ||p||^2
    double *s_pq = slot(c, S_COEF), *s_rn2 = slot(c, S_COEF + 1), *s_rz[2] = {slot(c, S_COEF + 2),
                                                                               slot(c, S_COEF + 3)};
    double *s_pn2 = slot(c, S_COEF + 4);
    vec_fill<double>(c->ex, x, n, 0.0);
    *iters = 0;
    *est_out = rhs_norm;
    if (rhs_norm <= tol) return JFNK_OK;
    vec_scale<double>(c->ex, g, c->nc, rhs, r, sign, nullptr, nullptr);
    const int maxit = c->opt.restart * c->opt.max_cycles;
    int cur = 0;
    for (int it = 1; it <= maxit; ++it) {
        precondition<T>(c, r, nullptr, z);
        {
            TimeScope ts(c, JFNK_TIMER_ARNOLDI, false);
            vec_dot<double, T>(c->ex, n, r, z, s_rz[cur]);
            vec_cg_dir<T>(c->ex, n, z, p, s_rz[cur], it == 1 ? nullptr : s_rz[cur ^ 1], s_pn2);
        }
        CHK(apply_op<double>(c, op, p, s_pn2, c->w));
        {
            TimeScope ts(c, JFNK_TIMER_ARNOLDI, false);
            vec_dot<double, double>(c->ex, n, p, c->w, s_pq);
            vec_cg_update(c->ex, n, p, c->w, x, r, s_rz[cur], s_pq, s_rn2);
        }
        CHK(check_launch(c));
        double h[2];
        CHK(read_slots(c, S_COEF, 2, h));
        *iters = it;
        if (!std::isfinite(h[0])) return fail(c, JFNK_E_NONFINITE, "CG: non-finite curvature");
        if (!(h[0] > 0.0)) {
            // x and r unchanged by this step; a first direction of
            // non-positive curvature is returned itself (truncated
            // Newton-CG, Nocedal and Wright Alg. 7.1): p = z = M r
            if (it == 1) HIPCHK(c, hipMemcpyAsync(x, p, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
            return JFNK_E_NOCONV;
        }
        const double rn = std::sqrt(h[1]);
        if (!std::isfinite(rn)) return fail(c, JFNK_E_NONFINITE, "CG: non-finite residual");
        *est_out = rn;
        if (rn <= tol) return JFNK_OK;
        cur ^= 1;
    }
    return JFNK_E_NOCONV;
}

// the Newton step's outer solve with the configured Krylov method
jfnk_status run_outer(jfnk_ctx *c, const double *rhs, double sign, double rhs_norm, double tol, double *x,
                      int *iters, double *est) {
    Range range("krylov");
    if (c->opt.outer_krylov == JFNK_OUTER_CG) {
        if (c->vprec == JFNK_F32) return pcg<float>(c, OP_FD, rhs, sign, rhs_norm, tol, x, iters, est);
        return pcg<double>(c, OP_FD, rhs, sign, rhs_norm, tol, x, iters, est);
    }
    return run_fgmres(c, OP_FD, rhs, sign, rhs_norm, tol, x, iters, est);
}

// ---------------------------------------------------------------------------
// inexact Newton with cubic backtracking (Sec. 3, setup)
// ---------------------------------------------------------------------------
bool variational(int kind) { return kind != JFNK_INVCOEF; }

// F, A(u) and ||F||^2 at state s into (Fo, Ao, slot)
jfnk_status eval_residual(jfnk_ctx *c, const double *s, double *Fo, double *Ao, int sl, bool timed) {
    const Level &L = c->lev[c->L];
    {
        TimeScope ts(c, timed ? JFNK_TIMER_RESID_FINE : JFNK_TIMER_COUNT);
        op_residual<double>(c->ex, L.g, c->ph, c->kap64, s, c->bm, Fo, Ao, slot(c, sl));
    }
    c->ge[c->L] += 1;
    return check_launch(c);
}

jfnk_status merit_energy(jfnk_ctx *c, const double *s, double *psi) {
    const Level &L = c->lev[c->L];
    op_energy(c->ex, L.g, c->ph, s, slot(c, S_ENER));
    vec_dot<double, double>(c->ex, c->n, c->bm, s, slot(c, S_BU));
    CHK(check_launch(c));
    double e[2];
    CHK(read_slots(c, S_ENER, 2, e));
    *psi = e[0] - e[1];
    return JFNK_OK;
}

// forget the coarse L-BFGS pairs: the next coarse solve records new ones
void qn_reset(jfnk_ctx *c) {
    if (c->opt.coarse_qn > 0) vec_fill<double>(c->ex, c->qn_state, 3, 0.0);
}

void report_init(jfnk_ctx *c, jfnk_report *rep) {
    std::memset(rep, 0, sizeof(*rep));
    for (int l = 0; l < JFNK_MAX_LEVELS; ++l) c->ge[l] = 0.0;
}

void report_finish(jfnk_ctx *c, jfnk_report *rep) {
    double cs[8];
    if (read_slots(c, S_COARSE, 8, cs) == JFNK_OK) {
        c->ge[0] += cs[3];
        rep->coarse_iters = (long long)cs[1];
        rep->neg_curv = (int)cs[4];
        rep->coarse_calls = (long long)cs[5];
        rep->last_shift = cs[0];
    }
    double eff = 0.0;
    for (int l = 0; l <= c->L; ++l) {
        rep->ge_level[l] = c->ge[l];
        rep->lambda[l] = c->lev[l].lam;
        eff += std::ldexp(c->ge[l], -c->prob.dim * (c->L - l));
    }
    rep->ge_effective = eff;
    if (c->opt.coarse_qn > 0) {
        double st[2] = {0.0, 0.0};
        if (hipMemcpyAsync(st, c->qn_state, sizeof(st), hipMemcpyDeviceToHost, c->st) == hipSuccess &&
            hipStreamSynchronize(c->st) == hipSuccess)
            rep->coarse_qn_pairs = st[0] != 0.0 ? (int)st[1] : 0;
    }
}

double line_cubic(double alpha, double ph, double phi0, double slope, bool have_prev, double ap, double pp) {
    double nw;
    if (!have_prev) {
        nw = -slope * alpha * alpha / (2.0 * (ph - phi0 - slope * alpha));
    } else {
        const double d1 = ph - phi0 - slope * alpha;
        const double d2 = pp - phi0 - slope * ap;
        const double a = (d1 / (alpha * alpha) - d2 / (ap * ap)) / (alpha - ap);
        const double b = (-ap * d1 / (alpha * alpha) + alpha * d2 / (ap * ap)) / (alpha - ap);
        if (a == 0.0) nw = -slope / (2.0 * b);
        else nw = (-b + std::sqrt(std::max(b * b - 3.0 * a * slope, 0.0))) / (3.0 * a);
    }
    if (!std::isfinite(nw)) nw = 0.5 * alpha;
    return std::min(std::max(nw, 0.1 * alpha), 0.5 * alpha);
}

jfnk_status newton(jfnk_ctx *c, jfnk_report *rep) {
    const jfnk_options &o = c->opt;
    CHK(eval_residual(c, c->u, c->F, c->Au, S_FN2, true));
    double fn2;
    CHK(read_slots(c, S_FN2, 1, &fn2));
    const double f0 = std::sqrt(fn2);
    rep->fnorm0 = f0;
    rep->fnorm = f0;
    double fn = f0;
    // energy merit of the current iterate, kept from the accepted trial point
    // of the previous step (the same kernels on the same data: bitwise equal
    // to evaluating it again)
    bool psi_known = false;
    double psi_u = 0.0;
    for (int k = 0; k <= o.newton_maxit; ++k) {
        if (!std::isfinite(fn)) return fail(c, JFNK_E_NONFINITE, "Newton: non-finite residual norm");
        if (fn <= std::max(o.newton_atol, o.newton_rtol * f0)) return JFNK_OK;
        if (k == o.newton_maxit) break;
        Range step("newton step");
        CHK(do_setup(c, c->u, c->mf));
        const double eta = o.forcing == JFNK_FORCING_PAPER ? std::min(0.5, fn) : std::min(0.5, fn / f0);
        // outer FD step numerator from the FP64 iterate
        vec_eps_num<double>(c->ex, c->lev[c->L].g, c->nc, c->u, root_eps(c, JFNK_F64, outer_mode(c)), o.eps_mode,
                            slot(c, S_NUM64));
        int its = 0;
        double est = 0.0;
        jfnk_status ks = run_outer(c, c->F, -1.0, fn, eta * fn, c->dx, &its, &est);
        if (ks == JFNK_E_NONFINITE || ks == JFNK_E_DEVICE) return ks;
        rep->linear_iters += its;
        // line search
        vec_dot<double, double>(c->ex, c->n, c->F, c->dx, slot(c, S_SLOPE));
        double slope_e;
        CHK(read_slots(c, S_SLOPE, 1, &slope_e));
        const bool use_e = variational(c->prob.kind) && o.merit == JFNK_MERIT_AUTO && slope_e < 0.0;
        double phi0, slope;
        if (use_e) {
            if (!psi_known) CHK(merit_energy(c, c->u, &psi_u));
            phi0 = psi_u;
            slope = slope_e;
        } else {
            phi0 = 0.5 * fn * fn;
            slope = -fn * fn;
        }
        double alpha = 1.0, ap = 0.0, pp = 0.0;
        bool have_prev = false, accepted = false;
        double fnt = 0.0, ph = 0.0;
        Range ls("line search");
        for (int it = 1; it <= o.ls_maxit; ++it) {
            vec_axpy(c->ex, c->n, c->u, alpha, c->dx, c->ut);
            CHK(eval_residual(c, c->ut, c->Ft, c->Aut, S_FT2, true));
            double ft2;
            CHK(read_slots(c, S_FT2, 1, &ft2));
            fnt = std::sqrt(ft2);
            if (use_e) CHK(merit_energy(c, c->ut, &ph));
            else ph = 0.5 * ft2;
            if (std::isfinite(ph) && ph <= phi0 + o.armijo * alpha * slope) { accepted = true; break; }
            if (use_e && std::isfinite(fnt) && fnt <= (1.0 - o.armijo * alpha) * fn) { accepted = true; break; }
            double nw;
            if (!std::isfinite(ph)) nw = 0.5 * alpha;
            else nw = line_cubic(alpha, ph, phi0, slope, have_prev, ap, pp);
            if (std::isfinite(ph)) { ap = alpha; pp = ph; have_prev = true; }
            else have_prev = false;
            alpha = nw;
        }
        if (!accepted) return fail(c, JFNK_E_NOCONV, "line search failed");
        psi_known = use_e;
        psi_u = ph;
        std::swap(c->u, c->ut);
        std::swap(c->Au, c->Aut);
        std::swap(c->F, c->Ft);
        fn = fnt;
        rep->fnorm = fn;
        if (rep->nhist < JFNK_MAX_HIST) {
            rep->fnorm_hist[rep->nhist] = fn;
            rep->alpha_hist[rep->nhist] = alpha;
            rep->eta_hist[rep->nhist] = eta;
            rep->lin_hist[rep->nhist] = its;
            rep->nhist++;
        }
        rep->newton_iters++;
    }
    return fail(c, JFNK_E_NOCONV, "Newton: iteration cap reached");
}

jfnk_status check_level(jfnk_ctx *c, int level) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (level < 0 || level > c->L) return fail(c, JFNK_E_INVAL, "level out of range");
    return JFNK_OK;
}

bool misaligned(const void *p, size_t a) { return p && ((uintptr_t)p % a) != 0; }

// kap = e^{coef} on a level into the level-sized scratch (precision T)
template <typename T> const T *coef_kap(jfnk_ctx *c, int level, const double *coef, T *scratch) {
    if (c->prob.kind != JFNK_INVCOEF) return nullptr;
    vec_exp<T>(c->ex, c->lev[level].g.nn, coef, scratch);
    return scratch;
}

// ---------------------------------------------------------------------------
// Scratch of jfnk_residual_static: the per-block partial sums of ||F||^2 in
// a file-scope device array, so that the call allocates nothing.  Every GPU
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives on that
// device (kept per device below), never through the array's name.
// ---------------------------------------------------------------------------
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[STATIC_MAX_DEVICES] = {};

// the scratch address on the current device (looked up once per device)
jfnk_status static_scratch(double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, JFNK_E_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(nullptr, JFNK_E_INVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, JFNK_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return JFNK_OK;
}

}  // namespace

// ===========================================================================
// C entry points
// ===========================================================================
extern "C" {

const char *jfnk_version(void) { return "libjfnk 0.1 (gfx950)"; }

void jfnk_abi_sizes(size_t out[3]) {
    out[0] = sizeof(jfnk_problem);
    out[1] = sizeof(jfnk_options);
    out[2] = sizeof(jfnk_report);
}

const char *jfnk_last_error(const jfnk_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

void jfnk_default_options(jfnk_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->nu_pre = 4;
    o->nu_post = 4;
    o->cheb_lo = 0.06;
    o->cheb_hi = 1.2;
    o->power_maxit = 30;
    o->power_fixed = 0;
    o->power_rtol = 1e-2;
    o->coarse_maxit = 0;
    o->coarse_atol = 1e-12;
    o->coarse_rtol = 1e-6;
    o->shift_gamma = 5.0;
    o->shift_max = 20;
    o->restart = 30;
    o->max_cycles = 20;
    o->newton_maxit = 50;
    o->newton_rtol = 1e-8;
    o->newton_atol = 0.0;
    o->ls_maxit = 30;
    o->armijo = 1e-4;
    o->vcycle_prec = JFNK_F64;
    o->eps_mode = JFNK_EPS_NORM;
    o->fd_root = 0.0;
    o->forcing = JFNK_FORCING_RELATIVE;
    o->merit = JFNK_MERIT_AUTO;
    o->seed = 0;
    o->kernel_path = 0;
    o->fd_form = 0;
    o->coarse_qn = 0;
    o->outer_krylov = JFNK_OUTER_FGMRES;
}

jfnk_status jfnk_workspace_bytes(const jfnk_problem *p, const jfnk_options *o, size_t *bytes) {
    std::string v = validate(p, o);
    if (!v.empty()) return fail(nullptr, JFNK_E_INVAL, v);
    if (!bytes) return fail(nullptr, JFNK_E_INVAL, "null bytes");
    jfnk_ctx tmp;
    tmp.prob = *p;
    tmp.opt = *o;
    tmp.nc = p->kind == JFNK_NEOHOOKE ? 3 : 1;
    tmp.vprec = o->vcycle_prec;
    Carve cv{nullptr};
    plan(&tmp, cv);
    *bytes = cv.off + 256;
    return JFNK_OK;
}

jfnk_status jfnk_create(const jfnk_problem *p, const jfnk_options *o, void *ws, size_t bytes, void *stream,
                        jfnk_ctx **out) {
    if (!out) return fail(nullptr, JFNK_E_INVAL, "null out");
    *out = nullptr;
    std::string v = validate(p, o);
    if (!v.empty()) return fail(nullptr, JFNK_E_INVAL, v);
    size_t need = 0;
    jfnk_workspace_bytes(p, o, &need);
    if (!ws) return fail(nullptr, JFNK_E_INVAL, "null workspace");
    if (misaligned(ws, 256)) return fail(nullptr, JFNK_E_INVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(nullptr, JFNK_E_NOMEM, "workspace too small");
    jfnk_ctx *c = new jfnk_ctx();
    c->prob = *p;
    c->opt = *o;
    c->nc = p->kind == JFNK_NEOHOOKE ? 3 : 1;
    c->vprec = o->vcycle_prec;
    c->L = p->nlevels - 1;
    c->ph = make_phys(*p);
    c->st = (hipStream_t)stream;
    Carve cv{(char *)ws};
    plan(c, cv);
    c->ex.st = c->st;
    c->ex.red.part = c->part;
    c->ex.path = o->kernel_path;
    // deferred reductions: the norms that only the next FD evaluation reads
    // (Chebyshev directions, smoothed corrections, restricted loads, the
    // preconditioned direction of the outer Krylov step)
    {
        int k = 0;
        auto reg = [&](double *sl) { c->lazy.buf[sl] = c->lazy_part + (size_t)(k++) * LAZY_CAP; };
        for (int l = 0; l < p->nlevels; ++l)
            for (int w : {L_D0, L_D1, L_S, L_B}) reg(lslot(c, l, w));
        reg(slot(c, S_ZN2));
        c->ex.lazy = &c->lazy;
    }
    for (int l = 0; l < JFNK_MAX_LEVELS; ++l) c->ge[l] = 0.0;
    hipError_t e = hipHostMalloc((void **)&c->hpin, 8 * sizeof(double), hipHostMallocDefault);
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&c->pev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(c->scal, 0, NSLOT * sizeof(double), c->st);
    if (e == hipSuccess) {
        qn_reset(c);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        g_err = std::string("jfnk_create: ") + hipGetErrorString(e);
        jfnk_destroy(c);
        return JFNK_E_DEVICE;
    }
    *out = c;
    return JFNK_OK;
}

void jfnk_destroy(jfnk_ctx *c) {
    if (!c) return;
    for (auto &t : c->timers)
        for (auto ev : t.ev) (void)hipEventDestroy(ev);
    if (c->t0) (void)hipEventDestroy(c->t0);
    if (c->t1) (void)hipEventDestroy(c->t1);
    for (auto ev : c->pev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->hpin) (void)hipHostFree(c->hpin);
    delete c;
}

jfnk_status jfnk_level_info(const jfnk_ctx *c, int level, int n[3], long long *nnodes, long long *ndof) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (level < 0 || level > c->L) return fail(const_cast<jfnk_ctx *>(c), JFNK_E_INVAL, "level out of range");
    const Grid &g = c->lev[level].g;
    if (n) { n[0] = g.nx; n[1] = g.ny; n[2] = g.nz; }
    if (nnodes) *nnodes = g.nn;
    if (ndof) *ndof = level_dofs(g, c->nc);
    return JFNK_OK;
}

jfnk_status jfnk_residual(jfnk_ctx *c, int level, int prec, const void *u, const void *coef, const void *b,
                          void *F) {
    CHK(check_level(c, level));
    if (!u || !F) return fail(c, JFNK_E_INVAL, "null u or F");
    if (prec != JFNK_F32 && prec != JFNK_F64) return fail(c, JFNK_E_INVAL, "bad precision");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    if (misaligned(u, esize(prec)) || misaligned(F, esize(prec)) || misaligned(b, esize(prec)))
        return fail(c, JFNK_E_INVAL, "misaligned array");
    const Grid &g = c->lev[level].g;
    if (prec == JFNK_F64) {
        const double *k = coef_kap<double>(c, level, (const double *)coef, c->tmpB);
        TimeScope ts(c, level == c->L ? JFNK_TIMER_RESID_FINE : JFNK_TIMER_COUNT);
        op_residual<double>(c->ex, g, c->ph, k, (const double *)u, (const double *)b, (double *)F, nullptr, nullptr);
    } else {
        const float *k = coef_kap<float>(c, level, (const double *)coef, (float *)c->tmpB);
        op_residual<float>(c->ex, g, c->ph, k, (const float *)u, (const float *)b, (float *)F, nullptr, nullptr);
    }
    return check_launch(c);
}

jfnk_status jfnk_residual_static(const jfnk_problem *p, int level, const double *u, const double *b, double *F,
                                 double *fnorm2, void *stream) {
    const std::string v = validate_problem(p);
    if (!v.empty()) return fail(nullptr, JFNK_E_INVAL, v);
    if (p->kind == JFNK_INVCOEF) return fail(nullptr, JFNK_E_INVAL, "INVCOEF needs a node-sized e^m array: use jfnk_residual");
    if (level < 0 || level >= p->nlevels) return fail(nullptr, JFNK_E_INVAL, "level out of range");
    if (!u || !F) return fail(nullptr, JFNK_E_INVAL, "null u or F");
    if (misaligned(u, 8) || misaligned(F, 8) || misaligned(b, 8) || misaligned(fnorm2, 8))
        return fail(nullptr, JFNK_E_INVAL, "misaligned array");
    double *part = nullptr;
    const jfnk_status s = static_scratch(&part);
    if (s != JFNK_OK) return s;
    Exec ex;
    ex.st = (hipStream_t)stream;
    ex.red = Red{part};
    ex.path = 0;
    ex.red_cap = STATIC_SCRATCH_DOUBLES;
    op_residual<double>(ex, level_grid(*p, level), make_phys(*p), nullptr, u, b, F, nullptr, fnorm2);
    if (ex.red_short)
        return fail(nullptr, JFNK_E_INVAL, "the grid needs more partial sums than the static scratch holds ("
                    + std::to_string(STATIC_SCRATCH_DOUBLES) + "): use jfnk_residual");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, JFNK_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return JFNK_OK;
}

jfnk_status jfnk_energy(jfnk_ctx *c, int level, const double *u, const double *b, double *psi) {
    CHK(check_level(c, level));
    if (!u || !psi) return fail(c, JFNK_E_INVAL, "null u or psi");
    if (!variational(c->prob.kind)) return fail(c, JFNK_E_INVAL, "INVCOEF has no energy");
    const Grid &g = c->lev[level].g;
    op_energy(c->ex, g, c->ph, u, slot(c, S_ENER));
    if (b) {
        vec_cast<double, double>(c->ex, g, c->nc, b, c->tmpA, nullptr);
        vec_dot<double, double>(c->ex, g.nn * c->nc, c->tmpA, u, slot(c, S_BU));
    } else {
        vec_fill<double>(c->ex, slot(c, S_BU), 1, 0.0);
    }
    CHK(check_launch(c));
    double e[2];
    CHK(read_slots(c, S_ENER, 2, e));
    *psi = e[0] - e[1];
    return JFNK_OK;
}

jfnk_status jfnk_jv(jfnk_ctx *c, int level, int prec, const void *u, const void *coef, const void *Au,
                    const void *v, double eps_override, void *Jv, double *eps_out) {
    CHK(check_level(c, level));
    if (!u || !v || !Jv) return fail(c, JFNK_E_INVAL, "null u, v or Jv");
    if (prec != JFNK_F32 && prec != JFNK_F64) return fail(c, JFNK_E_INVAL, "bad precision");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    const Grid &g = c->lev[level].g;
    const int nc = c->nc;
    if (prec == JFNK_F64) {
        const double *k = coef_kap<double>(c, level, (const double *)coef, c->tmpB);
        const double *A = (const double *)Au;
        if (!A) {
            op_residual<double>(c->ex, g, c->ph, k, (const double *)u, nullptr, c->tmpA, nullptr, nullptr);
            A = c->tmpA;
        }
        vec_eps_num<double>(c->ex, g, nc, (const double *)u, root_eps(c, JFNK_F64, outer_mode(c)), c->opt.eps_mode,
                            slot(c, S_DOT));
        vec_dot<double, double>(c->ex, g.nn * nc, (const double *)v, (const double *)v, slot(c, S_XN2));
        op_jv<double, double>(c->ex, outer_mode(c), g, c->ph, k, (const double *)u, A, (const double *)v,
                              slot(c, S_DOT), slot(c, S_XN2), eps_override, (double *)Jv);
    } else {
        const float *k = coef_kap<float>(c, level, (const double *)coef, (float *)c->tmpB);
        const float *A = (const float *)Au;
        if (!A) {
            op_residual<float>(c->ex, g, c->ph, k, (const float *)u, nullptr, (float *)c->tmpA, nullptr, nullptr);
            A = (const float *)c->tmpA;
        }
        vec_eps_num<float>(c->ex, g, nc, (const float *)u, root_eps(c, JFNK_F32, outer_mode(c)), c->opt.eps_mode,
                           slot(c, S_DOT));
        vec_dot<float, float>(c->ex, g.nn * nc, (const float *)v, (const float *)v, slot(c, S_XN2));
        op_jv<float, float>(c->ex, outer_mode(c), g, c->ph, k, (const float *)u, A, (const float *)v,
                            slot(c, S_DOT), slot(c, S_XN2), eps_override, (float *)Jv);
    }
    CHK(check_launch(c));
    if (eps_out) {
        // the kernels' step: eps_override, else num / ||v|| (0 for v = 0)
        double nv[2];
        CHK(read_slots(c, S_DOT, 1, nv));
        CHK(read_slots(c, S_XN2, 1, nv + 1));
        *eps_out = eps_override > 0.0 ? eps_override : (nv[1] > 0.0 ? nv[0] / std::sqrt(nv[1]) : 0.0);
    }
    return JFNK_OK;
}

static jfnk_status transfer_args(jfnk_ctx *c, int level, int prec, const void *a, const void *b) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (level < 1 || level > c->L) return fail(c, JFNK_E_INVAL, "transfer level must be in [1, L]");
    if (!a || !b) return fail(c, JFNK_E_INVAL, "null array");
    if (prec != JFNK_F32 && prec != JFNK_F64) return fail(c, JFNK_E_INVAL, "bad precision");
    return JFNK_OK;
}

jfnk_status mg_project(jfnk_ctx *c, int level, int prec, const void *xf, void *xc) {
    CHK(transfer_args(c, level, prec, xf, xc));
    const Grid &f = c->lev[level].g, &g = c->lev[level - 1].g;
    if (prec == JFNK_F64) tr_project<double, double>(c->ex, f, g, c->nc, (const double *)xf, (double *)xc);
    else tr_project<float, float>(c->ex, f, g, c->nc, (const float *)xf, (float *)xc);
    return check_launch(c);
}

jfnk_status mg_restrict(jfnk_ctx *c, int level, int prec, const void *rf, void *rc) {
    CHK(transfer_args(c, level, prec, rf, rc));
    const Grid &f = c->lev[level].g, &g = c->lev[level - 1].g;
    if (prec == JFNK_F64) tr_restrict<double>(c->ex, f, g, c->nc, (const double *)rf, (double *)rc, nullptr);
    else tr_restrict<float>(c->ex, f, g, c->nc, (const float *)rf, (float *)rc, nullptr);
    return check_launch(c);
}

jfnk_status mg_prolong_add(jfnk_ctx *c, int level, int prec, const void *cc, void *sf) {
    CHK(transfer_args(c, level, prec, cc, sf));
    const Grid &f = c->lev[level].g, &g = c->lev[level - 1].g;
    if (prec == JFNK_F64) tr_prolong_add<double>(c->ex, f, g, c->nc, (const double *)cc, (double *)sf, nullptr);
    else tr_prolong_add<float>(c->ex, f, g, c->nc, (const float *)cc, (float *)sf, nullptr);
    return check_launch(c);
}

jfnk_status mg_setup(jfnk_ctx *c, const double *u, const double *coef) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!u) return fail(c, JFNK_E_INVAL, "null u");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    if (c->prob.kind == JFNK_INVCOEF) {
        HIPCHK(c, hipMemcpyAsync(c->mf, coef, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->st));
        vec_exp<double>(c->ex, c->nn, coef, c->kap64);
    }
    for (int l = 0; l < JFNK_MAX_LEVELS; ++l) c->ge[l] = 0.0;
    return do_setup(c, u, c->mf);
}

jfnk_status mg_reset_eigvecs(jfnk_ctx *c) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    c->have_eigs = false;
    qn_reset(c);
    CHK(check_launch(c));
    return JFNK_OK;
}

jfnk_status mg_get_level(jfnk_ctx *c, int level, int which, void *out) {
    CHK(check_level(c, level));
    if (!out) return fail(c, JFNK_E_INVAL, "null out");
    if (!c->setup_done) return fail(c, JFNK_E_INVAL, "mg_setup has not run");
    const Level &L = c->lev[level];
    const void *src = which == 0 ? L.x : which == 1 ? L.Ax : which == 2 ? L.eig : which == 3 ? L.kap : nullptr;
    if (!src) return fail(c, JFNK_E_INVAL, "unknown or absent level quantity");
    const size_t n = (size_t)L.g.nn * (which == 3 ? 1 : c->nc);
    HIPCHK(c, hipMemcpyAsync(out, src, n * esize(c->vprec), hipMemcpyDeviceToDevice, c->st));
    return JFNK_OK;
}

jfnk_status mg_get_lambda(jfnk_ctx *c, double *lam) {
    if (!c || !lam) return fail(c, JFNK_E_INVAL, "null argument");
    for (int l = 0; l <= c->L; ++l) lam[l] = c->lev[l].lam;
    return JFNK_OK;
}

jfnk_status mg_smooth(jfnk_ctx *c, int level, const void *b, void *s, int nu, int s_is_zero) {
    CHK(check_level(c, level));
    if (level < 1) return fail(c, JFNK_E_INVAL, "smoothing needs level >= 1");
    if (!b || !s) return fail(c, JFNK_E_INVAL, "null b or s");
    if (!c->setup_done) return fail(c, JFNK_E_INVAL, "mg_setup has not run");
    const Level &L = c->lev[level];
    if (c->vprec == JFNK_F32) {
        if (!s_is_zero) vec_dot<float, float>(c->ex, L.g.nn * c->nc, (const float *)s, (const float *)s, lslot(c, level, L_S));
        chebyshev<float>(c, level, (const float *)b, (float *)s, nu, s_is_zero != 0, (float *)s, nullptr);
    } else {
        if (!s_is_zero) vec_dot<double, double>(c->ex, L.g.nn * c->nc, (const double *)s, (const double *)s, lslot(c, level, L_S));
        chebyshev<double>(c, level, (const double *)b, (double *)s, nu, s_is_zero != 0, (double *)s, nullptr);
    }
    return check_launch(c);
}

jfnk_status mg_coarse_solve(jfnk_ctx *c, const void *r0, void *s0, double *shift, int *iters, int *rounds) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!r0 || !s0) return fail(c, JFNK_E_INVAL, "null r0 or s0");
    if (!c->setup_done) return fail(c, JFNK_E_INVAL, "mg_setup has not run");
    double before[8];
    CHK(read_slots(c, S_COARSE, 8, before));
    if (c->vprec == JFNK_F32) vcycle<float>(c, 0, (const float *)r0, (float *)s0, nullptr);
    else vcycle<double>(c, 0, (const double *)r0, (double *)s0, nullptr);
    CHK(check_launch(c));
    double after[8];
    CHK(read_slots(c, S_COARSE, 8, after));
    if (shift) *shift = after[0];
    if (iters) *iters = (int)(after[1] - before[1]);
    if (rounds) *rounds = (int)after[2];
    return JFNK_OK;
}

jfnk_status mg_vcycle(jfnk_ctx *c, const double *b, double *s) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!b || !s) return fail(c, JFNK_E_INVAL, "null b or s");
    if (!c->setup_done) return fail(c, JFNK_E_INVAL, "mg_setup has not run");
    const Level &L = c->lev[c->L];
    if (c->vprec == JFNK_F32) {
        float *z = (float *)c->Z;   // restart slot 0 as the FP32 output
        vec_cast<double, float>(c->ex, L.g, c->nc, b, (float *)L.b, nullptr);
        vcycle<float>(c, c->L, (const float *)L.b, z, nullptr);
        vec_cast<float, double>(c->ex, L.g, c->nc, z, s, nullptr);
    } else {
        vec_cast<double, double>(c->ex, L.g, c->nc, b, c->tmpA, nullptr);
        vcycle<double>(c, c->L, c->tmpA, s, nullptr);
    }
    return check_launch(c);
}

// One Newton solve with load scale * b from u; u receives the last
// accepted iterate when write_back or on success.
static jfnk_status solve_once(jfnk_ctx *c, double *u, const double *coef, const double *b, double scale,
                              jfnk_report *rep, bool write_back, bool first) {
    Range range("jfnk_solve");
    report_init(c, rep);
    if (first) qn_reset(c);
    HIPCHK(c, hipMemsetAsync(c->scal + S_COARSE, 0, 8 * sizeof(double), c->st));
    if (!c->t0) {
        HIPCHK(c, hipEventCreate(&c->t0));
        HIPCHK(c, hipEventCreate(&c->t1));
    }
    HIPCHK(c, hipEventRecord(c->t0, c->st));
    const Grid &g = c->lev[c->L].g;
    HIPCHK(c, hipMemcpyAsync(c->u, u, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    if (b) vec_scale<double>(c->ex, g, c->nc, b, c->bm, scale, nullptr, nullptr);
    else vec_fill<double>(c->ex, c->bm, c->n, 0.0);
    if (c->prob.kind == JFNK_INVCOEF) {
        HIPCHK(c, hipMemcpyAsync(c->mf, coef, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->st));
        vec_exp<double>(c->ex, c->nn, coef, c->kap64);
    }
    c->have_eigs = false;
    jfnk_status s = newton(c, rep);
    if (s == JFNK_OK || write_back)
        HIPCHK(c, hipMemcpyAsync(u, c->u, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipEventRecord(c->t1, c->st));
    HIPCHK(c, hipEventSynchronize(c->t1));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->t0, c->t1);
    rep->time_ms = ms;
    report_finish(c, rep);
    rep->status = s;
    return s;
}

jfnk_status jfnk_solve(jfnk_ctx *c, double *u, const double *coef, const double *b, jfnk_report *rep) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!u) return fail(c, JFNK_E_INVAL, "null u");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    jfnk_report local;
    if (!rep) rep = &local;
    return solve_once(c, u, coef, b, 1.0, rep, true, true);
}

jfnk_status jfnk_solve_steps(jfnk_ctx *c, double *u, const double *coef, const double *b, int nsteps,
                             jfnk_report *rep) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!u) return fail(c, JFNK_E_INVAL, "null u");
    if (nsteps < 1) return fail(c, JFNK_E_INVAL, "nsteps must be >= 1");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    jfnk_report local, one;
    if (!rep) rep = &local;
    std::memset(rep, 0, sizeof(*rep));
    double t = 0.0, dt = 1.0 / nsteps;
    bool first = true;
    jfnk_status last = JFNK_OK;
    while (t < 1.0 - 1e-12) {
        const double step = std::min(dt, 1.0 - t);
        const double target = t + step >= 1.0 - 1e-12 ? 1.0 : t + step;   // the full load exactly
        last = solve_once(c, u, coef, b, target, &one, false, first);
        if (last == JFNK_E_DEVICE || last == JFNK_E_INVAL) return last;
        if (first) rep->fnorm0 = one.fnorm0;
        first = false;
        rep->newton_iters += one.newton_iters;
        rep->linear_iters += one.linear_iters;
        rep->coarse_calls += one.coarse_calls;
        rep->coarse_iters += one.coarse_iters;
        rep->coarse_qn_pairs = one.coarse_qn_pairs;
        rep->neg_curv += one.neg_curv;
        rep->ge_effective += one.ge_effective;
        for (int l = 0; l < JFNK_MAX_LEVELS; ++l) {
            rep->ge_level[l] += one.ge_level[l];
            rep->lambda[l] = one.lambda[l];
        }
        rep->last_shift = one.last_shift;
        rep->time_ms += one.time_ms;
        rep->fnorm = one.fnorm;
        if (rep->nhist < JFNK_MAX_HIST) {          // one history entry per attempted increment
            rep->fnorm_hist[rep->nhist] = one.fnorm;
            rep->alpha_hist[rep->nhist] = target;
            rep->eta_hist[rep->nhist] = step;
            rep->lin_hist[rep->nhist] = one.linear_iters;
            rep->nhist++;
        }
        if (last == JFNK_OK) {
            t = target;
        } else {
            dt = 0.5 * step;
            if (dt < 1e-6) break;
        }
    }
    const jfnk_status res = t >= 1.0 - 1e-12 ? JFNK_OK : (last == JFNK_OK ? JFNK_E_NOCONV : last);
    rep->status = res;
    return res;
}

jfnk_status jfnk_vjp(jfnk_ctx *c, int level, int wrt, const double *u, const double *coef, const double *lam,
                     double *out) {
    CHK(check_level(c, level));
    if (!u || !lam || !out) return fail(c, JFNK_E_INVAL, "null u, lam or out");
    if (wrt != 0 && wrt != 1) return fail(c, JFNK_E_INVAL, "wrt must be 0 or 1");
    if (wrt == 1 && c->prob.kind != JFNK_INVCOEF) return fail(c, JFNK_E_INVAL, "wrt = 1 needs INVCOEF");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    const Grid &g = c->lev[level].g;
    const double *k = coef_kap<double>(c, level, coef, c->tmpB);
    op_vjp(c->ex, g, c->ph, k, u, lam, wrt, out);
    return check_launch(c);
}

jfnk_status jfnk_adjoint_solve(jfnk_ctx *c, const double *u, const double *coef, const double *rhs, double rtol,
                               double *lam, jfnk_report *rep) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!u || !rhs || !lam) return fail(c, JFNK_E_INVAL, "null u, rhs or lam");
    if (c->prob.kind == JFNK_INVCOEF && !coef) return fail(c, JFNK_E_INVAL, "INVCOEF needs coef");
    jfnk_report local;
    if (!rep) rep = &local;
    Range range("adjoint solve");
    report_init(c, rep);
    qn_reset(c);
    HIPCHK(c, hipMemsetAsync(c->scal + S_COARSE, 0, 8 * sizeof(double), c->st));
    const Grid &g = c->lev[c->L].g;
    HIPCHK(c, hipMemcpyAsync(c->u, u, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    if (c->prob.kind == JFNK_INVCOEF) {
        HIPCHK(c, hipMemcpyAsync(c->mf, coef, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->st));
        vec_exp<double>(c->ex, c->nn, coef, c->kap64);
    }
    c->have_eigs = false;
    CHK(do_setup(c, c->u, c->mf));
    vec_cast<double, double>(c->ex, g, c->nc, rhs, c->lamv, slot(c, S_RN2));
    double rn2;
    CHK(read_slots(c, S_RN2, 1, &rn2));
    const double rn = std::sqrt(rn2);
    int its = 0;
    double est = 0.0;
    jfnk_status s = run_fgmres(c, OP_VJP, c->lamv, 1.0, rn, rtol * rn, lam, &its, &est);
    rep->linear_iters = its;
    rep->fnorm0 = rn;
    rep->fnorm = est;
    report_finish(c, rep);
    rep->status = s;
    return s;
}

jfnk_status jfnk_coef_gradient(jfnk_ctx *c, const double *u, const double *coef, const double *lam, double *grad) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (c->prob.kind != JFNK_INVCOEF) return fail(c, JFNK_E_INVAL, "the coefficient gradient needs INVCOEF");
    if (!u || !coef || !lam || !grad) return fail(c, JFNK_E_INVAL, "null u, coef, lam or grad");
    const Grid &g = c->lev[c->L].g;
    const double *k = coef_kap<double>(c, c->L, coef, c->tmpB);
    op_vjp(c->ex, g, c->ph, k, u, lam, 1, grad, -1.0);
    return check_launch(c);
}

jfnk_status jfnk_assemble_load(jfnk_ctx *c, int kind, const double *params, int nparams, double *b) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (!b || !params) return fail(c, JFNK_E_INVAL, "null b or params");
    const Grid &g = c->lev[c->L].g;
    if (kind == 0) {
        if (c->nc != 1) return fail(c, JFNK_E_INVAL, "Gaussian load is for scalar problems");
        const int per = g.dim + 2;
        if (nparams <= 0 || nparams % per) return fail(c, JFNK_E_INVAL, "nparams must be a multiple of dim+2");
        const int count = nparams / per;
        // parameters go to device scratch (tmpA, c->n doubles) first
        if ((long long)nparams > c->n) return fail(c, JFNK_E_INVAL, "too many load parameters for this grid");
        HIPCHK(c, hipMemcpyAsync(c->tmpA, params, nparams * sizeof(double), hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        load_gaussians(c->ex, g, c->tmpA, count, b);
    } else if (kind == 1) {
        if (c->nc != 3 || nparams != 3) return fail(c, JFNK_E_INVAL, "traction load needs NEOHOOKE and 3 params");
        load_traction(c->ex, g, params, b);
    } else {
        return fail(c, JFNK_E_INVAL, "unknown load kind");
    }
    return check_launch(c);
}

jfnk_status jfnk_stream_triad(const double *a, const double *b, double *c, long long n, double s, void *stream) {
    if (n < 0) return fail(nullptr, JFNK_E_INVAL, "negative n");
    if (n == 0) return JFNK_OK;
    if (!a || !b || !c) return fail(nullptr, JFNK_E_INVAL, "null array");
    if (misaligned(a, 16) || misaligned(b, 16) || misaligned(c, 16))
        return fail(nullptr, JFNK_E_INVAL, "arrays must be 16-byte aligned");
    stream_triad((hipStream_t)stream, a, b, c, n, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, JFNK_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return JFNK_OK;
}

jfnk_status jfnk_timer_enable(jfnk_ctx *c, int which, int enable) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (which < 0 || which >= JFNK_TIMER_COUNT) return fail(c, JFNK_E_INVAL, "unknown timer");
    TimerRec &t = c->timers[which];
    if (enable) {
        if (t.ev.empty()) {
            t.ev.resize(2 * 8192);
            for (auto &e : t.ev) HIPCHK(c, hipEventCreate(&e));
        }
        t.used = 0;
        t.on = true;
    } else {
        t.on = false;
    }
    return JFNK_OK;
}

jfnk_status jfnk_timer_read(jfnk_ctx *c, int which, long long *count, double *total_ms) {
    if (!c) return fail(nullptr, JFNK_E_INVAL, "null context");
    if (which < 0 || which >= JFNK_TIMER_COUNT) return fail(c, JFNK_E_INVAL, "unknown timer");
    TimerRec &t = c->timers[which];
    HIPCHK(c, hipStreamSynchronize(c->st));
    double tot = 0.0;
    for (size_t k = 0; k + 1 < t.used; k += 2) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, t.ev[k], t.ev[k + 1]));
        tot += ms;
    }
    if (count) *count = (long long)(t.used / 2);
    if (total_ms) *total_ms = tot;
    return JFNK_OK;
}

}  // extern "C"
