// Host-side launch interface of libjfnk's kernels.  Every function queues
// work on ex.st and returns immediately; slots are device doubles.
#pragma once
#include "common.hpp"
#include "reduce.hpp"

namespace jfnk {

struct Exec {
    hipStream_t st;
    Red red;
    int path;            // 0 auto, 1 node-centric, 2 z-marching tiles
    LazyTable *lazy = nullptr;   // deferred reductions (nullable)
    // > 0: red holds this many doubles, and a stencil launch that would need
    // more partial sums is not made (red_short is set instead); 0: unchecked
    // (the context's workspace sizes red for every launch it makes)
    long long red_cap = 0;
    mutable bool red_short = false;
    bool red_fits(int nb, int ns) const {
        if (red_cap <= 0 || (long long)nb * (ns > 0 ? ns : 1) <= red_cap) return true;
        red_short = true;
        return false;
    }
    // when set, recorded on st right after the next stencil kernel (before
    // its reduction finish) and cleared: lets a timer bracket that kernel
    mutable hipEvent_t ev_main_end = nullptr;
    void mark_main_end() const {
        if (ev_main_end) {
            (void)hipEventRecord(ev_main_end, st);
            ev_main_end = nullptr;
        }
    }
};

// ---- reductions into slots ------------------------------------------------------
// Partial-sum buffer for a reduction of nb blocks whose result goes to slot:
// the slot's own buffer when the slot is deferred, else the shared one.
inline Red red_for(const Exec &ex, const double *slot, int nb) {
    if (ex.lazy && slot && nb <= LAZY_CAP) {
        auto it = ex.lazy->buf.find(slot);
        if (it != ex.lazy->buf.end()) return Red{it->second};
    }
    return ex.red;
}
// After the producer: record the partials of a deferred slot, or run the
// finishing kernel (which writes the slot).
template <int NS, class Fin>
inline void finish_to(const Exec &ex, const double *slot, const Red &r, int nb, const Fin &fin) {
    if (ex.lazy && slot) {
        if (NS == 1 && r.part != ex.red.part) {
            ex.lazy->pend[slot] = Pending{r.part, nb};
            return;
        }
        ex.lazy->pend.erase(slot);
    }
    finish<NS>(ex.st, r, nb, fin);
}
// Write a deferred slot's value (for a consumer that reads the slot itself).
inline void materialize(const Exec &ex, double *slot) {
    if (!ex.lazy || !slot) return;
    auto it = ex.lazy->pend.find(slot);
    if (it == ex.lazy->pend.end()) return;
    finish<1>(ex.st, Red{const_cast<double *>(it->second.part)}, it->second.nb, FinStore<1>{slot});
    ex.lazy->pend.erase(it);
}
// FD step descriptor: a deferred ||v||^2 is summed by the consuming kernel.
inline FdStep make_fd(const Exec &ex, const double *num, const double *vn2, double fixed) {
    FdStep f{num, vn2, fixed};
    if (ex.lazy && vn2 && !(fixed > 0.0)) {
        auto it = ex.lazy->pend.find(vn2);
        if (it != ex.lazy->pend.end()) {
            f.part = it->second.part;
            f.nb = it->second.nb;
        }
    }
    return f;
}

// a1 residual: F = A(u) - b (b nullable), A(u) -> Aout (nullable), ||F||^2 -> nrm2 (nullable)
template <typename T>
void op_residual(const Exec &, const Grid &, const Phys &, const T *kap, const T *u, const T *b, T *F, T *Aout,
                 double *nrm2);
// FD evaluations (Sec. 1) take mode = M_FD_PLAIN ((A(x + eps v) - Ax)/eps
// with the cached Ax) or M_FD_DIFF (the element difference form; Ax unused).
// a5 FD Jacobian action
template <typename T, typename TV>
void op_jv(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax, const TV *v,
           const double *num, const double *vn2, double eps_fixed, T *Jv);
// a6 Chebyshev step with d_k (||d_k||^2 in vn2): s += d; r -= J d; dn = c1 d + c2 r
template <typename T>
void op_cheb_step(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax,
                  const T *d, const double *num, const double *vn2, T *r, T *s, T *dn, double c1, double c2,
                  double *dn_nrm2);
// first Chebyshev step from s = 0 with the direction b (||b||^2 in vn2):
// s = b / theta, r = b - (J b) / theta, dn = c1 s + c2 r; ||dn||^2 -> dn_nrm2
template <typename T>
void op_cheb_first(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax,
                   const T *b, const double *num, const double *vn2, T *r, T *s, T *dn, double inv_theta, double c1,
                   double c2, double *dn_nrm2);
// last Chebyshev step with d_k: sout = s + d_k + (c1 d_k + c2 (r - J d_k));
// ||sout||^2 -> s_nrm2 (nullable).  sout may alias s.
template <typename T>
void op_cheb_last(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax,
                  const T *d, const double *num, const double *vn2, const T *r, const T *s, T *sout, double c1,
                  double c2, double *s_nrm2);
// Chebyshev start from s: r = b - J s, d = r / theta
template <typename T>
void op_cheb_init(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax,
                  const T *s, const double *num, const double *vn2, const T *b, T *r, T *d, double inv_theta,
                  double *d_nrm2);
// a7 residual of the correction: t = b - J s
template <typename T>
void op_resid_jv(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax,
                 const T *s, const double *num, const double *vn2, const T *b, T *t);
// a4 power step: q = J v, out[0] = v.q, out[1] = ||q||^2
template <typename T>
void op_power(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax, const T *v,
              const double *num, const double *vn2, T *q, double *out);

// energy Psi_h(u) (element sum) -> out[0]   (FP64, variational kinds)
void op_energy(const Exec &, const Grid &, const Phys &, const double *u, double *out);
// exact VJP: out = scale J(u)^T lam (wrt 0) or scale (dF/dm)^T lam (wrt 1, kap = e^m)
void op_vjp(const Exec &, const Grid &, const Phys &, const double *kap, const double *u, const double *lam,
            int wrt, double *out, double scale = 1.0);

// ---- vectors (n = nodes, nc components, SoA) ---------------------------------
template <typename T> void vec_fill(const Exec &, T *x, long long n, T val);
// y = x on DoFs, 0 on Dirichlet nodes; ||y||^2 -> nrm2 (nullable)
template <typename TI, typename TO>
void vec_cast(const Exec &, const Grid &, int nc, const TI *x, TO *y, double *nrm2);
// y = a x on DoFs (0 on Dirichlet); ||y||^2 -> nrm2 (nullable); a = scale * (1/sqrt(*rs) if rs)
template <typename T>
void vec_scale(const Exec &, const Grid &, int nc, const T *x, T *y, double scale, const double *rs,
               double *nrm2);
// y = a x on DoFs (0 on Dirichlet) in precision TO; a and nrm2 as in vec_scale
template <typename TI, typename TO>
void vec_scale_cast(const Exec &, const Grid &, int nc, const TI *x, TO *y, double scale, const double *rs,
                    double *nrm2);
// FD step numerator of a level: root (1 + ||x||) (mode 0) or root mean(1 + |x|) (mode 1)
template <typename T>
void vec_eps_num(const Exec &, const Grid &, int nc, const T *x, double root, int mode, double *num);
// Chebyshev start from zero: r = b, d = b / theta, s = 0; ||d||^2
template <typename T>
void vec_cheb_zero(const Exec &, const Grid &, int nc, const T *b, T *r, T *d, T *s, double inv_theta,
                   double *d_nrm2);
// out = s + d on DoFs; ||out||^2 (out may alias s)
template <typename T>
void vec_add(const Exec &, const Grid &, int nc, const T *s, const T *d, T *out, double *nrm2);
// SplitMix64 start vector of a level, masked; ||v||^2
template <typename T>
void vec_random(const Exec &, const Grid &, int nc, unsigned long long seed, int level, T *v, double *nrm2);
// kap = exp(m) at every node
template <typename T> void vec_exp(const Exec &, long long n, const double *m, T *kap);
// sum x.y over n entries -> out
template <typename TA, typename TB>
void vec_dot(const Exec &, long long n, const TA *x, const TB *y, double *out);

// Arnoldi by classical Gram-Schmidt with delayed reorthogonalisation (DCGS2)
// on FP64 columns spaced by ld: V_0..V_{J-1} final, V_J the candidate u
// (projected once), w the new image.
// dcgs_dots: coef[0..J) = V^T u, coef[J..2J) = V^T w, coef[2J] = 1/r,
// coef[2J+1] = (u.w - s.b)/r, coef[2J+2] = r, with r = sqrt(u.u - s.s).
void dcgs_dots(const Exec &, long long n, const double *V, long long ld, int J, const double *w, double *coef);
// dcgs_update: V_J <- (u - V s)/r, V_{J+1} <- w - V b - coef[2J+1] V_J,
// ||V_{J+1}||^2 -> nrm2
void dcgs_update(const Exec &, long long n, double *V, long long ld, int J, const double *coef, const double *w,
                 double *nrm2);
// x += sum_j y_j Z_j (Z in TZ precision)
template <typename TZ>
void arn_combine(const Exec &, long long n, const TZ *Z, long long ld, int k, const double *y, double *x);
// y = x + a d (FP64)
// preconditioned CG: x += a p, r -= a q with a = *rz / *pq when *pq > 0
// (else nothing), ||r||^2 -> rn2; and p = z + (*rz / *rz_prev) p (rz_prev
// null: p = z), ||p||^2 -> pn2
void vec_cg_update(const Exec &, long long n, const double *p, const double *q, double *x, double *r,
                   const double *rz, const double *pq, double *rn2);
template <typename TZ>
void vec_cg_dir(const Exec &, long long n, const TZ *z, double *p, const double *rz, const double *rz_prev,
                double *pn2);
void vec_axpy(const Exec &, long long n, const double *x, double a, const double *d, double *y);

// ---- transfers (level l fine, l-1 coarse) -----------------------------------------
template <typename TI, typename TO>
void tr_project(const Exec &, const Grid &fine, const Grid &coarse, int nc, const TI *xf, TO *xc);
template <typename T>
void tr_restrict(const Exec &, const Grid &fine, const Grid &coarse, int nc, const T *rf, T *rc, double *nrm2);
template <typename T>
void tr_prolong_add(const Exec &, const Grid &fine, const Grid &coarse, int nc, const T *cc, T *sf,
                    double *nrm2);

// ---- coarse solve (Algorithm 1, level 0) ------------------------------------------
constexpr int QN_MAX = 32;   // secant pairs of the coarse L-BFGS preconditioner
// qn_state layout: [0] 0 none / 1 built, [1] pairs kept, [2] gamma,
// [3 + i] 1/(s_i.y_i), then s_a.y_b and y_a.y_b ([a][b], QN_MAX columns)
constexpr int QN_OFF_SY = 3 + QN_MAX;
constexpr int QN_OFF_YY = QN_OFF_SY + QN_MAX * QN_MAX;
constexpr int QN_STATE_LEN = QN_OFF_YY + QN_MAX * QN_MAX;
struct CoarseArgs {
    int maxit, shift_max;
    double atol, rtol, gamma;
    double *stats;      // [0] last shift, [1] total CG iterations, [2] rounds, [3] FD evaluations,
                        // [4] negative-curvature exits (accumulated over calls)
    // L-BFGS preconditioner (CG-QN), qn_m > 0 pairs: the first call records
    // every CG step's pair into qn_rec ([2][qn_cap][nn], level precision)
    // and keeps a uniform sample in qn_pairs ([2][qn_m][nn]); qn_state
    // (QN_STATE_LEN doubles) as laid out above
    int qn_m = 0, qn_cap = 0;
    void *qn_rec = nullptr, *qn_pairs = nullptr;
    double *qn_state = nullptr;
};
// whether the coarse solve of this level runs in the one-workgroup kernel
// that keeps the level in LDS (the one that supports the L-BFGS preconditioner)
bool coarse_small(const Grid &, int kind, size_t elem_bytes);
// elements of the work array the generic coarse solver needs
size_t coarse_work_elems(const Grid &, int nc);
template <typename T>
void coarse_solve(const Exec &, int mode, const Grid &, const Phys &, const T *kap, const T *x, const T *Ax,
                  const double *num, const T *b, T *s, T *work, const CoarseArgs &);
int coarse_max_nodes();

// ---- loads ---------------------------------------------------------------------------
void load_gaussians(const Exec &, const Grid &, const double *prm, int count, double *b);
void load_traction(const Exec &, const Grid &, const double *t, double *b);

// streaming calibration c = a + s b (FP64, n elements, a, b, c 16-byte aligned)
void stream_triad(hipStream_t st, const double *a, const double *b, double *c, long long n, double s);

}  // namespace jfnk
