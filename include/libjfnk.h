/*
 * libjfnk -- Jacobian-free Newton-Krylov with a Jacobian-free geometric
 * multigrid preconditioner on one AMD MI355X (gfx950).
 *
 * Method: H. Kothari, A. Kopanicakova, R. Krause, "A Multigrid
 * Preconditioner for Jacobian-free Newton-Krylov Methods" (arXiv
 * 2103.13890).  Section numbers below refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 * Grids.  Level l (0 = coarsest, L = nlevels-1 = finest, Sec. 2) is a
 *   uniform box grid with n_k / 2^(L-l) cubic elements of edge h 2^(L-l) per
 *   axis.  Nodal arrays are C-order [nz+1][ny+1][nx+1] (x fastest,
 *   boundary nodes included); 2D grids use [ny+1][nx+1].  Vector fields
 *   (NEOHOOKE, 3 components) are SoA: [3][nz+1][ny+1][nx+1].
 * DoFs.  Nodes on faces named in jfnk_problem.dirichlet hold Dirichlet
 *   data (taken from the state u passed in); every other node is a DoF.
 *   Residuals, Jacobian actions and Krylov vectors are 0 on Dirichlet
 *   nodes.
 * Memory.  Every array argument is a DEVICE pointer owned by the caller,
 *   element type double (JFNK_F64) or float (JFNK_F32) as stated; it must
 *   stay valid until the work queued on the context's stream has run.
 *   The library never allocates device memory: all of its state lives in
 *   the caller's workspace (jfnk_workspace_bytes / jfnk_create).  Report
 *   and scalar out-parameters are HOST pointers.
 * Streams.  A context is bound to one HIP stream.  Primitive calls
 *   (residual, jv, vjp, transfers, vcycle) are queued asynchronously;
 *   calls that make host decisions (mg_setup's power method, solves,
 *   coarse solve, anything returning a host scalar) synchronise it.
 * Errors.  Every call returns a jfnk_status and never aborts.  Arguments
 *   are validated before anything is queued (JFNK_E_INVAL); HIP failures
 *   give JFNK_E_DEVICE.  jfnk_last_error() returns a message.
 * Threads.  One context per host thread; no global mutable state.
 */
#ifndef LIBJFNK_H
#define LIBJFNK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JFNK_MAX_LEVELS 12
#define JFNK_MAX_RESTART 31
#define JFNK_MAX_HIST 128

typedef enum {
    JFNK_OK = 0,
    JFNK_E_INVAL = 1,      /* bad argument, nothing was queued */
    JFNK_E_NOMEM = 2,      /* workspace too small */
    JFNK_E_DEVICE = 3,     /* a HIP call failed */
    JFNK_E_NOCONV = 4,     /* Newton / line search / Krylov did not converge */
    JFNK_E_BREAKDOWN = 5,  /* Krylov breakdown before the tolerance */
    JFNK_E_NONFINITE = 6   /* a norm became NaN or Inf */
} jfnk_status;

/* Residuals (Sec. 3 problem statements; see jfnk_residual). */
typedef enum {
    JFNK_BRATU = 0,     /* Psi = int 1/2|grad u|^2 - lam e^u; Gauss 2^d points    */
    JFNK_PLAP = 1,      /* regularised p-Laplacian, element-mean coefficient      */
    JFNK_INVCOEF = 2,   /* -div(e^m (1+u^2) grad u) = f, element-mean coefficient  */
    JFNK_NEOHOOKE = 3,  /* compressible Neo-Hookean solid, Gauss 2x2x2, 3 comps   */
    JFNK_PLAP_GAUSS = 4 /* regularised p-Laplacian, coefficient at each of the 2^d
                           Gauss points; param p, delta as for PLAP             */
} jfnk_kind;

typedef enum { JFNK_F64 = 0, JFNK_F32 = 1 } jfnk_prec;

/* Finite-difference step of the Jacobian action (Sec. 1):
 * NORM  eps = root (1 + ||x||_2) / ||v||_2
 * PAPER eps = root * mean_i (1 + |x_i|) / ||v||_2   (the paper's choice)
 * root = sqrt(machine epsilon of the level precision) unless overridden;
 * norms and means over the DoFs of the level. */
typedef enum { JFNK_EPS_NORM = 0, JFNK_EPS_PAPER = 1 } jfnk_eps_mode;

/* Forcing term of the inexact Newton step (Sec. 3, setup):
 * RELATIVE eta_k = min(0.5, ||F_k|| / ||F_0||);  PAPER eta_k = min(0.5, ||F_k||). */
typedef enum { JFNK_FORCING_RELATIVE = 0, JFNK_FORCING_PAPER = 1 } jfnk_forcing;

/* Line-search merit: AUTO = the energy Psi_h for variational residuals
 * (Sec. 3 poses every problem as an energy minimisation), 1/2||F||^2
 * otherwise; RESIDUAL = always 1/2||F||^2. */
typedef enum { JFNK_MERIT_AUTO = 0, JFNK_MERIT_RESIDUAL = 1 } jfnk_merit;

/* Outer Krylov solver of the Newton step (jfnk_options.outer_krylov). */
typedef enum { JFNK_OUTER_FGMRES = 0, JFNK_OUTER_CG = 1 } jfnk_outer;

#define JFNK_FACE_XLO 1u
#define JFNK_FACE_XHI 2u
#define JFNK_FACE_YLO 4u
#define JFNK_FACE_YHI 8u
#define JFNK_FACE_ZLO 16u
#define JFNK_FACE_ZHI 32u
#define JFNK_FACES_ALL 63u

typedef struct {
    int kind;           /* jfnk_kind */
    int dim;            /* 2 or 3 (NEOHOOKE: 3) */
    int n[3];           /* elements per axis on the finest level; n[2] unused in 2D */
    double h;           /* element edge on the finest level */
    unsigned dirichlet; /* JFNK_FACE_* bits */
    double param[4];    /* BRATU: lambda | PLAP: p, delta | NEOHOOKE: E, nu */
    int nlevels;        /* >= 1; every n_k must be divisible by 2^(nlevels-1) */
} jfnk_problem;

typedef struct {
    /* Chebyshev smoother (Sec. 2): degree nu, interval [lo, hi] * lambda_l */
    int nu_pre, nu_post;
    double cheb_lo, cheb_hi;            /* 0.06, 1.2 */
    /* power method (Sec. 2): <= power_maxit iterations or relative change < power_rtol */
    int power_maxit, power_fixed;       /* power_fixed != 0: exactly power_maxit iterations */
    double power_rtol;
    /* coarse CG with negative-curvature exit and shift loop (Sec. 2, Algorithm 1) */
    int coarse_maxit;                   /* 0: number of coarse DoFs */
    double coarse_atol, coarse_rtol;    /* stop at ||r|| <= max(atol, rtol ||r_coarse||) */
    double shift_gamma;                 /* 5 */
    int shift_max;                      /* cap on shift rounds */
    /* outer flexible GMRES and inexact Newton (Sec. 3, setup) */
    int restart, max_cycles;            /* 30, restarts per Newton step */
    int newton_maxit;
    double newton_rtol, newton_atol;    /* stop at ||F|| <= max(atol, rtol ||F_0||) */
    int ls_maxit;                       /* line-search trials per Newton step (>= 1) */
    double armijo;                      /* sufficient-decrease constant, in (0, 1); 1e-4 */
    int vcycle_prec;                    /* jfnk_prec of every multigrid level */
    int eps_mode;                       /* jfnk_eps_mode */
    double fd_root;                     /* > 0: replaces sqrt(machine eps) in the FD step */
    int forcing;                        /* jfnk_forcing */
    int merit;                          /* jfnk_merit */
    unsigned long long seed;            /* power-method start vectors (SplitMix64) */
    int kernel_path;                    /* 0 auto, 1 node-centric, 2 z-marching tiles */
    /* How the FD quotient (F(x + eps v) - F(x)) / eps is evaluated (same
     * quotient, same eps, different rounding):
     * 0 auto: element difference form on the multigrid levels, two residual
     *   evaluations (the paper's black-box form) for the outer FP64 J v;
     * 1 two residual evaluations everywhere; 2 difference form everywhere.
     * The difference form computes r_e(x + eps v) - r_e(x) per element
     * without subtracting two nearly equal vectors (see jfnk_jv). */
    int fd_form;
    /* L-BFGS preconditioner of the coarse CG (CG-QN; Sec. 2, coarse level
     * solver, and Sec. 3, setup): 0 plain CG; m in [1, 32] secant pairs (the
     * paper uses 20).  The first coarse solve of a solve (jfnk_solve,
     * jfnk_solve_steps, jfnk_adjoint_solve; after jfnk_create or
     * mg_reset_eigvecs for the mg_* calls) runs plain CG and records every
     * step's pair s = alpha p, y = alpha (J - shift I) p; the steps
     * floor(i t / m), i < m, of its t steps (all of them if t <= m) with
     * s.y > 0 are kept, oldest first.  Every later coarse CG of the solve is
     * preconditioned by their two-loop recursion with H_0 = (s.y / y.y) I of
     * the newest kept pair. */
    int coarse_qn;
    /* Krylov solver of the Newton step J dx = -F (Sec. 3, setup):
     * JFNK_OUTER_FGMRES flexible GMRES(restart), right-preconditioned by one
     * V-cycle per step; JFNK_OUTER_CG the paper's CG-MG: conjugate gradients
     * preconditioned by one V-cycle per step, at most restart * max_cycles
     * steps, stopped at ||r|| <= eta ||F|| or at a direction p with
     * p.Jp <= 0 (the step so far is kept; on the first direction that
     * direction itself, the preconditioned residual, as truncated
     * Newton-CG does).  CG assumes a symmetric J: it
     * is meant for the variational kinds, not JFNK_INVCOEF.
     * jfnk_adjoint_solve always uses FGMRES. */
    int outer_krylov;
} jfnk_options;

typedef struct {
    int status;                          /* jfnk_status of the solve */
    int newton_iters, linear_iters;
    double fnorm0, fnorm;
    int nhist;                           /* entries used in the *_hist arrays */
    double fnorm_hist[JFNK_MAX_HIST];    /* ||F|| after each Newton step */
    double alpha_hist[JFNK_MAX_HIST];    /* accepted line-search step */
    double eta_hist[JFNK_MAX_HIST];      /* forcing term */
    int lin_hist[JFNK_MAX_HIST];         /* Krylov iterations per Newton step */
    double ge_level[JFNK_MAX_LEVELS];    /* gradient evaluations per level */
    double ge_effective;                 /* sum_l 2^(-d (L-l)) GE_l (Sec. 3) */
    double lambda[JFNK_MAX_LEVELS];      /* last power-method estimates */
    long long coarse_calls, coarse_iters;
    int neg_curv;                        /* coarse negative-curvature exits */
    double last_shift;                   /* lambda_c+ of the last coarse solve */
    double time_ms;                      /* wall time of the solve (stream events) */
    int coarse_qn_pairs;                 /* L-BFGS pairs kept (coarse_qn > 0), else 0 */
} jfnk_report;

typedef struct jfnk_ctx jfnk_ctx;

/* ---- lifecycle --------------------------------------------------------- */

/* Defaults: nu 4/4, [0.06,1.2], power 30 / 1e-2, coarse rtol 1e-6, atol
 * 1e-12, gamma 5, restart 30 (at most JFNK_MAX_RESTART), Newton rtol 1e-8,
 * F64 levels, NORM step, RELATIVE forcing, AUTO merit, seed 0, plain coarse
 * CG (coarse_qn 0), FGMRES outer solver. */
void jfnk_default_options(jfnk_options *opt);

/* Bytes of device workspace a context for (prob, opt) needs. */
jfnk_status jfnk_workspace_bytes(const jfnk_problem *prob, const jfnk_options *opt,
                                 size_t *bytes);

/* Create a context.  workspace: device memory of >= jfnk_workspace_bytes
 * bytes, 256-byte aligned, owned by the caller and kept alive as long as
 * the context.  stream: a hipStream_t (NULL = the null stream). */
jfnk_status jfnk_create(const jfnk_problem *prob, const jfnk_options *opt,
                        void *workspace, size_t bytes, void *stream, jfnk_ctx **out);
void jfnk_destroy(jfnk_ctx *ctx);
const char *jfnk_last_error(const jfnk_ctx *ctx);   /* ctx may be NULL */
const char *jfnk_version(void);
/* sizeof(jfnk_problem), sizeof(jfnk_options), sizeof(jfnk_report): lets a
 * binding check its mirrors of the three structs. */
void jfnk_abi_sizes(size_t out[3]);

/* Element counts per axis, node count and DoF count (components included). */
jfnk_status jfnk_level_info(const jfnk_ctx *ctx, int level, int n[3],
                            long long *nnodes, long long *ndof);

/* ---- a1: residual ------------------------------------------------------- */
/* F = A_l(u; coef) - b on the DoFs of level l, 0 on Dirichlet nodes.  A_l is
 * the gradient of the discrete energy (Sec. 1: F = grad Psi) assembled with
 * first-order elements on grid l (Sec. 3).  coef: nodal coefficient field m
 * of INVCOEF (NULL otherwise); b: load, NULL for none.  All arrays have the
 * level's node layout and the precision prec. */
jfnk_status jfnk_residual(jfnk_ctx *ctx, int level, int prec, const void *u,
                          const void *coef, const void *b, void *F);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the FP64 residual
 * F = A_l(u) - b of jfnk_residual without a context.  prob describes the
 * grid and the residual as for jfnk_workspace_bytes (INVCOEF excepted: its
 * e^m needs a node-sized array); level in [0, nlevels); u, b (nullable), F:
 * FP64 device arrays of that level's node layout; fnorm2 (device, nullable)
 * receives ||F||^2; stream: a hipStream_t (NULL: the default stream).  The
 * same kernels as jfnk_residual, with their per-block partial sums in a
 * 128 KB static device array instead of a workspace: no hipMalloc, hipFree
 * or other allocation is made.  Each GPU has one such array, shared by every
 * call on it, so calls that overlap on one GPU race (one stream, or ordered
 * streams, per GPU).  Asynchronous.  Errors (jfnk_last_error(NULL)):
 * JFNK_E_INVAL for an invalid problem, level or pointer, INVCOEF, or a grid
 * whose launch needs more partial sums than the array holds (very tall
 * grids: use jfnk_residual); JFNK_E_DEVICE for a HIP error. */
jfnk_status jfnk_residual_static(const jfnk_problem *prob, int level, const double *u, const double *b,
                                 double *F, double *fnorm2, void *stream);

/* Discrete energy Psi_h(u) - b.u on level l (FP64, variational kinds).
 * Blocks; the value goes to *psi (host). */
jfnk_status jfnk_energy(jfnk_ctx *ctx, int level, const double *u, const double *b,
                        double *psi);

/* ---- a5: finite-difference Jacobian action ----------------------------- */
/* Jv = (A_l(u + eps v) - A_l(u)) / eps (Sec. 1; the load cancels).  Au:
 * A_l(u) if cached by the caller, or NULL to compute it.  eps_override > 0
 * replaces the eps rule; otherwise eps follows options.eps_mode.  v = 0
 * gives Jv = 0.  eps_out (host, nullable): the step used; asking for it
 * synchronises the stream. */
jfnk_status jfnk_jv(jfnk_ctx *ctx, int level, int prec, const void *u, const void *coef,
                    const void *Au, const void *v, double eps_override, void *Jv,
                    double *eps_out);

/* ---- a3, a7, a8: transfers (Sec. 2, transfer operators) ---------------- */
/* level: the FINE level l >= 1 of the pair (l, l-1).
 * mg_project    x_c = P x_f: 2^-d I^T x_f at coarse interior nodes (row
 *               sums normalised on natural-boundary faces so constants are
 *               preserved), injection at coarse Dirichlet nodes.
 * mg_restrict   r_c = I^T r_f, 0 at coarse Dirichlet nodes.
 * mg_prolong_add s_f += I c_c (multilinear interpolation). */
jfnk_status mg_project(jfnk_ctx *ctx, int level, int prec, const void *x_fine, void *x_coarse);
jfnk_status mg_restrict(jfnk_ctx *ctx, int level, int prec, const void *r_fine, void *r_coarse);
jfnk_status mg_prolong_add(jfnk_ctx *ctx, int level, int prec, const void *c_coarse,
                           void *s_fine);

/* ---- a2, a3, a4: multigrid setup at a Newton iterate ------------------- */
/* Projects u (and coef) to every level, caches A_l(x_l), and estimates the
 * largest eigenvalue lambda_l of each smoothed level's FD Jacobian by the
 * power method (Sec. 2, smoothers), warm-started from the previous call's
 * eigenvectors after the first.  u, coef: FP64 on the finest level.
 * Synchronises (the power method's stopping test runs on the host). */
jfnk_status mg_setup(jfnk_ctx *ctx, const double *u_fine, const double *coef_fine);
/* Forget the stored eigenvectors: the next mg_setup starts from random vectors. */
jfnk_status mg_reset_eigvecs(jfnk_ctx *ctx);
/* Copy a setup quantity of a level into out (level precision):
 * which 0: projected iterate x_l, 1: A_l(x_l), 2: power-method eigenvector,
 * 3: e^{m_l} (INVCOEF). */
jfnk_status mg_get_level(jfnk_ctx *ctx, int level, int which, void *out);
/* lambda_l for l = 0..L (host array of nlevels; level 0 reports 0). */
jfnk_status mg_get_lambda(jfnk_ctx *ctx, double *lam);

/* ---- a6, a9, a10: smoother, coarse solve, V-cycle ----------------------- */
/* nu Chebyshev steps on J_l s = b at the setup state of level l >= 1
 * (level precision), from s (s_is_zero != 0: from 0 without reading s). */
jfnk_status mg_smooth(jfnk_ctx *ctx, int level, const void *b, void *s, int nu, int s_is_zero);
/* The coarse branch of Algorithm 1 on level 0: CG with the negative-
 * curvature exit, shifted while lambda_c < 0.  r0, s0: level precision.
 * shift, iters, rounds (host, nullable): final lambda_c+, total CG
 * iterations, shift rounds.  Synchronises. */
jfnk_status mg_coarse_solve(jfnk_ctx *ctx, const void *r0, void *s0, double *shift,
                            int *iters, int *rounds);
/* s = MG(b): one V(nu_pre, nu_post) cycle of Algorithm 1 from the finest
 * level at the current setup state.  b, s: FP64 finest-level arrays; with
 * FP32 levels they are converted on entry and exit. */
jfnk_status mg_vcycle(jfnk_ctx *ctx, const double *b_fine, double *s_fine);

/* ---- a11, a12: inexact Newton solve ------------------------------------- */
/* Solves F(u) = A(u; coef) - b = 0 on the finest level from the initial u
 * (FP64, overwritten with the last accepted iterate) by inexact Newton
 * with cubic backtracking (Sec. 3, setup), each step by right-
 * preconditioned flexible GMRES(restart) in FP64 whose preconditioner is one
 * V-cycle (Algorithm 1) in the level precision.  coef, b: nullable.  rep:
 * host, nullable.  Returns JFNK_OK when ||F|| <= max(atol, rtol ||F_0||). */
jfnk_status jfnk_solve(jfnk_ctx *ctx, double *u, const double *coef, const double *b,
                       jfnk_report *rep);

/* Load stepping (Sec. 3, the hyperelastic example applies its boundary data
 * in increments): solves with the loads (k / nsteps) b for k = 1..nsteps,
 * each increment a jfnk_solve from the previous increment's solution.  A
 * failed increment is retried with half the step (down to 1e-6 of the load).
 * u: FP64, in the initial iterate, out the solution of the last accepted
 * increment.  rep (host, nullable) sums the iteration counts and GE over all
 * increments; its histories hold one entry per attempted increment: fnorm,
 * alpha = load fraction reached, eta = increment size, lin = Krylov
 * iterations.  JFNK_OK when the full load was reached. */
jfnk_status jfnk_solve_steps(jfnk_ctx *ctx, double *u, const double *coef, const double *b,
                             int nsteps, jfnk_report *rep);

/* ---- a13, a14: exact vector-Jacobian products --------------------------- */
/* wrt 0: out = J_l(u)^T lam on the DoFs (exact element Jacobians; equal to
 *        J lam for the variational kinds).
 * wrt 1: out = (dF/dm)^T lam at every node (INVCOEF only).
 * FP64 arrays of level l. */
jfnk_status jfnk_vjp(jfnk_ctx *ctx, int level, int wrt, const double *u, const double *coef,
                     const double *lam, double *out);

/* ---- a15: adjoint solve --------------------------------------------------- */
/* Solves J(u)^T lam = rhs on the finest level by flexible GMRES with the
 * exact VJP as operator and one V-cycle of the multigrid set up at u as
 * preconditioner, to ||rhs - J^T lam|| <= rtol ||rhs||.  lam: FP64, output. */
jfnk_status jfnk_adjoint_solve(jfnk_ctx *ctx, const double *u, const double *coef,
                               const double *rhs, double rtol, double *lam, jfnk_report *rep);

/* Gradient of a loss L(u(m)) with respect to the coefficient field, by the
 * implicit-function theorem: with F(u(m); m) = 0 and lam solving
 * J(u)^T lam = dL/du (jfnk_adjoint_solve), dL/dm = -(dF/dm)^T lam
 * (jfnk_vjp with wrt 1, negated here).  INVCOEF only; u, coef, lam, grad:
 * FP64 finest-level arrays, grad at every node.  Errors: JFNK_E_INVAL for
 * another kind or a null pointer. */
jfnk_status jfnk_coef_gradient(jfnk_ctx *ctx, const double *u, const double *coef, const double *lam,
                               double *grad);

/* ---- load vectors ---------------------------------------------------------- */
/* kind 0: b_i = sum_e sum_q w_q f(x_q) phi_i(x_q), 2^d Gauss points, with
 *         f(x) = sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2)); params holds, per
 *         Gaussian, (c_x, c_y[, c_z], w, a); nparams = count * (dim + 2),
 *         at most the number of finest-level nodes (the parameters are
 *         staged in a node-sized device scratch array).
 * kind 1: surface traction t = (t_x, t_y, t_z) on the x = x_max face
 *         (NEOHOOKE), 2x2 Gauss per face cell; nparams = 3.
 * b: FP64 finest-level array (zero on Dirichlet nodes).
 * Errors: JFNK_E_INVAL for a null pointer, an unknown kind, a kind that does
 * not fit the problem, or a parameter count that is not one of the above. */
jfnk_status jfnk_assemble_load(jfnk_ctx *ctx, int kind, const double *params, int nparams,
                               double *b);

/* ---- measurement ----------------------------------------------------------- */
/* The achievable HBM rate, for reading the kernels' roofline fractions:
 * c = a + s b over n FP64 elements (device arrays, 16-byte aligned, no
 * aliasing of c with a or b), a dense grid-wide sweep with 16-byte accesses
 * and the non-temporal hint, 24 bytes per element.  Asynchronous on stream
 * (NULL: the default stream).  Errors: JFNK_E_INVAL for n < 0, a null or
 * misaligned array; JFNK_E_DEVICE for a launch error. */
jfnk_status jfnk_stream_triad(const double *a, const double *b, double *c, long long n, double s,
                              void *stream);

/* Kernel classes that can be timed with stream events around each launch. */
typedef enum {
    JFNK_TIMER_CHEB_FINE = 0,   /* interior fused Chebyshev steps on the finest level */
    JFNK_TIMER_JV_OUTER = 1,    /* FP64 outer FD Jacobian action */
    JFNK_TIMER_RESID_FINE = 2,  /* FP64 finest-level residual */
    JFNK_TIMER_ARNOLDI = 3,     /* Gram-Schmidt passes of FGMRES; the vector steps of CG */
    JFNK_TIMER_COUNT = 4
} jfnk_timer;
/* enable != 0 starts recording (clearing earlier records); 0 stops. */
jfnk_status jfnk_timer_enable(jfnk_ctx *ctx, int timer, int enable);
/* Launch count and summed duration (ms) of the records so far.  Synchronises. */
jfnk_status jfnk_timer_read(jfnk_ctx *ctx, int timer, long long *count, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* LIBJFNK_H */
