"""Jacobian-free multigrid (oracle; test infrastructure).

Follows Sec. 1 (finite-difference Jacobian action), Sec. 2 (transfer
operators, Chebyshev smoother with a power-method eigenvalue estimate,
shifted coarse CG with a negative-curvature exit) and Algorithm 1 (the
V(nu1, nu2)-cycle).  Readings where the paper is silent or ambiguous:

* FD step: eps = root (1 + ||x||_2) / ||v||_2 ('norm', the default) or the
  paper's eps = root * mean_i(1 + |x_i|) / ||v||_2 ('paper'); root is
  sqrt(machine epsilon) unless a test overrides it.  Norms and means run
  over the DoFs of the level.  v = 0 gives J v = 0.
* What is differenced: (A(x + eps v) - A(x)) / eps with the load-free
  operator A and a cached A(x) per level.  The load cancels in the
  difference, so this is the paper's (F(x + eps v) - F(x)) / eps.
* Level operators: the same energy discretised on the coarser grid at the
  projected iterate (rediscretisation), each level keeping A(x_l).
* Chebyshev: the three-term recurrence for the interval
  [0.06 lam_l, 1.2 lam_l]; "nu smoothing steps" is a polynomial of degree
  nu, i.e. nu updates of s, the last of which needs no new residual.
* Power method: Rayleigh-quotient estimate lam_k = v^T J v with ||v|| = 1;
  stop when |lam_k - lam_{k-1}| < rtol |lam_k| or after maxit iterations;
  a fixed count is also supported.  Start: SplitMix64 vector (``rng``) at
  the first Newton step, the previous eigenvector afterwards.
* Coarse CG: on (J - lam_c+ I) s = r from the current s; exit with
  negative curvature when p^T A_s p <= 0, returning the Rayleigh quotient
  p^T A_s p / p^T p of the operator in use; otherwise stop at
  ||r|| <= max(atol, rtol ||r_coarse||) or maxit iterations (default: the
  number of coarse DoFs) and return lam_c = 0.  Shift loop of Algorithm 1
  with gamma = 5, capped at shift_max rounds.
* Coarse L-BFGS preconditioner (CG-QN, Sec. 2 coarse level solver and
  Sec. 3 setup, after Morales and Nocedal 2000), optional (coarse_qn = m
  secant pairs; the paper's experiments use 20).  The first coarse CG of a
  solve runs unpreconditioned and records every step's pair
  s_k = alpha_k p_k, y_k = alpha_k (J - shift I) p_k.  Uniform sampling
  over the t recorded steps keeps the pairs at steps floor(i t / m),
  i = 0..m-1 (all of them when t <= m), of which those with s^T y > 0
  form the preconditioner, oldest first.  It is applied by the two-loop
  recursion with H_0 = (s^T y / y^T y) I of the newest kept pair, and
  every later coarse CG of the solve (shifted ones included) is
  preconditioned CG with it: same negative-curvature test p^T A_s p <= 0,
  same Rayleigh quotient, same stop on the unpreconditioned residual.
"""
from dataclasses import dataclass, field

import numpy as np

from .problems import apply_A, _mask
from .rng import splitmix_uniform
from .transfer import project, prolong, restrict

EPS64 = 2.0 ** -52


@dataclass
class MGOptions:
    nu_pre: int = 3
    nu_post: int = 3
    cheb_lo: float = 0.06
    cheb_hi: float = 1.2
    power_maxit: int = 30
    power_rtol: float = 1e-2
    power_fixed: bool = False
    coarse_maxit: int = 0            # 0: number of coarse DoFs
    coarse_atol: float = 1e-12
    coarse_rtol: float = 1e-6
    shift_gamma: float = 5.0
    shift_max: int = 20
    coarse_qn: int = 0               # L-BFGS secant pairs of the coarse CG (0: none)
    eps_mode: str = 'norm'           # 'norm' or 'paper'
    fd_root: float = np.sqrt(EPS64)  # sqrt of the machine epsilon
    seed: int = 0


@dataclass
class Level:
    grid: object
    x: np.ndarray
    m: object
    Ax: np.ndarray = None
    eps_num: float = 0.0
    lam: float = 0.0
    eig: np.ndarray = None
    power_iters: int = 0
    qn: dict = None                  # coarse level: the solve's L-BFGS state


@dataclass
class Stats:
    ge: dict = field(default_factory=dict)          # level -> gradient evaluations
    neg_curv: int = 0
    shifts: list = field(default_factory=list)
    coarse_iters: list = field(default_factory=list)

    def count(self, level):
        self.ge[level] = self.ge.get(level, 0) + 1

    def effective_ge(self, dim, L):
        """GE = sum_l 2^(-d (L - l)) GE_l (Sec. 3)."""
        return sum(2.0 ** (-dim * (L - l)) * n for l, n in self.ge.items())


def dof_norm(grid, v):
    return float(np.sqrt(np.sum(_mask(grid, 1 if v.ndim == grid.dim else v.shape[0], v) ** 2)))


def eps_numerator(grid, x, opts):
    """The factor of 1/||v|| in the FD step for iterate x on this grid."""
    dof = grid.dof_mask()
    xs = x[dof] if x.ndim == grid.dim else x[:, dof]
    if opts.eps_mode == 'norm':
        return opts.fd_root * (1.0 + float(np.sqrt(np.sum(xs * xs))))
    if opts.eps_mode == 'paper':
        return opts.fd_root * float(np.mean(1.0 + np.abs(xs)))
    raise ValueError(opts.eps_mode)


def fd_jv(problem, grid, x, Ax, v, m, eps):
    """(A(x + eps v) - A(x)) / eps on the DoFs (Sec. 1); v acts on the DoFs
    only (Dirichlet entries of v are ignored: they are not unknowns)."""
    if eps == 0.0:
        return np.zeros_like(v)
    nc = 1 if v.ndim == grid.dim else v.shape[0]
    return (apply_A(problem, grid, x + eps * _mask(grid, nc, v), m) - Ax) / eps


def level_jv(problem, lev, v, stats=None, level=None):
    nv = dof_norm(lev.grid, v)
    if stats is not None:
        stats.count(level)
    if nv == 0.0:
        return np.zeros_like(v)
    return fd_jv(problem, lev.grid, lev.x, lev.Ax, v, lev.m, lev.eps_num / nv)


# ---------------------------------------------------------------------------
def power_method(Jv, v0, maxit, rtol, fixed):
    """Largest eigenvalue by the power method with Rayleigh quotients."""
    v = v0 / np.sqrt(np.sum(v0 * v0))
    lam_prev = None
    lam = 0.0
    it = 0
    for it in range(1, maxit + 1):
        w = Jv(v)
        lam = float(np.sum(v * w))
        nw = float(np.sqrt(np.sum(w * w)))
        if nw == 0.0:
            break
        v = w / nw
        if not fixed and lam_prev is not None and abs(lam - lam_prev) < rtol * abs(lam):
            break
        lam_prev = lam
    return lam, v, it


def random_start(grid, ncomp, seed, level):
    shape = grid.node_shape if ncomp == 1 else (ncomp,) + grid.node_shape
    v = splitmix_uniform(seed, level, int(np.prod(shape))).reshape(shape)
    return _mask(grid, ncomp, v)


def chebyshev(Jv, b, s, nu, lam, lo, hi, s_is_zero=False):
    """nu steps of the three-term Chebyshev iteration for J s = b on [lo lam, hi lam]."""
    if nu <= 0:
        return s
    a, bb = lo * lam, hi * lam
    theta, delta = 0.5 * (bb + a), 0.5 * (bb - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b.copy() if s_is_zero else b - Jv(s)
    d = r / theta
    for k in range(nu):
        s = s + d
        if k == nu - 1:
            break
        r = r - Jv(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return s


def lbfgs_apply(pairs, r):
    """H r for the L-BFGS inverse approximation of the pairs (s_i, y_i),
    oldest first: the two-loop recursion with H_0 = (s^T y / y^T y) I of the
    newest pair (Nocedal and Wright, Numerical Optimization, Alg. 7.4)."""
    if not pairs:
        return r.copy()
    q = r.copy()
    rho = [1.0 / float(np.sum(s * y)) for s, y in pairs]
    a = [0.0] * len(pairs)
    for i in range(len(pairs) - 1, -1, -1):
        s, y = pairs[i]
        a[i] = rho[i] * float(np.sum(s * q))
        q = q - a[i] * y
    s, y = pairs[-1]
    z = (float(np.sum(s * y)) / float(np.sum(y * y))) * q
    for i in range(len(pairs)):
        s, y = pairs[i]
        bi = rho[i] * float(np.sum(y * z))
        z = z + (a[i] - bi) * s
    return z


def uniform_sample(t, m):
    """Indices of the m steps kept out of t recorded ones (uniform sampling)."""
    if t <= m:
        return list(range(t))
    return [(i * t) // m for i in range(m)]


def cg_shifted(Jv, b, s, shift, maxit, tol, prec=None, record=None):
    """CG on (J - shift I) s = b from s with the negative-curvature exit,
    preconditioned by prec (a function r -> M^-1 r) when given; record, a
    list, receives every step's pair (alpha p, alpha A_s p).

    Returns (s, lam_c, iterations): lam_c < 0 is the Rayleigh quotient of
    the shifted operator at the direction with non-positive curvature,
    lam_c = 0 when CG ended normally.
    """
    def As(v):
        return Jv(v) - shift * v
    r = b - As(s) if np.any(s) else b.copy()
    if np.sqrt(float(np.sum(r * r))) <= tol:
        return s, 0.0, 0
    z = prec(r) if prec is not None else r
    p = z.copy()
    rz = float(np.sum(r * z))
    for it in range(1, maxit + 1):
        q = As(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            return s, pq / float(np.sum(p * p)), it
        alpha = rz / pq
        if record is not None:
            record.append((alpha * p, alpha * q))
        s = s + alpha * p
        r = r - alpha * q
        if np.sqrt(float(np.sum(r * r))) <= tol:
            return s, 0.0, it
        z = prec(r) if prec is not None else r
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return s, 0.0, maxit


def coarse_solve(Jv, r0, n_dof, opts, stats=None, qn=None):
    """The coarse branch of Algorithm 1: CG, then shifted CG while lam_c < 0.
    With opts.coarse_qn > 0 and a state dict qn: the first call records the
    secant pairs, later ones (and this call's shifted rounds) precondition."""
    maxit = opts.coarse_maxit if opts.coarse_maxit > 0 else n_dof
    tol = max(opts.coarse_atol, opts.coarse_rtol * float(np.sqrt(np.sum(r0 * r0))))
    use_qn = opts.coarse_qn > 0 and qn is not None
    record = None
    if use_qn and qn.get('pairs') is None:
        record = []

    def prec():
        if use_qn and qn.get('pairs') is not None:
            return lambda r: lbfgs_apply(qn['pairs'], r)
        return None
    shift = 0.0
    s = np.zeros_like(r0)
    s, lam_c, it = cg_shifted(Jv, r0, s, shift, maxit, tol, prec(), record)
    if record is not None:
        kept = [record[i] for i in uniform_sample(len(record), opts.coarse_qn)]
        qn['pairs'] = [(sk, yk) for sk, yk in kept if float(np.sum(sk * yk)) > 0.0]
    iters = [it]
    rounds = 0
    while lam_c < 0.0 and rounds < opts.shift_max:
        if stats is not None:
            stats.neg_curv += 1
        shift = opts.shift_gamma * min(lam_c, shift)
        s, lam_c, it = cg_shifted(Jv, r0, s, shift, maxit, tol, prec())
        iters.append(it)
        rounds += 1
    if stats is not None:
        stats.shifts.append(shift)
        stats.coarse_iters.append(iters)
    return s, shift, iters


# ---------------------------------------------------------------------------
def make_grids(finest, nlevels):
    """Grids from coarsest (index 0) to finest (index nlevels-1)."""
    g = [finest]
    for _ in range(nlevels - 1):
        g.append(g[-1].coarsen())
    return g[::-1]


def mg_setup(problem, grids, u, m, opts, prev_eigs=None, stats=None, qn=None):
    """Project the iterate (and coefficient), cache A_l(x_l), estimate lam_l.
    qn: the solve's coarse L-BFGS state (a dict kept across Newton steps)."""
    L = len(grids) - 1
    xs, ms = [None] * (L + 1), [None] * (L + 1)
    xs[L], ms[L] = u, m
    for l in range(L, 0, -1):
        xs[l - 1] = project(grids[l - 1], grids[l], xs[l])
        if m is not None:
            ms[l - 1] = project(grids[l - 1], grids[l], ms[l])
    levels = []
    for l in range(L + 1):
        lev = Level(grid=grids[l], x=xs[l], m=ms[l])
        lev.Ax = apply_A(problem, grids[l], xs[l], ms[l])
        if stats is not None:
            stats.count(l)
        lev.eps_num = eps_numerator(grids[l], xs[l], opts)
        levels.append(lev)
    levels[0].qn = qn
    for l in range(1, L + 1):
        lev = levels[l]
        v0 = prev_eigs[l] if prev_eigs is not None else random_start(lev.grid, problem.ncomp, opts.seed, l)
        lev.lam, lev.eig, lev.power_iters = power_method(
            lambda v, lev=lev, l=l: level_jv(problem, lev, v, stats, l),
            v0, opts.power_maxit, opts.power_rtol, opts.power_fixed)
    return levels


def vcycle(problem, levels, l, b, opts, stats=None):
    """Algorithm 1: s_l = MG(x_l, F(x_l), b_l, l)."""
    lev = levels[l]

    def Jv(v):
        return level_jv(problem, lev, v, stats, l)
    if l == 0:
        s, _, _ = coarse_solve(Jv, b, lev.grid.n_dof(problem.ncomp), opts, stats, lev.qn)
        return s
    s = np.zeros_like(b)
    s = chebyshev(Jv, b, s, opts.nu_pre, lev.lam, opts.cheb_lo, opts.cheb_hi, s_is_zero=True)
    t = b - Jv(s)
    rc = restrict(levels[l - 1].grid, lev.grid, t)
    c = vcycle(problem, levels, l - 1, rc, opts, stats)
    s = s + prolong(levels[l - 1].grid, lev.grid, c)
    s = chebyshev(Jv, b, s, opts.nu_post, lev.lam, opts.cheb_lo, opts.cheb_hi)
    return s
