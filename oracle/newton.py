"""Inexact Jacobian-free Newton with cubic backtracking (oracle; test infrastructure).

Sec. 1: x <- x + alpha dx with J(x) dx = -F(x); Sec. 3 (setup): inexact
Newton whose direction satisfies ||J dx + F|| <= eta ||F||, a cubic
backtracking line search (Dennis and Schnabel, Alg. A6.3.1), and the
multigrid-preconditioned Krylov solve.  Readings:

* forcing: eta_k = min(0.5, ||F_k|| / ||F_0||) ('relative', default) --
  scale-free; the paper's eta_k = min(0.5, ||F_k||) is 'paper'.
* stop: ||F|| <= max(atol, rtol ||F_0||).
* merit: the problems of Sec. 3 are energy minimisations, so for the
  variational residuals the merit is the energy, phi(alpha) =
  Psi_h(x + alpha dx), with the exact slope F(x)^T dx (F = grad Psi).
  The non-variational inverse-coefficient residual, and any step that is
  not a descent direction of Psi, use phi = 1/2 ||F||^2 with slope
  -||F||^2.  Sufficient decrease phi <= phi(0) + 1e-4 alpha slope; a step
  whose residual norm drops to (1 - 1e-4 alpha) ||F|| is also accepted,
  because near the root energy differences fall below rounding.  First
  backtrack quadratic, later ones cubic through the two latest trials,
  each new step kept in [0.1, 0.5] times the previous; a non-finite merit
  halves alpha.
* outer solver: flexible GMRES(30), preconditioned by one V-cycle
  ('fgmres', default), or the paper's CG with the V-cycle as preconditioner
  ('cg', at most restart * max_cycles steps).
* outer J v: the finite-difference quotient on the finest level at the
  Newton iterate, the same operator the finest smoother uses.

Pins: the solution satisfies the discrete equations (F = 0 to the
tolerance) and converges to the manufactured and closed-form solutions at
O(h^2) (tests/test_oracle_problems.py, tests/test_oracle_solve.py).
"""
from dataclasses import dataclass, field

import numpy as np

from .krylov import fgmres, pcg
from .mg import MGOptions, Stats, level_jv, make_grids, mg_setup, vcycle
from .problems import _mask, apply_A, energy

VARIATIONAL = ('bratu', 'plap', 'plap_gauss', 'neohooke')


@dataclass
class NewtonOptions:
    rtol: float = 1e-8
    atol: float = 0.0
    maxit: int = 50
    forcing: str = 'relative'
    restart: int = 30
    max_cycles: int = 20
    ls_maxit: int = 30
    armijo: float = 1e-4
    merit: str = 'auto'              # 'auto': energy if variational; 'residual'
    outer: str = 'fgmres'            # 'fgmres' or 'cg'
    f0: float = 0.0                  # > 0: ||F_0|| of the solve this one continues
                                     # (from its saved iterate); the forcing and the
                                     # stop are relative to it


@dataclass
class Report:
    status: str = 'ok'
    newton_iters: int = 0
    linear_iters: int = 0
    fnorm: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    eta: list = field(default_factory=list)
    lin: list = field(default_factory=list)
    lams: list = field(default_factory=list)
    stats: Stats = field(default_factory=Stats)


def _norm(v):
    return float(np.sqrt(np.sum(v * v)))


def line_search(trial, phi0, slope, maxit, armijo, fnorm0=None):
    """Backtracking on phi(alpha); returns (alpha, trials) or (None, trials).

    trial(alpha) returns (phi(alpha), ||F(x + alpha dx)||); with fnorm0 set,
    a trial whose residual norm is <= (1 - armijo alpha) fnorm0 is accepted
    as well.
    """
    alpha = 1.0
    prev = None
    for it in range(1, maxit + 1):
        ph, fn = trial(alpha)
        if np.isfinite(ph) and ph <= phi0 + armijo * alpha * slope:
            return alpha, it
        if fnorm0 is not None and np.isfinite(fn) and fn <= (1.0 - armijo * alpha) * fnorm0:
            return alpha, it
        if not np.isfinite(ph):
            new = 0.5 * alpha
        elif prev is None:
            new = -slope * alpha ** 2 / (2.0 * (ph - phi0 - slope * alpha))
        else:
            ap, pp = prev
            d1 = ph - phi0 - slope * alpha
            d2 = pp - phi0 - slope * ap
            a = (d1 / alpha ** 2 - d2 / ap ** 2) / (alpha - ap)
            b = (-ap * d1 / alpha ** 2 + alpha * d2 / ap ** 2) / (alpha - ap)
            if a == 0.0:
                new = -slope / (2.0 * b)
            else:
                new = (-b + np.sqrt(max(b * b - 3.0 * a * slope, 0.0))) / (3.0 * a)
        if not np.isfinite(new):
            new = 0.5 * alpha
        new = min(max(new, 0.1 * alpha), 0.5 * alpha)
        prev = (alpha, ph) if np.isfinite(ph) else None
        alpha = new
    return None, maxit


def solve(problem, finest, nlevels, u0, b, m=None, mg_opts=None, opts=None, report=None):
    """Solve F(u) = A(u) - b = 0 from u0.  Returns (u, Report)."""
    mg_opts = mg_opts or MGOptions()
    opts = opts or NewtonOptions()
    rep = report or Report()
    st = rep.stats
    grids = make_grids(finest, nlevels)
    L = nlevels - 1
    g = grids[L]
    nc = problem.ncomp
    u = u0.copy()
    Au = apply_A(problem, g, u, m)
    st.count(L)
    F = _mask(g, nc, Au - b)
    rep.fnorm.append(_norm(F))
    f0 = opts.f0 if opts.f0 > 0.0 else rep.fnorm[0]
    eigs = None
    qn = {}                                   # coarse L-BFGS pairs, built once per solve
    for k in range(opts.maxit + 1):
        fn = _norm(F)
        if not np.isfinite(fn):
            rep.status = 'nonfinite'
            return u, rep
        if fn <= max(opts.atol, opts.rtol * f0):
            rep.status = 'ok'
            return u, rep
        if k == opts.maxit:
            break
        levels = mg_setup(problem, grids, u, m, mg_opts, eigs, st, qn)
        eigs = [lev.eig for lev in levels]
        rep.lams.append([lev.lam for lev in levels])
        eta = min(0.5, fn / f0) if opts.forcing == 'relative' else min(0.5, fn)
        fine = levels[L]

        def A(z):
            return level_jv(problem, fine, z, st, L)

        def M(v):
            return vcycle(problem, levels, L, v, mg_opts, st)
        if opts.outer == 'cg':
            dx, its, _, _ = pcg(A, -F, M, eta * fn, opts.restart * opts.max_cycles)
        else:
            dx, its, _, _ = fgmres(A, -F, M, eta * fn, opts.restart, opts.max_cycles)
        rep.linear_iters += its
        rep.lin.append(its)
        rep.eta.append(eta)
        trials = {}
        slope_e = float(np.sum(F * dx))
        use_energy = problem.kind in VARIATIONAL and opts.merit == 'auto' and slope_e < 0.0

        def trial(alpha):
            ut = u + alpha * dx
            At = apply_A(problem, g, ut, m)
            st.count(L)
            Ft = _mask(g, nc, At - b)
            trials[alpha] = (ut, At, Ft)
            fnt = _norm(Ft)
            if use_energy:
                return energy(problem, g, ut, b), fnt
            return 0.5 * fnt * fnt, fnt
        if use_energy:
            alpha, _ = line_search(trial, energy(problem, g, u, b), slope_e, opts.ls_maxit,
                                   opts.armijo, fn)
        else:
            alpha, _ = line_search(trial, 0.5 * fn * fn, -fn * fn, opts.ls_maxit, opts.armijo)
        if alpha is None:
            rep.status = 'noconv'
            return u, rep
        u, Au, F = trials[alpha]
        rep.alpha.append(alpha)
        rep.newton_iters += 1
        rep.fnorm.append(_norm(F))
    rep.status = 'noconv'
    return u, rep


def load_steps(problem, finest, nlevels, u0, b_final, nsteps, m=None, mg_opts=None, opts=None):
    """Apply the load in nsteps equal increments, halving a failed increment.

    Increment k solves at k / nsteps of the load; the last one at the full
    load exactly.  A failed increment is retried at half its size, and the
    halved size is kept for the rest of the path."""
    u = u0.copy()
    t, dt = 0.0, 1.0 / nsteps
    reports = []
    while t < 1.0 - 1e-12:
        step = min(dt, 1.0 - t)
        # increments k / nsteps of the load; the last one is the full load exactly
        target = 1.0 if t + step >= 1.0 - 1e-12 else t + step
        un, rep = solve(problem, finest, nlevels, u, target * b_final, m, mg_opts, opts)
        reports.append((target, rep))
        if rep.status == 'ok':
            u, t = un, target
        else:
            dt = 0.5 * step
            if dt < 1e-6:
                break
    return u, reports
