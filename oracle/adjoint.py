"""Adjoint solve and coefficient gradient (oracle; test infrastructure).

For the inverse-coefficient problem F(u; m) = 0 and the misfit
L(m) = 1/2 ||u(m) - u_obs||^2 over the DoFs, the implicit-function theorem
gives dL/dm = -(dF/dm)^T lam with J(u)^T lam = u - u_obs.  The adjoint
system is solved with flexible GMRES, the operator being the exact
transpose (``derivatives.vjp``) and the preconditioner one V-cycle of the
Jacobian-free multigrid set up at the converged state (Algorithm 1).

Pins: central differences of L along seeded directions; the dot-product
identity of the VJP (tests/test_oracle_adjoint.py).
"""
import numpy as np

from .derivatives import vjp, vjp_coef
from .krylov import fgmres
from .mg import MGOptions, Stats, make_grids, mg_setup, vcycle
from .problems import _mask


def adjoint_solve(problem, finest, nlevels, u, m, rhs, mg_opts=None, rtol=1e-12,
                  restart=30, max_cycles=20, stats=None):
    mg_opts = mg_opts or MGOptions()
    stats = stats or Stats()
    grids = make_grids(finest, nlevels)
    L = nlevels - 1
    levels = mg_setup(problem, grids, u, m, mg_opts, None, stats, {})
    rhs = _mask(finest, problem.ncomp, rhs)

    def A(lam):
        return vjp(problem, finest, u, lam, m)

    def M(v):
        return vcycle(problem, levels, L, v, mg_opts, stats)
    tol = rtol * float(np.sqrt(np.sum(rhs * rhs)))
    lam, its, est, ok = fgmres(A, rhs, M, tol, restart, max_cycles)
    return lam, its, ok


def misfit(finest, u, u_obs):
    d = _mask(finest, 1, u - u_obs)
    return 0.5 * float(np.sum(d * d))


def gradient(problem, finest, nlevels, u, m, u_obs, mg_opts=None, rtol=1e-12):
    """dL/dm for L = 1/2 ||u - u_obs||^2 at a converged state u."""
    lam, its, ok = adjoint_solve(problem, finest, nlevels, u, m, u - u_obs, mg_opts, rtol)
    return -vjp_coef(problem, finest, u, lam, m), lam, its, ok
