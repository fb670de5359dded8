"""Exact derivatives of the discrete residuals (oracle; test infrastructure).

The solver itself never uses these: the method applies J only through the
finite-difference quotient of Sec. 1.  They exist to check it, and for the
adjoint of the inverse-coefficient problem, which needs the exact
transpose J^T lambda.  Each is the derivative of the element vector r_e of
``problems`` with respect to the corner values, written out by hand:

* 'bratu'      J_e = K_e - lam sum_q w_q exp(u_q) phi_a phi_b          (symmetric)
* 'plap'       J_e = k_e K_e + (p-2)(delta^2+s_e)^((p-4)/2)/|e| (K_e u)(K_e u)^T
* 'plap_gauss' the same at each Gauss point with grad u there
* 'invcoef'    J_e = k_e K_e + (kbar_e ubar_e / 4) (K_e u) 1^T      (not symmetric)
               dF/dm_a contribution: (1/8) e^{m_a} (1 + ubar_e^2) K_e u_e
* 'neohooke'   dP = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T

Pins: directional central differences of F; dot-product identity
<J v, w> = <v, J^T w>; symmetry for the variational problems; the Q1
stencil for the linear limits (tests/test_oracle_derivatives.py).
"""
import numpy as np

from .fe import element_stiffness, reference_rule
from .problems import _deformation, _mask, lame


def _elem_jvp(problem, grid, u, v, m, transpose):
    dim, h = grid.dim, grid.h
    kind, prm = problem.kind, problem.params
    K = element_stiffness(dim, h)
    vol = h ** dim
    if kind == 'neohooke':
        return _neohooke_jvp(grid, grid.gather(u), grid.gather(v), prm)
    ue, ve = grid.gather(u), grid.gather(v)
    Ku = np.einsum('ab,b...->a...', K, ue)
    Kv = np.einsum('ab,b...->a...', K, ve)
    if kind == 'bratu':
        phi, _, w, _ = reference_rule(dim)
        uq = np.einsum('qa,a...->q...', phi, ue)
        vq = np.einsum('qa,a...->q...', phi, ve)
        return Kv - prm['lam'] * np.einsum('q,q...,qa->a...', w * vol, np.exp(uq) * vq, phi)
    if kind == 'plap':
        p, delta = prm['p'], prm['delta']
        s = np.einsum('a...,a...->...', ue, Ku) / vol
        k = (delta ** 2 + s) ** ((p - 2.0) / 2.0)
        dk = (p - 2.0) * (delta ** 2 + s) ** ((p - 4.0) / 2.0) / vol
        return k * Kv + dk * Ku * np.einsum('a...,a...->...', Ku, ve)
    if kind == 'plap_gauss':
        p, delta = prm['p'], prm['delta']
        _, dphi, w, _ = reference_rule(dim)
        out = np.zeros_like(ue)
        for q in range(len(w)):
            B = dphi[q] / h
            gu = np.einsum('ak,a...->k...', B, ue)
            gv = np.einsum('ak,a...->k...', B, ve)
            t = delta ** 2 + np.sum(gu * gu, axis=0)
            flux = t ** ((p - 2.0) / 2.0) * gv + (p - 2.0) * t ** ((p - 4.0) / 2.0) * np.sum(gu * gv, axis=0) * gu
            out += w[q] * vol * np.einsum('ak,k...->a...', B, flux)
        return out
    if kind == 'invcoef':
        me = grid.gather(m)
        kbar = np.mean(np.exp(me), axis=0)
        ubar = np.mean(ue, axis=0)
        k = kbar * (1.0 + ubar ** 2)
        c = kbar * ubar / 4.0                       # d k_e / d u_a, same for every corner
        if not transpose:
            return k * Kv + c * Ku * np.sum(ve, axis=0)
        return k * Kv + c * np.einsum('a...,a...->...', ve, Ku)[None]
    raise ValueError(kind)


def _neohooke_jvp(grid, ue, ve, prm):
    mu, lam = lame(prm['E'], prm['nu'])
    _, dphi, w, _ = reference_rule(3)
    vol = grid.h ** 3
    out = np.zeros_like(ue)
    for q in range(len(w)):
        B = dphi[q] / grid.h
        Fd = _deformation(grid.h, ue, q)
        dF = np.einsum('ia...,aj->...ij', ve, B)
        J = np.linalg.det(Fd)
        Finv = np.linalg.inv(Fd)
        FinvT = np.swapaxes(Finv, -1, -2)
        lnJ = np.log(J)
        tr = np.einsum('...ij,...ji->...', Finv, dF)
        term = FinvT @ np.swapaxes(dF, -1, -2) @ FinvT
        dP = mu * dF + (mu - lam * lnJ)[..., None, None] * term + (lam * tr)[..., None, None] * FinvT
        out += w[q] * vol * np.einsum('...ij,aj->ia...', dP, B)
    return out


def jvp(problem, grid, u, v, m=None):
    """Exact J(u) v on the DoF space (v is masked to the DoFs first)."""
    v = _mask(grid, problem.ncomp, v)
    re = _elem_jvp(problem, grid, u, v, m, transpose=False)
    return _mask(grid, problem.ncomp, grid.scatter(re, 1 if problem.ncomp > 1 else 0))


def vjp(problem, grid, u, lam, m=None):
    """Exact J(u)^T lam on the DoF space."""
    lam = _mask(grid, problem.ncomp, lam)
    if problem.kind == 'invcoef':
        re = _elem_jvp(problem, grid, u, lam, m, transpose=True)
    else:   # symmetric element Jacobians
        re = _elem_jvp(problem, grid, u, lam, m, transpose=False)
    return _mask(grid, problem.ncomp, grid.scatter(re, 1 if problem.ncomp > 1 else 0))


def vjp_coef(problem, grid, u, lam, m):
    """(dF/dm)^T lam for 'invcoef', a nodal field over all nodes."""
    assert problem.kind == 'invcoef'
    lam = _mask(grid, 1, lam)
    K = element_stiffness(grid.dim, grid.h)
    ue, le, me = grid.gather(u), grid.gather(lam), grid.gather(m)
    ubar = np.mean(ue, axis=0)
    lKu = np.einsum('a...,ab,b...->...', le, K, ue)
    n = 2 ** grid.dim
    re = np.exp(me) / n * ((1.0 + ubar ** 2) * lKu)[None]
    return grid.scatter(re)


def assembled_jacobian(problem, grid, u, m=None):
    """Dense J on the DoF space, built column by column from the exact JVP.

    Returns (J, dof_index) where dof_index maps columns to flat node indices
    (component-major for vector fields).  Tiny grids only.
    """
    nc = problem.ncomp
    shape = grid.node_shape if nc == 1 else (nc,) + grid.node_shape
    dof = grid.dof_mask() if nc == 1 else np.broadcast_to(grid.dof_mask(), shape)
    idx = np.flatnonzero(dof.reshape(-1))
    J = np.zeros((idx.size, idx.size))
    e = np.zeros(int(np.prod(shape)))
    for c, j in enumerate(idx):
        e[:] = 0.0
        e[j] = 1.0
        J[:, c] = jvp(problem, grid, u, e.reshape(shape), m).reshape(-1)[idx]
    return J, idx
