"""Energies Psi_h and residuals F(u) = grad Psi_h (oracle; test infrastructure).

The method assumes the nonlinear system is the gradient of an energy,
F = grad Psi (Sec. 1, Jacobian-free Newton-Krylov paragraph), discretised
with first-order finite elements (Sec. 3).  This module evaluates, for a
state u on a Grid,

    A(u)  = sum_e  r_e(u_e)            (element vectors scattered to nodes)
    F(u)  = A(u) - b                   (b: load vector)

and zeroes both at Dirichlet nodes, where u holds the boundary data.

Problems (element vector r_e, corner index a):

* 'bratu'      Psi = int 1/2 |grad u|^2 - lam exp(u)            (Sec. 3, Bratu)
               r_e = K_e u_e - lam sum_q w_q exp(u_h(x_q)) phi_a(x_q)
* 'plap'       regularised p-Laplacian, element-mean coefficient:
               s_e = u_e^T K_e u_e / |e|   (mean of |grad u_h|^2 on e)
               Psi_e = |e|/p (delta^2 + s_e)^(p/2)
               r_e = (delta^2 + s_e)^((p-2)/2) K_e u_e
* 'plap_gauss' the same energy with the coefficient at each Gauss point
* 'invcoef'    -div(e^m (1 + u^2) grad u) = f, element-mean coefficient
               k_e = mean_a(e^{m_a}) (1 + mean_a(u_a)^2),  r_e = k_e K_e u_e
               (not the gradient of an energy)
* 'neohooke'   Psi = int mu/2 (tr C - 3) - mu ln J + lam/2 (ln J)^2
               (Sec. 3, hyperelasticity), first Piola stress
               P = mu (Fd - Fd^-T) + lam ln J Fd^-T,  Fd = I + grad u
               r_e[i, a] = sum_q w_q sum_j P_ij(x_q) d_j phi_a(x_q)

Pins: F = grad Psi_h by central differences; O(h^2) manufactured-solution
convergence; the 1D Bratu closed form; Q1 stencils for the linear limits;
the homogeneous-deformation patch test for the solid
(tests/test_oracle_problems.py).  'invcoef' has no energy: it is pinned by
its manufactured solution and by its p = 2 / m = 0 / u = 0 linear limit.
"""
from dataclasses import dataclass, field

import numpy as np

from .fe import element_stiffness, reference_rule


@dataclass
class Problem:
    kind: str
    params: dict = field(default_factory=dict)

    @property
    def ncomp(self):
        return 3 if self.kind == 'neohooke' else 1


def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson's ratio (Sec. 3)."""
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def _mask(grid, ncomp, v):
    m = grid.dirichlet_mask()
    v = v.copy()
    if ncomp == 1:
        v[m] = 0.0
    else:
        v[:, m] = 0.0
    return v


# ---------------------------------------------------------------------------
# element vectors
# ---------------------------------------------------------------------------
def element_vectors(problem, grid, u, m=None):
    """r_e for every element: shape (2^d,)+elem_shape, or (3, 8)+elem_shape."""
    me = grid.gather(m) if problem.kind == 'invcoef' else None
    return element_vectors_from_corners(problem, grid.dim, grid.h, grid.gather(u), me)


def element_vectors_from_corners(problem, dim, h, ue, me=None):
    """r_e from corner values ue (2^d, ...) or (3, 8, ...); me: corner m values."""
    kind, prm = problem.kind, problem.params
    K = element_stiffness(dim, h)
    vol = h ** dim
    if kind == 'neohooke':
        return _neohooke_vectors(h, ue, prm)
    Ku = np.einsum('ab,b...->a...', K, ue)
    if kind == 'bratu':
        phi, _, w, _ = reference_rule(dim)
        uq = np.einsum('qa,a...->q...', phi, ue)
        src = np.einsum('q,q...,qa->a...', w * vol, np.exp(uq), phi)
        return Ku - prm['lam'] * src
    if kind == 'plap':
        p, delta = prm['p'], prm['delta']
        s = np.einsum('a...,a...->...', ue, Ku) / vol
        return (delta ** 2 + s) ** ((p - 2.0) / 2.0) * Ku
    if kind == 'plap_gauss':
        p, delta = prm['p'], prm['delta']
        _, dphi, w, _ = reference_rule(dim)
        out = np.zeros_like(ue)
        for q in range(len(w)):
            g = np.einsum('ak,a...->k...', dphi[q] / h, ue)
            kq = (delta ** 2 + np.sum(g * g, axis=0)) ** ((p - 2.0) / 2.0)
            out += w[q] * vol * kq * np.einsum('ak,k...->a...', dphi[q] / h, g)
        return out
    if kind == 'invcoef':
        kbar = np.mean(np.exp(me), axis=0)
        ubar = np.mean(ue, axis=0)
        return kbar * (1.0 + ubar ** 2) * Ku
    raise ValueError(kind)


def _deformation(h, ue, q):
    """Fd = I + grad u at Gauss point q in every element, shape elem+(3,3)."""
    _, dphi, _, _ = reference_rule(3)
    G = np.einsum('ia...,aj->...ij', ue, dphi[q] / h)
    return np.eye(3) + G


def _neohooke_vectors(h, ue, prm):
    mu, lam = lame(prm['E'], prm['nu'])
    _, dphi, w, _ = reference_rule(3)
    vol = h ** 3
    out = np.zeros_like(ue)
    for q in range(len(w)):
        Fd = _deformation(h, ue, q)
        J = np.linalg.det(Fd)
        with np.errstate(invalid='ignore', divide='ignore'):
            lnJ = np.where(J > 0, np.log(np.where(J > 0, J, 1.0)), np.nan)
        FinvT = np.swapaxes(np.linalg.inv(Fd), -1, -2)
        P = mu * (Fd - FinvT) + (lam * lnJ)[..., None, None] * FinvT
        out += w[q] * vol * np.einsum('...ij,aj->ia...', P, dphi[q] / h)
    return out


# ---------------------------------------------------------------------------
# global operators
# ---------------------------------------------------------------------------
def apply_A(problem, grid, u, m=None):
    """A(u): assembled element vectors, zero at Dirichlet nodes."""
    re = element_vectors(problem, grid, u, m)
    nc = 1 if problem.ncomp > 1 else 0
    return _mask(grid, problem.ncomp, grid.scatter(re, ncomp_axes=nc))


def residual(problem, grid, u, b, m=None):
    """F(u) = A(u) - b, zero at Dirichlet nodes."""
    A = apply_A(problem, grid, u, m)
    return _mask(grid, problem.ncomp, A - b) if b is not None else A


def residual_at(problem, grid, u, b, nodes, m=None):
    """F at selected nodes only (flat node indices), by summing the element
    vectors of the elements around each node; for checks at sizes where a
    full assembly is too slow.  Returns (ncomp, len(nodes)) or (len(nodes),)."""
    nodes = np.asarray(nodes)
    d = grid.dim
    coords = np.unravel_index(nodes, grid.node_shape)            # (z, y, x) order
    xyz = [coords[d - 1 - k] for k in range(d)]                   # x, y[, z]
    nc = problem.ncomp
    out = np.zeros((nc, nodes.size))
    uf = u.reshape((nc, -1)) if nc > 1 else u.reshape((1, -1))
    mf = m.reshape(-1) if m is not None else None
    for e in range(2 ** d):
        bits = [(e >> k) & 1 for k in range(d)]
        org = [xyz[k] - bits[k] for k in range(d)]
        ok = np.ones(nodes.size, dtype=bool)
        for k in range(d):
            ok &= (org[k] >= 0) & (org[k] < grid.n[k])
        if not ok.any():
            continue
        corner_idx = []
        for a in range(2 ** d):
            ab = [(a >> k) & 1 for k in range(d)]
            c = [np.where(ok, org[k], 0) + ab[k] for k in range(d)]
            corner_idx.append(np.ravel_multi_index(tuple(reversed(c)), grid.node_shape))
        corner_idx = np.array(corner_idx)                          # (2^d, N)
        ue = uf[:, corner_idx] if nc > 1 else uf[0][corner_idx]
        me = mf[corner_idx] if mf is not None else None
        re = element_vectors_from_corners(problem, d, grid.h, ue, me)
        if nc > 1:
            out += np.where(ok, re[:, e], 0.0)
        else:
            out[0] += np.where(ok, re[e], 0.0)
    dm = grid.dirichlet_mask().reshape(-1)[nodes]
    if b is not None:
        bf = b.reshape((nc, -1)) if nc > 1 else b.reshape((1, -1))
        out -= bf[:, nodes]
    out[:, dm] = 0.0
    return out if nc > 1 else out[0]


def energy(problem, grid, u, b=None):
    """Psi_h(u) - b.u for the variational problems."""
    dim, h = grid.dim, grid.h
    prm = problem.params
    vol = h ** dim
    K = element_stiffness(dim, h)
    ext = 0.0 if b is None else float(np.sum(_mask(grid, problem.ncomp, b) * u))
    if problem.kind == 'neohooke':
        mu, lam = lame(prm['E'], prm['nu'])
        _, _, w, _ = reference_rule(3)
        ue = grid.gather(u)
        tot = 0.0
        for q in range(len(w)):
            Fd = _deformation(grid.h, ue, q)
            J = np.linalg.det(Fd)
            if np.any(J <= 0):
                return np.inf
            IC = np.einsum('...ij,...ij->...', Fd, Fd)
            lnJ = np.log(J)
            tot += w[q] * vol * np.sum(0.5 * mu * (IC - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2)
        return tot - ext
    ue = grid.gather(u)
    Ku = np.einsum('ab,b...->a...', K, ue)
    quad = np.einsum('a...,a...->...', ue, Ku)
    if problem.kind == 'bratu':
        phi, _, w, _ = reference_rule(dim)
        uq = np.einsum('qa,a...->q...', phi, ue)
        return float(np.sum(0.5 * quad) - prm['lam'] * np.sum(
            np.einsum('q,q...->...', w * vol, np.exp(uq)))) - ext
    if problem.kind == 'plap':
        p, delta = prm['p'], prm['delta']
        return float(np.sum(vol / p * (delta ** 2 + quad / vol) ** (p / 2.0))) - ext
    if problem.kind == 'plap_gauss':
        p, delta = prm['p'], prm['delta']
        _, dphi, w, _ = reference_rule(dim)
        tot = 0.0
        for q in range(len(w)):
            g = np.einsum('ak,a...->k...', dphi[q] / h, ue)
            tot += w[q] * vol * np.sum((delta ** 2 + np.sum(g * g, axis=0)) ** (p / 2.0) / p)
        return float(tot) - ext
    raise ValueError('no energy for ' + problem.kind)


# ---------------------------------------------------------------------------
# load vectors
# ---------------------------------------------------------------------------
def load_from_function(grid, f):
    """b_i = sum_e sum_q w_q f(x_q) phi_i(x_q), 2^d Gauss points; 0 on Dirichlet."""
    phi, _, w, xi = reference_rule(grid.dim)
    re = np.zeros((2 ** grid.dim,) + grid.elem_shape)
    for q in range(len(w)):
        fq = f(*grid.quad_points(xi[q]))
        re += (w[q] * grid.h ** grid.dim) * fq * phi[q].reshape((-1,) + (1,) * grid.dim)
    return _mask(grid, 1, grid.scatter(re))


def gaussian_source(centres, widths, amps):
    """f(x) = sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2))."""
    centres = np.asarray(centres, float)
    widths = np.asarray(widths, float)
    amps = np.asarray(amps, float)

    def f(*x):
        out = 0.0
        for c, wd, a in zip(centres, widths, amps):
            r2 = sum((x[k] - c[k]) ** 2 for k in range(len(x)))
            out = out + a * np.exp(-r2 / (2.0 * wd * wd))
        return out
    return f


def traction_load(grid, t, axis=0, side=1):
    """b[i, node] = int_face t_i phi_node dA on one face, 2x2 Gauss per face cell."""
    assert grid.dim == 3
    t = np.asarray(t, float)
    face_axes = [k for k in range(3) if k != axis]
    phi, _, w, _ = reference_rule(2)
    b = np.zeros((3,) + grid.node_shape)
    pos = 0 if side == 0 else grid.n[axis]
    na, nb = grid.n[face_axes[0]], grid.n[face_axes[1]]
    face = np.zeros((nb + 1, na + 1))
    for a in range(4):
        wa = np.sum(w * phi[:, a]) * grid.h ** 2
        ax, bx = a & 1, (a >> 1) & 1
        face[bx:bx + nb, ax:ax + na] += wa
    idx = [slice(None)] * 3
    idx[2 - axis] = pos
    for i in range(3):
        bi = b[i]
        # array axes of the face slice are (2-face_axes[1], 2-face_axes[0]) order
        sub = face if face_axes[1] > face_axes[0] else face.T
        bi[tuple(idx)] = t[i] * sub
    return _mask(grid, 3, b)
