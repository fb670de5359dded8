"""Pins of the oracle's transfer operators (Sec. 2, transfer operators).

* I reproduces multilinear functions exactly (nested Q1 spaces).
* Galerkin identity I^T K_fine I = K_coarse for the Q1 stiffness on all
  nodes (nested spaces with exact integration).
* P maps constants to constants (the stated purpose of the 2^-d factor);
  at coarse interior nodes P equals 2^-d I^T exactly.
* R is the transpose of I on the DoF spaces.
"""
import numpy as np

from oracle.fe import Grid
from oracle.problems import Problem, apply_A
from oracle.transfer import interpolation, project, prolong, restrict

ALL3 = [(a, s) for a in range(3) for s in range(2)]


def test_interpolation_reproduces_multilinear():
    c = Grid([3, 2, 4], 0.5, [])
    fine = Grid([6, 4, 8], 0.25, [])

    def fun(x, y, z):
        return (1 + 2 * x) * (3 - y) * (0.5 + z) + 0.7
    xc = fun(*c.node_coords())
    I = interpolation(c)
    xf = (I @ xc.reshape(-1)).reshape(fine.node_shape)
    assert np.max(np.abs(xf - fun(*fine.node_coords()))) < 1e-14


def _full_stiffness(g):
    pb = Problem('plap', {'p': 2.0, 'delta': 1.0})
    n = g.n_nodes
    K = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        K[:, j] = apply_A(pb, g, e.reshape(g.node_shape)).reshape(-1)
    return K


def test_galerkin_identity():
    fine = Grid([4, 2, 4], 0.25, [])
    coarse = fine.coarsen()
    I = interpolation(coarse).toarray()
    Kf, Kc = _full_stiffness(fine), _full_stiffness(coarse)
    assert np.max(np.abs(I.T @ Kf @ I - Kc)) < 1e-14


def test_projection_preserves_constants():
    fine = Grid([8, 4, 6], 0.125, [(0, 0)])
    coarse = fine.coarsen()
    x = np.full(fine.node_shape, 2.5)
    assert np.max(np.abs(project(coarse, fine, x) - 2.5)) == 0.0
    rng = np.random.default_rng(4)
    y = rng.normal(size=fine.node_shape)
    py = project(coarse, fine, y)
    IT = interpolation(coarse).T @ y.reshape(-1)
    inner = (slice(1, -1),) * 3
    assert np.max(np.abs(py[inner] - (IT.reshape(coarse.node_shape) / 8.0)[inner])) == 0.0
    assert np.all(py[:, :, 0] == y[::2, ::2, 0])   # Dirichlet face: injection


def test_restriction_is_transpose():
    fine = Grid([8, 6, 4], 0.125, ALL3)
    coarse = fine.coarsen()
    rng = np.random.default_rng(5)
    r = rng.normal(size=fine.node_shape)
    r[fine.dirichlet_mask()] = 0
    c = rng.normal(size=coarse.node_shape)
    c[coarse.dirichlet_mask()] = 0
    lhs = np.sum(restrict(coarse, fine, r) * c)
    rhs = np.sum(r * prolong(coarse, fine, c))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
