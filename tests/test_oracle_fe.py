"""Pins of the oracle's Q1 discretisation against closed forms.

* The assembled Q1 stiffness equals the classical stencils
  (2D: 8/3 centre, -1/3 for all eight neighbours; 3D: 8h/3 centre,
  0 across faces, -h/6 across edges, -h/12 across corners).
* Discrete sine modes are eigenvectors with the closed-form eigenvalues
  2D: (8 - 2a - 2b - 4ab)/3,  3D: h (8/3 - 2/3 (ab+ac+bc) - 2/3 abc),
  a = cos(k_x pi h) etc.
Both stencils follow from integrating products of the 1D hat-function
stiffness [1,-1;-1,1]/h and mass h[1/3,1/6;1/6,1/3] (tensor structure),
independently of the oracle's quadrature-based element matrix.
"""
import itertools

import numpy as np

from oracle.fe import Grid
from oracle.problems import Problem, apply_A

ALL2 = [(a, s) for a in range(2) for s in range(2)]
ALL3 = [(a, s) for a in range(3) for s in range(2)]


def _linear_problem():
    return Problem('plap', {'p': 2.0, 'delta': 1.0})


def test_stencil_2d():
    g = Grid([6, 6], 1 / 6, ALL2)
    e = np.zeros(g.node_shape)
    e[3, 3] = 1.0
    col = apply_A(_linear_problem(), g, e)
    want = np.zeros(g.node_shape)
    want[2:5, 2:5] = -1.0 / 3.0
    want[3, 3] = 8.0 / 3.0
    assert np.max(np.abs(col - want)) < 1e-14


def test_stencil_3d():
    h = 0.25
    g = Grid([6, 6, 6], h, ALL3)
    e = np.zeros(g.node_shape)
    e[3, 3, 3] = 1.0
    col = apply_A(_linear_problem(), g, e)
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        nz = abs(dx) + abs(dy) + abs(dz)
        want = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[nz]
        assert abs(col[3 + dz, 3 + dy, 3 + dx] - want) < 1e-14
    col[2:5, 2:5, 2:5] = 0.0
    assert np.max(np.abs(col)) == 0.0


def test_bratu_linear_limit_is_stiffness():
    g = Grid([5, 7], 0.1, ALL2)
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, g.node_shape)
    u[g.dirichlet_mask()] = 0
    a = apply_A(Problem('bratu', {'lam': 0.0}), g, u)
    b = apply_A(_linear_problem(), g, u)
    assert np.max(np.abs(a - b)) < 1e-14


def test_sine_mode_eigenvalues_2d():
    n = 8
    h = 1.0 / n
    g = Grid([n, n], h, ALL2)
    x, y = g.node_coords()
    for kx, ky in [(1, 1), (3, 5), (7, 7), (2, 6)]:
        phi = np.sin(kx * np.pi * x) * np.sin(ky * np.pi * y)
        a, b = np.cos(kx * np.pi * h), np.cos(ky * np.pi * h)
        lam = (8 - 2 * a - 2 * b - 4 * a * b) / 3
        Kphi = apply_A(_linear_problem(), g, phi)
        assert np.max(np.abs(Kphi - lam * phi)) < 1e-13


def test_sine_mode_eigenvalues_3d():
    n = 6
    h = 1.0 / n
    g = Grid([n, n, n], h, ALL3)
    x, y, z = g.node_coords()
    for kx, ky, kz in [(1, 1, 1), (5, 5, 5), (2, 3, 4)]:
        phi = np.sin(kx * np.pi * x) * np.sin(ky * np.pi * y) * np.sin(kz * np.pi * z)
        a, b, c = (np.cos(k * np.pi * h) for k in (kx, ky, kz))
        lam = h * (8 / 3 - 2 / 3 * (a * b + a * c + b * c) - 2 / 3 * a * b * c)
        Kphi = apply_A(_linear_problem(), g, phi)
        assert np.max(np.abs(Kphi - lam * phi)) < 1e-14


def test_dirichlet_rows_vanish_and_natural_faces_stay():
    g = Grid([4, 2, 2], 0.25, [(0, 0)])
    m = g.dirichlet_mask()
    assert m[:, :, 0].all() and not m[:, :, 1:].any()
    assert g.n_dof(3) == 3 * 4 * 3 * 3
