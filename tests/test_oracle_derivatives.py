"""Pins of the oracle's exact derivatives and of its FD Jacobian action.

* Exact JVP against central differences of F (O(t^2) truncation).
* Dot-product identity <J v, w> = <v, J^T w> for the VJP.
* Symmetry of the assembled Jacobian for the variational problems
  (Sec. 1: F = grad Psi gives a symmetric J).
* Coefficient VJP against central differences in m.
* FD Jv (Sec. 1) against the exact JVP: error of the order of the step.
"""
import numpy as np
import pytest

from oracle.derivatives import assembled_jacobian, jvp, vjp, vjp_coef
from oracle.fe import Grid
from oracle.mg import EPS64, fd_jv
from oracle.problems import Problem, apply_A, residual

ALL = {2: [(a, s) for a in range(2) for s in range(2)],
       3: [(a, s) for a in range(3) for s in range(2)]}
CASES = [
    ('bratu', 2, {'lam': 5.0}),
    ('plap', 3, {'p': 3.0, 'delta': 1e-2}),
    ('plap_gauss', 3, {'p': 3.0, 'delta': 1e-2}),
    ('invcoef', 3, {}),
    ('neohooke', 3, {'E': 1.0, 'nu': 0.3}),
]


def _setup(kind, dim, prm, seed=0):
    rng = np.random.default_rng(seed)
    if kind == 'neohooke':
        g = Grid([4, 2, 2], 0.25, [(0, 0)])
        shape = (3,) + g.node_shape
        scale = 0.05
    else:
        g = Grid([4] * dim, 0.25, ALL[dim])
        shape = g.node_shape
        scale = 0.8
    dm = g.dirichlet_mask()

    def vec(s):
        v = s * rng.uniform(-1, 1, shape)
        if len(shape) == g.dim:
            v[dm] = 0
        else:
            v[:, dm] = 0
        return v
    m = 0.5 * rng.normal(size=g.node_shape) if kind == 'invcoef' else None
    return Problem(kind, prm), g, vec(scale), vec(1.0), vec(1.0), m


@pytest.mark.parametrize('kind,dim,prm', CASES)
def test_jvp_matches_central_difference(kind, dim, prm):
    pb, g, u, v, _, m = _setup(kind, dim, prm)
    t = 1e-5
    fd = (apply_A(pb, g, u + t * v, m) - apply_A(pb, g, u - t * v, m)) / (2 * t)
    ex = jvp(pb, g, u, v, m)
    assert np.max(np.abs(fd - ex)) <= 1e-7 * np.max(np.abs(ex))


@pytest.mark.parametrize('kind,dim,prm', CASES)
def test_vjp_dot_product(kind, dim, prm):
    pb, g, u, v, w, m = _setup(kind, dim, prm, 1)
    lhs = np.sum(jvp(pb, g, u, v, m) * w)
    rhs = np.sum(v * vjp(pb, g, u, w, m))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


@pytest.mark.parametrize('kind,dim,prm', [c for c in CASES if c[0] != 'invcoef'])
def test_assembled_jacobian_symmetric(kind, dim, prm):
    pb, g, u, _, _, m = _setup(kind, dim, prm, 2)
    J, _ = assembled_jacobian(pb, g, u, m)
    assert np.max(np.abs(J - J.T)) <= 1e-14 * np.max(np.abs(J)) * 10


def test_invcoef_jacobian_not_symmetric():
    pb, g, u, _, _, m = _setup('invcoef', 3, {}, 3)
    J, _ = assembled_jacobian(pb, g, u, m)
    assert np.max(np.abs(J - J.T)) > 1e-3 * np.max(np.abs(J))


def test_coefficient_vjp_central_difference():
    pb, g, u, _, lam, m = _setup('invcoef', 3, {}, 4)
    b = np.zeros(g.node_shape)
    gm = vjp_coef(pb, g, u, lam, m)
    rng = np.random.default_rng(9)
    for _ in range(3):
        dm = rng.normal(size=g.node_shape)
        t = 1e-5
        fd = np.sum(lam * (residual(pb, g, u, b, m + t * dm) - residual(pb, g, u, b, m - t * dm))) / (2 * t)
        assert abs(fd - np.sum(gm * dm)) <= 1e-8 * max(1.0, abs(fd))


@pytest.mark.parametrize('kind,dim,prm', CASES)
def test_fd_jv_against_exact(kind, dim, prm):
    pb, g, u, v, _, m = _setup(kind, dim, prm, 5)
    Au = apply_A(pb, g, u, m)
    ex = jvp(pb, g, u, v, m)
    nv = np.sqrt(np.sum(v * v))
    eps = np.sqrt(EPS64) * (1 + np.sqrt(np.sum(u * u))) / nv
    err = np.max(np.abs(fd_jv(pb, g, u, Au, v, m, eps) - ex)) / np.max(np.abs(ex))
    assert err < 1e-6
