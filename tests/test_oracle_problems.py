"""Pins of the oracle's residuals.

* F = grad Psi_h: central differences of the discrete energy (written from
  the energies of Sec. 3) against F along random directions.
* Manufactured solutions: with f derived symbolically (sympy) from each
  strong form, the discrete solution converges at O(h^2) in the nodal max
  norm (error ratio near 4 per halving of h).
* 1D Bratu closed form u = -2 ln[cosh((x - 1/2) t / 2) / cosh(t / 4)],
  t = sqrt(2 lam) cosh(t / 4) (lower root, found with scipy's brentq).
* Neo-Hookean patch test: under a homogeneous deformation the stress is
  constant, so the residual vanishes at every interior node.
* The Gauss-point p-Laplacian: for p = 2 both p-Laplacian residuals are the
  exact Q1 stiffness (2^d Gauss points integrate it exactly), and on an
  affine state the gradient is the same at every point, so the Gauss and
  element-mean residuals agree there; elsewhere they differ.  Its 2D
  manufactured solution converges at O(h^2).
"""
import numpy as np
import pytest
import scipy.optimize
import sympy

from oracle import newton
from oracle.fe import Grid
from oracle.mg import MGOptions
from oracle.problems import Problem, apply_A, energy, load_from_function, residual

ALL = {1: [(0, 0), (0, 1)], 2: [(a, s) for a in range(2) for s in range(2)],
       3: [(a, s) for a in range(3) for s in range(2)]}


def _rand_state(g, rng, scale=0.5, nc=1):
    shape = g.node_shape if nc == 1 else (nc,) + g.node_shape
    u = scale * rng.uniform(-1, 1, shape)
    if nc == 1:
        u[g.dirichlet_mask()] = 0
    else:
        u[:, g.dirichlet_mask()] = 0
    return u


@pytest.mark.parametrize('kind,dim,prm', [
    ('bratu', 2, {'lam': 5.0}),
    ('bratu', 3, {'lam': 2.0}),
    ('plap', 3, {'p': 3.0, 'delta': 1e-2}),
    ('plap', 2, {'p': 4.0, 'delta': 0.1}),
    ('plap_gauss', 3, {'p': 3.0, 'delta': 1e-2}),
])
def test_residual_is_energy_gradient(kind, dim, prm):
    rng = np.random.default_rng(11)
    g = Grid([5] * dim, 0.2, ALL[dim])
    pb = Problem(kind, prm)
    u = _rand_state(g, rng)
    b = _rand_state(g, rng, 0.1)
    F = residual(pb, g, u, b)
    for _ in range(3):
        d = _rand_state(g, rng, 1.0)
        t = 1e-5
        fd = (energy(pb, g, u + t * d, b) - energy(pb, g, u - t * d, b)) / (2 * t)
        assert abs(fd - np.sum(F * d)) <= 1e-7 * max(1.0, abs(fd))


def test_neohooke_is_energy_gradient():
    rng = np.random.default_rng(12)
    g = Grid([4, 2, 2], 0.25, [(0, 0)])
    pb = Problem('neohooke', {'E': 1.0, 'nu': 0.3})
    u = _rand_state(g, rng, 0.05, 3)
    b = _rand_state(g, rng, 0.01, 3)
    F = residual(pb, g, u, b)
    for _ in range(3):
        d = _rand_state(g, rng, 1.0, 3)
        t = 1e-6
        fd = (energy(pb, g, u + t * d, b) - energy(pb, g, u - t * d, b)) / (2 * t)
        assert abs(fd - np.sum(F * d)) <= 1e-7 * max(1e-3, abs(fd))


def test_neohooke_patch_test():
    rng = np.random.default_rng(13)
    g = Grid([4, 3, 3], 0.25, [(0, 0)])
    G = 0.1 * rng.uniform(-1, 1, (3, 3))
    x = g.node_coords()
    u = np.stack([sum(G[i, j] * x[j] for j in range(3)) for i in range(3)])
    A = apply_A(Problem('neohooke', {'E': 1.0, 'nu': 0.3}), g, u)
    interior = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.max(np.abs(A[interior])) < 1e-14
    assert np.max(np.abs(A)) > 1e-4          # boundary nodes carry the traction
    zero = apply_A(Problem('neohooke', {'E': 1.0, 'nu': 0.3}), g, 0 * u)
    assert np.max(np.abs(zero)) == 0.0


# ---------------------------------------------------------------------------
def _solve(pb, g, levels, b, m=None, rtol=1e-11):
    nc = pb.ncomp
    shape = g.node_shape if nc == 1 else (nc,) + g.node_shape
    u, rep = newton.solve(pb, g, levels, np.zeros(shape), b, m,
                          MGOptions(nu_pre=3, nu_post=3), newton.NewtonOptions(rtol=rtol))
    assert rep.status == 'ok', rep.status
    return u


def _mms(dim, strong, u_expr, xs):
    f_expr = strong(u_expr)
    f = sympy.lambdify(xs, f_expr, 'numpy')
    u = sympy.lambdify(xs, u_expr, 'numpy')
    return f, u


def _rates(errs):
    return [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]


@pytest.mark.slow
def test_mms_plap_3d():
    X = sympy.symbols('x y z')
    p, delta = 3, sympy.Rational(1, 100)
    ue = sympy.sin(sympy.pi * X[0]) * sympy.sin(sympy.pi * X[1]) * sympy.sin(sympy.pi * X[2])
    grad = [sympy.diff(ue, v) for v in X]
    k = (delta ** 2 + sum(gi ** 2 for gi in grad)) ** sympy.Rational(p - 2, 2)
    f_expr = -sum(sympy.diff(k * gi, v) for gi, v in zip(grad, X))
    f = sympy.lambdify(X, f_expr, 'numpy')
    uex = sympy.lambdify(X, ue, 'numpy')
    pb = Problem('plap', {'p': float(p), 'delta': 0.01})
    errs = []
    for n in (8, 16, 32):
        g = Grid([n] * 3, 1.0 / n, ALL[3])
        u = _solve(pb, g, 2, load_from_function(g, f))
        errs.append(np.max(np.abs(u - uex(*g.node_coords()))))
    r = _rates(errs)
    assert r[-1] > 3.5 and r[-1] < 4.6, (errs, r)


def test_mms_bratu_2d():
    X = sympy.symbols('x y')
    lam = 5.0
    ue = sympy.Rational(1, 2) * sympy.sin(sympy.pi * X[0]) * sympy.sin(sympy.pi * X[1])
    f_expr = -sum(sympy.diff(ue, v, 2) for v in X) - lam * sympy.exp(ue)
    f = sympy.lambdify(X, f_expr, 'numpy')
    uex = sympy.lambdify(X, ue, 'numpy')
    pb = Problem('bratu', {'lam': lam})
    errs = []
    for n in (16, 32, 64):
        g = Grid([n] * 2, 1.0 / n, ALL[2])
        u = _solve(pb, g, 3, load_from_function(g, f))
        errs.append(np.max(np.abs(u - uex(*g.node_coords()))))
    r = _rates(errs)
    assert 3.5 < r[-1] < 4.6, (errs, r)


@pytest.mark.slow
def test_mms_invcoef_3d():
    X = sympy.symbols('x y z')
    ue = sympy.sin(sympy.pi * X[0]) * sympy.sin(sympy.pi * X[1]) * sympy.sin(sympy.pi * X[2])
    me = sympy.Rational(3, 10) * sympy.cos(2 * X[0] + X[1] - X[2])
    coef = sympy.exp(me) * (1 + ue ** 2)
    f_expr = -sum(sympy.diff(coef * sympy.diff(ue, v), v) for v in X)
    f = sympy.lambdify(X, f_expr, 'numpy')
    uex = sympy.lambdify(X, ue, 'numpy')
    mex = sympy.lambdify(X, me, 'numpy')
    pb = Problem('invcoef')
    errs = []
    for n in (8, 16, 32):
        g = Grid([n] * 3, 1.0 / n, ALL[3])
        m = mex(*g.node_coords()) * np.ones(g.node_shape)
        u = _solve(pb, g, 2, load_from_function(g, f), m)
        errs.append(np.max(np.abs(u - uex(*g.node_coords()))))
    r = _rates(errs)
    assert 3.5 < r[-1] < 4.6, (errs, r)


def test_bratu_1d_closed_form():
    lam = 1.0
    theta = scipy.optimize.brentq(lambda t: t - np.sqrt(2 * lam) * np.cosh(t / 4), 0.0, 4.0)

    def exact(x):
        return -2.0 * np.log(np.cosh((x - 0.5) * theta / 2) / np.cosh(theta / 4))
    pb = Problem('bratu', {'lam': lam})
    errs = []
    for n in (32, 64, 128):
        g = Grid([n], 1.0 / n, ALL[1])
        u = _solve(pb, g, 3, np.zeros(g.node_shape))
        errs.append(np.max(np.abs(u - exact(g.node_coords()[0]))))
    r = _rates(errs)
    assert 3.8 < r[-1] < 4.2, (errs, r)
    assert errs[-1] < 1e-5


@pytest.mark.parametrize('dim', [2, 3])
def test_plap_gauss_reductions(dim):
    rng = np.random.default_rng(21)
    g = Grid([4] * dim, 0.25, ALL[dim])
    zero = np.zeros(g.node_shape)
    u = _rand_state(g, rng)
    for prm in ({'p': 2.0, 'delta': 0.3}, {'p': 3.0, 'delta': 1e-2}):
        Fg = apply_A(Problem('plap_gauss', prm), g, u)
        Fm = apply_A(Problem('plap', prm), g, u)
        if prm['p'] == 2.0:
            assert np.max(np.abs(Fg - Fm)) < 1e-13
        else:
            assert np.max(np.abs(Fg - Fm)) > 1e-3
    xs = g.node_coords()
    aff = 0.2 + sum((0.5 - 0.3 * k) * x for k, x in enumerate(xs))
    prm = {'p': 3.0, 'delta': 1e-2}
    assert np.max(np.abs(apply_A(Problem('plap_gauss', prm), g, aff) - apply_A(Problem('plap', prm), g, aff))) < 1e-13
    assert abs(energy(Problem('plap_gauss', prm), g, aff, zero) - energy(Problem('plap', prm), g, aff, zero)) < 1e-13


def test_mms_plap_gauss_2d():
    X = sympy.symbols('x y')
    p, delta = 3, sympy.Rational(1, 10)
    ue = sympy.sin(sympy.pi * X[0]) * sympy.sin(sympy.pi * X[1])
    grad = [sympy.diff(ue, v) for v in X]
    k = (delta ** 2 + sum(gi ** 2 for gi in grad)) ** sympy.Rational(p - 2, 2)
    f = sympy.lambdify(X, -sum(sympy.diff(k * gi, v) for gi, v in zip(grad, X)), 'numpy')
    uex = sympy.lambdify(X, ue, 'numpy')
    pb = Problem('plap_gauss', {'p': float(p), 'delta': 0.1})
    errs = []
    for n in (16, 32, 64):
        g = Grid([n] * 2, 1.0 / n, ALL[2])
        u = _solve(pb, g, 2, load_from_function(g, f))
        errs.append(np.max(np.abs(u - uex(*g.node_coords()))))
    r = _rates(errs)
    assert r[-1] > 3.5 and r[-1] < 4.6, (errs, r)
