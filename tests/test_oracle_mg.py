"""Pins of the oracle's multigrid components (Sec. 2, Algorithm 1).

* Power method: converges to the closed-form largest sine-mode eigenvalue
  of the Q1 Laplacian, and the paper's 30-iteration / 1e-2 rule gives an
  estimate within a few percent of it.
* Chebyshev: on an eigenvector with eigenvalue mu the error after a degree
  nu iteration is T_nu((theta - mu)/delta) / T_nu(theta/delta) times the
  initial error (numpy's Chebyshev series, not the recurrence).
* Coarse CG: matches a dense solve on an SPD system; on an indefinite
  system (Bratu at u = 3) it exits with negative curvature, shifts, and the
  returned correction solves the shifted system (dense solve).
* V-cycle: as a stationary iteration on the linear Q1 Laplacian its
  convergence factor is small and does not grow with the number of levels.
"""
import numpy as np
from numpy.polynomial import chebyshev as C

from oracle.derivatives import assembled_jacobian
from oracle.fe import Grid
from oracle.mg import (Level, MGOptions, Stats, chebyshev, coarse_solve, eps_numerator, fd_jv,
                       level_jv, make_grids, mg_setup, power_method, random_start, vcycle)
from oracle.problems import Problem, apply_A

ALL2 = [(a, s) for a in range(2) for s in range(2)]
ALL3 = [(a, s) for a in range(3) for s in range(2)]
LIN = Problem('plap', {'p': 2.0, 'delta': 1.0})


def _lam_max_2d(n):
    """Largest closed-form eigenvalue (8 - 2a - 2b - 4ab)/3 over all sine modes."""
    c = np.cos(np.arange(1, n) * np.pi / n)
    a, b = np.meshgrid(c, c)
    return float(np.max((8 - 2 * a - 2 * b - 4 * a * b) / 3))


def _level(pb, g, x, m=None, opts=None):
    lev = Level(grid=g, x=x, m=m)
    lev.Ax = apply_A(pb, g, x, m)
    lev.eps_num = eps_numerator(g, x, opts or MGOptions())
    return lev


def test_power_method_largest_eigenvalue():
    n = 8
    g = Grid([n, n], 1.0 / n, ALL2)
    lev = _level(LIN, g, np.zeros(g.node_shape))
    lam_max = _lam_max_2d(n)
    v0 = random_start(g, 1, 0, 1)
    lam, _, _ = power_method(lambda v: level_jv(LIN, lev, v), v0, 3000, 0.0, True)
    assert abs(lam - lam_max) < 1e-8 * lam_max
    lam30, _, it = power_method(lambda v: level_jv(LIN, lev, v), v0, 30, 1e-2, False)
    assert it <= 30 and 0.9 * lam_max < lam30 <= lam_max * (1 + 1e-12)


def test_chebyshev_damping_factor():
    n = 16
    h = 1.0 / n
    g = Grid([n, n], h, ALL2)
    lev = _level(LIN, g, np.zeros(g.node_shape))
    x, y = g.node_coords()
    lam_max = _lam_max_2d(n)
    lo, hi = 0.06, 1.2
    al, be = lo * lam_max, hi * lam_max
    theta, delta = (al + be) / 2, (be - al) / 2
    for kx, ky in [(1, 1), (4, 9), (15, 15)]:
        phi = np.sin(kx * np.pi * x) * np.sin(ky * np.pi * y)
        ca, cb = np.cos(kx * np.pi * h), np.cos(ky * np.pi * h)
        mu = (8 - 2 * ca - 2 * cb - 4 * ca * cb) / 3
        b = mu * phi
        for nu in (1, 3, 5):
            s = chebyshev(lambda v: level_jv(LIN, lev, v), b, np.zeros_like(b), nu, lam_max, lo, hi,
                          s_is_zero=True)
            Tn = C.Chebyshev.basis(nu)
            factor = Tn((theta - mu) / delta) / Tn(theta / delta)
            assert np.max(np.abs((phi - s) - factor * phi)) < 1e-9


def test_chebyshev_from_nonzero_start():
    n = 8
    g = Grid([n, n], 1.0 / n, ALL2)
    lev = _level(LIN, g, np.zeros(g.node_shape))
    J, idx = assembled_jacobian(LIN, g, np.zeros(g.node_shape))
    rng = np.random.default_rng(1)
    s0 = np.zeros(g.node_shape)
    s0[g.dof_mask()] = rng.normal(size=idx.size)
    b = np.zeros(g.node_shape)
    b[g.dof_mask()] = rng.normal(size=idx.size)
    lam = np.linalg.eigvalsh(J).max()
    s = chebyshev(lambda v: level_jv(LIN, lev, v), b, s0, 4, lam, 0.06, 1.2)
    # closed form: e_4 = p(J) e_0 with the Chebyshev residual polynomial
    e0 = np.linalg.solve(J, b[g.dof_mask()]) - s0[g.dof_mask()]
    al, be = 0.06 * lam, 1.2 * lam
    theta, delta = (al + be) / 2, (be - al) / 2
    w, V = np.linalg.eigh(J)
    p = C.Chebyshev.basis(4)((theta - w) / delta) / C.Chebyshev.basis(4)(theta / delta)
    e4 = V @ (p * (V.T @ e0))
    got = np.linalg.solve(J, b[g.dof_mask()]) - s[g.dof_mask()]
    assert np.max(np.abs(got - e4)) < 1e-8 * np.max(np.abs(e0))


def test_coarse_cg_spd_matches_dense():
    g = Grid([8, 8], 1.0 / 8, ALL2)
    pb = Problem('bratu', {'lam': 5.0})
    rng = np.random.default_rng(2)
    x = np.zeros(g.node_shape)
    x[g.dof_mask()] = 0.3 * rng.uniform(size=int(g.dof_mask().sum()))
    lev = _level(pb, g, x)
    J, idx = assembled_jacobian(pb, g, x)
    assert np.linalg.eigvalsh(J).min() > 0
    r0 = np.zeros(g.node_shape)
    r0[g.dof_mask()] = rng.normal(size=idx.size)
    opts = MGOptions(coarse_rtol=1e-10)
    s, shift, _ = coarse_solve(lambda v: level_jv(pb, lev, v), r0, idx.size, opts)
    assert shift == 0.0
    ref = np.linalg.solve(J, r0[g.dof_mask()])
    assert np.max(np.abs(s[g.dof_mask()] - ref)) < 1e-6 * np.max(np.abs(ref))


def test_coarse_cg_indefinite_shift():
    g = Grid([8, 8], 1.0 / 8, ALL2)
    pb = Problem('bratu', {'lam': 5.0})
    x = np.full(g.node_shape, 3.0)
    x[g.dirichlet_mask()] = 0
    lev = _level(pb, g, x)
    J, idx = assembled_jacobian(pb, g, x)
    ev = np.linalg.eigvalsh(J)
    assert (ev < 0).sum() == 4                   # indefinite
    r0 = np.zeros(g.node_shape)
    r0[g.dof_mask()] = np.sin(np.arange(idx.size))
    st = Stats()
    opts = MGOptions(coarse_rtol=1e-10)
    s, shift, iters = coarse_solve(lambda v: level_jv(pb, lev, v), r0, idx.size, opts, st)
    assert st.neg_curv >= 1 and shift < 0 and len(iters) >= 2
    assert np.linalg.eigvalsh(J - shift * np.eye(idx.size)).min() > 0
    ref = np.linalg.solve(J - shift * np.eye(idx.size), r0[g.dof_mask()])
    assert np.max(np.abs(s[g.dof_mask()] - ref)) < 1e-5 * np.max(np.abs(ref))


def _vcycle_factor(n, nlev, dim):
    faces = ALL2 if dim == 2 else ALL3
    g = Grid([n] * dim, 1.0 / n, faces)
    grids = make_grids(g, nlev)
    opts = MGOptions(nu_pre=3, nu_post=3)
    levels = mg_setup(LIN, grids, np.zeros(g.node_shape), None, opts)
    rng = np.random.default_rng(3)
    b = rng.normal(size=g.node_shape)
    b[g.dirichlet_mask()] = 0
    s = np.zeros_like(b)
    rn = []
    top = levels[-1]
    for _ in range(6):
        r = b - level_jv(LIN, top, s)
        rn.append(np.sqrt(np.sum(r * r)))
        s = s + vcycle(LIN, levels, nlev - 1, r, opts)
    return (rn[-1] / rn[1]) ** (1 / 4)


def test_vcycle_level_independent():
    f2 = _vcycle_factor(16, 2, 2)
    f4 = _vcycle_factor(64, 4, 2)
    f3d = _vcycle_factor(16, 3, 3)
    # two-grid bound of V(3,3): 1 / T_3(theta/delta)^2 ~ 0.23 on [0.06, 1.2] lam
    bound = 1.0 / C.Chebyshev.basis(3)(0.63 / 0.57) ** 2
    assert max(f2, f4, f3d) < bound, (f2, f4, f3d, bound)
    assert abs(f4 - f2) < 0.02


def test_fd_jv_zero_direction():
    g = Grid([4, 4], 0.25, ALL2)
    lev = _level(LIN, g, np.zeros(g.node_shape))
    assert np.all(level_jv(LIN, lev, np.zeros(g.node_shape)) == 0.0)
    assert np.all(fd_jv(LIN, g, lev.x, lev.Ax, np.ones(g.node_shape), None, 0.0) == 0.0)
