"""Pins of the oracle's L-BFGS coarse preconditioner (CG-QN: Sec. 2, coarse
level solver; Sec. 3, setup, after Morales and Nocedal 2000).

* The two-loop recursion equals the dense BFGS inverse update
  H+ = (I - rho s y^T) H (I - rho y s^T) + rho s s^T applied pair by pair
  from H_0 = gamma I (an independent matrix formula).
* Quadratic termination: the n pairs of an n-step CG run on an SPD system
  give H = A^-1 (a classical property of BFGS with exact line searches on a
  quadratic), so H r matches a dense solve.
* Preconditioned CG with the exact inverse converges in one step.
* Uniform sampling keeps steps floor(i t / m), all of them when t <= m.
* On the coarse Bratu systems: the first coarse solve records at most m
  pairs with positive curvature and returns the same correction as plain
  CG; a later solve is preconditioned, reaches the dense solution and needs
  fewer iterations; on the indefinite system the preconditioned solve still
  exits with negative curvature, shifts, and solves the shifted system.
"""
import numpy as np

from oracle.derivatives import assembled_jacobian
from oracle.fe import Grid
from oracle.mg import (Level, MGOptions, Stats, cg_shifted, coarse_solve, eps_numerator, lbfgs_apply,
                       level_jv, uniform_sample)
from oracle.problems import Problem, apply_A

ALL2 = [(a, s) for a in range(2) for s in range(2)]


def _spd(n, seed, cond=30.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


def _level(pb, g, x):
    lev = Level(grid=g, x=x, m=None)
    lev.Ax = apply_A(pb, g, x, None)
    lev.eps_num = eps_numerator(g, x, MGOptions())
    return lev


def test_two_loop_equals_dense_bfgs():
    n = 12
    A = _spd(n, 1)
    rng = np.random.default_rng(2)
    pairs = []
    for _ in range(5):
        s = rng.normal(size=n)
        pairs.append((s, A @ s))
    s_m, y_m = pairs[-1]
    H = (s_m @ y_m) / (y_m @ y_m) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / (s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    r = rng.normal(size=n)
    ref = H @ r
    got = lbfgs_apply(pairs, r)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # secant condition of the newest pair: H y = s
    assert np.allclose(lbfgs_apply(pairs, pairs[-1][1]), pairs[-1][0], rtol=1e-10, atol=1e-12)


def test_quadratic_termination():
    n = 10
    A = _spd(n, 3, cond=20.0)
    b = np.random.default_rng(4).normal(size=n)
    rec = []
    s, lam, it = cg_shifted(lambda v: A @ v, b, np.zeros(n), 0.0, n, 0.0, None, rec)
    assert lam == 0.0 and len(rec) == n
    assert all(float(sk @ yk) > 0 for sk, yk in rec)
    Ainv = np.linalg.inv(A)
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        assert np.max(np.abs(lbfgs_apply(rec, e) - Ainv[:, j])) < 1e-8 * np.max(np.abs(Ainv))


def test_pcg_exact_inverse_one_step():
    n = 15
    A = _spd(n, 5, cond=1e3)
    b = np.random.default_rng(6).normal(size=n)
    s, lam, it = cg_shifted(lambda v: A @ v, b, np.zeros(n), 0.0, n, 1e-12 * np.linalg.norm(b),
                            lambda r: np.linalg.solve(A, r))
    assert it == 1 and lam == 0.0
    assert np.max(np.abs(A @ s - b)) < 1e-10 * np.max(np.abs(b))


def test_uniform_sample():
    assert uniform_sample(5, 20) == [0, 1, 2, 3, 4]
    assert uniform_sample(20, 20) == list(range(20))
    got = uniform_sample(45, 20)
    assert got == [(i * 45) // 20 for i in range(20)]
    assert got[0] == 0 and got[-1] == 42 and len(set(got)) == 20


def test_coarse_qn_spd():
    g = Grid([8, 8], 1.0 / 8, ALL2)
    pb = Problem('bratu', {'lam': 5.0})
    rng = np.random.default_rng(7)
    x = np.zeros(g.node_shape)
    x[g.dof_mask()] = 0.3 * rng.uniform(size=int(g.dof_mask().sum()))
    lev = _level(pb, g, x)
    J, idx = assembled_jacobian(pb, g, x)
    Jv = lambda v: level_jv(pb, lev, v)          # noqa: E731
    opts0 = MGOptions(coarse_rtol=1e-10)
    opts = MGOptions(coarse_rtol=1e-10, coarse_qn=6)
    r1 = np.zeros(g.node_shape)
    r1[g.dof_mask()] = rng.normal(size=idx.size)
    qn = {}
    s_plain, _, it_plain = coarse_solve(Jv, r1, idx.size, opts0)
    s_rec, _, it_rec = coarse_solve(Jv, r1, idx.size, opts, None, qn)
    # recording run: plain CG, bitwise
    assert it_rec == it_plain and np.array_equal(s_rec, s_plain)
    pairs = qn['pairs']
    assert 0 < len(pairs) <= 6 and all(float(np.sum(s * y)) > 0 for s, y in pairs)
    # a second right-hand side: preconditioned, fewer steps, same solution
    r2 = np.zeros(g.node_shape)
    r2[g.dof_mask()] = rng.normal(size=idx.size)
    s_p, _, it_p = coarse_solve(Jv, r2, idx.size, opts0)
    s_q, _, it_q = coarse_solve(Jv, r2, idx.size, opts, None, qn)
    assert it_q[0] < it_p[0]
    ref = np.linalg.solve(J, r2[g.dof_mask()])
    assert np.max(np.abs(s_q[g.dof_mask()] - ref)) < 1e-6 * np.max(np.abs(ref))


def test_coarse_qn_indefinite_shift():
    g = Grid([8, 8], 1.0 / 8, ALL2)
    pb = Problem('bratu', {'lam': 5.0})
    # pairs recorded on the SPD system at u = 0.3 U, then used at u = 3
    rng = np.random.default_rng(8)
    x0 = np.zeros(g.node_shape)
    x0[g.dof_mask()] = 0.3 * rng.uniform(size=int(g.dof_mask().sum()))
    lev0 = _level(pb, g, x0)
    idx_n = int(g.dof_mask().sum())
    r0 = np.zeros(g.node_shape)
    r0[g.dof_mask()] = np.sin(np.arange(idx_n))
    opts = MGOptions(coarse_rtol=1e-10, coarse_qn=20)
    qn = {}
    coarse_solve(lambda v: level_jv(pb, lev0, v), r0, idx_n, opts, None, qn)
    assert qn['pairs']
    x = np.full(g.node_shape, 3.0)
    x[g.dirichlet_mask()] = 0
    lev = _level(pb, g, x)
    J, idx = assembled_jacobian(pb, g, x)
    st = Stats()
    s, shift, iters = coarse_solve(lambda v: level_jv(pb, lev, v), r0, idx.size, opts, st, qn)
    assert st.neg_curv >= 1 and shift < 0 and len(iters) >= 2
    assert np.linalg.eigvalsh(J - shift * np.eye(idx.size)).min() > 0
    ref = np.linalg.solve(J - shift * np.eye(idx.size), r0[g.dof_mask()])
    assert np.max(np.abs(s[g.dof_mask()] - ref)) < 1e-5 * np.max(np.abs(ref))
