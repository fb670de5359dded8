"""The paper's solver settings and its minimal-surface experiment in the oracle
(Sec. 3: minimal surface; setup; Tables 1 and 2).

* Minimal surface = the p-Laplacian energy with p = 1, delta = 1:
  Psi = int sqrt(1 + |grad u|^2).  On an affine state the element-mean
  coefficient is exact, so Psi_h is the area of the plane,
  sqrt(1 + a^2 + b^2) on the unit square, and F vanishes at every interior
  node (a plane is a minimal surface).
* Scherk's first surface z = ln(cos(2(y - 1/2)) / cos(2(x - 1/2))) / 2
  solves the minimal-surface equation; with its values as Dirichlet data
  the oracle's CG-MG Newton solution converges to it at O(h^2) in the max
  norm (error ratios > 3.5 per halving of h).
* The preset settings are the constants the paper states
  (tests/golden/paper_setup.txt).
* Table 2 trends on Q1 grids with the paper's 25 x 25 coarse mesh, L1-L3:
  Bratu needs the same number of Newton steps on every level and a
  level-independent number of effective gradient evaluations; the minimal
  surface needs more Newton steps as the mesh is refined.  The counts stay
  within one Newton step and two CG-MG steps of the paper's
  (tests/golden/paper_table2.txt; the paper's elements are triangles).
"""
import os

import numpy as np
import pytest

from oracle import newton as ON
from oracle.fe import Grid
from oracle.mg import MGOptions
from oracle.problems import Problem, energy, residual
from paper_2103_13890_amd import workloads as W

ALL2 = [(a, s) for a in range(2) for s in range(2)]
HERE = os.path.dirname(__file__)
MINSURF = Problem('plap', {'p': 1.0, 'delta': 1.0})


def _golden(name):
    rows = []
    for line in open(os.path.join(HERE, 'golden', name)):
        line = line.strip()
        if line and not line.startswith('#'):
            rows.append(line.split())
    return rows


def paper_mg_options():
    return MGOptions(nu_pre=5, nu_post=5, power_maxit=30, power_rtol=1e-2, eps_mode='paper', coarse_atol=1e-12,
                     coarse_rtol=0.0, coarse_qn=20, shift_gamma=5.0)


def paper_newton_options():
    return ON.NewtonOptions(rtol=0.0, atol=1e-6, forcing='paper', outer='cg')


def test_minsurf_affine_state_is_a_plane():
    n = 8
    g = Grid([n, n], 1.0 / n, ALL2)
    X, Y = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n)
    a, b = 0.7, -0.4
    u = 0.3 + a * X + b * Y
    zero = np.zeros(g.node_shape)
    assert abs(energy(MINSURF, g, u, zero) - np.sqrt(1 + a * a + b * b)) < 1e-14
    assert np.max(np.abs(residual(MINSURF, g, u, zero))) < 1e-14


def test_scherk_surface_convergence():
    def scherk(x, y):
        return np.log(np.cos(2.0 * (y - 0.5)) / np.cos(2.0 * (x - 0.5))) / 2.0
    errs = []
    for n, L in ((8, 2), (16, 3), (32, 4)):
        g = Grid([n, n], 1.0 / n, ALL2)
        X, Y = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n)
        ex = scherk(X, Y)
        u0 = np.zeros(g.node_shape)
        m = g.dirichlet_mask()
        u0[m] = ex[m]
        u, rep = ON.solve(MINSURF, g, L, u0, np.zeros(g.node_shape), None, MGOptions(nu_pre=5, nu_post=5),
                          ON.NewtonOptions(rtol=1e-10, outer='cg'))
        assert rep.status == 'ok'
        assert np.array_equal(u[m], ex[m])
        errs.append(np.max(np.abs(u - ex)))
    assert errs[-1] < 5e-5
    assert all(errs[i] / errs[i + 1] > 3.5 for i in range(len(errs) - 1)), errs


def test_preset_settings_are_the_papers():
    gd = {k: float(v) for k, v in _golden('paper_setup.txt')}
    o = W.PAPER_OPTIONS
    assert o['nu_pre'] == o['nu_post'] == gd['nu_paper']
    assert o['power_maxit'] == gd['power_maxit'] and o['power_rtol'] == gd['power_rtol']
    assert o['coarse_atol'] == gd['coarse_atol'] and o['coarse_rtol'] == 0.0
    assert o['shift_gamma'] == gd['shift_gamma'] and o['coarse_qn'] == gd['lbfgs_pairs']
    assert o['newton_atol'] == gd['newton_atol_paper'] and o['newton_rtol'] == 0.0
    assert o['outer_krylov'] == 1 and o['forcing'] == 1 and o['eps_mode'] == 1
    for name in ('bratu2d-800', 'minsurf2d-800'):
        w = W.WORKLOADS[name]
        assert w['n'] == (800, 800) and w['nlevels'] == 6 and (w['n'][0] >> 5) == 25
    assert W.WORKLOADS['minsurf2d-800']['params'] == (1.0, 1.0)


def _solve(name, level):
    n = 25 << level
    w = W.scaled(name, (n, n), nlevels=level + 1)
    g = Grid(w['n'], w['h'], w['faces'])
    pb = MINSURF if name.startswith('minsurf') else Problem('bratu', {'lam': w['params'][0]})
    u0 = W.dirichlet_state(w)
    u, rep = ON.solve(pb, g, level + 1, u0, np.zeros(g.node_shape), None, paper_mg_options(),
                      paper_newton_options())
    assert rep.status == 'ok'
    assert rep.fnorm[-1] <= 1e-6
    return rep


@pytest.mark.parametrize('problem', ['bratu', 'minsurf'])
def test_table2_trends(problem):
    table = {(r[0], r[1]): (int(r[2]), int(r[3])) for r in _golden('paper_table2.txt')}
    name = 'bratu2d-800' if problem == 'bratu' else 'minsurf2d-800'
    ins, cgs, ges = [], [], []
    for level in (1, 2, 3):
        rep = _solve(name, level)
        ins.append(rep.newton_iters)
        cgs.append(rep.linear_iters)
        ges.append(rep.stats.effective_ge(2, level))
        p_in, p_cg = table[(problem, 'L%d' % level)]
        assert abs(rep.newton_iters - p_in) <= 1, (level, rep.newton_iters, p_in)
        assert abs(rep.linear_iters - p_cg) <= 2, (level, rep.linear_iters, p_cg)
    if problem == 'bratu':
        assert len(set(ins)) == 1, ins
        assert max(ges) < 1.25 * min(ges), ges
    else:
        assert ins[0] < ins[1] < ins[2], ins
        assert cgs[0] < cgs[1] < cgs[2], cgs
