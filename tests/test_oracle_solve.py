"""Solver-level checks of the oracle.

* The paper's constants (tests/golden/paper_setup.txt, each line cited to
  its section) are the oracle's defaults.
* Bratu, lam = 5: the number of effective gradient evaluations and of
  Newton steps does not grow with the number of levels -- the trend of
  Tables 1 and 2 (qualitative: the paper's meshes and outer solver differ).
* The regularised p-Laplacian is strictly convex: two starting guesses give
  the same solution.
* Bratu above the critical parameter (lam = 7 > 6.81 in 2D) has no
  solution: the solver must report failure, not a converged state.
"""
import os

import numpy as np

from oracle import newton
from oracle.fe import Grid
from oracle.mg import MGOptions
from oracle.problems import Problem, gaussian_source, load_from_function, residual

ALL2 = [(a, s) for a in range(2) for s in range(2)]
ALL3 = [(a, s) for a in range(3) for s in range(2)]
GOLDEN = os.path.join(os.path.dirname(__file__), 'golden', 'paper_setup.txt')


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith('#'):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_defaults_are_the_papers_constants():
    gd = _golden()
    o = MGOptions()
    assert o.cheb_lo == gd['cheb_lo'] and o.cheb_hi == gd['cheb_hi']
    assert o.power_maxit == gd['power_maxit'] and o.power_rtol == gd['power_rtol']
    assert o.shift_gamma == gd['shift_gamma'] and o.coarse_atol == gd['coarse_atol']


def test_bratu_level_independence():
    ges, ins = [], []
    for n, L in [(32, 3), (64, 4), (128, 5)]:
        g = Grid([n, n], 1.0 / n, ALL2)
        u, rep = newton.solve(Problem('bratu', {'lam': 5.0}), g, L, np.zeros(g.node_shape),
                              np.zeros(g.node_shape), None,
                              MGOptions(nu_pre=3, nu_post=3, power_fixed=True, power_maxit=10),
                              newton.NewtonOptions(rtol=1e-8))
        assert rep.status == 'ok'
        ges.append(rep.stats.effective_ge(2, L - 1))
        ins.append(rep.newton_iters)
    assert max(ges) < 1.25 * min(ges), ges
    assert max(ins) - min(ins) <= 1, ins


def test_plap_unique_solution():
    g = Grid([8, 8, 8], 1.0 / 8, ALL3)
    pb = Problem('plap', {'p': 3.0, 'delta': 1e-2})
    rng = np.random.default_rng(1)
    b = load_from_function(g, gaussian_source(rng.uniform(0.2, 0.8, (4, 3)),
                                              rng.uniform(0.05, 0.15, 4), rng.normal(size=4)))
    sols = []
    for u0 in (np.zeros(g.node_shape), 0.1 * rng.uniform(-1, 1, g.node_shape)):
        u0[g.dirichlet_mask()] = 0
        u, rep = newton.solve(pb, g, 2, u0, b, None, MGOptions(nu_pre=4, nu_post=4),
                              newton.NewtonOptions(rtol=1e-12))
        assert rep.status == 'ok'
        assert np.linalg.norm(residual(pb, g, u, b)) <= 1e-12 * np.linalg.norm(residual(pb, g, u0, b))
        sols.append(u)
    assert np.linalg.norm(sols[0] - sols[1]) <= 1e-9 * np.linalg.norm(sols[0])


def test_bratu_supercritical_fails():
    g = Grid([16, 16], 1.0 / 16, ALL2)
    u, rep = newton.solve(Problem('bratu', {'lam': 7.0}), g, 2, np.zeros(g.node_shape),
                          np.zeros(g.node_shape), None, MGOptions(),
                          newton.NewtonOptions(rtol=1e-8, maxit=12))
    assert rep.status != 'ok'
