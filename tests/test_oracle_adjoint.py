"""Pin of the oracle's gradient: central differences of the misfit.

L(m) = 1/2 ||u(m) - u_obs||^2 with u(m) the solution of the inverse
coefficient problem; the adjoint gradient must match (L(m + t dm) -
L(m - t dm)) / 2t along seeded directions to the O(t^2) truncation.
"""
import numpy as np

from oracle import newton
from oracle.adjoint import gradient, misfit
from oracle.fe import Grid
from oracle.mg import MGOptions
from oracle.problems import Problem, gaussian_source, load_from_function

ALL3 = [(a, s) for a in range(3) for s in range(2)]


def test_gradient_central_difference():
    g = Grid([8, 8, 8], 1.0 / 8, ALL3)
    pb = Problem('invcoef')
    rng = np.random.default_rng(7)
    f = gaussian_source(rng.uniform(0.2, 0.8, (4, 3)), rng.uniform(0.1, 0.2, 4), 10 * rng.normal(size=4))
    b = load_from_function(g, f)
    m = 0.3 * rng.normal(size=g.node_shape)
    opts = MGOptions(nu_pre=3, nu_post=3)
    nopts = newton.NewtonOptions(rtol=1e-13)

    def solve(mm):
        u, rep = newton.solve(pb, g, 2, np.zeros(g.node_shape), b, mm, opts, nopts)
        assert rep.status == 'ok'
        return u
    u = solve(m)
    u_obs = solve(m + 0.2 * rng.normal(size=g.node_shape))
    gm, lam, its, ok = gradient(pb, g, 2, u, m, u_obs, opts)
    assert ok
    for _ in range(2):
        dm = rng.normal(size=g.node_shape)
        t = 1e-4 / np.max(np.abs(dm))
        fd = (misfit(g, solve(m + t * dm), u_obs) - misfit(g, solve(m - t * dm), u_obs)) / (2 * t)
        assert abs(fd - np.sum(gm * dm)) <= 1e-6 * abs(fd), (fd, np.sum(gm * dm))
