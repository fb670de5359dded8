"""Pins of the oracle's checkers and solver control logic.

* ``residual_at`` (the F(u) checker of every sampled full-size comparison)
  equals the assembled ``residual`` at every node of small grids that mix
  Dirichlet and natural faces: 2D Bratu, the 3D scalar kinds (element-mean
  and Gauss-point p-Laplacian, the inverse-coefficient residual with its
  field m) and the three-component Neo-Hookean residual.  For p = 2 the
  p-Laplacian residual is K u - b, and ``residual_at`` reproduces the
  closed-form Q1 stencils at interior nodes and at nodes on a natural face,
  where only the elements on one side exist.
* ``traction_load`` (the beam's load, Sec. 3 hyperelasticity): the total
  force is the traction times the face area, the nodal weights on the
  loaded face are h^2 (1/4, 1/2, 1) at its corners, edges and interior, and
  no other node is loaded.
* ``load_steps``: one step is a plain solve; the increments are t_k = k/n
  of the load with the last one the full load exactly; a failed increment is
  halved and the halved step is kept.
* ``line_search`` (Sec. 3 setup: cubic backtracking, Dennis and Schnabel
  Alg. A6.3.1): on an analytic quadratic the first backtrack is its
  minimiser; on an analytic cubic the second backtrack is the cubic's
  minimiser (-b + sqrt(b^2 - 3 a phi'(0))) / (3 a); steps are safeguarded to
  [0.1, 0.5] times the previous one; the sufficient-decrease test accepts
  at its boundary and rejects just above it; a non-finite merit halves the
  step; the residual-norm test accepts on its own.
* ``pcg`` (the paper's outer CG-MG): non-positive curvature on the first
  direction returns that direction, the preconditioned residual (the
  truncated Newton-CG rule of Nocedal and Wright, Alg. 7.1).
* ``solve`` continued from a saved iterate with ``NewtonOptions.f0`` keeps
  the original solve's forcing and stop (the full-size references are
  computed in pieces this way).
"""
import numpy as np
import pytest

from oracle import newton
from oracle.fe import Grid
from oracle.krylov import pcg
from oracle.problems import Problem, residual, residual_at, traction_load

MIXED2 = [(0, 0), (1, 1)]                   # x = 0 and y = 1 Dirichlet, the others natural
MIXED3 = [(0, 0), (1, 1), (2, 0)]


def _state(shape, rng, scale, mask=None, nc=1):
    u = scale * rng.uniform(-1, 1, shape if nc == 1 else (nc,) + shape)
    if mask is not None:
        if nc == 1:
            u[mask] = 0
        else:
            u[:, mask] = 0
    return u


@pytest.mark.parametrize('kind,prm,n,faces', [
    ('bratu', {'lam': 3.0}, (7, 5), MIXED2),
    ('plap', {'p': 3.0, 'delta': 1e-2}, (5, 4, 3), MIXED3),
    ('plap', {'p': 1.0, 'delta': 1.0}, (6, 5), MIXED2),
    ('plap_gauss', {'p': 3.0, 'delta': 1e-2}, (5, 4, 3), MIXED3),
    ('invcoef', {}, (5, 4, 3), MIXED3),
    ('neohooke', {'E': 1.0, 'nu': 0.3}, (5, 3, 2), [(0, 0)]),
])
def test_residual_at_equals_residual_everywhere(kind, prm, n, faces):
    rng = np.random.default_rng(5)
    g = Grid(n, 1.0 / n[0], faces)
    pb = Problem(kind, prm)
    nc = pb.ncomp
    scale = 0.02 if kind == 'neohooke' else 0.5      # keeps every Neo-Hookean element uninverted
    u = _state(g.node_shape, rng, scale, g.dirichlet_mask(), nc)
    u += 0.0 if nc > 1 else 0.1 * _state(g.node_shape, rng, 1.0) * g.dirichlet_mask()   # boundary data
    b = _state(g.node_shape, rng, 0.1, None, nc)
    m = 0.5 * rng.normal(size=g.node_shape) if kind == 'invcoef' else None
    full = residual(pb, g, u, b, m)
    nodes = np.arange(g.n_nodes)
    at = residual_at(pb, g, u, b, nodes, m)
    ref = full.reshape((nc, -1)) if nc > 1 else full.reshape(-1)
    assert at.shape == ref.shape
    assert np.max(np.abs(at - ref)) <= 1e-14 * np.max(np.abs(ref))
    # a shuffled subset with repeats gives the same values
    sub = rng.choice(g.n_nodes, 17)
    at2 = residual_at(pb, g, u, b, sub, m)
    assert np.array_equal(at2, at[..., sub])


def test_residual_at_linear_stencils_3d():
    """p = 2: F = K u - b.  3D Q1 stencil (K row at a node, in units of h):
    interior 8/3 at the centre, 0 at face neighbours, -1/6 at edge and -1/12
    at corner neighbours; on a natural face 4/3 at the centre, -1/12 at the
    4 in-face diagonal neighbours, -1/6 at the 4 edge neighbours off the face,
    -1/12 at the 4 corner neighbours off the face."""
    rng = np.random.default_rng(8)
    n = (6, 5, 4)
    h = 0.25
    g = Grid(n, h, [(1, 0), (1, 1), (2, 0), (2, 1), (0, 1)])   # x = 0 natural
    pb = Problem('plap', {'p': 2.0, 'delta': 0.3})
    u = rng.uniform(-1, 1, g.node_shape)
    u[g.dirichlet_mask()] = 0
    zero = np.zeros_like(u)

    def stencil(z, y, x, face):
        acc = 0.0
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in ((0, 1) if face else (-1, 0, 1)):
                    c = abs(dx) + abs(dy) + abs(dz)
                    if face:
                        if c == 0:
                            wgt = 4 / 3
                        elif c == 1:
                            wgt = 0.0
                        elif c == 2:
                            wgt = -1 / 12 if dx == 0 else -1 / 6
                        else:
                            wgt = -1 / 12
                    else:
                        wgt = (8 / 3, 0.0, -1 / 6, -1 / 12)[c]
                    acc += wgt * u[z + dz, y + dy, x + dx]
        return h * acc

    pts = [(2, 2, 3, False), (1, 3, 1, False), (2, 2, 0, True), (1, 1, 0, True), (3, 4, 0, True)]
    nodes = [np.ravel_multi_index(p[:3], g.node_shape) for p in pts]
    F = residual_at(pb, g, u, zero, nodes)
    for k, (z, y, x, face) in enumerate(pts):
        assert abs(F[k] - stencil(z, y, x, face)) <= 1e-14, (pts[k], F[k], stencil(z, y, x, face))


def test_residual_at_linear_stencils_2d():
    """2D Q1 stencil: interior 8/3 at the centre, -1/3 at all 8 neighbours;
    on a natural edge 4/3 at the centre, -1/6 at the 2 neighbours along the
    edge, -1/3 at the neighbour off the edge and at the 2 diagonal ones."""
    rng = np.random.default_rng(9)
    g = Grid((6, 5), 0.2, [(0, 0), (0, 1), (1, 1)])            # y = 0 natural
    pb = Problem('bratu', {'lam': 0.0})
    u = rng.uniform(-1, 1, g.node_shape)
    u[g.dirichlet_mask()] = 0
    zero = np.zeros_like(u)
    y, x = 2, 3
    ref_int = 8 / 3 * u[y, x] - 1 / 3 * (u[y - 1:y + 2, x - 1:x + 2].sum() - u[y, x])
    y0 = 0
    ref_edge = (4 / 3 * u[y0, x] - 1 / 6 * (u[y0, x - 1] + u[y0, x + 1]) - 1 / 3 * u[y0 + 1, x]
                - 1 / 3 * (u[y0 + 1, x - 1] + u[y0 + 1, x + 1]))
    F = residual_at(pb, g, u, zero, [np.ravel_multi_index((y, x), g.node_shape),
                                     np.ravel_multi_index((y0, x), g.node_shape)])
    assert abs(F[0] - ref_int) <= 1e-14 and abs(F[1] - ref_edge) <= 1e-14


def test_traction_load_weights_and_total_force():
    n = (4, 3, 2)
    h = 0.5
    g = Grid(n, h, [(0, 0)])
    t = np.array([0.3, -1.2, 0.7])
    b = traction_load(g, t)
    assert b.shape == (3,) + g.node_shape
    area = (n[1] * h) * (n[2] * h)
    for i in range(3):
        assert abs(b[i].sum() - t[i] * area) <= 1e-14 * area
        face = b[i][:, :, -1]                 # x = n_x h, array axes (z, y)
        assert not np.any(b[i][:, :, :-1])
        ny1, nz1 = n[1] + 1, n[2] + 1
        for z in range(nz1):
            for y in range(ny1):
                onb = (y in (0, ny1 - 1)) + (z in (0, nz1 - 1))
                wgt = h * h * (1.0, 0.5, 0.25)[onb]
                assert abs(face[z, y] - t[i] * wgt) <= 1e-15
    # the clamped face x = 0 carries nothing even when it is the loaded one
    b0 = traction_load(g, t, axis=0, side=0)
    assert not np.any(b0)


def test_load_steps_control(monkeypatch):
    calls = []
    bf = np.array([1.0, -2.0, 3.0])

    def fake_solve(problem, finest, nlevels, u0, b, m=None, mg_opts=None, opts=None, report=None):
        calls.append(b.copy())
        rep = newton.Report()
        k = len(calls)
        rep.status = 'noconv' if k == 2 else 'ok'          # the second increment fails once
        return u0 + 0.0 * b[0], rep

    monkeypatch.setattr(newton, 'solve', fake_solve)
    u, reps = newton.load_steps(None, None, 2, np.zeros(1), bf, 10)
    fr = [float(c @ bf / (bf @ bf)) for c in calls]
    assert np.allclose(fr[:3], [0.1, 0.2, 0.15], rtol=0, atol=1e-15)
    # after the failure the halved increment 0.05 is kept up to the full load
    assert np.allclose(np.diff(fr[2:]), 0.05, rtol=0, atol=1e-12)
    assert np.array_equal(calls[-1], bf)                 # the last increment is the full load exactly
    assert reps[-1][0] == 1.0 and [r.status for _, r in reps].count('noconv') == 1
    assert len(calls) == 3 + 17
    # ten plain increments: t_k = k / 10, the last one exactly 1
    calls.clear()

    def ok_solve(problem, finest, nlevels, u0, b, *rest, **kw):
        calls.append(b.copy())
        return u0, newton.Report()

    monkeypatch.setattr(newton, 'solve', ok_solve)
    newton.load_steps(None, None, 2, np.zeros(1), bf, 10)
    fr = [float(c @ bf / (bf @ bf)) for c in calls]
    assert len(calls) == 10 and np.allclose(fr, np.arange(1, 11) / 10, rtol=0, atol=1e-15)
    assert np.array_equal(calls[-1], bf)


def test_load_steps_single_step_is_a_solve():
    g = Grid((8, 8), 1 / 8, [(a, s) for a in range(2) for s in range(2)])
    pb = Problem('bratu', {'lam': 2.0})
    rng = np.random.default_rng(4)
    b = 0.1 * rng.normal(size=g.node_shape)
    b[g.dirichlet_mask()] = 0
    from oracle.mg import MGOptions
    mo = MGOptions(nu_pre=2, nu_post=2, power_fixed=True, power_maxit=5)
    no = newton.NewtonOptions(rtol=1e-10)
    u1, r1 = newton.solve(pb, g, 2, np.zeros(g.node_shape), b, None, mo, no)
    u2, reps = newton.load_steps(pb, g, 2, np.zeros(g.node_shape), b, 1, None, mo, no)
    assert r1.status == 'ok' and len(reps) == 1 and reps[0][0] == 1.0
    assert np.array_equal(u1, u2)


def test_solve_continued_from_a_saved_iterate():
    """A solve stopped after two Newton steps and continued from its iterate
    with NewtonOptions.f0 = the first solve's ||F_0|| takes the same forcing
    and stop: it meets ||F|| <= rtol ||F_0|| of the original start and reaches
    the uninterrupted solve's root; without f0 its forcing starts again at
    0.5 and its stop is relative to the continued start."""
    g = Grid((16, 16), 1 / 16, [(a, s) for a in range(2) for s in range(2)])
    pb = Problem('bratu', {'lam': 5.0})
    b = np.zeros(g.node_shape)
    from oracle.mg import MGOptions
    mo = MGOptions(nu_pre=2, nu_post=2, power_fixed=True, power_maxit=5)
    u0 = np.zeros(g.node_shape)
    uf, rf = newton.solve(pb, g, 2, u0, b, None, mo, newton.NewtonOptions(rtol=1e-10))
    assert rf.status == 'ok' and rf.newton_iters >= 3
    f0 = rf.fnorm[0]
    u2, r2 = newton.solve(pb, g, 2, u0, b, None, mo, newton.NewtonOptions(rtol=1e-10, maxit=2))
    assert r2.status == 'noconv' and r2.newton_iters == 2
    uc, rc = newton.solve(pb, g, 2, u2, b, None, mo, newton.NewtonOptions(rtol=1e-10, f0=f0))
    assert rc.status == 'ok'
    assert rc.fnorm[-1] <= 1e-10 * f0
    assert rc.eta[0] == min(0.5, rc.fnorm[0] / f0)
    assert np.linalg.norm(uc - uf) <= 1e-9 * np.linalg.norm(uf)
    # the same continuation without f0: forcing and stop relative to F(u2)
    _, rn = newton.solve(pb, g, 2, u2, b, None, mo, newton.NewtonOptions(rtol=1e-10, maxit=1))
    assert rn.eta[0] == 0.5


def _run_ls(phi, phi0, slope, maxit=10, armijo=1e-4, fnorm=None, fnorm0=None):
    alphas = []

    def trial(a):
        alphas.append(a)
        return phi(a), (fnorm(a) if fnorm else np.inf)
    a, it = newton.line_search(trial, phi0, slope, maxit, armijo, fnorm0)
    return a, it, alphas


def test_line_search_quadratic_minimiser():
    c = 1.5                                     # phi = -a + c a^2: minimiser 1 / (2c) = 1/3
    a, it, al = _run_ls(lambda x: -x + c * x * x, 0.0, -1.0)
    assert it == 2 and al[0] == 1.0
    assert abs(al[1] - 1.0 / 3.0) <= 1e-15 and a == al[1]


def test_line_search_cubic_minimiser():
    a3, b3 = -2.06, 3.26                        # phi = -x + b3 x^2 + a3 x^3
    phi = (lambda x: -x + b3 * x * x + a3 * x ** 3)
    a, it, al = _run_ls(phi, 0.0, -1.0)
    assert it == 3
    assert abs(al[1] - 1.0 / (2.0 * (a3 + b3))) <= 1e-15         # quadratic backtrack first
    xmin = (-b3 + np.sqrt(b3 * b3 - 3.0 * a3 * (-1.0))) / (3.0 * a3)
    assert 0.1 * al[1] < xmin < 0.5 * al[1]
    assert abs(al[2] - xmin) <= 1e-12 and a == al[2]


def test_line_search_safeguards_and_armijo_boundary():
    # a steep quadratic: the raw step 1/(2 c) = 0.025 is raised to 0.1
    a, it, al = _run_ls(lambda x: -x + 20.0 * x * x, 0.0, -1.0)
    assert al[:2] == [1.0, 0.1]
    # a flat one: phi(1) = -5e-5 misses the sufficient decrease, and the raw
    # step 1 / (2 (1 - 5e-5)) is lowered to 0.5
    a, it, al = _run_ls(lambda x: -x + 0.99995 * x * x, 0.0, -1.0)
    assert al[:2] == [1.0, 0.5] and a == 0.5
    phi0, slope, arm = 1.0, -0.5, 1e-4
    edge = phi0 + arm * 1.0 * slope
    a, it, al = _run_ls(lambda x: edge if x == 1.0 else phi0 - 1.0, phi0, slope)
    assert a == 1.0 and it == 1
    a, it, al = _run_ls(lambda x: np.nextafter(edge, np.inf) if x == 1.0 else phi0 - 1.0, phi0, slope)
    assert it == 2 and a == al[1] < 1.0
    # a non-finite merit halves the step
    a, it, al = _run_ls(lambda x: np.inf if x > 0.6 else -x, 0.0, -1.0)
    assert al[:2] == [1.0, 0.5] and a == 0.5
    # the residual-norm test accepts where the merit does not
    a, it, al = _run_ls(lambda x: 5.0, 0.0, -1.0, fnorm=lambda x: 0.9, fnorm0=1.0)
    assert a == 1.0 and it == 1
    a, it, al = _run_ls(lambda x: 5.0, 0.0, -1.0, maxit=3, fnorm=lambda x: 1.0, fnorm0=1.0)
    assert a is None and it == 3


def test_pcg_first_direction_at_negative_curvature():
    A = np.diag([-3.0, 1.0])
    b = np.array([1.0, 1.0])
    x, its, rn, ok = pcg(lambda v: A @ v, b, lambda v: 2.0 * v, 1e-12, 10)
    assert not ok and its == 1
    assert np.array_equal(x, 2.0 * b)            # the preconditioned residual z = M b
