"""Parity at the benchmark configurations' full sizes (besides 256^3, which
tests/test_gpu_fullsize.py covers), in the launch configuration the
benchmark uses (automatic kernel choice).

* 2D Bratu 32^2 (lam = 5): tests/test_gpu_solve.py solves it in full.
* p-Laplacian 128^3, FP64 multigrid: F(u), J v and the load compared with
  the oracle on the whole grid; the solve to 1e-8 is checked by the
  oracle's residual of the GPU solution (a property at any size: the
  solution satisfies the oracle's discrete equations to the tolerance).
* Neo-Hookean beam 256 x 64 x 64: F(u) and J v on 2048 sampled nodes, the
  traction load on the whole grid.
* Inverse coefficient 128^3: F(u; m), both VJPs and the load on the whole
  grid; the adjoint gradient is checked through the oracle's formulas at the
  GPU's forward and adjoint states (J^T lam = u - u_obs, g = -(dF/dm)^T lam)
  and against central differences of the misfit along a seeded direction.

* The paper's three experiments at their finest refinement with the
  paper's settings (Bratu and minimal surface 800^2 on 6 levels, the beam
  160 x 16 x 16 on 5): the solve keeps the Dirichlet data, and the oracle's
  residual of the GPU solution on the whole grid is within 2x the absolute
  stopping bound 1e-6.

Tolerances as elsewhere: single evaluations 1e-12 relative (1e-10 for J v
at a test step eps = 1e-2 (1 + ||u||)/||v||, where the quotient amplifies
rounding by 1/eps_rel); solves: oracle residual <= 2x the stopping bound.
"""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import make_ctx, oracle_grid, oracle_problem, rel, to_dev, to_np
from oracle import derivatives as OD
from oracle import mg as OM
from oracle import problems as OP
from paper_2103_13890_amd import api
from paper_2103_13890_amd import workloads as W


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _gauss_load(ctx, w):
    c, wd, a = W.gaussian_params(w.get('load_seed', 1), 16, 3)
    b = api.jfnk_assemble_load(ctx, 0, W.gaussian_param_array(c, wd, a))
    ref = OP.load_from_function(oracle_grid(w), OP.gaussian_source(c, wd, a))
    return b, ref


def test_plap128_config():
    w = W.WORKLOADS['plap3d-128']
    pb, g = oracle_problem(w), oracle_grid(w)
    ctx = make_ctx(w)
    L = ctx.nlevels - 1
    b, bref = _gauss_load(ctx, w)
    assert rel(to_np(b), bref) < 1e-13
    u = 0.3 * W.rough_state(w['n'], w['faces'], 21)
    v = W.normal_vector(w['n'], w['faces'], 22)
    F = api.jfnk_residual(ctx, L, to_dev(u), None, b)
    assert rel(to_np(F), OP.residual(pb, g, u, bref)) < 1e-12
    eps = 1e-2 * (1 + np.linalg.norm(u)) / np.linalg.norm(v)
    Jv = api.jfnk_jv(ctx, L, to_dev(u), to_dev(v), eps_override=eps)
    assert rel(to_np(Jv), OM.fd_jv(pb, g, u, OP.apply_A(pb, g, u), v, None, eps)) < 1e-12
    # the configured solve (FP64 levels), then the FP32-multigrid variant
    f0 = np.linalg.norm(OP.residual(pb, g, np.zeros_like(u), bref))
    for prec, crtol in ((0, 1e-6), (1, 1e-3)):
        c2 = ctx if prec == 0 else make_ctx(w, vcycle_prec=1, coarse_rtol=crtol)
        us = to_dev(np.zeros_like(u))
        rep = api.jfnk_solve(c2, us, None, b)
        assert rep['status'] == 'ok', rep
        fo = np.linalg.norm(OP.residual(pb, g, to_np(us), bref))
        assert fo <= 2e-8 * f0, (prec, fo / f0)


def test_neohooke_config_sampled():
    w = W.WORKLOADS['neohooke-256x64']
    pb, g = oracle_problem(w), oracle_grid(w)
    ctx = make_ctx(w)
    L = ctx.nlevels - 1
    t = W.traction(w.get('traction_seed', 2))
    b = api.jfnk_assemble_load(ctx, 1, t)
    bref = OP.traction_load(g, t)
    assert rel(to_np(b), bref) < 1e-14
    u = 0.002 * W.rough_state(w['n'], w['faces'], 31, ncomp=3)   # |grad u| < 1: no inverted elements
    v = W.normal_vector(w['n'], w['faces'], 32, ncomp=3)
    nodes = np.random.default_rng(33).choice(g.n_nodes, 2048, replace=False)
    F = to_np(api.jfnk_residual(ctx, L, to_dev(u), None, b)).reshape(3, -1)[:, nodes]
    assert _maxrel(F, OP.residual_at(pb, g, u, bref, nodes)) < 1e-12
    eps = 1e-2 * (1 + np.linalg.norm(u)) / np.linalg.norm(v)
    Jv = to_np(api.jfnk_jv(ctx, L, to_dev(u), to_dev(v), eps_override=eps)).reshape(3, -1)[:, nodes]
    zero = np.zeros_like(u)
    ref = (OP.residual_at(pb, g, u + eps * v, zero, nodes) - OP.residual_at(pb, g, u, zero, nodes)) / eps
    assert _maxrel(Jv, ref) < 1e-10


def test_invcoef128_config_and_gradient():
    w = W.WORKLOADS['invcoef3d-128']
    pb, g = oracle_problem(w), oracle_grid(w)
    ctx = make_ctx(w, newton_rtol=1e-12)
    L = ctx.nlevels - 1
    b, bref = _gauss_load(ctx, w)
    assert rel(to_np(b), bref) < 1e-13
    m = W.matern_field(w['n'], w['h'], w.get('m_seed', 3))
    m_obs = W.matern_field(w['n'], w['h'], w.get('obs_seed', 4))
    md = to_dev(m)
    # single evaluations on the whole grid
    u = 0.3 * W.rough_state(w['n'], w['faces'], 41)
    lam = W.normal_vector(w['n'], w['faces'], 42)
    F = api.jfnk_residual(ctx, L, to_dev(u), md, b)
    assert rel(to_np(F), OP.residual(pb, g, u, bref, m)) < 1e-12
    assert rel(to_np(api.jfnk_vjp(ctx, L, 0, to_dev(u), to_dev(lam), md)), OD.vjp(pb, g, u, lam, m)) < 1e-12
    assert rel(to_np(api.jfnk_vjp(ctx, L, 1, to_dev(u), to_dev(lam), md)), OD.vjp_coef(pb, g, u, lam, m)) < 1e-12
    # forward solves at m and m_obs, adjoint gradient of 1/2 ||u - u_obs||^2
    def solve(mm):
        us = ctx.empty(L).zero_()
        rep = api.jfnk_solve(ctx, us, to_dev(mm), b)
        assert rep['status'] == 'ok', rep
        return us
    us, uo = solve(m), solve(m_obs)
    mask = g.dirichlet_mask()
    rhs = to_np(us) - to_np(uo)
    rhs[mask] = 0
    lam_g, arep = api.jfnk_adjoint_solve(ctx, us, to_dev(rhs), md, rtol=1e-12)
    assert arep['ok'], arep
    # the oracle's formulas at the GPU states
    un, ln = to_np(us), to_np(lam_g)
    adj_res = OD.vjp(pb, g, un, ln, m) - rhs
    adj_res[mask] = 0
    assert np.linalg.norm(adj_res) <= 1e-10 * np.linalg.norm(rhs)
    grad = to_np(api.jfnk_coef_gradient(ctx, us, md, lam_g))
    assert rel(grad, -OD.vjp_coef(pb, g, un, ln, m)) < 1e-12
    # central differences of the misfit along a seeded direction
    dm = W.matern_field(w['n'], w['h'], 43)
    tstep = 1e-4 / np.max(np.abs(dm))

    def misfit(mm):
        d = to_np(solve(mm)) - to_np(uo)
        d[mask] = 0
        return 0.5 * float(np.sum(d * d))
    fd = (misfit(m + tstep * dm) - misfit(m - tstep * dm)) / (2 * tstep)
    assert abs(fd - float(np.sum(grad * dm))) <= 1e-5 * abs(fd)


def test_neohooke_config_load_stepped_solve():
    """The configured beam solve: 10 load steps, FP32 multigrid.  The oracle's
    residual at 2048 sampled nodes of the GPU solution is at the stopping
    level (each increment stops at 1e-8 of its initial residual, about a
    tenth of the load), far below the load itself."""
    w = W.WORKLOADS['neohooke-256x64']
    pb, g = oracle_problem(w), oracle_grid(w)
    ctx = make_ctx(w)
    L = ctx.nlevels - 1
    t = W.traction(w.get('traction_seed', 2))
    b = api.jfnk_assemble_load(ctx, 1, t)
    u = ctx.empty(L).zero_()
    rep = api.jfnk_solve_steps(ctx, u, w['load_steps'], None, b)
    assert rep['status'] == 'ok', rep
    assert rep['alpha_hist'][-1] == 1.0
    un, bn = to_np(u), to_np(b)
    nodes = np.random.default_rng(34).choice(g.n_nodes, 2048, replace=False)
    Fo = OP.residual_at(pb, g, un, bn, nodes)
    bmax = np.max(np.abs(bn))
    assert np.max(np.abs(Fo)) <= 1e-6 * bmax, np.max(np.abs(Fo)) / bmax
    # a finite deformation: the tip moves by a few percent of the length
    assert 0.05 < float(u.abs().max()) < 2.0


@pytest.mark.parametrize('name', ['bratu2d-800', 'minsurf2d-800', 'beam3d-160x16x16'])
def test_paper_presets_full_size(name):
    w = W.WORKLOADS[name]
    pb, g = oracle_problem(w), oracle_grid(w)
    u0 = W.dirichlet_state(w)
    ctx = make_ctx(w)
    u = to_dev(u0)
    print(f'{name}: GPU solve with the paper settings', flush=True)
    rep = api.jfnk_solve(ctx, u, None, to_dev(np.zeros_like(u0)))
    assert rep['status'] == 'ok', rep
    assert rep['fnorm'] <= 1e-6
    un = to_np(u)
    m = g.dirichlet_mask()
    if un.ndim == len(w['n']):
        assert np.array_equal(un[m], u0[m])
    else:
        assert np.array_equal(un[:, m], u0[:, m])
    print(f'{name}: oracle residual on the whole grid', flush=True)
    F = OP.residual(pb, g, un, np.zeros_like(un))
    assert np.linalg.norm(F) <= 2e-6, np.linalg.norm(F)
