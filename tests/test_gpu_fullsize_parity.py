"""Converged solutions and gradients at the full configuration sizes against
the oracle's own tight solves (stored by tests/golden/make_fullsize_refs.py,
which calls only oracle/ and the seeded generators).

At these sizes a small residual does not bound the solution error tightly
(the p-Laplacian's smallest Jacobian eigenvalue at 128^3 is ~1e-7 of its
largest), so both sides solve to ||F|| <= 1e-12 ||F_0|| (Sec. 1: F(x*) = 0)
and the solutions are compared directly:

* on the stored 8192 seeded nodes, ||u_gpu - u_ora|| / ||u_ora|| <= 1e-8;
* the whole-grid 2-norms agree to 1e-8 relative.

Configurations:
* the p-Laplacian on 128^3, with FP64 and with FP32 multigrid levels;
* the inverse-coefficient problem on 128^3: u(m), u(m_obs), the adjoint state
  lam of J(u)^T lam = u - u_obs and the gradient -(dF/dm)^T lam of
  1/2 ||u - u_obs||^2;
* the p-Laplacian on 256^3 (the benchmark grid), FP32 and FP64 levels.  Here
  the FP64 residual has a rounding floor near 3.1e-12 ||F_0||: the oracle's
  tenth Newton step (23 V-cycles) moved u by 7e-16 relative and left ||F||
  at 3.147e-12 (from 3.153e-12), so its reference is the iterate after nine
  steps, and the GPU solves to 1e-11 (it stops near 4e-12).
* the Neo-Hookean beam 256 x 64 x 64: its first load increment (a tenth of
  the traction), FP32 levels.  Here the FP64 residual has a rounding floor
  near 2e-11 ||F_0||: the oracle's last Newton steps no longer lowered it
  (2.204e-11, then 2.195e-11), so its reference is that iterate, and the GPU
  solves to 3e-11.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import make_ctx, to_dev, to_np
from paper_2103_13890_amd import api
from paper_2103_13890_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'golden')
BAR = 1e-8


def _ref(name):
    path = os.path.join(GOLDEN, f'ref_{name}.npz')
    if not os.path.exists(path):
        # the oracle's solve at this size takes hours on one core; until its
        # result is committed the comparison cannot run
        pytest.skip(f'{path} not written yet: python tests/golden/make_fullsize_refs.py {name}')
    return np.load(path)


def _cmp(tag, g_full, nodes, ref_vals, ref_norm):
    g = to_np(g_full).reshape(-1)
    e_s = np.linalg.norm(g[nodes] - ref_vals) / np.linalg.norm(ref_vals)
    e_n = abs(np.linalg.norm(g) - float(ref_norm)) / float(ref_norm)
    print(f'{tag}: sampled rel diff {e_s:.2e}, norm rel diff {e_n:.2e}', flush=True)
    assert e_s <= BAR and e_n <= BAR, (tag, e_s, e_n)


def _gauss_load(ctx, w):
    c, wd, a = W.gaussian_params(w.get('load_seed', 1), 16, 3)
    return api.jfnk_assemble_load(ctx, 0, W.gaussian_param_array(c, wd, a))


@pytest.mark.parametrize('prec', [0, 1])
def test_plap128_solution(prec):
    w = W.WORKLOADS['plap3d-128']
    r = _ref('plap3d-128')
    over = dict(newton_rtol=1e-12, vcycle_prec=prec)
    if prec == 1:
        over['coarse_rtol'] = 1e-3
    ctx = make_ctx(w, **over)
    b = _gauss_load(ctx, w)
    u = ctx.empty(ctx.nlevels - 1)
    rep = api.jfnk_solve(ctx, u, None, b)
    assert rep['status'] == 'ok', rep
    _cmp(f'plap 128^3 vcycle_prec {prec}', u, r['nodes'], r['u'], r['u_norm'])


def test_invcoef128_solution_adjoint_gradient():
    w = W.WORKLOADS['invcoef3d-128']
    r = _ref('invcoef3d-128')
    ctx = make_ctx(w, newton_rtol=1e-12)
    L = ctx.nlevels - 1
    b = _gauss_load(ctx, w)
    m = to_dev(W.matern_field(w['n'], w['h'], w.get('m_seed', 3)))
    m_obs = to_dev(W.matern_field(w['n'], w['h'], w.get('obs_seed', 4)))

    def solve(mm):
        u = ctx.empty(L)
        rep = api.jfnk_solve(ctx, u, mm, b)
        assert rep['status'] == 'ok', rep
        return u
    u, uo = solve(m), solve(m_obs)
    _cmp('invcoef u(m)', u, r['nodes'], r['u'], r['u_norm'])
    _cmp('invcoef u(m_obs)', uo, r['nodes'], r['u_obs'], r['u_obs_norm'])
    mask = to_dev(W.boundary_mask(w['n'], w['faces']))
    rhs = (u - uo).masked_fill(mask, 0.0)
    lam, arep = api.jfnk_adjoint_solve(ctx, u, rhs, m, rtol=1e-12)
    assert arep['ok'], arep
    _cmp('invcoef adjoint lam', lam, r['nodes'], r['lam'], r['lam_norm'])
    g = api.jfnk_coef_gradient(ctx, u, m, lam)
    _cmp('invcoef gradient', g, r['nodes'], r['grad'], r['grad_norm'])
    mis = 0.5 * float((rhs * rhs).sum())
    assert abs(mis - float(r['misfit'])) <= BAR * float(r['misfit'])


@pytest.mark.parametrize('prec', [0, 1])
def test_plap256_solution(prec):
    w = W.WORKLOADS['plap3d-256']
    r = _ref('plap3d-256')
    ctx = make_ctx(w, newton_rtol=1e-11, vcycle_prec=prec, coarse_rtol=1e-3 if prec else 1e-6)
    b = _gauss_load(ctx, w)
    u = ctx.empty(ctx.nlevels - 1)
    rep = api.jfnk_solve(ctx, u, None, b)
    assert rep['status'] == 'ok', rep
    _cmp(f'plap 256^3 vcycle_prec {prec}', u, r['nodes'], r['u'], r['u_norm'])


def test_neohooke_first_increment():
    w = W.WORKLOADS['neohooke-256x64']
    r = _ref('neohooke-256x64')
    ctx = make_ctx(w, newton_rtol=3e-11)
    t = W.traction(w.get('traction_seed', 2))
    b = api.jfnk_assemble_load(ctx, 1, t)
    b1 = (1.0 / w['load_steps']) * b           # the first increment's load, as the load stepping scales it
    u = ctx.empty(ctx.nlevels - 1)
    rep = api.jfnk_solve(ctx, u, None, b1)
    assert rep['status'] == 'ok', rep
    _cmp('neohooke first increment', u, r['nodes'], r['u'], r['u_norm'])
