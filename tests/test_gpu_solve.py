"""GPU solves against the oracle.

Both sides solve to ||F|| <= 1e-12 ||F_0|| from the same start; the
solutions must agree to 1e-8 relative (the solution is the root of F, not a
path-dependent quantity, so the two iterations may differ).  The FP32
V-cycle only changes the preconditioner: its FP64 outer Newton reaches the
same root.  Gradient of the misfit through the adjoint: 1e-8 against the
oracle's gradient, and central differences of the misfit computed with the
GPU solver itself.
"""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import make_ctx, ncomp, oracle_grid, oracle_mg_options, oracle_problem, rel, small, to_dev, to_np
from oracle import newton as ON
from oracle import adjoint as OA
from oracle import problems as OP
from paper_2103_13890_amd import _lib, api
from paper_2103_13890_amd import workloads as W


def _load(w):
    if w['kind'] in ('plap', 'plap_gauss', 'invcoef'):
        c, wd, a = W.gaussian_params(1, 16, 3)
        return OP.load_from_function(oracle_grid(w), OP.gaussian_source(c, wd, a))
    if w['kind'] == 'neohooke':
        return 0.1 * OP.traction_load(oracle_grid(w), W.traction(2))
    return np.zeros(oracle_grid(w).node_shape)


def _oracle_solve(w, b, m=None, rtol=1e-12):
    g = oracle_grid(w)
    shape = g.node_shape if ncomp(w) == 1 else (3,) + g.node_shape
    u, rep = ON.solve(oracle_problem(w), g, w['nlevels'], np.zeros(shape), b, m, oracle_mg_options(w),
                      ON.NewtonOptions(rtol=rtol))
    assert rep.status == 'ok'
    return u, rep


@pytest.mark.parametrize('kind', ['bratu2d', 'plap', 'plap_gauss', 'neohooke-solve'])
def test_solution_parity_f64(kind):
    # the Neo-Hookean residual has a rounding floor near 1e-12 relative
    rtol = 1e-11 if kind.startswith('neohooke') else 1e-12
    w = small(kind)
    b = _load(w)
    ref, orep = _oracle_solve(w, b, rtol=rtol)
    ctx = make_ctx(w, newton_rtol=rtol)
    u = to_dev(np.zeros_like(ref))
    rep = api.jfnk_solve(ctx, u, None, to_dev(b))
    assert rep['status'] == 'ok', rep
    assert rel(to_np(u), ref) < 1e-8
    # the oracle's residual at the GPU solution
    F = OP.residual(oracle_problem(w), oracle_grid(w), to_np(u), b)
    assert np.linalg.norm(F) <= 10 * rtol * orep.fnorm[0]


def test_bratu_config_solution():
    w = W.WORKLOADS['bratu2d-32']
    b = np.zeros(oracle_grid(w).node_shape)
    ref, _ = _oracle_solve(w, b)
    ctx = make_ctx(w, newton_rtol=1e-12)
    u = to_dev(np.zeros_like(ref))
    rep = api.jfnk_solve(ctx, u, None, to_dev(b))
    assert rep['status'] == 'ok'
    assert rel(to_np(u), ref) < 1e-8
    assert 3 <= rep['newton_iters'] <= 8


def test_fp32_vcycle_reaches_same_root():
    # both sides to ||F|| <= 1e-12 ||F_0||, where the solution bar of 1e-8
    # is meaningful on this grid; the FP32 levels' kernels themselves are
    # compared with the oracle step by step in test_gpu_fp32_mg.py
    w = W.scaled('plap3d-128', (64, 64, 64), nlevels=4)
    b = _load(w)
    ref, _ = _oracle_solve(w, b, rtol=1e-12)
    its = {}
    for prec, rtol_c in ((1, 1e-3), (0, 1e-6)):
        ctx = make_ctx(w, vcycle_prec=prec, coarse_rtol=rtol_c, newton_rtol=1e-12)
        u = to_dev(np.zeros_like(ref))
        rep = api.jfnk_solve(ctx, u, None, to_dev(b))
        assert rep['status'] == 'ok', rep
        e = rel(to_np(u), ref)
        print(f'vcycle_prec {prec}: {rep["newton_iters"]} Newton, {rep["linear_iters"]} Krylov, '
              f'relative difference to the oracle {e:.2e}', flush=True)
        assert e < 1e-8
        its[prec] = rep['linear_iters']
    # the FP32 V-cycle is as good a preconditioner as the FP64 one
    assert its[1] <= its[0] + max(2, its[0] // 4), its


def test_fp32_vcycle_gauss_kind():
    # the Gauss-point p-Laplacian with FP32 levels (its FP32 difference-form
    # kernels in the V-cycle) reaches the oracle's root as the FP64 solve does
    w = small('plap_gauss')
    b = _load(w)
    ref, _ = _oracle_solve(w, b, rtol=1e-12)
    ctx = make_ctx(w, vcycle_prec=1, coarse_rtol=1e-3, newton_rtol=1e-12)
    u = to_dev(np.zeros_like(ref))
    rep = api.jfnk_solve(ctx, u, None, to_dev(b))
    assert rep['status'] == 'ok', rep
    assert rel(to_np(u), ref) < 1e-8


def test_invcoef_solve_and_gradient():
    w = W.scaled('invcoef3d-128', (16, 16, 16), nlevels=3)
    g = oracle_grid(w)
    b = _load(w)
    m = W.matern_field(w['n'], w['h'], 3)
    m_obs = W.matern_field(w['n'], w['h'], 4)
    u_ref, _ = _oracle_solve(w, b, m)
    uo_ref, _ = _oracle_solve(w, b, m_obs)
    ctx = make_ctx(w, newton_rtol=1e-12)
    u = to_dev(np.zeros(g.node_shape))
    rep = api.jfnk_solve(ctx, u, to_dev(m), to_dev(b))
    assert rep['status'] == 'ok'
    assert rel(to_np(u), u_ref) < 1e-8
    # gradient of 1/2 ||u - u_obs||^2
    grad_ref, _, _, ok = OA.gradient(oracle_problem(w), g, w['nlevels'], u_ref, m, uo_ref, oracle_mg_options(w))
    assert ok
    rhs = to_np(u) - uo_ref
    rhs[g.dirichlet_mask()] = 0
    lam, arep = api.jfnk_adjoint_solve(ctx, u, to_dev(rhs), to_dev(m), rtol=1e-12)
    gm = to_np(api.jfnk_coef_gradient(ctx, u, to_dev(m), lam))
    assert rel(gm, grad_ref) < 1e-8
    # the gradient call is the coefficient VJP negated, bit for bit
    assert np.array_equal(gm, -to_np(api.jfnk_vjp(ctx, w['nlevels'] - 1, 1, u, lam, to_dev(m))))


def test_edge_cases():
    # no interior DoFs: the solve returns at once with F = 0
    w = W.scaled('plap3d-128', (2, 2, 2), nlevels=1)
    w['n'] = (1, 1, 1)
    ctx = make_ctx(w)
    u = to_dev(np.zeros((2, 2, 2)))
    rep = api.jfnk_solve(ctx, u, None, to_dev(np.zeros((2, 2, 2))))
    assert rep['status'] == 'ok' and rep['newton_iters'] == 0
    # zero load: u = 0 is the root
    w = small('plap')
    ctx = make_ctx(w)
    u = to_dev(np.zeros(oracle_grid(w).node_shape))
    rep = api.jfnk_solve(ctx, u, None, None)
    assert rep['status'] == 'ok' and not torch.any(u)
    # supercritical Bratu has no solution: failure is reported
    w = W.scaled('bratu2d-32', (16, 16), nlevels=2)
    w['params'] = (7.0,)
    ctx = make_ctx(w, newton_maxit=12)
    u = to_dev(np.zeros(oracle_grid(w).node_shape))
    rep = api.jfnk_solve(ctx, u, None, None)
    assert rep['status'] != 'ok'


def _status(rep):
    return rep['status'] if isinstance(rep['status'], str) else _lib.STATUS.get(rep['status'], rep['status'])


def test_failure_injection():
    """Failures forced from the host return their status codes and leave
    finite state: a NaN in the start state (non-finite residual), a Newton
    cap of one step, a sufficient-decrease constant of 0.9999 with one trial
    (a Newton step on a convex energy decreases it by about half the linear
    prediction, so the line search fails), and a Neo-Hookean load beyond what the increments can
    carry (inverted elements, halved increments)."""
    w = small('plap')
    g = oracle_grid(w)
    b = to_dev(0.1 * W.normal_vector(w['n'], w['faces'], 300))
    ctx = make_ctx(w)
    u0 = np.zeros(g.node_shape)
    u0[3, 4, 5] = np.nan
    rep = api.jfnk_solve(ctx, to_dev(u0), None, b)
    assert _status(rep) == 'nonfinite', rep
    assert 'non-finite' in rep['error']
    ctx = make_ctx(w, newton_maxit=1)
    u = to_dev(np.zeros(g.node_shape))
    rep = api.jfnk_solve(ctx, u, None, b)
    assert _status(rep) == 'noconv' and rep['newton_iters'] == 1, rep
    assert bool(torch.isfinite(u).all()) and bool(u.abs().max() > 0)
    ctx = make_ctx(w, armijo=0.9999, ls_maxit=1)
    u = to_dev(np.zeros(g.node_shape))
    rep = api.jfnk_solve(ctx, u, None, b)
    assert _status(rep) == 'noconv' and rep['newton_iters'] == 0, rep
    assert 'line search' in rep['error'] and not torch.any(u)
    # a traction 500 times the configured one on a short beam, one increment
    # allowed three Newton steps: every increment fails and is halved until
    # the step falls below 1e-6; u keeps the last accepted increment
    wn = small('neohooke-solve')
    gn = oracle_grid(wn)
    ctx = make_ctx(wn, newton_maxit=3)
    t = 500.0 * W.traction(wn.get('traction_seed', 2))
    bn = api.jfnk_assemble_load(ctx, 1, t)
    u = to_dev(np.zeros((3,) + gn.node_shape))
    rep = api.jfnk_solve_steps(ctx, u, 1, None, bn)
    assert _status(rep) in ('noconv', 'nonfinite'), rep
    tg = rep['alpha_hist']
    assert tg[0] == 1.0 and all(tg[k + 1] < tg[k] or tg[k + 1] > tg[k] for k in range(len(tg) - 1))
    assert bool(torch.isfinite(u).all())


def test_autograd_solve_gradients():
    """JFNKSolve: d/dm and d/db of 1/2 ||u - u_obs||^2 by torch autograd
    against the oracle's adjoint gradient and adjoint state."""
    w = W.scaled('invcoef3d-128', (16, 16, 16), nlevels=3)
    g = oracle_grid(w)
    b = _load(w)
    m = W.matern_field(w['n'], w['h'], 3)
    m_obs = W.matern_field(w['n'], w['h'], 4)
    u_ref, _ = _oracle_solve(w, b, m)
    uo_ref, _ = _oracle_solve(w, b, m_obs)
    grad_ref, lam_ref, _, ok = OA.gradient(oracle_problem(w), g, w['nlevels'], u_ref, m, uo_ref,
                                           oracle_mg_options(w))
    assert ok
    ctx = make_ctx(w, newton_rtol=1e-12)
    md = to_dev(m).requires_grad_(True)
    bd = to_dev(b).requires_grad_(True)
    u = api.JFNKSolve.apply(md, bd, ctx, None, 1e-12)
    assert rel(to_np(u), u_ref) < 1e-8
    d = u - to_dev(uo_ref)
    d = d.masked_fill(to_dev(g.dirichlet_mask()), 0.0)
    loss = 0.5 * (d * d).sum()
    loss.backward()
    assert rel(to_np(md.grad), grad_ref) < 1e-8
    assert rel(to_np(bd.grad), lam_ref) < 1e-8


def test_load_steps_neohooke():
    """Load stepping: the GPU increments reach the oracle's load-stepped root.
    Each increment stops at 1e-10 relative: the FP64 rounding floor of the
    Neo-Hookean residual (about 4e-16 absolute here) sits near 1e-11 of the
    full load's initial residual, so smaller increments cannot reach 1e-11."""
    w = small('neohooke-solve')
    b = _load(w)
    g = oracle_grid(w)
    rtol = 1e-10
    ref, reps = ON.load_steps(oracle_problem(w), g, w['nlevels'], np.zeros((3,) + g.node_shape), b, 3,
                              mg_opts=oracle_mg_options(w), opts=ON.NewtonOptions(rtol=rtol))
    assert all(r.status == 'ok' for _, r in reps)
    ctx = make_ctx(w, newton_rtol=rtol)
    u = to_dev(np.zeros_like(ref))
    rep = api.jfnk_solve_steps(ctx, u, 3, None, to_dev(b))
    assert rep['status'] == 'ok', rep
    assert rel(to_np(u), ref) < 1e-8
    assert rep['alpha_hist'][-1] == 1.0
    # one increment equals a plain solve
    u1 = to_dev(np.zeros_like(ref))
    rep1 = api.jfnk_solve_steps(ctx, u1, 1, None, to_dev(b))
    u2 = to_dev(np.zeros_like(ref))
    rep2 = api.jfnk_solve(ctx, u2, None, to_dev(b))
    assert rep1['status'] == rep2['status'] == 'ok'
    assert torch.equal(u1, u2)
