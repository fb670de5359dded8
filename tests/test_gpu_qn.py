"""CG-QN on the GPU against the oracle (Sec. 2, coarse level solver; Sec. 3,
setup): the coarse CG preconditioned by L-BFGS pairs recorded by the first
coarse CG of a solve.

* Coarse solves on the 8 x 8 Bratu coarse grid (FD step 1e-2, FP64): the
  recording solve, a preconditioned solve of another right-hand side, and,
  after a new setup at an indefinite state, a preconditioned solve that
  exits with negative curvature and shifts.  Iteration and round counts
  exactly; corrections to 1e-9 and shifts to 1e-10, except on the
  indefinite preconditioned solve: there the shift is the Rayleigh quotient
  of a PCG direction built through the two-loop recursion, whose dot
  products sum in a different order on each side, so shift and correction
  agree to 1e-8.
* V-cycles on the small p-Laplacian (ragged 36 x 20 x 12, 3 levels): the
  first records, the second preconditions; 1e-9 against the oracle.
* A solve with coarse_qn = 20 (FP64 and FP32 levels) reaches the oracle's
  CG-QN solution to 1e-8 relative and keeps between 1 and 20 pairs.  (The
  pairs come from the first Newton step's coarse Jacobian; on the
  p-Laplacian from u = 0 that is delta times the Laplacian, which describes
  the later Jacobians poorly, so fewer coarse iterations are not expected
  here: the preconditioned solve of the same Jacobian above shows them.)
* The generic coarse solver (vectors in global memory) on the Neo-Hookean
  coarse level and on a 2D Bratu coarse level with 1369 nodes: a recording
  and a preconditioned solve, iteration counts exact, corrections to 1e-9.
* Options: coarse_qn outside [0, 32] is rejected at creation.
"""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import make_ctx, oracle_grid, oracle_mg_options, oracle_problem, rel, small, to_dev, to_np
from oracle import mg as OM
from oracle import newton as ON
from oracle import problems as OP
from paper_2103_13890_amd import api
from paper_2103_13890_amd import workloads as W


def test_coarse_qn_solves():
    w = W.scaled('bratu2d-32', (16, 16), nlevels=2)
    g = oracle_grid(w)
    grids = OM.make_grids(g, 2)
    pb = oracle_problem(w)
    opts = oracle_mg_options(w, fd_root=1e-2, coarse_rtol=1e-10, power_fixed=True, power_maxit=10,
                             coarse_qn=6)
    ctx = make_ctx(w, fd_root=1e-2, coarse_rtol=1e-10, coarse_qn=6)
    qn = {}
    n0 = grids[0].n_dof()
    r0 = np.sin(np.arange(grids[0].n_nodes)).reshape(grids[0].node_shape)
    r0[grids[0].dirichlet_mask()] = 0
    r1 = np.cos(0.7 * np.arange(grids[0].n_nodes)).reshape(grids[0].node_shape)
    r1[grids[0].dirichlet_mask()] = 0
    iters_seen = []
    for uval, rhs in ((0.3, r0), (0.3, r1), (3.0, r0)):
        u = np.full(g.node_shape, uval)
        u[g.dirichlet_mask()] = 0
        api.mg_setup(ctx, to_dev(u))
        levels = OM.mg_setup(pb, grids, u, None, opts, None, None, qn)
        s, shift, its, rounds = api.mg_coarse_solve(ctx, to_dev(rhs))
        ref, shift_o, iters_o = OM.coarse_solve(lambda x: OM.level_jv(pb, levels[0], x), rhs, n0, opts,
                                                None, qn)
        assert qn['pairs'], 'the first solve keeps pairs'
        assert its == sum(iters_o) and rounds == len(iters_o) - 1, (uval, its, iters_o)
        tol_shift, tol_s = (1e-8, 1e-8) if uval == 3.0 else (1e-10, 1e-9)
        assert abs(shift - shift_o) <= tol_shift * max(1.0, abs(shift_o)), (shift, shift_o)
        assert rel(to_np(s), ref) < tol_s
        if uval == 3.0:
            assert shift < 0 and rounds >= 1
        if len(iters_seen) == 1:
            # the preconditioned solve of the SPD Jacobian the pairs came from
            # needs fewer steps than plain CG on the same system
            plain = oracle_mg_options(w, fd_root=1e-2, coarse_rtol=1e-10)
            _, _, it_plain = OM.coarse_solve(lambda x: OM.level_jv(pb, levels[0], x), rhs, n0, plain)
            assert its < it_plain[0], (its, it_plain)
        iters_seen.append(its)


def test_vcycle_qn():
    w = small('plap')
    u = 1.0 * W.rough_state(w['n'], w['faces'], 170)
    g = oracle_grid(w)
    xs = g.node_coords()
    bump = np.prod([np.sin(np.pi * x / (w['n'][k] * w['h'])) for k, x in enumerate(xs)], axis=0)
    u = bump + 1e-3 * u
    u[g.dirichlet_mask()] = 0
    ctx = make_ctx(w, fd_root=1e-2, power_fixed=1, power_maxit=10, coarse_rtol=1e-10, coarse_qn=20)
    api.mg_setup(ctx, to_dev(u))
    opts = oracle_mg_options(w, fd_root=1e-2, power_fixed=True, power_maxit=10, coarse_rtol=1e-10,
                             coarse_qn=20)
    qn = {}
    levels = OM.mg_setup(oracle_problem(w), OM.make_grids(g, ctx.nlevels), u, None, opts, None, None, qn)
    for seed in (171, 172):
        v = W.normal_vector(w['n'], w['faces'], seed)
        s = api.mg_vcycle(ctx, to_dev(v))
        ref = OM.vcycle(oracle_problem(w), levels, ctx.nlevels - 1, v, opts)
        assert rel(to_np(s), ref) < 1e-9
    assert qn['pairs']


@pytest.mark.parametrize('prec', [0, 1])
def test_solve_qn(prec):
    w = small('plap')
    c, wd, a = W.gaussian_params(1, 16, 3)
    b = OP.load_from_function(oracle_grid(w), OP.gaussian_source(c, wd, a))
    g = oracle_grid(w)
    opts = oracle_mg_options(w, coarse_qn=20)
    ref, orep = ON.solve(oracle_problem(w), g, w['nlevels'], np.zeros(g.node_shape), b, None, opts,
                         ON.NewtonOptions(rtol=1e-12))
    assert orep.status == 'ok'
    reps = {}
    for qn in (0, 20):
        ctx = make_ctx(w, newton_rtol=1e-12, vcycle_prec=prec, coarse_qn=qn,
                       coarse_rtol=1e-6 if prec == 0 else 1e-3)
        u = to_dev(np.zeros_like(ref))
        rep = api.jfnk_solve(ctx, u, None, to_dev(b))
        assert rep['status'] == 'ok', rep
        assert rel(to_np(u), ref) < 1e-8
        reps[qn] = rep
    assert reps[0]['coarse_qn_pairs'] == 0 and 1 <= reps[20]['coarse_qn_pairs'] <= 20


@pytest.mark.parametrize('kind', ['neohooke', 'bratu2d-large'])
def test_generic_coarse_qn(kind):
    # the generic coarse solver (vectors in global memory): the Neo-Hookean
    # coarse level, and a scalar coarse level with more than 1024 nodes
    if kind == 'neohooke':
        w = small('neohooke')
        nc = 3
    else:
        w = W.scaled('bratu2d-32', (72, 72), nlevels=2)
        nc = 1
    g = oracle_grid(w)
    grids = OM.make_grids(g, w['nlevels'])
    g0 = grids[0]
    assert nc == 3 or g0.n_nodes > 1024
    pb = oracle_problem(w)
    xs = g.node_coords()
    bump = np.prod([np.sin(np.pi * x / (w['n'][k] * w['h'])) for k, x in enumerate(xs)], axis=0)
    u = 0.01 * np.stack([bump, 0.5 * bump, -bump]) if nc == 3 else 0.3 * bump
    mask = g.dirichlet_mask()
    if nc == 3:
        u[:, mask] = 0
    else:
        u[mask] = 0
    opts = oracle_mg_options(w, fd_root=1e-2, coarse_rtol=1e-10, power_fixed=True, power_maxit=10, coarse_qn=8)
    ctx = make_ctx(w, fd_root=1e-2, coarse_rtol=1e-10, power_fixed=1, power_maxit=10, coarse_qn=8)
    api.mg_setup(ctx, to_dev(u))
    qn = {}
    levels = OM.mg_setup(pb, grids, u, None, opts, None, None, qn)
    n0 = g0.n_dof(nc)
    shape0 = g0.node_shape if nc == 1 else (3,) + g0.node_shape
    m0 = g0.dirichlet_mask()
    for seed in (180, 181):
        rhs = np.random.default_rng(seed).normal(size=shape0)
        if nc == 3:
            rhs[:, m0] = 0
        else:
            rhs[m0] = 0
        print(f'{kind} coarse rhs seed {seed}', flush=True)
        s, shift, its, rounds = api.mg_coarse_solve(ctx, to_dev(rhs))
        ref, shift_o, iters_o = OM.coarse_solve(lambda x: OM.level_jv(pb, levels[0], x), rhs, n0, opts, None, qn)
        assert its == sum(iters_o) and rounds == len(iters_o) - 1, (its, iters_o)
        assert rel(to_np(s), ref) < 1e-9
        assert 0 < len(qn['pairs']) <= 8


def test_qn_option_checks():
    w = small('plap')
    with pytest.raises(api.JfnkError):
        make_ctx(w, coarse_qn=33)
    with pytest.raises(api.JfnkError):
        make_ctx(w, coarse_qn=-1)
