"""GPU parity: every libjfnk entry point against the oracle on the same
seeded inputs, at ragged sizes that span several blocks.

Tolerances (relative 2-norms):
* residual F(u), FP64: 1e-12 (two FP64 summation orders differ by ~1e-16).
* FD Jacobian action with a test step eps = 1e-2 (1 + ||u||)/||v||: 1e-12;
  the step itself: 1e-14; at the configured step: 1e-7 -- the quotient
  amplifies O(1e-16) differences in A by 1/(relative step) ~ 1e8, so two
  correct FP64 implementations differ by ~1e-8 there (the measured values
  are printed).
* transfers: 1e-14 (a few rounded multiply-adds).
* multigrid components run with the large test step (fd_root = 1e-2) so that
  FD noise does not mask parity: 1e-10.
* exact VJPs: 1e-12.
"""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import (make_ctx, ncomp, oracle_grid, oracle_mg_options, oracle_problem, rel, small, to_dev,
                     to_np)
from oracle import derivatives as OD
from oracle import mg as OM
from oracle import problems as OP
from oracle import transfer as OT
from paper_2103_13890_amd import _lib, api
from paper_2103_13890_amd import workloads as W

KINDS = ['bratu2d', 'bratu3d', 'plap', 'plap_gauss', 'minsurf', 'invcoef', 'neohooke']


def _inputs(w, seed, smooth=False):
    nc = ncomp(w)
    scale = 0.01 if w['kind'] == 'neohooke' else (0.3 if w['kind'] == 'bratu' else 1.0)
    u = scale * W.rough_state(w['n'], w['faces'], seed, ncomp=nc)
    if smooth:
        g = oracle_grid(w)
        xs = g.node_coords()
        bump = np.prod([np.sin(np.pi * x / (w['n'][k] * w['h'])) for k, x in enumerate(xs)], axis=0)
        u = scale * (bump if nc == 1 else np.stack([bump, 0.5 * bump, -bump])) + 1e-3 * u
        if nc == 1:
            u[g.dirichlet_mask()] = 0
        else:
            u[:, g.dirichlet_mask()] = 0
    v = W.normal_vector(w['n'], w['faces'], seed + 1, ncomp=nc)
    m = W.matern_field(w['n'], w['h'], seed + 2) if w['kind'] == 'invcoef' else None
    b = 0.1 * W.normal_vector(w['n'], w['faces'], seed + 3, ncomp=nc)
    return u, v, m, b


@pytest.mark.parametrize('kind', KINDS)
@pytest.mark.parametrize('smooth', [False, True])
@pytest.mark.parametrize('path', [1, 2])
def test_residual_f64(kind, smooth, path):
    w = small(kind)
    ctx = make_ctx(w, kernel_path=path)
    u, v, m, b = _inputs(w, 100, smooth)
    F = api.jfnk_residual(ctx, ctx.nlevels - 1, to_dev(u), to_dev(m) if m is not None else None, to_dev(b))
    ref = OP.residual(oracle_problem(w), oracle_grid(w), u, b, m)
    assert rel(to_np(F), ref) < 1e-12
    # bitwise reproducible
    F2 = api.jfnk_residual(ctx, ctx.nlevels - 1, to_dev(u), to_dev(m) if m is not None else None, to_dev(b))
    assert torch.equal(F, F2)


@pytest.mark.parametrize('kind', KINDS)
@pytest.mark.parametrize('path', [1, 2])
def test_residual_f32_reported(kind, path):
    w = small(kind)
    ctx = make_ctx(w, kernel_path=path)
    u, v, m, b = _inputs(w, 101, True)
    F = api.jfnk_residual(ctx, ctx.nlevels - 1, to_dev(u, torch.float32), to_dev(m) if m is not None else None,
                          to_dev(b, torch.float32))
    ref = OP.residual(oracle_problem(w), oracle_grid(w), u, b, m)
    assert rel(to_np(F), ref) < 1e-4


@pytest.mark.parametrize('kind', KINDS)
def test_residual_coarse_levels(kind):
    w = small(kind)
    ctx = make_ctx(w)
    g = oracle_grid(w)
    for level in range(ctx.nlevels - 2, -1, -1):
        g = g.coarsen()
        wl = dict(w, n=g.n, h=g.h)
        u, v, m, b = _inputs(wl, 102 + level, True)
        F = api.jfnk_residual(ctx, level, to_dev(u), to_dev(m) if m is not None else None, to_dev(b))
        assert rel(to_np(F), OP.residual(oracle_problem(w), g, u, b, m)) < 1e-12


@pytest.mark.parametrize('kind', KINDS)
@pytest.mark.parametrize('path,form', [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_jv_f64(kind, path, form):
    """form 1: two residual evaluations; form 2: element difference form."""
    w = small(kind)
    ctx = make_ctx(w, kernel_path=path, fd_form=form)
    L = ctx.nlevels - 1
    u, v, m, b = _inputs(w, 110, True)
    pb, g = oracle_problem(w), oracle_grid(w)
    md = to_dev(m) if m is not None else None
    Au = OP.apply_A(pb, g, u, m)
    # test step
    eps_t = 1e-2 * (1 + np.linalg.norm(u)) / np.linalg.norm(v)
    Jv, eps = api.jfnk_jv(ctx, L, to_dev(u), to_dev(v), md, eps_override=eps_t, want_eps=True)
    assert eps == eps_t
    assert rel(to_np(Jv), OM.fd_jv(pb, g, u, Au, v, m, eps_t)) < 1e-12
    # configured step (norm rule): step and quotient
    Jv, eps = api.jfnk_jv(ctx, L, to_dev(u), to_dev(v), md, want_eps=True)
    eps_o = OM.eps_numerator(g, u, OM.MGOptions()) / OM.dof_norm(g, v)
    assert abs(eps - eps_o) <= 1e-14 * eps_o
    dev = rel(to_np(Jv), OM.fd_jv(pb, g, u, Au, v, m, eps_o))
    print(f'J v at the configured step, {kind} path {path} form {form}: {dev:.2e}', flush=True)
    assert dev < 1e-7
    # against the exact derivative: FD truncation + rounding only
    assert rel(to_np(Jv), OD.jvp(pb, g, u, v, m)) < 1e-5


# Row-tiled kernel shapes: x extents that are a multiple of 64 (the last node
# column has its own loader), two wavefronts with a partial second one,
# natural faces on the high sides, several y tiles and z chunks (below 128
# elements in x, chunks go down to one plane: the 64 x 30 x 31 case asks for
# more tiles than its 32 planes times its y tiles, so each chunk is one plane).
TILE_CASES = [
    ('plap', (64, 17, 9), W.ALL3),
    ('plap', (64, 30, 31), [(0, 0), (1, 0), (2, 1)]),
    ('plap', (64, 17, 9), [(0, 0), (1, 0), (2, 0)]),
    ('plap_gauss', (64, 17, 9), W.ALL3),
    ('plap_gauss', (128, 9, 5), [(0, 0), (1, 1), (2, 0)]),
    ('invcoef', (100, 19, 7), [(0, 1), (1, 1), (2, 0)]),
    ('bratu', (33, 9, 13), W.ALL3),
    # the tiled kernel's widest rows: 512 threads (8 wavefronts) per block,
    # the last node column (x = 512) finished through the extra-column path
    ('plap', (512, 10, 10), [(0, 0), (1, 1), (2, 0)]),
    ('invcoef', (512, 9, 11), W.ALL3),
]


def _tile_workload(kind, n, faces):
    base = {'plap': 'plap3d-128', 'plap_gauss': 'plap3d-128', 'invcoef': 'invcoef3d-128',
            'bratu': 'plap3d-128'}[kind]
    w = W.scaled(base, n, nlevels=1, vcycle_prec=0)
    w['faces'] = faces
    if kind == 'bratu':
        w.update(kind='bratu', params=(2.0,))
    if kind == 'plap_gauss':
        w.update(kind='plap_gauss')
    return w


@pytest.mark.parametrize('case', range(len(TILE_CASES)))
def test_tiled_shapes(case):
    kind, n, faces = TILE_CASES[case]
    w = _tile_workload(kind, n, faces)
    pb, g = oracle_problem(w), oracle_grid(w)
    u, v, m, b = _inputs(w, 120 + case, True)
    md = to_dev(m) if m is not None else None
    Au = OP.apply_A(pb, g, u, m)
    eps_t = 1e-2 * (1 + np.linalg.norm(u)) / np.linalg.norm(v)
    for path in (1, 2):
        ctx = make_ctx(w, kernel_path=path, fd_form=2)
        F = api.jfnk_residual(ctx, 0, to_dev(u), md, to_dev(b))
        assert rel(to_np(F), OP.residual(pb, g, u, b, m)) < 1e-12, path
        Jv = api.jfnk_jv(ctx, 0, to_dev(u), to_dev(v), md, eps_override=eps_t)
        assert rel(to_np(Jv), OM.fd_jv(pb, g, u, Au, v, m, eps_t)) < 1e-12, path
        Jv32 = api.jfnk_jv(ctx, 0, to_dev(u, torch.float32), to_dev(v, torch.float32), md, eps_override=eps_t)
        assert rel(to_np(Jv32), OM.fd_jv(pb, g, u, Au, v, m, eps_t)) < 1e-4, path


@pytest.mark.parametrize('kind', KINDS)
@pytest.mark.parametrize('path', [1, 2])
def test_jv_f32_difference_form(kind, path):
    """FP32: the difference form keeps the quotient accurate on smooth
    directions where two FP32 residual evaluations cancel."""
    w = small(kind)
    L = len(oracle_grid(w).n) and w['nlevels'] - 1
    u, v, m, b = _inputs(w, 112, True)
    g = oracle_grid(w)
    xs = g.node_coords()
    smooth = np.prod([np.sin(np.pi * x / (w['n'][k] * w['h'])) for k, x in enumerate(xs)], axis=0)
    vs = smooth if ncomp(w) == 1 else np.stack([smooth, smooth, smooth])
    pb = oracle_problem(w)
    md = to_dev(m) if m is not None else None
    ex = OD.jvp(pb, g, u, vs, m)
    errs = {}
    for form in (1, 2):
        ctx = make_ctx(w, kernel_path=path, fd_form=form)
        Jv = api.jfnk_jv(ctx, L, to_dev(u, torch.float32), to_dev(vs, torch.float32), md)
        errs[form] = rel(to_np(Jv), ex)
    assert errs[2] < 2e-3, errs
    assert errs[2] <= errs[1] * 1.5, errs


def test_jv_paper_step_and_zero_direction():
    w = small('plap')
    ctx = make_ctx(w, eps_mode=1)
    L = ctx.nlevels - 1
    u, v, m, b = _inputs(w, 111, True)
    g = oracle_grid(w)
    _, eps = api.jfnk_jv(ctx, L, to_dev(u), to_dev(v), want_eps=True)
    eps_o = OM.eps_numerator(g, u, OM.MGOptions(eps_mode='paper')) / OM.dof_norm(g, v)
    assert abs(eps - eps_o) <= 1e-14 * eps_o
    Jv, eps = api.jfnk_jv(ctx, L, to_dev(u), to_dev(0 * v), want_eps=True)
    assert eps == 0.0 and not torch.any(Jv)


@pytest.mark.parametrize('kind', ['bratu2d', 'plap', 'neohooke'])
def test_transfers(kind):
    w = small(kind)
    ctx = make_ctx(w)
    grids = OM.make_grids(oracle_grid(w), ctx.nlevels)
    nc = ncomp(w)
    for l in range(ctx.nlevels - 1, 0, -1):
        gf, gc = grids[l], grids[l - 1]
        wf = dict(w, n=gf.n, h=gf.h)
        wc = dict(w, n=gc.n, h=gc.h)
        x = W.rough_state(gf.n, [], 120 + l, ncomp=nc)           # nonzero boundary data too
        xc = api.mg_project(ctx, l, to_dev(x))
        assert rel(to_np(xc), OT.project(gc, gf, x)) < 1e-14
        r = W.normal_vector(gf.n, w['faces'], 121 + l, ncomp=nc)
        rc = api.mg_restrict(ctx, l, to_dev(r))
        assert rel(to_np(rc), OT.restrict(gc, gf, r)) < 1e-14
        c = W.normal_vector(gc.n, w['faces'], 122 + l, ncomp=nc)
        s = W.normal_vector(gf.n, w['faces'], 123 + l, ncomp=nc)
        sd = to_dev(s)
        api.mg_prolong_add(ctx, l, to_dev(c), sd)
        assert rel(to_np(sd), s + OT.prolong(gc, gf, c)) < 1e-14


def _setup_both(w, u, m, **mg_over):
    ctx = make_ctx(w, fd_root=1e-2, power_fixed=1, power_maxit=10, **mg_over)
    api.mg_setup(ctx, to_dev(u), to_dev(m) if m is not None else None)
    opts = oracle_mg_options(w, fd_root=1e-2, power_fixed=True, power_maxit=10)
    grids = OM.make_grids(oracle_grid(w), ctx.nlevels)
    levels = OM.mg_setup(oracle_problem(w), grids, u, m, opts)
    return ctx, levels, opts


@pytest.mark.parametrize('kind', ['bratu2d', 'plap', 'plap_gauss', 'minsurf', 'invcoef', 'neohooke'])
@pytest.mark.parametrize('form', [1, 2])
def test_mg_setup(kind, form):
    w = small(kind)
    u, v, m, b = _inputs(w, 130, True)
    ctx, levels, _ = _setup_both(w, u, m, fd_form=form)
    lam = api.mg_get_lambda(ctx)
    for l, lev in enumerate(levels):
        assert rel(to_np(api.mg_get_level(ctx, l, 'x')), lev.x) < 1e-14
        assert rel(to_np(api.mg_get_level(ctx, l, 'Ax')), lev.Ax) < 1e-12
        if l >= 1:
            assert abs(lam[l] - lev.lam) < 1e-10 * abs(lev.lam)
            assert rel(to_np(api.mg_get_level(ctx, l, 'eig')), lev.eig) < 1e-9


@pytest.mark.parametrize('kind', ['bratu2d', 'plap', 'plap_gauss', 'minsurf', 'neohooke'])
@pytest.mark.parametrize('form', [1, 2])
def test_smoother(kind, form):
    w = small(kind)
    u, v, m, b = _inputs(w, 140, True)
    ctx, levels, opts = _setup_both(w, u, m, fd_form=form)
    pb = oracle_problem(w)
    for l in range(1, ctx.nlevels):
        lev = levels[l]
        gl = lev.grid
        bl = W.normal_vector(gl.n, w['faces'], 141 + l, ncomp=ncomp(w))
        s0 = W.normal_vector(gl.n, w['faces'], 151 + l, ncomp=ncomp(w))
        # every degree path: nu = 1 (no J v), 2 (start and last step), 3 and
        # more (fused first step from s = 0, plain steps, fused last step)
        for nu in (1, 2, 3, 5):
            for zero in (True, False):
                s = to_dev(s0)
                api.mg_smooth(ctx, l, to_dev(bl), s, nu, zero)
                ref = OM.chebyshev(lambda x: OM.level_jv(pb, lev, x), bl, 0 * s0 if zero else s0, nu, lev.lam,
                                   opts.cheb_lo, opts.cheb_hi, s_is_zero=zero)
                assert rel(to_np(s), ref) < 1e-10, (l, nu, zero)


def test_coarse_solve_spd_and_shift():
    # Bratu on an 8 x 8 coarse grid: SPD at u = 0.3 sin, indefinite at u = 3 (4 negative eigenvalues)
    w = W.scaled('bratu2d-32', (16, 16), nlevels=2)
    g = oracle_grid(w)
    grids = OM.make_grids(g, 2)
    pb = oracle_problem(w)
    for uval, expect_shift in ((0.3, False), (3.0, True)):
        u = np.full(g.node_shape, uval)
        u[g.dirichlet_mask()] = 0
        ctx = make_ctx(w, fd_root=1e-2, coarse_rtol=1e-10)
        api.mg_setup(ctx, to_dev(u))
        opts = oracle_mg_options(w, fd_root=1e-2, coarse_rtol=1e-10, power_fixed=True, power_maxit=10)
        levels = OM.mg_setup(pb, grids, u, None, opts)
        r0 = np.sin(np.arange(grids[0].n_nodes)).reshape(grids[0].node_shape)
        r0[grids[0].dirichlet_mask()] = 0
        s, shift, its, rounds = api.mg_coarse_solve(ctx, to_dev(r0))
        st = OM.Stats()
        ref, shift_o, iters_o = OM.coarse_solve(lambda x: OM.level_jv(pb, levels[0], x), r0,
                                                grids[0].n_dof(), opts, st)
        assert (shift < 0) == expect_shift
        assert abs(shift - shift_o) <= 1e-10 * max(1.0, abs(shift_o))
        assert its == sum(iters_o) and rounds == len(iters_o) - 1
        assert rel(to_np(s), ref) < 1e-9


@pytest.mark.parametrize('kind', ['bratu2d', 'plap', 'plap_gauss', 'minsurf', 'invcoef', 'neohooke'])
@pytest.mark.parametrize('form', [1, 2])
def test_vcycle(kind, form):
    w = small(kind)
    u, v, m, b = _inputs(w, 160, True)
    ctx, levels, opts = _setup_both(w, u, m, coarse_rtol=1e-10, fd_form=form)
    opts.coarse_rtol = 1e-10
    s = api.mg_vcycle(ctx, to_dev(v))
    ref = OM.vcycle(oracle_problem(w), levels, ctx.nlevels - 1, v, opts)
    assert rel(to_np(s), ref) < 1e-9


@pytest.mark.parametrize('kind', KINDS)
def test_vjp(kind):
    w = small(kind)
    ctx = make_ctx(w)
    L = ctx.nlevels - 1
    u, v, m, b = _inputs(w, 170, True)
    pb, g = oracle_problem(w), oracle_grid(w)
    md = to_dev(m) if m is not None else None
    out = api.jfnk_vjp(ctx, L, 0, to_dev(u), to_dev(v), md)
    assert rel(to_np(out), OD.vjp(pb, g, u, v, m)) < 1e-12
    if kind == 'invcoef':
        gm = api.jfnk_vjp(ctx, L, 1, to_dev(u), to_dev(v), md)
        assert rel(to_np(gm), OD.vjp_coef(pb, g, u, v, m)) < 1e-12


@pytest.mark.parametrize('kind', ['bratu2d', 'plap', 'plap_gauss', 'minsurf', 'neohooke'])
def test_energy(kind):
    w = small(kind)
    ctx = make_ctx(w)
    u, v, m, b = _inputs(w, 180, True)
    psi = api.jfnk_energy(ctx, ctx.nlevels - 1, to_dev(u), to_dev(b))
    ref = OP.energy(oracle_problem(w), oracle_grid(w), u, b)
    assert abs(psi - ref) <= 1e-12 * max(1.0, abs(ref))


def test_gaussian_load():
    w = small('plap')
    ctx = make_ctx(w)
    c, wd, a = W.gaussian_params(1, 16, 3)
    b = api.jfnk_assemble_load(ctx, 0, W.gaussian_param_array(c, wd, a))
    ref = OP.load_from_function(oracle_grid(w), OP.gaussian_source(c, wd, a))
    assert rel(to_np(b), ref) < 1e-13


def test_load_parameters_beyond_grid_refused():
    # 16 sources x 5 parameters = 80 doubles against a 3^3-node grid: the
    # parameters are staged in a node-sized device buffer, so the call is
    # refused before any copy or launch
    w = W.scaled('plap3d-128', (2, 2, 2), nlevels=1)
    ctx = make_ctx(w)
    c, wd, a = W.gaussian_params(1, 16, 3)
    with pytest.raises(api.JfnkError) as err:
        api.jfnk_assemble_load(ctx, 0, W.gaussian_param_array(c, wd, a))
    assert err.value.status == _lib.E_INVAL
    # one source (5 doubles) fits and matches the oracle
    c1, wd1, a1 = c[:1], wd[:1], a[:1]
    b = api.jfnk_assemble_load(ctx, 0, W.gaussian_param_array(c1, wd1, a1))
    ref = OP.load_from_function(oracle_grid(w), OP.gaussian_source(c1, wd1, a1))
    assert rel(to_np(b), ref) < 1e-13


def test_traction_load():
    w = small('neohooke')
    ctx = make_ctx(w)
    t = W.traction(2)
    b = api.jfnk_assemble_load(ctx, 1, t)
    ref = OP.traction_load(oracle_grid(w), t)
    assert rel(to_np(b), ref) < 1e-14
