"""FP32 multigrid levels against the oracle, in the benchmark's launch shapes.

The benchmark solve runs every multigrid level in FP32 (vcycle_prec = 1):
the FD Jacobian action in the element difference form, the fused Chebyshev
steps (first, interior and last), the power method, the transfers and the
coarse CG (Sec. 2 smoothers and coarse solver; Algorithm 1).  Here each of
them is compared with the oracle's FP64 algorithm on the same inputs.

* Grid: the p-Laplacian (p = 3, delta = 1e-2) on 128 x 64 x 64 elements,
  4 levels.  The two finest levels take the FP32 row-tiled kernel (128 and
  64 elements in x, the second with one-plane z chunks), 32 x 16 x 16 the
  node kernel, and the 16 x 8 x 8 coarse grid (735 DoFs) the coarse kernel.
* 256^3 (the benchmark's finest level): the smoother from s = 0 and from
  s != 0 with degree 4, i.e. the fused first step, the interior step and the
  fused last step in the benchmark's 256-thread row tiles, against the
  oracle's Chebyshev iteration on the whole grid.
* Step: fd_root = 1e-2 on every level, so that FD truncation is not the
  difference being measured; with the same step the GPU's difference form
  and the oracle's quotient of two residuals are the same quotient up to
  rounding.
* The oracle evaluates at the GPU's FP32 level states (exact in FP64) and
  with the GPU's lambda_l, so the comparison isolates the FP32 arithmetic of
  the kernels from the rounding of the states to FP32.  The states
  themselves are checked against the oracle's projection to FP32 rounding
  (2^-24 relative per entry), and the power method's lambda_l against the
  oracle's.

Bars (relative 2-norms), from FP32 arithmetic (unit roundoff
u = 2^-24 = 6e-8), with the values measured on MI355X in brackets:
* x_l 1e-7 [2.6e-8]: one rounding of the oracle's projection;
* lambda_l 1e-6 [6e-8] and the eigenvector 1e-5 [2e-7]: ten power steps,
  each an FD product in FP32;
* A_l(x_l) 1e-4 [1.7e-7 coarsest .. 1.9e-5 finest]: the element stiffness
  applied to a smooth FP32 state cancels (4 x_a minus four neighbours of the
  same size leaves O(h^2 |x|)), so rounding errors of |x| size grow like
  1/h^2 relative to the result;
* smoother and V-cycle outputs 1e-5 [1.1e-6, 1.8e-6] on 128 x 64 x 64, and
  the 256^3 smoother 1e-4 [4.5e-5]: the same cancellation, four times
  larger at half the mesh size.
"""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import make_ctx, oracle_grid, oracle_mg_options, oracle_problem, rel, to_dev, to_np
from oracle import mg as OM
from oracle import problems as OP
from paper_2103_13890_amd import api
from paper_2103_13890_amd import workloads as W

U32 = 2.0 ** -24


def _w128():
    return W.scaled('plap3d-128', (128, 64, 64), nlevels=4, vcycle_prec=1, coarse_rtol=1e-6)


def _smooth_state(w, seed, amp=0.3):
    g = oracle_grid(w)
    xs = g.node_coords()
    bump = np.prod([np.sin(np.pi * x / (w['n'][k] * w['h'])) for k, x in enumerate(xs)], axis=0)
    u = amp * bump + 1e-3 * W.rough_state(w['n'], w['faces'], seed)
    u[g.dirichlet_mask()] = 0
    return u


def _f32(a):
    """An FP64 array rounded to FP32 (as the GPU levels hold it), back in FP64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


OVER = dict(fd_root=1e-2, power_fixed=1, power_maxit=10)


@pytest.fixture(scope='module')
def setup128():
    w = _w128()
    u = _smooth_state(w, 200)
    ctx = make_ctx(w, **OVER)
    api.mg_setup(ctx, to_dev(u))
    pb = oracle_problem(w)
    opts = oracle_mg_options(w, fd_root=1e-2, power_fixed=True, power_maxit=10, coarse_rtol=1e-6)
    grids = OM.make_grids(oracle_grid(w), ctx.nlevels)
    ora = OM.mg_setup(pb, grids, u, None, opts)          # the oracle's own setup (FP64 states)
    lam = api.mg_get_lambda(ctx)
    # the oracle's levels at the GPU's FP32 states and eigenvalue estimates
    at = []
    for l in range(ctx.nlevels):
        x = to_np(api.mg_get_level(ctx, l, 'x'))
        lev = OM.Level(grid=grids[l], x=x, m=None)
        lev.Ax = OP.apply_A(pb, grids[l], x)
        lev.eps_num = OM.eps_numerator(grids[l], x, opts)
        lev.lam = lam[l]
        at.append(lev)
    return dict(w=w, ctx=ctx, pb=pb, opts=opts, ora=ora, at=at, lam=lam)


def test_fp32_setup(setup128):
    s = setup128
    ctx, ora, at = s['ctx'], s['ora'], s['at']
    for l in range(ctx.nlevels):
        x = at[l].x
        ex = rel(x, ora[l].x)
        assert ex <= 1e-7, (l, ex)
        assert np.array_equal(x, _f32(x))                # FP32 values
        eA = rel(to_np(api.mg_get_level(ctx, l, 'Ax')), at[l].Ax)
        print(f'level {l}: x {ex:.2e}, A(x) {eA:.2e}', flush=True)
        assert eA <= 1e-4, (l, eA)
        if l >= 1:
            el = abs(s['lam'][l] - ora[l].lam) / abs(ora[l].lam)
            ev = rel(to_np(api.mg_get_level(ctx, l, 'eig')), ora[l].eig)
            print(f'level {l}: lambda {el:.2e}, eigenvector {ev:.2e}', flush=True)
            assert el <= 1e-6 and ev <= 1e-5, (l, el, ev)


def test_fp32_smoother(setup128):
    s = setup128
    ctx, w, pb, at, opts = s['ctx'], s['w'], s['pb'], s['at'], s['opts']
    worst = 0.0
    for l in range(1, ctx.nlevels):
        lev = at[l]
        gl = lev.grid
        bl = _f32(W.normal_vector(gl.n, w['faces'], 210 + l))
        s0 = _f32(W.normal_vector(gl.n, w['faces'], 220 + l))
        for nu in (1, 2, 3, 4):
            for zero in (True, False):
                sd = to_dev(s0, torch.float32)
                api.mg_smooth(ctx, l, to_dev(bl, torch.float32), sd, nu, zero)
                ref = OM.chebyshev(lambda x: OM.level_jv(pb, lev, x), bl, 0 * s0 if zero else s0, nu, lev.lam,
                                   opts.cheb_lo, opts.cheb_hi, s_is_zero=zero)
                e = rel(to_np(sd), ref)
                worst = max(worst, e)
                assert e <= 1e-5, (l, nu, zero, e)
    print(f'FP32 smoother, worst relative difference {worst:.2e}', flush=True)


def test_fp32_vcycle(setup128):
    s = setup128
    ctx, w, pb, at, opts = s['ctx'], s['w'], s['pb'], s['at'], s['opts']
    L = ctx.nlevels - 1
    for seed in (230, 231):
        b = W.normal_vector(w['n'], w['faces'], seed)
        sv = to_np(api.mg_vcycle(ctx, to_dev(b)))
        # the V-cycle rounds its FP64 input to the FP32 level on entry
        ref = OM.vcycle(pb, at, L, _f32(b), opts)
        e = rel(sv, ref)
        print(f'FP32 V-cycle (seed {seed}): relative difference {e:.2e}', flush=True)
        assert e <= 1e-5, e


def test_fp32_transfers(setup128):
    s = setup128
    ctx, w = s['ctx'], s['w']
    from oracle import transfer as OT
    grids = [lev.grid for lev in s['at']]
    for l in range(ctx.nlevels - 1, 0, -1):
        gf, gc = grids[l], grids[l - 1]
        r = _f32(W.normal_vector(gf.n, w['faces'], 240 + l))
        rc = to_np(api.mg_restrict(ctx, l, to_dev(r, torch.float32)))
        assert rel(rc, OT.restrict(gc, gf, r)) <= 8 * U32
        c = _f32(W.normal_vector(gc.n, w['faces'], 250 + l))
        sf = _f32(W.normal_vector(gf.n, w['faces'], 260 + l))
        sd = to_dev(sf, torch.float32)
        api.mg_prolong_add(ctx, l, to_dev(c, torch.float32), sd)
        assert rel(to_np(sd), sf + OT.prolong(gc, gf, c)) <= 8 * U32


def test_fp32_smoother_256_bench_shape():
    """The benchmark's finest level (256^3, FP32 row tiles of 256 threads):
    degree-4 Chebyshev from s = 0 (fused first step, interior step, fused
    last step: the pre-smoother) and from s != 0 (start, two interior steps,
    last step: the post-smoother), on the whole grid."""
    w = dict(W.WORKLOADS['plap3d-256'])
    w['options'] = dict(w['options'], vcycle_prec=1)
    pb, g = oracle_problem(w), oracle_grid(w)
    print('256^3: states', flush=True)
    u = _smooth_state(w, 270)
    ctx = make_ctx(w, fd_root=1e-2, power_fixed=1, power_maxit=3)
    api.mg_setup(ctx, to_dev(u))
    L = ctx.nlevels - 1
    x = to_np(api.mg_get_level(ctx, L, 'x'))
    assert rel(x, u) <= 1e-7
    opts = oracle_mg_options(w, fd_root=1e-2)
    lev = OM.Level(grid=g, x=x, m=None)
    print('256^3: oracle A(x)', flush=True)
    lev.Ax = OP.apply_A(pb, g, x)
    lev.eps_num = OM.eps_numerator(g, x, opts)
    lev.lam = api.mg_get_lambda(ctx)[L]
    b = _f32(W.normal_vector(w['n'], w['faces'], 271))
    s0 = _f32(W.normal_vector(w['n'], w['faces'], 272))
    for zero in (True, False):
        sd = to_dev(s0, torch.float32)
        api.mg_smooth(ctx, L, to_dev(b, torch.float32), sd, 4, zero)
        print(f'256^3: oracle Chebyshev from {"0" if zero else "s"}', flush=True)
        ref = OM.chebyshev(lambda v: OM.level_jv(pb, lev, v), b, 0 * s0 if zero else s0, 4, lev.lam,
                           opts.cheb_lo, opts.cheb_hi, s_is_zero=zero)
        e = rel(to_np(sd), ref)
        print(f'256^3 FP32 smoother from {"0" if zero else "s"}: relative difference {e:.2e}', flush=True)
        assert e <= 1e-4, (zero, e)
