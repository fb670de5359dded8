#!/usr/bin/env python3
"""Benchmark: DoF/s to a 1e-8 relative nonlinear residual on one MI355X.

Workload (default plap3d-256): the regularised p-Laplacian (p = 3,
delta = 1e-2) on the unit cube, 256^3 Q1 elements (16,581,375 DoFs), load =
16 seeded Gaussians, 6 multigrid levels, Chebyshev degree 4, FGMRES(30).
One step = one full inexact-Newton solve from u = 0 to ||F|| <= 1e-8 ||F_0||
with the FP32 V-cycle (FP64 outer Newton, outer FD Jv, Arnoldi and norms).
The same solve with FP64 levels is timed for comparison.

Printed JSON line: value = DoF / (seconds per solve) of the FP32-multigrid
solve; roofline = the fine-level kernel class with the largest share of the
timed region, measured with HIP events around each of its launches;
fine_residual = FP64 F(u) GB/s over rotating buffers (and the same with the
p-Laplacian coefficient at each Gauss point, against the FP64 VALU peak);
cpu_baseline = the
NumPy oracle on the host (see --help).  The paper's own experiments (Bratu
and minimal surface on 800 x 800 elements, the Neo-Hookean beam on
160 x 16 x 16, with its solver settings: CG-MG, V(5, 5), shifted coarse
CG-QN, ||F|| <= 1e-6) are solved as well and reported beside the paper's
Table 1-3 counts, with Bratu and the minimal surface also at every
refinement level L1..L5 (Table 2; --no-paper skips all of them).
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print('[bench]', *a, file=sys.stderr, flush=True)


HBM_PEAK_GBS = 8000.0

# algorithmic bytes per fine node of each timed kernel class
BYTES_PER_NODE = {
    'cheb_step_f32': 7 * 4,   # difference form: reads x, d, r, s; writes r, s, d'
    'cheb_step_f64': 7 * 8,
    'outer_jv': 8 + 8 + 4 + 8,   # reads u, A(u) (FP64), z (FP32); writes Jv (FP64)
    'outer_jv_f64': 4 * 8,
    'resid_fine': 4 * 8,      # reads u, b; writes F and A(u)
}


HERE = os.path.dirname(os.path.abspath(__file__))
STENCIL_SOURCES = ['common.hpp', 'access.hpp', 'elem.hpp', 'reduce.hpp', 'stencil.hpp', 'stencil_tiled.hpp',
                   'ops_stencil.inc']
TRAFFIC_FILES = {'cheb_step_f32': 'cheb_step_f32_plap3d-256_hbm_traffic.md',
                 'resid_f64': 'resid_f64_plap3d-256_hbm_traffic.md'}


def stencil_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(HERE, 'paper_2103_13890_amd', 'csrc', f), 'rb') as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    name = TRAFFIC_FILES.get(kernel)
    path = os.path.join(HERE, 'profiles', name) if name else None
    if not path or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ':' in line and not line.startswith(('#', ' ', '|')):
                k, v = line.split(':', 1)
                vals[k.strip()] = v.strip()
    if vals.get('kernel_source_sha256_16') != stencil_hash() or 'traffic_bytes_per_launch' not in vals:
        return None
    return int(vals['traffic_bytes_per_launch'])


def build_problem(w):
    from paper_2103_13890_amd import api
    return api.make_problem(w['kind'], w['n'], w['h'], w['faces'], w['params'], w['nlevels'])


def make_load(ctx, w):
    from paper_2103_13890_amd import api
    from paper_2103_13890_amd import workloads as W
    c, wd, a = W.gaussian_params(w.get('load_seed', 1), 16, len(w['n']))
    return api.jfnk_assemble_load(ctx, 0, W.gaussian_param_array(c, wd, a))


def timed_solves(ctx, b, steps, warmup, timers=True, u0=None):
    """Solve from 0 (or from u0, which carries Dirichlet data) warmup + steps times."""
    import torch
    from paper_2103_13890_amd import api
    from paper_2103_13890_amd import _lib
    u = ctx.empty(ctx.nlevels - 1)

    def start():
        if u0 is None:
            u.zero_()
        else:
            u.copy_(u0)
    for i in range(warmup):
        start()
        rep = api.jfnk_solve(ctx, u, None, b)
        log(f'warmup {i}: {rep["status"]} newton {rep["newton_iters"]} krylov {rep["linear_iters"]} '
            f'{rep["time_ms"]:.1f} ms')
    tids = [_lib.TIMER_CHEB_FINE, _lib.TIMER_JV_OUTER, _lib.TIMER_RESID_FINE, _lib.TIMER_ARNOLDI]
    if timers:
        for t in tids:
            api.jfnk_timer_enable(ctx, t, True)
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        start()
        reps.append(api.jfnk_solve(ctx, u, None, b))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = {}
    if timers:
        for t in tids:
            tim[t] = api.jfnk_timer_read(ctx, t)
            api.jfnk_timer_enable(ctx, t, False)
    for i, r in enumerate(reps):
        log(f'step {i}: {r["status"]} newton {r["newton_iters"]} krylov {r["linear_iters"]} '
            f'GE {r["ge_effective"]:.1f} {r["time_ms"]:.1f} ms')
    return u, reps, (t1 - t0) / steps, tim


def residual_gbps(ctx, w, nsets=4, launches=100):
    """FP64 F(u) on the finest level, rotating over nsets buffer sets."""
    import torch
    from paper_2103_13890_amd import api
    from paper_2103_13890_amd import _lib
    L = ctx.nlevels - 1
    sets = []
    for k in range(nsets):
        u = torch.rand(ctx.node_shape(L), dtype=torch.float64, device=ctx.device) * 0.1
        b = torch.rand_like(u) * 1e-6
        sets.append((u, b, torch.empty_like(u)))
    for k in range(nsets):
        api.jfnk_residual(ctx, L, sets[k][0], None, sets[k][1], sets[k][2])
    api.jfnk_timer_enable(ctx, _lib.TIMER_RESID_FINE, True)
    for i in range(launches):
        u, b, F = sets[i % nsets]
        api.jfnk_residual(ctx, L, u, None, b, F)
    cnt, ms = api.jfnk_timer_read(ctx, _lib.TIMER_RESID_FINE)
    api.jfnk_timer_enable(ctx, _lib.TIMER_RESID_FINE, False)
    _, nn, _ = ctx.level_info(L)
    avg = ms / cnt
    gbs = 24.0 * nn / (avg * 1e-3) / 1e9
    del sets
    return {'gbps': gbs, 'frac': gbs / HBM_PEAK_GBS, 'avg_us': avg * 1e3, 'launches': cnt,
            'bytes_per_launch': 24 * nn, 'buffers': f'{nsets} rotating sets of u, b, F (FP64)'}


# FP64 operations per element of the Gauss-point p-Laplacian residual as the
# element routine is written (an FMA counts 2, a square root 1): gradients at
# the Gauss points 84, |g_q|^2 and the coefficient 8 x 8, fluxes 24, the
# scatter back to the corners 104
GAUSS_FLOPS_PER_ELEM = 84 + 64 + 24 + 104
FP64_VALU_PEAK_TFLOPS = 78.6


def gauss_residual(w):
    """FP64 F(u) of the p-Laplacian with its coefficient at each of the 8
    Gauss points (instead of the element mean) on the same grid: HBM rate
    and FP64 VALU rate."""
    from paper_2103_13890_amd import api
    prob = api.make_problem('plap_gauss', w['n'], w['h'], w['faces'], w['params'], w['nlevels'])
    ctx = api.Context(prob, api.default_options(vcycle_prec=0))
    r = residual_gbps(ctx, w)
    ne = 1
    for k in w['n']:
        ne *= k
    tf = GAUSS_FLOPS_PER_ELEM * ne / (r['avg_us'] * 1e-6) / 1e12
    r.update({'flops_per_element': GAUSS_FLOPS_PER_ELEM, 'tflops_fp64': tf,
              'frac_fp64_valu': tf / FP64_VALU_PEAK_TFLOPS, 'valu_peak_tflops': FP64_VALU_PEAK_TFLOPS})
    del ctx
    return r


def host_cpu():
    """The host's CPU model and the threads this process may use."""
    model = 'unknown'
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def cpu_baseline(w, rep, ndof):
    """The NumPy oracle's time for the same solve, extrapolated from timed
    units of the oracle at full size on the host:

    * t_Jv[l]: an FD product level_jv on each level l (the unit that every
      gradient evaluation, GE, stands for; the fastest of two or three);
    * one mg_setup with two fixed power steps, its GEs counted by the
      oracle's own Stats: its time beyond those GEs is the per-setup work
      outside GEs (projections, FD step numerators);
    * one V-cycle (Algorithm 1) on those levels, its GEs counted: its time
      beyond them is the per-cycle vector work (Chebyshev recurrences,
      transfers, coarse CG);
    * FGMRES cycles of 3 and 6 iterations with a diagonal operator and the
      identity preconditioner: the DCGS2 Arnoldi cost c0 + c1 (j + 1) of an
      iteration with j + 1 basis vectors, the diagonal product subtracted.

    T = sum_l GE_l t_Jv[l] + N_K (V-cycle work outside GEs) + N_Newton
    (setup work outside GEs) + sum over the solve's FGMRES iterations of
    c0 + c1 (j + 1), with GE_l, N_K, N_Newton and the iterations per Newton
    step (restart 30) those of the GPU solve in rep.  Residual evaluations
    are priced as FD products (slightly more), so T errs toward a slower
    oracle only by that."""
    from oracle import krylov as OK
    from oracle import mg as OM
    from oracle.fe import Grid
    from oracle.problems import Problem
    from paper_2103_13890_amd import workloads as W
    o = w['options']
    g = Grid(w['n'], w['h'], w['faces'])
    pb = Problem('plap', {'p': w['params'][0], 'delta': w['params'][1]})
    opts = OM.MGOptions(nu_pre=o['nu_pre'], nu_post=o['nu_post'], power_fixed=True, power_maxit=2,
                        coarse_rtol=1e-6)
    grids = OM.make_grids(g, w['nlevels'])
    L = w['nlevels'] - 1
    u = 0.01 * W.rough_state(w['n'], w['faces'], 7)
    wall0, cpu0 = time.perf_counter(), time.process_time()

    st_setup = OM.Stats()
    t0 = time.perf_counter()
    levels = OM.mg_setup(pb, grids, u, None, opts, None, st_setup)
    t_setup = time.perf_counter() - t0
    t_jv = []
    for l in range(L + 1):
        v = W.normal_vector(grids[l].n, w['faces'], 300 + l)
        best = np.inf
        for _ in range(3 if l < L else 2):          # the fastest of a few: first touches excluded
            t0 = time.perf_counter()
            OM.level_jv(pb, levels[l], v)
            best = min(best, time.perf_counter() - t0)
        t_jv.append(best)
    st_v = OM.Stats()
    bL = W.normal_vector(w['n'], w['faces'], 310)
    t0 = time.perf_counter()
    OM.vcycle(pb, levels, L, bL, opts, st_v)
    t_v = time.perf_counter() - t0
    d = 1.0 + np.random.default_rng(11).random(bL.shape)
    t0 = time.perf_counter()
    for _ in range(3):
        _ = d * bL
    t_diag = (time.perf_counter() - t0) / 3
    t_k = {}
    for k in (3, 6):
        t0 = time.perf_counter()
        OK.fgmres(lambda z: d * z, bL, lambda v: v, 0.0, restart=k, max_cycles=1)
        t_k[k] = time.perf_counter() - t0 - k * t_diag
    wall = time.perf_counter() - wall0
    cpu = time.process_time() - cpu0
    # t_k = k c0 + c1 k (k + 1) / 2
    c1 = max(0.0, (t_k[6] - 2.0 * t_k[3]) / 9.0)
    c0 = max(0.0, (t_k[3] - 6.0 * c1) / 3.0)

    ge = rep['ge_level']
    ge_v = [st_v.ge.get(l, 0) for l in range(L + 1)]
    ge_s = [st_setup.ge.get(l, 0) for l in range(L + 1)]
    v_extra = max(0.0, t_v - sum(ge_v[l] * t_jv[l] for l in range(L + 1)))
    s_extra = max(0.0, t_setup - sum(ge_s[l] * t_jv[l] for l in range(L + 1)))
    nk, nn = rep['linear_iters'], rep['newton_iters']
    t_arn = 0.0
    for n in rep['lin_hist'][:nn]:
        for i in range(n):
            t_arn += c0 + c1 * (i % 30 + 1)
    t_ge = sum(ge[l] * t_jv[l] for l in range(L + 1))
    T = t_ge + nk * v_extra + nn * s_extra + t_arn
    model, avail = host_cpu()
    return {'value': ndof / T, 'unit': 'DoF/s', 'cores': round(cpu / wall, 2), 'kind': 'oracle',
            'extrapolated': True, 'seconds_per_solve': T, 'host_cpu': model, 'host_threads_available': avail,
            'sample_seconds': round(wall, 1),
            'units_s': {'jv_per_level': [round(t, 4) for t in t_jv], 'mg_setup_2_power_steps': round(t_setup, 3),
                        'vcycle': round(t_v, 3), 'vcycle_ge_per_level': ge_v, 'arnoldi_c0': round(c0, 4),
                        'arnoldi_c1_per_basis_vector': round(c1, 4)},
            'breakdown_s': {'gradient_evaluations': round(t_ge, 1), 'vcycle_vector_work': round(nk * v_extra, 1),
                            'setup_outside_ge': round(nn * s_extra, 1), 'arnoldi': round(t_arn, 1)},
            'sample': (f'timed on the host at full size ({"x".join(map(str, w["n"]))}, {wall:.0f} s): one FD '
                       f'product per level, one mg_setup (2 power steps), one V-cycle and FGMRES(3), FGMRES(6) '
                       f'Arnoldi cycles of the NumPy oracle (FP64); extrapolated to this solve\'s counts '
                       f'({nn} Newton steps, {nk} FGMRES iterations, GE per level {[round(x) for x in ge]}); '
                       f'cores = process CPU time / wall time over the sample')}


ORACLE_PARAMS = {'bratu': ('lam',), 'plap': ('p', 'delta'), 'invcoef': (), 'neohooke': ('E', 'nu')}


def oracle_table():
    """The oracle (NumPy FP64, as it stands) timed on the host: F(u), an FD
    product and one V-cycle on the 128^3 and 256^3 p-Laplacian grids (the
    fastest of a few calls; the V-cycle once, on levels set up with two
    fixed power steps), and full solves to ||F|| <= 1e-8 ||F_0|| from u = 0
    of the 2D Bratu 32^2, the p-Laplacian 128^3 and the inverse-coefficient
    problem 128^3 (at m) with their configured multigrid (FP64 levels).
    The 256^3 solve is the extrapolation of the default run's cpu_baseline."""
    from oracle import mg as OM
    from oracle import newton as ON
    from oracle import problems as OP
    from oracle.fe import Grid
    from oracle.problems import Problem
    from paper_2103_13890_amd import workloads as W
    model, avail = host_cpu()
    wall0, cpu0 = time.perf_counter(), time.process_time()

    def setup(name):
        w = W.WORKLOADS[name]
        pb = Problem(w['kind'], dict(zip(ORACLE_PARAMS[w['kind']], w['params'])))
        g = Grid(w['n'], w['h'], w['faces'])
        o = w['options']
        mo = OM.MGOptions(nu_pre=o.get('nu_pre', 4), nu_post=o.get('nu_post', 4),
                          power_fixed=bool(o.get('power_fixed', 0)), power_maxit=o.get('power_maxit', 30),
                          coarse_rtol=1e-6)
        return w, pb, g, mo

    def best(fn, k):
        t = np.inf
        for _ in range(k):
            t0 = time.perf_counter()
            fn()
            t = min(t, time.perf_counter() - t0)
        return t
    units = {}
    for name in ('plap3d-128', 'plap3d-256'):
        w, pb, g, mo = setup(name)
        u = 0.01 * W.rough_state(w['n'], w['faces'], 7)
        b = np.zeros_like(u)
        reps = 3 if name.endswith('128') else 2
        t_f = best(lambda: OP.residual(pb, g, u, b), reps)
        mo2 = OM.MGOptions(nu_pre=mo.nu_pre, nu_post=mo.nu_post, power_fixed=True, power_maxit=2,
                           coarse_rtol=1e-6)
        levels = OM.mg_setup(pb, OM.make_grids(g, w['nlevels']), u, None, mo2)
        v = W.normal_vector(w['n'], w['faces'], 8)
        t_jv = best(lambda: OM.level_jv(pb, levels[-1], v), reps)
        t0 = time.perf_counter()
        OM.vcycle(pb, levels, w['nlevels'] - 1, v, mo2)
        t_v = time.perf_counter() - t0
        units[name] = {'residual_s': t_f, 'fd_jv_s': t_jv, 'vcycle_s': t_v}
        log(f'oracle units {name}: F {t_f:.3f} s, J v {t_jv:.3f} s, V-cycle {t_v:.2f} s')
        del levels
    solves = {}
    for name in ('bratu2d-32', 'plap3d-128', 'invcoef3d-128'):
        w, pb, g, mo = setup(name)
        if w['kind'] == 'bratu':
            b, m = np.zeros(g.node_shape), None
        else:
            c, wd, a = W.gaussian_params(w.get('load_seed', 1), 16, len(w['n']))
            b = OP.load_from_function(g, OP.gaussian_source(c, wd, a))
            m = W.matern_field(w['n'], w['h'], w.get('m_seed', 3)) if w['kind'] == 'invcoef' else None
        t0 = time.perf_counter()
        _, rep = ON.solve(pb, g, w['nlevels'], np.zeros(g.node_shape), b, m, mo, ON.NewtonOptions(rtol=1e-8))
        sec = time.perf_counter() - t0
        ndof = int(np.sum(g.dof_mask()))
        solves[name] = {'seconds': sec, 'dof_per_s': ndof / sec, 'dofs': ndof, 'status': rep.status,
                        'newton': rep.newton_iters, 'krylov': rep.linear_iters}
        log(f'oracle solve {name}: {rep.status}, {sec:.1f} s, {rep.newton_iters} Newton, '
            f'{rep.linear_iters} Krylov')
    wall = time.perf_counter() - wall0
    return {'kind': 'oracle', 'host_cpu': model, 'host_threads_available': avail,
            'cores': round((time.process_time() - cpu0) / wall, 2), 'units': units, 'solves_to_1e-8': solves,
            'seconds': round(wall, 1)}


def sampled_check(ctx, w, u, b, nsamp=4096):
    """The oracle's residual at sampled nodes of the FP32-MG solution: how far
    the GPU's F(u) is from the oracle's there, and how small the oracle's
    F(u) is, both relative to the largest sampled load entry."""
    from oracle.fe import Grid
    from oracle.problems import Problem, residual_at
    from paper_2103_13890_amd import api
    g = Grid(w['n'], w['h'], w['faces'])
    pb = Problem('plap', {'p': w['params'][0], 'delta': w['params'][1]})
    L = ctx.nlevels - 1
    F = api.jfnk_residual(ctx, L, u, None, b).cpu().numpy().reshape(-1)
    un, bn = u.cpu().numpy(), b.cpu().numpy()
    rng = np.random.default_rng(5)
    nodes = rng.choice(g.n_nodes, nsamp, replace=False)
    Fo = residual_at(pb, g, un, bn, nodes)
    scale = max(float(np.max(np.abs(bn.reshape(-1)[nodes]))), 1e-300)
    return {'nodes': nsamp, 'max_abs_diff_over_max_load': float(np.max(np.abs(F[nodes] - Fo)) / scale),
            'oracle_max_abs_residual_over_max_load': float(np.max(np.abs(Fo)) / scale)}


# Tables 1 and 2 (and 3, shifted CG-QN column), finest row: Newton steps,
# CG-MG steps, total gradient evaluations (the paper's elements and meshes)
# and average GE per CG-MG step (AGE, Table 2)
PAPER_FINEST = {'bratu2d-800': {'level': 'L5', 'newton': 3, 'cg_mg': 9, 'ge': 238, 'age': 26.53},
                'minsurf2d-800': {'level': 'L5', 'newton': 9, 'cg_mg': 41, 'ge': 931, 'age': 22.79},
                'beam3d-160x16x16': {'level': 'L4', 'newton': 5, 'cg_mg': 39, 'ge': 733, 'age': 18.76}}


def paper_mode_solves(steps):
    """The paper's three experiments at their finest refinement with the
    paper's solver settings (CG-MG outer solver, V(5, 5), shifted coarse
    CG-QN, stop at ||F|| <= 1e-6): Bratu and minimal surface on 800 x 800
    Q1 elements (6 levels from the 25 x 25 coarse mesh), the Neo-Hookean
    beam on 160 x 16 x 16 (5 levels from 10 x 1 x 1)."""
    import torch
    from paper_2103_13890_amd import api
    from paper_2103_13890_amd import workloads as W
    out = {}
    for name in ('bratu2d-800', 'minsurf2d-800', 'beam3d-160x16x16'):
        w = W.WORKLOADS[name]
        ctx = api.Context(build_problem(w), api.default_options(**w['options']))
        _, _, ndof = ctx.level_info(ctx.nlevels - 1)
        u0 = torch.from_numpy(W.dirichlet_state(w)).to('cuda')
        b = torch.zeros_like(u0)
        log(f'paper settings: {name}')
        _, reps, sec, _ = timed_solves(ctx, b, steps, 1, timers=False, u0=u0)
        r = reps[-1]
        out[name] = {'ms_per_solve': sec * 1e3, 'dofs': ndof, 'ok': all(x['status'] == 'ok' for x in reps),
                     'newton': r['newton_iters'], 'cg_mg': r['linear_iters'], 'fnorm': r['fnorm'],
                     'ge_effective': r['ge_effective'], 'ge_level': r['ge_level'],
                     'age': r['ge_effective'] / max(r['linear_iters'], 1),
                     'coarse_calls': r['coarse_calls'], 'coarse_cg_iters': r['coarse_iters'],
                     'neg_curv': r['neg_curv'], 'coarse_qn_pairs': r['coarse_qn_pairs'],
                     'paper': PAPER_FINEST[name]}
        log(f'{name}: {sec * 1e3:.1f} ms/solve, Newton {r["newton_iters"]}, CG-MG {r["linear_iters"]}, '
            f'GE {r["ge_effective"]:.1f}')
        del ctx
        torch.cuda.empty_cache()
    return out


# Table 2 (the paper's meshes): Newton and CG-MG steps per refinement level,
# L1..L5 for Bratu and the minimal surface, L1..L4 for the beam
PAPER_TABLE2 = {'bratu2d-800': [(3, 7), (3, 9), (3, 9), (3, 9), (3, 9)],
                'minsurf2d-800': [(6, 13), (7, 18), (8, 25), (9, 32), (9, 41)],
                'beam3d-160x16x16': [(9, 28), (5, 15), (5, 20), (5, 39)]}


def paper_levels():
    """Table 2's trend on Q1 grids with the paper's settings, one untimed
    solve each: Bratu and the minimal surface at L1..L5 (25 * 2^k elements
    per axis on k + 1 levels), the beam at L1..L4 (10 * 2^k x 2^k x 2^k)."""
    import torch
    from paper_2103_13890_amd import api
    from paper_2103_13890_amd import workloads as W
    out = {}
    for name in ('bratu2d-800', 'minsurf2d-800', 'beam3d-160x16x16'):
        rows = []
        for k in range(1, len(PAPER_TABLE2[name]) + 1):
            n = (10 << k, 1 << k, 1 << k) if name.startswith('beam') else (25 << k, 25 << k)
            w = W.scaled(name, n, nlevels=k + 1)
            ctx = api.Context(build_problem(w), api.default_options(**w['options']))
            u = torch.from_numpy(W.dirichlet_state(w)).to('cuda')
            rep = api.jfnk_solve(ctx, u, None, torch.zeros_like(u))
            p_in, p_cg = PAPER_TABLE2[name][k - 1]
            rows.append({'level': f'L{k}', 'ok': rep['status'] == 'ok', 'newton': rep['newton_iters'],
                         'cg_mg': rep['linear_iters'], 'ge_effective': rep['ge_effective'],
                         'paper_newton': p_in, 'paper_cg_mg': p_cg})
            del ctx
        out[name] = rows
        log(f'{name} by level: Newton {[r["newton"] for r in rows]}, CG-MG {[r["cg_mg"] for r in rows]}, '
            f'GE {[round(r["ge_effective"], 1) for r in rows]}')
    return out


def oracle_reference(workload):
    """The oracle's stored tight solve for this workload, if there is one."""
    path = os.path.join(HERE, 'tests', 'golden', f'ref_{workload}.npz')
    return np.load(path) if os.path.exists(path) else None


def compare_to_reference(u, ref):
    """||u - u_ora|| / ||u_ora|| on the reference's sampled nodes, and the
    relative difference of the whole-grid 2-norms."""
    g = u.double().cpu().numpy().reshape(-1)
    s = g[ref['nodes']]
    return {'sampled': float(np.linalg.norm(s - ref['u']) / np.linalg.norm(ref['u'])),
            'norm': float(abs(np.linalg.norm(g) - float(ref['u_norm'])) / float(ref['u_norm']))}


def triad_gbps(n, nsets=4, launches=40):
    """c = a + s b over FP64 arrays of n entries (the fine level's node
    count), rotating over nsets buffer sets as the F(u) timing does
    (libjfnk's streaming calibration kernel): the HBM rate a dense sweep of
    arrays of this size reaches, beside the 8 TB/s peak."""
    import torch
    from paper_2103_13890_amd import api
    sets = [(torch.rand(n, dtype=torch.float64, device='cuda'), torch.rand(n, dtype=torch.float64, device='cuda'),
             torch.empty(n, dtype=torch.float64, device='cuda')) for _ in range(nsets)]
    for a, b, c in sets:
        api.jfnk_stream_triad(a, b, c)
    a, b, c = sets[0]
    ok = bool(torch.equal(c, a + 0.5 * b))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(launches):
        api.jfnk_stream_triad(*sets[i % nsets])
    e1.record()
    torch.cuda.synchronize()
    avg = e0.elapsed_time(e1) / launches
    gbs = 24.0 * n / (avg * 1e-3) / 1e9
    del sets
    return {'gbps': gbs, 'frac_of_peak': gbs / HBM_PEAK_GBS, 'avg_us': avg * 1e3, 'bytes_per_launch': 24 * n,
            'launches': launches, 'buffers': f'{nsets} rotating sets of a, b, c (FP64, {n} entries)', 'check': ok}


def copy_calibration(nbytes=1 << 30, launches=5):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device='cuda')
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(launches):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({'copy_bytes_read': nbytes, 'copy_bytes_written': nbytes, 'launches': launches}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--workload', default='plap3d-256')
    ap.add_argument('--no-fp64', action='store_true', help='skip the FP64-multigrid comparison solve')
    ap.add_argument('--no-cpu', action='store_true', help='skip the oracle CPU baseline')
    ap.add_argument('--no-qn', action='store_true',
                    help='skip the FP32-MG solve with the L-BFGS coarse preconditioner (CG-QN)')
    ap.add_argument('--no-paper', action='store_true',
                    help="skip the paper's three experiments solved with its solver settings")
    ap.add_argument('--no-gauss', action='store_true',
                    help='skip the FP64 residual with the coefficient at each Gauss point')
    ap.add_argument('--no-paper-fd', action='store_true',
                    help="skip the FP32-MG solve with the paper's black-box FD quotient on the levels")
    ap.add_argument('--no-triad', action='store_true', help='skip the streaming triad calibration')
    ap.add_argument('--kernel-path', type=int, default=0)
    ap.add_argument('--oracle-table', action='store_true',
                    help='only time the oracle on the host (units at 128^3 and 256^3, full solves of the '
                         '2D Bratu, p-Laplacian 128^3 and inverse-coefficient configurations) and exit')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='only run a 1 GiB device copy (to scale HBM counters) and exit')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) != 1:
        print('bench.py runs on exactly one GPU: libjfnk has no multi-GPU path', file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.oracle_table:
        print(json.dumps(oracle_table()), flush=True)
        return
    import torch
    from paper_2103_13890_amd import api
    from paper_2103_13890_amd import workloads as W

    w = W.WORKLOADS[args.workload]
    prob = build_problem(w)
    opts32 = api.default_options(**dict(w['options'], vcycle_prec=1, coarse_rtol=1e-3,
                                        kernel_path=args.kernel_path))
    log(f'workload {args.workload}: creating FP32-multigrid context')
    ctx = api.Context(prob, opts32)
    L = ctx.nlevels - 1
    _, nn, ndof = ctx.level_info(L)
    b = make_load(ctx, w)
    u32, reps32, sec32, tim = timed_solves(ctx, b, args.steps, args.warmup)
    value = ndof / sec32
    ok32 = all(r['status'] == 'ok' for r in reps32)
    # roofline of the dominant fine-level kernel class in the timed region
    from paper_2103_13890_amd import _lib
    cls = {_lib.TIMER_CHEB_FINE: 'cheb_step_f32', _lib.TIMER_JV_OUTER: 'outer_jv',
           _lib.TIMER_RESID_FINE: 'resid_fine'}
    shares = {cls[t]: tim[t] for t in cls}
    dom = max(shares, key=lambda k: shares[k][1])
    cnt, ms = shares[dom]
    avg_ms = ms / max(cnt, 1)
    achieved = BYTES_PER_NODE[dom] * nn / (avg_ms * 1e-3) / 1e9
    arn_cnt, arn_ms = tim[_lib.TIMER_ARNOLDI]
    traffic = measured_traffic(dom)
    roofline = {'bound': 'hbm', 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                'frac': round(achieved / HBM_PEAK_GBS, 4),
                'traffic': round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                'traffic_bytes_per_launch': traffic, 'kernel': dom,
                'avg_launch_us': round(avg_ms * 1e3, 2), 'launches': cnt,
                'bytes_per_launch': BYTES_PER_NODE[dom] * nn,
                'share_of_step': round(ms / (sec32 * 1e3 * args.steps), 4)}
    kernel_shares = {k: {'launches': v[0], 'ms_total': round(v[1], 3),
                         'share': round(v[1] / (sec32 * 1e3 * args.steps), 4)} for k, v in shares.items()}
    kernel_shares['arnoldi_dcgs2'] = {'launches': arn_cnt, 'ms_total': round(arn_ms, 3),
                                     'share': round(arn_ms / (sec32 * 1e3 * args.steps), 4)}
    ge32 = reps32[-1]['ge_effective']
    log(f'FP32-MG: {sec32 * 1e3:.1f} ms/solve, {value:.3e} DoF/s, dominant {dom} {achieved:.0f} GB/s')

    extra = {}
    if not args.no_qn:
        # the paper's CG-QN coarse solver (20 secant pairs), same FP32-MG solve
        del ctx
        torch.cuda.empty_cache()
        ctxq = api.Context(prob, api.default_options(**dict(w['options'], vcycle_prec=1, coarse_rtol=1e-3,
                                                            coarse_qn=20, kernel_path=args.kernel_path)))
        bq = make_load(ctxq, w)
        uq, repsq, secq, _ = timed_solves(ctxq, bq, max(1, min(args.steps, 2)), 1, timers=False)
        rq = repsq[-1]
        extra['fp32_mg_coarse_qn'] = {
            'ms_per_step': secq * 1e3, 'value': ndof / secq, 'ok': all(r['status'] == 'ok' for r in repsq),
            'newton': rq['newton_iters'], 'krylov': rq['linear_iters'], 'pairs': rq['coarse_qn_pairs'],
            'coarse_calls': rq['coarse_calls'], 'coarse_cg_iters': rq['coarse_iters'],
            'ge_effective': rq['ge_effective'],
            'rel_diff_vs_plain_cg_solution': float(torch.linalg.norm(uq - u32) / torch.linalg.norm(u32))}
        log(f'FP32-MG with CG-QN: {secq * 1e3:.1f} ms/solve, coarse CG {rq["coarse_iters"]} iterations in '
            f'{rq["coarse_calls"]} calls ({rq["coarse_qn_pairs"]} pairs)')
        del ctxq, uq, bq
        torch.cuda.empty_cache()
        ctx = None
    u64 = rep64 = None
    if not args.no_paper_fd:
        # the paper's black-box FD quotient (F(x + eps v) - F(x)) / eps on the
        # FP32 levels, eps from the FP32 machine epsilon (fd_form 1)
        del ctx
        torch.cuda.empty_cache()
        ctxp = api.Context(prob, api.default_options(**dict(w['options'], vcycle_prec=1, coarse_rtol=1e-3,
                                                            fd_form=1, kernel_path=args.kernel_path)))
        bp = make_load(ctxp, w)
        up, repsp, secp, _ = timed_solves(ctxp, bp, max(1, min(args.steps, 2)), 1, timers=False)
        rp = repsp[-1]
        extra['fp32_mg_paper_quotient'] = {
            'ms_per_step': secp * 1e3, 'value': ndof / secp, 'ok': all(r['status'] == 'ok' for r in repsp),
            'status': rp['status'], 'newton': rp['newton_iters'], 'krylov': rp['linear_iters'],
            'ge_effective': rp['ge_effective'], 'final_rel_residual': rp['fnorm'] / rp['fnorm0'],
            'rel_diff_vs_difference_form_solution': float(torch.linalg.norm(up - u32) / torch.linalg.norm(u32))}
        log(f'FP32-MG with the black-box quotient: {rp["status"]}, {secp * 1e3:.1f} ms/solve, Newton '
            f'{rp["newton_iters"]}, FGMRES {rp["linear_iters"]}')
        del ctxp, up, bp
        torch.cuda.empty_cache()
        ctx = None
    if not args.no_fp64:
        del ctx
        torch.cuda.empty_cache()
        opts64 = api.default_options(**dict(w['options'], vcycle_prec=0, coarse_rtol=1e-6,
                                            kernel_path=args.kernel_path))
        log('creating FP64-multigrid context')
        ctx64 = api.Context(prob, opts64)
        b64 = make_load(ctx64, w)
        u64, reps64, sec64, _ = timed_solves(ctx64, b64, args.steps, args.warmup, timers=False)
        ok64 = all(r['status'] == 'ok' for r in reps64)
        rep64 = reps64[-1]
        extra['fp64_mg'] = {'value': ndof / sec64, 'ms_per_step': sec64 * 1e3, 'ok': ok64,
                            'newton': reps64[-1]['newton_iters'], 'krylov': reps64[-1]['linear_iters'],
                            'ge_effective': reps64[-1]['ge_effective'],
                            'final_rel_residual': reps64[-1]['fnorm'] / reps64[-1]['fnorm0']}
        extra['fp32_over_fp64_speedup'] = sec64 / sec32
        extra['rel_diff_fp32_vs_fp64_solution'] = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        log(f'FP64-MG: {sec64 * 1e3:.1f} ms/solve; speedup {sec64 / sec32:.2f}')
        # tight FP64 solve (to 1e-11, near the FP64 floor at this size) for the error statement
        del ctx64
        torch.cuda.empty_cache()
        opts_t = api.default_options(**dict(w['options'], vcycle_prec=0, coarse_rtol=1e-6, newton_rtol=1e-11,
                                            kernel_path=args.kernel_path))
        ctxt = api.Context(prob, opts_t)
        ut = ctxt.empty(L)
        rt = api.jfnk_solve(ctxt, ut, None, b64)
        extra['rel_err_vs_tight_fp64_solution'] = {
            'fp32_mg': float(torch.linalg.norm(u32 - ut) / torch.linalg.norm(ut)),
            'fp64_mg': float(torch.linalg.norm(u64 - ut) / torch.linalg.norm(ut)),
            'tight_status': rt['status'], 'tight_rel_residual': rt['fnorm'] / rt['fnorm0']}
        ref = oracle_reference(args.workload)
        if ref is not None:
            extra['rel_err_vs_oracle_solution'] = {
                'fp32_mg': compare_to_reference(u32, ref), 'fp64_mg': compare_to_reference(u64, ref),
                'reference': f'tests/golden/ref_{args.workload}.npz: the oracle\'s FP64 Newton iterate at '
                             f'||F|| = {float(ref["f"]) / float(ref["f0"]):.2e} ||F_0||, '
                             f'{len(ref["nodes"])} seeded nodes and the whole-grid 2-norm'}
            log(f'vs the oracle solution: {extra["rel_err_vs_oracle_solution"]}')
        fres = residual_gbps(ctxt, w)
        tr = measured_traffic('resid_f64')
        fres['traffic'] = round(tr / (fres['avg_us'] * 1e-6) / 1e9, 1) if tr else None
        fres['traffic_bytes_per_launch'] = tr
        extra['fine_residual_f64'] = fres
        log(f'fine F(u) FP64: {fres["gbps"]:.0f} GB/s ({fres["avg_us"]:.1f} us)')
        try:
            extra['oracle_sampled_residual'] = sampled_check(ctxt, w, u32, b64)
        except Exception as e:      # the check is informative only
            extra['oracle_sampled_residual'] = f'skipped: {e}'
        del ctxt
    if w['kind'] == 'plap' and not args.no_gauss:
        torch.cuda.empty_cache()
        fg = gauss_residual(w)
        extra['fine_residual_f64_gauss'] = fg
        log(f'fine F(u) FP64, coefficient at the Gauss points: {fg["avg_us"]:.1f} us, {fg["gbps"]:.0f} GB/s, '
            f'{fg["tflops_fp64"]:.1f} TFLOP/s FP64')
    if not args.no_paper:
        extra['paper_settings'] = paper_mode_solves(max(1, min(args.steps, 3)))
        extra['paper_table2_levels'] = paper_levels()
    if not args.no_triad:
        torch.cuda.empty_cache()
        extra['hbm_triad_calibration'] = triad_gbps(nn)
        log(f'streaming triad: {extra["hbm_triad_calibration"]["gbps"]:.0f} GB/s')
    cpu = None
    if not args.no_cpu:
        log('timing the oracle sample on the host')
        cpu = cpu_baseline(w, rep64 if rep64 is not None else reps32[-1], ndof)
        log(f'oracle (extrapolated): {cpu["seconds_per_solve"]:.0f} s/solve from a {cpu["sample_seconds"]} s sample')

    out = {
        'metric': 'DoF/s to 1e-8 nonlinear residual, FP32-MG vs FP64-MG; fine F(u) HBM GB/s',
        'value': value, 'unit': 'DoF/s', 'n_gpus': 1, 'steps': args.steps, 'warmup': args.warmup,
        'ms_per_step': sec32 * 1e3, 'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'f64 outer / f32 multigrid', 'data': 'synthetic',
        'config': {'workload': args.workload, 'elements': list(w['n']), 'dofs': ndof, 'levels': w['nlevels'],
                   'cheb_degree': w['options']['nu_pre'], 'restart': 30, 'newton_rtol': 1e-8,
                   'discretisation': 'Q1, element-mean coefficient'},
        'ok': ok32, 'newton_iters': reps32[-1]['newton_iters'], 'krylov_iters': reps32[-1]['linear_iters'],
        'ge_effective': ge32, 'final_rel_residual': reps32[-1]['fnorm'] / reps32[-1]['fnorm0'],
        'coarse': {'calls': reps32[-1]['coarse_calls'], 'cg_iters': reps32[-1]['coarse_iters'],
                   'neg_curv': reps32[-1]['neg_curv']},
        'roofline': roofline, 'kernel_shares': kernel_shares, 'cpu_baseline': cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
