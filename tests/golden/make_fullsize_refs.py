"""Write the oracle's tight solutions at the full benchmark sizes (test data).

For each configuration the oracle (FP64 NumPy; nothing of the GPU path is
imported) solves F(u) = 0 from u = 0 to ||F|| <= 1e-12 ||F_0|| (the
Neo-Hookean increment to 1e-11) and stores, in tests/golden/ref_<name>.npz:

  nodes         8192 node indices drawn with numpy.random.default_rng(2024)
                (per component for the three-component beam: flat indices
                into the (3, nodes) array)
  u             the solution at those nodes
  u_norm        ||u||_2 over the whole grid
  f0, f         ||F(0)||_2 and ||F(u)||_2
  newton, krylov  the oracle's iteration counts

The inverse-coefficient configuration also stores u_obs (the solution at the
second seeded field), the adjoint state lam of J(u)^T lam = u - u_obs and the
gradient g = -(dF/dm)^T lam of L(m) = 1/2 ||u - u_obs||^2 (Sec. 1: F(x*) = 0;
the adjoint of the implicit-function theorem), each at the nodes and as a
2-norm.

Inputs come from paper_2103_13890_amd/workloads.py (seeded generators, no
arithmetic of the method).  Usage:

    python tests/golden/make_fullsize_refs.py plap3d-128 invcoef3d-128 plap3d-256 neohooke-256x64

Each configuration runs in its own process; the 256^3 solve takes hours on
one core.  Options: --out DIR writes the files there instead; --progress
prints a line at every finest-level V-cycle and every Newton step (the
oracle's arithmetic is untouched: the V-cycle and setup functions the
Newton loop calls are wrapped by a logger).

A long solve can run in pieces: --checkpoint FILE saves the Newton iterate
(with ||F(0)||) at the start of every Newton step, and --resume FILE
continues the oracle's Newton solve from that iterate with forcing and stop
relative to the same ||F(0)|| (NewtonOptions.f0).  The root is the same
whatever the path; only the iteration counts stored with it then cover the
last piece.  --checkpoint-f32 stores the iterate rounded to FP32 and
compressed (a 256^3 iterate then fits a 64 MB transfer); the continued solve
starts from that rounded iterate, which moves its path, not its root.
--from-checkpoint FILE stores the saved iterate itself, with its residual
as the oracle evaluates it: for a solve whose last Newton steps no longer
lower ||F|| (its FP64 rounding floor, above the requested tolerance).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import adjoint as OA          # noqa: E402
from oracle import newton as ON           # noqa: E402
from oracle import problems as OP         # noqa: E402
from oracle.fe import Grid                # noqa: E402
from oracle.mg import MGOptions           # noqa: E402
from oracle.problems import Problem       # noqa: E402
from paper_2103_13890_amd import workloads as W   # noqa: E402

PARAMS = {'plap': ('p', 'delta'), 'invcoef': (), 'neohooke': ('E', 'nu')}
OUT = HERE
CHECKPOINT = None
CHECKPOINT_F32 = False
RESUME = None
FROM_CHECKPOINT = None


def _progress():
    """Log every finest-level V-cycle and every multigrid setup (one per
    Newton step) that the oracle's Newton loop runs."""
    vcycle, setup = ON.vcycle, ON.mg_setup
    count = {'v': 0, 's': 0}

    def vcycle_logged(problem, levels, l, b, opts, stats=None):
        count['v'] += 1
        _log(f'V-cycle {count["v"]}')
        return vcycle(problem, levels, l, b, opts, stats)

    def setup_logged(*a, **k):
        count['s'] += 1
        _log(f'setup {count["s"]} (Newton step)')
        return setup(*a, **k)
    ON.vcycle = vcycle_logged
    ON.mg_setup = setup_logged
NSAMPLE = 8192
SAMPLE_SEED = 2024


def _log(*a):
    print(time.strftime('%H:%M:%S'), *a, flush=True)


def _setup(name):
    w = W.WORKLOADS[name]
    pb = Problem(w['kind'], dict(zip(PARAMS[w['kind']], w['params'])))
    g = Grid(w['n'], w['h'], w['faces'])
    o = w['options']
    # FP64 multigrid settings of the configuration (the oracle has no FP32 levels)
    mo = MGOptions(nu_pre=o.get('nu_pre', 4), nu_post=o.get('nu_post', 4), coarse_rtol=1e-6)
    return w, pb, g, mo


def _nodes(count_total):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(count_total, NSAMPLE, replace=False))


def _solve(pb, g, L, b, m, mo, rtol, tag):
    rep = ON.Report()
    t = time.time()
    nc = pb.ncomp
    if FROM_CHECKPOINT:
        # the saved Newton iterate itself, with its residual from the oracle
        ck = np.load(FROM_CHECKPOINT)
        u = ck['u'].astype(np.float64)
        fn = float(np.linalg.norm(OP._mask(g, nc, OP.apply_A(pb, g, u, m) - b)))
        rep.fnorm = [float(ck['f0']), fn]
        rep.status = 'checkpoint'
        rep.newton_iters = rep.linear_iters = -1
        _log(f'{tag}: iterate of {FROM_CHECKPOINT}, |F|/|F0| = {fn / float(ck["f0"]):.3e}')
        return u, rep
    u0 = np.zeros(g.node_shape if nc == 1 else (nc,) + g.node_shape)
    # ||F(0)||, as the Newton solve computes it
    f0 = float(np.linalg.norm(OP._mask(g, nc, OP.apply_A(pb, g, u0, m) - b)))
    opts = ON.NewtonOptions(rtol=rtol, maxit=60)
    if RESUME:
        ck = np.load(RESUME)
        u0, f0 = ck['u'].astype(np.float64), float(ck['f0'])
        opts = ON.NewtonOptions(rtol=rtol, f0=f0, maxit=60)
        _log(f'{tag}: resuming from {RESUME} (||F(0)|| = {f0:.6e})')
    if CHECKPOINT:
        setup = ON.mg_setup

        def setup_saving(problem, grids, u, *a, **k):
            tmp = CHECKPOINT + '.tmp.npz'             # replaced in one step: a kill leaves the last one whole
            if CHECKPOINT_F32:
                np.savez_compressed(tmp, u=u.astype(np.float32), f0=f0)
            else:
                np.savez(tmp, u=u, f0=f0)
            os.replace(tmp, CHECKPOINT)
            _log(f'checkpoint written to {CHECKPOINT}')
            return setup(problem, grids, u, *a, **k)
        ON.mg_setup = setup_saving
    u, rep = ON.solve(pb, g, L, u0, b, m, mo, opts, rep)
    if RESUME:
        rep.fnorm[0] = f0                             # the target and the stored f0 refer to F(0)
    _log(f'{tag}: {rep.status}, {rep.newton_iters} Newton, {rep.linear_iters} Krylov, '
         f'|F|/|F0| = {rep.fnorm[-1] / rep.fnorm[0]:.3e}, {time.time() - t:.0f} s')
    if rep.status != 'ok':
        raise RuntimeError(f'{tag}: oracle solve failed ({rep.status})')
    return u, rep


def _gauss_load(w, g):
    c, wd, a = W.gaussian_params(w.get('load_seed', 1), 16, 3)
    return OP.load_from_function(g, OP.gaussian_source(c, wd, a))


def make(name):
    w, pb, g, mo = _setup(name)
    L = w['nlevels']
    out = {}
    if w['kind'] == 'plap':
        b = _gauss_load(w, g)
        u, rep = _solve(pb, g, L, b, None, mo, 1e-12, name)
        nodes = _nodes(g.n_nodes)
        out.update(nodes=nodes, u=u.reshape(-1)[nodes], u_norm=np.linalg.norm(u))
    elif w['kind'] == 'invcoef':
        b = _gauss_load(w, g)
        m = W.matern_field(w['n'], w['h'], w.get('m_seed', 3))
        m_obs = W.matern_field(w['n'], w['h'], w.get('obs_seed', 4))
        u, rep = _solve(pb, g, L, b, m, mo, 1e-12, name + ' at m')
        uo, _ = _solve(pb, g, L, b, m_obs, mo, 1e-12, name + ' at m_obs')
        t = time.time()
        grad, lam, its, ok = OA.gradient(pb, g, L, u, m, uo, mo, rtol=1e-12)
        _log(f'{name}: adjoint {its} Krylov, ok {ok}, {time.time() - t:.0f} s')
        if not ok:
            raise RuntimeError('adjoint solve failed')
        nodes = _nodes(g.n_nodes)
        out.update(nodes=nodes, u=u.reshape(-1)[nodes], u_norm=np.linalg.norm(u),
                   u_obs=uo.reshape(-1)[nodes], u_obs_norm=np.linalg.norm(uo),
                   lam=lam.reshape(-1)[nodes], lam_norm=np.linalg.norm(lam),
                   grad=grad.reshape(-1)[nodes], grad_norm=np.linalg.norm(grad),
                   misfit=OA.misfit(g, u, uo))
    elif w['kind'] == 'neohooke':
        # the first of the configuration's load increments
        t = W.traction(w.get('traction_seed', 2))
        b = (1.0 / w['load_steps']) * OP.traction_load(g, t)   # the first increment's load, as scaled by the solver
        u, rep = _solve(pb, g, L, b, None, mo, 1e-11, name + ' first increment')
        nodes = _nodes(3 * g.n_nodes)
        out.update(nodes=nodes, u=u.reshape(-1)[nodes], u_norm=np.linalg.norm(u),
                   load_fraction=1.0 / w['load_steps'])
    else:
        raise KeyError(name)
    out.update(f0=rep.fnorm[0], f=rep.fnorm[-1], newton=rep.newton_iters, krylov=rep.linear_iters)
    path = os.path.join(OUT, f'ref_{name}.npz')
    np.savez_compressed(path, **{k: np.asarray(v) for k, v in out.items()})
    _log(f'wrote {path}')


if __name__ == '__main__':
    args = sys.argv[1:]
    if '--out' in args:
        i = args.index('--out')
        OUT = args[i + 1]
        del args[i:i + 2]
    if '--progress' in args:
        args.remove('--progress')
        _progress()
    if '--from-checkpoint' in args:
        i = args.index('--from-checkpoint')
        FROM_CHECKPOINT = args[i + 1]
        del args[i:i + 2]
    if '--checkpoint-f32' in args:
        args.remove('--checkpoint-f32')
        CHECKPOINT_F32 = True
    for opt in ('--checkpoint', '--resume'):
        if opt in args:
            i = args.index(opt)
            if opt == '--checkpoint':
                CHECKPOINT = args[i + 1]
            else:
                RESUME = args[i + 1]
            del args[i:i + 2]
    for nm in args:
        make(nm)
