"""Parity at the full 256^3 benchmark size (16,974,593 nodes), in the launch
configuration the benchmark times (automatic kernel choice: the row-tiled
kernels), on 4096 seeded sample nodes the oracle evaluates one by one.

Tolerances (max abs difference over the samples, relative to the largest
sampled magnitude): F(u) FP64 1e-12; FD Jacobian action at a test step
eps = 1e-2 (1 + ||u||) / ||v|| in FP64 1e-10 (both the plain quotient and
the element difference form); the FP32 difference form 1e-4."""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from _common import make_ctx, oracle_grid, oracle_problem, to_dev
from oracle import problems as OP
from paper_2103_13890_amd import api
from paper_2103_13890_amd import workloads as W

NSAMP = 4096


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope='module')
def data():
    w = W.WORKLOADS['plap3d-256']
    g = oracle_grid(w)
    u = 0.3 * W.rough_state(w['n'], w['faces'], 7)
    v = W.normal_vector(w['n'], w['faces'], 8)
    b = 0.1 * W.normal_vector(w['n'], w['faces'], 9)
    nodes = np.random.default_rng(10).choice(g.n_nodes, NSAMP, replace=False)
    eps = 1e-2 * (1 + np.linalg.norm(u)) / np.linalg.norm(v)
    pb = oracle_problem(w)
    zero = np.zeros_like(u)
    A0 = OP.residual_at(pb, g, u, zero, nodes)
    A1 = OP.residual_at(pb, g, u + eps * v, zero, nodes)
    return dict(w=w, u=u, v=v, b=b, nodes=nodes, eps=eps, F=OP.residual_at(pb, g, u, b, nodes),
                Jv=(A1 - A0) / eps)


@pytest.mark.parametrize('form', [1, 2])
def test_fullsize_residual_and_jv(data, form):
    w = data['w']
    ctx = make_ctx(w, fd_form=form, vcycle_prec=1, coarse_rtol=1e-3)
    L = ctx.nlevels - 1
    nodes = data['nodes']
    u, v = to_dev(data['u']), to_dev(data['v'])
    F = api.jfnk_residual(ctx, L, u, None, to_dev(data['b']))
    assert _maxrel(F.reshape(-1)[nodes].cpu().numpy(), data['F']) < 1e-12
    Jv = api.jfnk_jv(ctx, L, u, v, eps_override=data['eps'])
    assert _maxrel(Jv.reshape(-1)[nodes].cpu().numpy(), data['Jv']) < 1e-10
    if form == 2:
        Jv32 = api.jfnk_jv(ctx, L, u.float(), v.float(), eps_override=data['eps'])
        assert _maxrel(Jv32.reshape(-1)[nodes].double().cpu().numpy(), data['Jv']) < 1e-4
    del ctx
    torch.cuda.empty_cache()


def test_residual_beyond_tiled_limit():
    """A grid past the tiled kernel's limit of 2^28 nodes per array
    (512 x 768 x 704 elements: 278 M nodes, 2.2 GB per FP64 array), where F(u)
    runs on the node kernel with 64-bit node indices; through the entry point
    that needs no context (the workspace of a context this size is tens of
    GB).  F at 4096 seeded nodes against the oracle (1e-12), ||F||^2 against
    the sum of squares of F (1e-12)."""
    n = (512, 768, 704)
    w = W.scaled('plap3d-256', n, nlevels=7)       # coarsest 8 x 12 x 11
    p = api.make_problem(w['kind'], w['n'], w['h'], w['faces'], w['params'], w['nlevels'])
    shape = (n[2] + 1, n[1] + 1, n[0] + 1)
    nn = shape[0] * shape[1] * shape[2]
    assert nn >= 1 << 28
    print(f'{nn} nodes', flush=True)
    gen = torch.Generator(device='cuda').manual_seed(600)
    u = 0.6 * (torch.rand(shape, dtype=torch.float64, device='cuda', generator=gen) - 0.5)
    b = 0.1 * torch.randn(shape, dtype=torch.float64, device='cuda', generator=gen)
    n2 = torch.zeros(1, dtype=torch.float64, device='cuda')
    F = api.jfnk_residual_static(p, w['nlevels'] - 1, u, b, None, n2)
    nodes = np.random.default_rng(601).choice(nn, NSAMP, replace=False)
    Fs = F.reshape(-1)[torch.from_numpy(nodes).cuda()].cpu().numpy()
    s2 = float((F * F).sum())
    un, bn = u.cpu().numpy(), b.cpu().numpy()
    del u, b, F
    torch.cuda.empty_cache()
    Fo = OP.residual_at(oracle_problem(w), oracle_grid(w), un, bn, nodes)
    e = _maxrel(Fs, Fo)
    print(f'278M-node F(u): max relative difference {e:.2e} at {NSAMP} nodes', flush=True)
    assert e < 1e-12
    assert abs(float(n2[0]) - s2) <= 1e-12 * s2
