"""Thin Python binding of libjfnk (include/libjfnk.h).

Every function has the name of its C entry point and takes torch tensors
on the context's GPU; it checks dtype, device, contiguity and size, passes
the device pointers through, and raises RuntimeError with the library's
message on a non-zero status.  No arithmetic of the method happens here.
"""
import ctypes

import torch

from . import _lib
from ._lib import F32, F64

FACE_BITS = {(0, 0): 1, (0, 1): 2, (1, 0): 4, (1, 1): 8, (2, 0): 16, (2, 1): 32}


def faces_to_mask(faces):
    """Dirichlet faces as (axis, side) pairs -> JFNK_FACE_* bit mask."""
    m = 0
    for f in faces:
        m |= FACE_BITS[tuple(f)]
    return m


class JfnkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f'libjfnk {_lib.STATUS.get(status, status)}: {msg}')
        self.status = status


def default_options(**kw):
    lib = _lib.load()
    o = _lib.Options()
    lib.jfnk_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f'unknown option {k}')
        setattr(o, k, v)
    return o


def make_problem(kind, n, h, faces, params=(), nlevels=1):
    p = _lib.Problem()
    p.kind = _lib.KINDS[kind] if isinstance(kind, str) else int(kind)
    p.dim = len(n)
    for k in range(3):
        p.n[k] = int(n[k]) if k < len(n) else 0
    p.h = float(h)
    p.dirichlet = faces_to_mask(faces)
    for k in range(4):
        p.param[k] = float(params[k]) if k < len(params) else 0.0
    p.nlevels = int(nlevels)
    return p


class Context:
    """A libjfnk context on one GPU; owns its workspace tensor."""

    def __init__(self, problem, options=None, device='cuda'):
        self.lib = _lib.load()
        self.problem = problem
        self.options = options if options is not None else default_options()
        nbytes = ctypes.c_size_t()
        self._check(None, self.lib.jfnk_workspace_bytes(ctypes.byref(problem), ctypes.byref(self.options),
                                                         ctypes.byref(nbytes)))
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device('cuda', torch.cuda.current_device())
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        self._check(None, self.lib.jfnk_create(ctypes.byref(problem), ctypes.byref(self.options),
                                                ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                                ctypes.c_void_p(stream), ctypes.byref(h)))
        self.h = h
        self.nlevels = problem.nlevels
        self.ncomp = 3 if problem.kind == _lib.NEOHOOKE else 1
        self.dim = problem.dim
        self.vprec = self.options.vcycle_prec

    def _check(self, h, status):
        if status != _lib.OK:
            msg = self.lib.jfnk_last_error(h)
            raise JfnkError(status, msg.decode() if msg else '')

    def check(self, status):
        self._check(self.h, status)

    def close(self):
        if getattr(self, 'h', None):
            self.lib.jfnk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- shapes -----------------------------------------------------------
    def level_info(self, level):
        n = (ctypes.c_int * 3)()
        nn = ctypes.c_longlong()
        nd = ctypes.c_longlong()
        self.check(self.lib.jfnk_level_info(self.h, level, n, ctypes.byref(nn), ctypes.byref(nd)))
        return tuple(n), nn.value, nd.value

    def node_shape(self, level, comps=True):
        n, _, _ = self.level_info(level)
        sh = (n[1] + 1, n[0] + 1) if self.dim == 2 else (n[2] + 1, n[1] + 1, n[0] + 1)
        return ((self.ncomp,) + sh) if (comps and self.ncomp > 1) else sh

    def empty(self, level, dtype=torch.float64, comps=True):
        return torch.zeros(self.node_shape(level, comps), dtype=dtype, device=self.device)

    def level_dtype(self):
        return torch.float32 if self.vprec == F32 else torch.float64


def _ptr(t, ctx, level, dtype, comps=True, name='array'):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f'{name} must be a torch tensor')
    if t.device != ctx.device:
        raise ValueError(f'{name} is on {t.device}, context on {ctx.device}')
    if t.dtype != dtype:
        raise TypeError(f'{name} has dtype {t.dtype}, expected {dtype}')
    if not t.is_contiguous():
        raise ValueError(f'{name} must be contiguous')
    want = 1
    for s in ctx.node_shape(level, comps):
        want *= s
    if t.numel() != want:
        raise ValueError(f'{name} has {t.numel()} entries, level {level} needs {want}')
    return ctypes.c_void_p(t.data_ptr())


def _prec(dtype):
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError('arrays must be float32 or float64')


# ---- a1 -------------------------------------------------------------------------
def jfnk_residual(ctx, level, u, coef=None, b=None, F=None):
    dt = u.dtype
    F = ctx.empty(level, dt) if F is None else F
    ctx.check(ctx.lib.jfnk_residual(ctx.h, level, _prec(dt), _ptr(u, ctx, level, dt, name='u'),
                                    _ptr(coef, ctx, level, torch.float64, False, 'coef'),
                                    _ptr(b, ctx, level, dt, name='b'), _ptr(F, ctx, level, dt, name='F')))
    return F


def jfnk_residual_static(problem, level, u, b=None, F=None, fnorm2=None):
    """F = A_l(u) - b without a context (no allocation by the library); the
    arrays are FP64 tensors on the current GPU with the level's node layout,
    fnorm2 (optional) a one-element FP64 tensor that receives ||F||^2.  Runs
    on the current torch stream."""
    lib = _lib.load()
    n = [problem.n[k] >> (problem.nlevels - 1 - level) for k in range(problem.dim)]
    nc = 3 if problem.kind == _lib.NEOHOOKE else 1
    shape = tuple(k + 1 for k in reversed(n))
    shape = ((nc,) + shape) if nc > 1 else shape
    numel = 1
    for s in shape:
        numel *= s
    F = torch.empty(shape, dtype=torch.float64, device=u.device) if F is None else F
    for name, t, want in (('u', u, numel), ('b', b, numel), ('F', F, numel), ('fnorm2', fnorm2, 1)):
        if t is None:
            continue
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != want:
            raise ValueError(f'{name} must be a contiguous FP64 GPU tensor of {want} entries')
    stream = torch.cuda.current_stream(u.device).cuda_stream
    p = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
    st = lib.jfnk_residual_static(ctypes.byref(problem), int(level), p(u), p(b), p(F), p(fnorm2),
                                  ctypes.c_void_p(stream))
    if st != _lib.OK:
        msg = lib.jfnk_last_error(None)
        raise JfnkError(st, msg.decode() if msg else '')
    return F


def jfnk_energy(ctx, level, u, b=None):
    out = ctypes.c_double()
    ctx.check(ctx.lib.jfnk_energy(ctx.h, level, _ptr(u, ctx, level, torch.float64, name='u'),
                                  _ptr(b, ctx, level, torch.float64, name='b'), ctypes.byref(out)))
    return out.value


# ---- a5 -------------------------------------------------------------------------
def jfnk_jv(ctx, level, u, v, coef=None, Au=None, eps_override=0.0, Jv=None, want_eps=False):
    dt = u.dtype
    Jv = ctx.empty(level, dt) if Jv is None else Jv
    eps = ctypes.c_double()
    ctx.check(ctx.lib.jfnk_jv(ctx.h, level, _prec(dt), _ptr(u, ctx, level, dt, name='u'),
                              _ptr(coef, ctx, level, torch.float64, False, 'coef'),
                              _ptr(Au, ctx, level, dt, name='Au'), _ptr(v, ctx, level, dt, name='v'),
                              float(eps_override), _ptr(Jv, ctx, level, dt, name='Jv'),
                              ctypes.byref(eps) if want_eps else None))
    return (Jv, eps.value) if want_eps else Jv


# ---- a3, a7, a8 -------------------------------------------------------------------
def mg_project(ctx, level, xf, xc=None):
    dt = xf.dtype
    xc = ctx.empty(level - 1, dt) if xc is None else xc
    ctx.check(ctx.lib.mg_project(ctx.h, level, _prec(dt), _ptr(xf, ctx, level, dt), _ptr(xc, ctx, level - 1, dt)))
    return xc


def mg_restrict(ctx, level, rf, rc=None):
    dt = rf.dtype
    rc = ctx.empty(level - 1, dt) if rc is None else rc
    ctx.check(ctx.lib.mg_restrict(ctx.h, level, _prec(dt), _ptr(rf, ctx, level, dt), _ptr(rc, ctx, level - 1, dt)))
    return rc


def mg_prolong_add(ctx, level, cc, sf):
    dt = cc.dtype
    ctx.check(ctx.lib.mg_prolong_add(ctx.h, level, _prec(dt), _ptr(cc, ctx, level - 1, dt), _ptr(sf, ctx, level, dt)))
    return sf


# ---- a2-a4 -------------------------------------------------------------------------
def mg_setup(ctx, u, coef=None):
    L = ctx.nlevels - 1
    ctx.check(ctx.lib.mg_setup(ctx.h, _ptr(u, ctx, L, torch.float64, name='u'),
                               _ptr(coef, ctx, L, torch.float64, False, 'coef')))


def mg_reset_eigvecs(ctx):
    ctx.check(ctx.lib.mg_reset_eigvecs(ctx.h))


def mg_get_level(ctx, level, which):
    """which: 'x', 'Ax', 'eig' or 'kap' (e^m)."""
    k = {'x': 0, 'Ax': 1, 'eig': 2, 'kap': 3}[which]
    out = ctx.empty(level, ctx.level_dtype(), comps=(k != 3))
    ctx.check(ctx.lib.mg_get_level(ctx.h, level, k, ctypes.c_void_p(out.data_ptr())))
    torch.cuda.synchronize(ctx.device)
    return out


def mg_get_lambda(ctx):
    arr = (ctypes.c_double * ctx.nlevels)()
    ctx.check(ctx.lib.mg_get_lambda(ctx.h, arr))
    return list(arr)


# ---- a6, a9, a10 -----------------------------------------------------------------------
def mg_smooth(ctx, level, b, s, nu, s_is_zero=False):
    dt = ctx.level_dtype()
    ctx.check(ctx.lib.mg_smooth(ctx.h, level, _ptr(b, ctx, level, dt, name='b'), _ptr(s, ctx, level, dt, name='s'),
                                int(nu), int(bool(s_is_zero))))
    return s


def mg_coarse_solve(ctx, r0, s0=None):
    dt = ctx.level_dtype()
    s0 = ctx.empty(0, dt) if s0 is None else s0
    sh, it, rd = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
    ctx.check(ctx.lib.mg_coarse_solve(ctx.h, _ptr(r0, ctx, 0, dt, name='r0'), _ptr(s0, ctx, 0, dt, name='s0'),
                                      ctypes.byref(sh), ctypes.byref(it), ctypes.byref(rd)))
    return s0, sh.value, it.value, rd.value


def mg_vcycle(ctx, b, s=None):
    L = ctx.nlevels - 1
    s = ctx.empty(L, torch.float64) if s is None else s
    ctx.check(ctx.lib.mg_vcycle(ctx.h, _ptr(b, ctx, L, torch.float64, name='b'),
                                _ptr(s, ctx, L, torch.float64, name='s')))
    return s


# ---- a11, a12 -------------------------------------------------------------------------
def jfnk_solve(ctx, u, coef=None, b=None, raise_on_fail=False):
    """Solve F(u) = 0 in place from the given u; returns the report dict."""
    L = ctx.nlevels - 1
    rep = _lib.Report()
    st = ctx.lib.jfnk_solve(ctx.h, _ptr(u, ctx, L, torch.float64, name='u'),
                            _ptr(coef, ctx, L, torch.float64, False, 'coef'),
                            _ptr(b, ctx, L, torch.float64, name='b'), ctypes.byref(rep))
    d = rep.to_dict(ctx.nlevels)
    if st != _lib.OK:
        msg = ctx.lib.jfnk_last_error(ctx.h)
        d['error'] = msg.decode() if msg else ''
        if raise_on_fail or st in (_lib.E_INVAL, _lib.E_DEVICE):
            raise JfnkError(st, d['error'])
    return d


def jfnk_solve_steps(ctx, u, nsteps, coef=None, b=None, raise_on_fail=False):
    """Load stepping: solve with loads (k / nsteps) b, k = 1..nsteps, in place;
    returns the summed report dict (see jfnk_solve_steps in libjfnk.h)."""
    L = ctx.nlevels - 1
    rep = _lib.Report()
    st = ctx.lib.jfnk_solve_steps(ctx.h, _ptr(u, ctx, L, torch.float64, name='u'),
                                  _ptr(coef, ctx, L, torch.float64, False, 'coef'),
                                  _ptr(b, ctx, L, torch.float64, name='b'), int(nsteps), ctypes.byref(rep))
    d = rep.to_dict(ctx.nlevels)
    if st != _lib.OK:
        msg = ctx.lib.jfnk_last_error(ctx.h)
        d['error'] = msg.decode() if msg else ''
        if raise_on_fail or st in (_lib.E_INVAL, _lib.E_DEVICE):
            raise JfnkError(st, d['error'])
    return d


# ---- a13, a14, a15 ------------------------------------------------------------------------
def jfnk_vjp(ctx, level, wrt, u, lam, coef=None, out=None):
    out = ctx.empty(level, torch.float64, comps=(wrt == 0)) if out is None else out
    ctx.check(ctx.lib.jfnk_vjp(ctx.h, level, int(wrt), _ptr(u, ctx, level, torch.float64, name='u'),
                               _ptr(coef, ctx, level, torch.float64, False, 'coef'),
                               _ptr(lam, ctx, level, torch.float64, name='lam'),
                               _ptr(out, ctx, level, torch.float64, wrt == 0, 'out')))
    return out


def jfnk_adjoint_solve(ctx, u, rhs, coef=None, rtol=1e-10, lam=None, raise_on_fail=True):
    L = ctx.nlevels - 1
    lam = ctx.empty(L, torch.float64) if lam is None else lam
    rep = _lib.Report()
    st = ctx.lib.jfnk_adjoint_solve(ctx.h, _ptr(u, ctx, L, torch.float64, name='u'),
                                    _ptr(coef, ctx, L, torch.float64, False, 'coef'),
                                    _ptr(rhs, ctx, L, torch.float64, name='rhs'), float(rtol),
                                    _ptr(lam, ctx, L, torch.float64, name='lam'), ctypes.byref(rep))
    d = rep.to_dict(ctx.nlevels)
    if st != _lib.OK and raise_on_fail:
        msg = ctx.lib.jfnk_last_error(ctx.h)
        raise JfnkError(st, msg.decode() if msg else '')
    d['ok'] = st == _lib.OK
    return lam, d


def jfnk_coef_gradient(ctx, u, coef, lam, out=None):
    L = ctx.nlevels - 1
    out = ctx.empty(L, torch.float64, comps=False) if out is None else out
    ctx.check(ctx.lib.jfnk_coef_gradient(ctx.h, _ptr(u, ctx, L, torch.float64, name='u'),
                                         _ptr(coef, ctx, L, torch.float64, False, 'coef'),
                                         _ptr(lam, ctx, L, torch.float64, name='lam'),
                                         _ptr(out, ctx, L, torch.float64, False, 'out')))
    return out


# ---- loads and timers -----------------------------------------------------------------------
def jfnk_assemble_load(ctx, kind, params, b=None):
    L = ctx.nlevels - 1
    b = ctx.empty(L, torch.float64) if b is None else b
    arr = (ctypes.c_double * len(params))(*[float(p) for p in params])
    ctx.check(ctx.lib.jfnk_assemble_load(ctx.h, int(kind), arr, len(params), _ptr(b, ctx, L, torch.float64, name='b')))
    return b


def jfnk_stream_triad(a, b, c, s=0.5):
    """c = a + s b on FP64 GPU tensors of equal size (the HBM calibration
    sweep), on the current torch stream."""
    lib = _lib.load()
    for name, t in (('a', a), ('b', b), ('c', c)):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != a.numel():
            raise ValueError(f'{name} must be a contiguous FP64 GPU tensor of {a.numel()} entries')
    stream = torch.cuda.current_stream(a.device).cuda_stream
    st = lib.jfnk_stream_triad(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                               ctypes.c_void_p(c.data_ptr()), a.numel(), float(s), ctypes.c_void_p(stream))
    if st != _lib.OK:
        msg = lib.jfnk_last_error(None)
        raise JfnkError(st, msg.decode() if msg else '')
    return c


def jfnk_timer_enable(ctx, which, enable=True):
    ctx.check(ctx.lib.jfnk_timer_enable(ctx.h, int(which), int(bool(enable))))


def jfnk_timer_read(ctx, which):
    cnt = ctypes.c_longlong()
    ms = ctypes.c_double()
    ctx.check(ctx.lib.jfnk_timer_read(ctx.h, int(which), ctypes.byref(cnt), ctypes.byref(ms)))
    return cnt.value, ms.value


# ---- a15: differentiable solve ----------------------------------------------------------------
class JFNKSolve(torch.autograd.Function):
    """u = JFNKSolve.apply(coef, b, ctx, u0, adjoint_rtol): the root of
    F(u; coef) = A(u; coef) - b on the finest level (jfnk_solve from u0, or
    from 0).  Backward (implicit-function theorem): with J(u)^T lam = dL/du
    (jfnk_adjoint_solve, the multigrid of the converged u as preconditioner),
    dL/dcoef = -(dF/dcoef)^T lam (jfnk_vjp, wrt 1) and dL/db = lam.  coef is
    the INVCOEF field m (None for the other kinds); its gradient comes from
    jfnk_coef_gradient."""

    @staticmethod
    def forward(fctx, coef, b, ctx, u0=None, adjoint_rtol=1e-10):
        L = ctx.nlevels - 1
        u = ctx.empty(L, torch.float64).zero_() if u0 is None else u0.detach().clone()
        jfnk_solve(ctx, u, None if coef is None else coef.detach(), None if b is None else b.detach(),
                   raise_on_fail=True)
        fctx.jctx = ctx
        fctx.rtol = adjoint_rtol
        fctx.has_coef = coef is not None
        fctx.save_for_backward(u, coef.detach() if coef is not None else None)
        return u

    @staticmethod
    def backward(fctx, gu):
        ctx = fctx.jctx
        u, coef = fctx.saved_tensors
        lam, _ = jfnk_adjoint_solve(ctx, u, gu.contiguous().to(torch.float64), coef=coef, rtol=fctx.rtol)
        g_coef = None
        if fctx.has_coef and fctx.needs_input_grad[0]:
            g_coef = jfnk_coef_gradient(ctx, u, coef, lam)
        g_b = lam if fctx.needs_input_grad[1] else None
        return g_coef, g_b, None, None, None
