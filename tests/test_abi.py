"""The C ABI without a GPU: every function include/libjfnk.h declares is
exported by libjfnk.so and bound by the Python layer, the ctypes mirrors
have the library's struct sizes, and the host-side entry points (defaults,
workspace sizing, argument validation) behave as documented."""
import ctypes
import os
import re

import pytest

from paper_2103_13890_amd import _lib, api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'libjfnk.h')


def _declared():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'^[a-z_ ]+[ *]+((?:jfnk|mg)_[a-z0-9_]+)\s*\(', text, flags=re.M)))


@pytest.fixture(scope='module')
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip('libjfnk.so is not built')
    return _lib.load()


def test_header_declares_the_path():
    names = _declared()
    for need in ('jfnk_residual', 'jfnk_jv', 'mg_setup', 'mg_project', 'mg_restrict', 'mg_prolong_add',
                 'mg_vcycle', 'jfnk_solve', 'jfnk_solve_steps', 'jfnk_vjp', 'jfnk_adjoint_solve'):
        assert need in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = _declared()
    assert names, 'no declarations parsed'
    for n in names:
        assert hasattr(lib, n), n           # dlsym succeeds
    assert sorted(_lib.EXPORTS) == names


def test_struct_sizes_match(lib):
    out = (ctypes.c_size_t * 3)()
    lib.jfnk_abi_sizes(out)
    assert list(out) == [ctypes.sizeof(_lib.Problem), ctypes.sizeof(_lib.Options), ctypes.sizeof(_lib.Report)]


def test_defaults(lib):
    o = _lib.Options()
    lib.jfnk_default_options(ctypes.byref(o))
    assert (o.nu_pre, o.nu_post, o.power_maxit, o.restart) == (4, 4, 30, 30)
    assert (o.cheb_lo, o.cheb_hi, o.power_rtol, o.shift_gamma) == (0.06, 1.2, 1e-2, 5.0)
    assert o.newton_rtol == 1e-8 and o.vcycle_prec == _lib.F64 and o.eps_mode == _lib.EPS_NORM
    assert lib.jfnk_version().decode().startswith('libjfnk')


def _bytes(lib, prob, opt):
    n = ctypes.c_size_t(0)
    st = lib.jfnk_workspace_bytes(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(n))
    return st, n.value


def test_workspace_and_validation(lib):
    opt = api.default_options(nu_pre=4)
    prob = api.make_problem('plap', (32, 32, 32), 1 / 32, [(a, s) for a in range(3) for s in range(2)], (3.0, 1e-2), 3)
    st, n = _bytes(lib, prob, opt)
    assert st == _lib.OK and n > 0
    # more levels or FP32 levels change the plan; the finest FP64 vectors dominate
    st32, n32 = _bytes(lib, prob, api.default_options(vcycle_prec=_lib.F32))
    assert st32 == _lib.OK and 0 < n32
    assert n >= 8 * 33 ** 3 * 10
    bad = [
        ('restart', dict(restart=32)),
        ('restart', dict(restart=0)),
        ('fd_form', dict(fd_form=3)),
        ('kernel_path', dict(kernel_path=5)),
        ('cheb', dict(cheb_lo=1.5)),
        ('armijo', dict(armijo=1.0)),
        ('armijo', dict(armijo=0.0)),
    ]
    for what, over in bad:
        st, _ = _bytes(lib, prob, api.default_options(**over))
        assert st == _lib.E_INVAL, what
        assert lib.jfnk_last_error(None)
    # element counts not divisible by 2^(nlevels-1)
    p2 = api.make_problem('plap', (30, 32, 32), 1 / 32, [], (3.0, 1e-2), 3)
    assert _bytes(lib, p2, opt)[0] == _lib.E_INVAL
    # the coarsest grid must fit the one-workgroup coarse solver
    p3 = api.make_problem('plap', (64, 64, 64), 1 / 64, [], (3.0, 1e-2), 1)
    assert _bytes(lib, p3, opt)[0] == _lib.E_INVAL
    # Neo-Hookean needs a valid Poisson ratio and 3D
    p4 = api.make_problem('neohooke', (16, 4, 4), 1 / 4, [(0, 0)], (1.0, 0.5), 2)
    assert _bytes(lib, p4, opt)[0] == _lib.E_INVAL
    p5 = api.make_problem('neohooke', (16, 4), 1 / 4, [(0, 0)], (1.0, 0.3), 2)
    assert _bytes(lib, p5, opt)[0] == _lib.E_INVAL


def test_null_arguments_rejected(lib):
    assert lib.jfnk_workspace_bytes(None, None, None) == _lib.E_INVAL
    # a null context is rejected by every entry point before any device work
    assert lib.jfnk_residual(None, 0, 0, None, None, None, None) == _lib.E_INVAL
    assert lib.jfnk_solve(None, None, None, None, None) == _lib.E_INVAL
    assert lib.jfnk_solve_steps(None, None, None, None, 1, None) == _lib.E_INVAL
    assert lib.mg_vcycle(None, None, None) == _lib.E_INVAL
