"""Seeded synthetic inputs and workload presets.

This module holds no arithmetic of the method: it draws random numbers,
builds boolean boundary masks and describes problem sizes.  Both the GPU
path and the CPU oracle take their inputs from here (as NumPy arrays), so
the two are compared on identical data.

Workloads (all synthetic; the paper uses analytic PDEs, no datasets):

* bratu2d-32      2D Bratu, lam = 5, unit square, 32 x 32 Q1, 3 levels,
                  Chebyshev degree 3, 10 power iterations, FP64
* plap3d-128      3D p-Laplacian p = 3, delta = 1e-2, unit cube, 128^3, 5
                  levels, f = sum of 16 seeded Gaussians (seed 1), FP64
* plap3d-256      the same on 256^3 (16.6M DoFs), 6 levels, degree 4,
                  FP32 V-cycle (FP64 for the comparison run)
* neohooke-256x64 Neo-Hookean beam [0,4] x [0,1]^2, 256 x 64 x 64, E = 1,
                  nu = 0.3, clamped at x = 0, seeded traction on x = 4
                  (seed 2) in 10 load steps, 5 levels, FP32 V-cycle
* invcoef3d-128   -div(e^m (1 + u^2) grad u) = f on 128^3, m a Matern-like
                  field (sigma 0.5, length 0.1, seed 3), u_obs from a second
                  field (seed 4), 5 levels
* bratu2d-800     the paper's Bratu experiment on Q1 elements: lam = 5, a
                  25 x 25 coarse mesh refined five times (800 x 800, 6
                  levels), solved with the paper's settings (PAPER_OPTIONS)
* beam3d-160x16x16 the paper's hyperelastic beam (0, 10) x (0, 1)^2: Neo-Hookean,
                  E = 10, nu = 0.3, clamped at x = 0, the rotational data
                  u_2 at x = 10, no load; the 10 x 1 x 1 coarse mesh refined
                  four times (5 levels); paper settings
* minsurf2d-800   the paper's minimal-surface experiment on the same
                  hierarchy: the p-Laplacian energy with p = 1, delta = 1 is
                  int sqrt(1 + |grad u|^2); u = 0 on x = 0, 1 and u = x(1 - x)
                  on y = 0, 1; paper settings
"""
import numpy as np

ALL2 = [(0, 0), (0, 1), (1, 0), (1, 1)]
ALL3 = [(a, s) for a in range(3) for s in range(2)]


def node_shape(n):
    """Node-array shape (z, y, x order) of a grid with n = (nx, ny[, nz]) elements."""
    return tuple(k + 1 for k in reversed(n))


def boundary_mask(n, faces):
    """Boolean mask of the nodes lying on the given (axis, side) faces."""
    m = np.zeros(node_shape(n), dtype=bool)
    d = len(n)
    for axis, side in faces:
        idx = [slice(None)] * d
        idx[d - 1 - axis] = 0 if side == 0 else n[axis]
        m[tuple(idx)] = True
    return m


# ---- random inputs ----------------------------------------------------------------
def gaussian_params(seed=1, count=16, dim=3):
    """Centres U[0.2, 0.8]^d, widths U[0.05, 0.15], amplitudes N(0, 1) (this draw order)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.2, 0.8, (count, dim))
    w = rng.uniform(0.05, 0.15, count)
    a = rng.normal(size=count)
    return c, w, a


def gaussian_param_array(c, w, a):
    """Flat (c_x, c_y[, c_z], w, a) per Gaussian, the layout of jfnk_assemble_load."""
    return np.concatenate([np.concatenate([c[k], [w[k], a[k]]]) for k in range(len(w))])


def traction(seed=2, tau=2e-3):
    """tau times a seeded unit vector."""
    rng = np.random.default_rng(seed)
    s = rng.normal(size=3)
    return tau * s / np.linalg.norm(s)


def matern_field(n, h, seed, sigma=0.5, ell=0.1, nu=1.0):
    """Gaussian random field on the nodes with a Matern-like spectrum.

    White noise is filtered in Fourier space by (ell^-2 + |k|^2)^(-(nu + d/2)/2)
    on a grid padded to twice the size (to weaken periodic wrap-around),
    cropped to the nodes, then shifted and scaled to mean 0, std sigma.
    """
    shape = node_shape(n)
    d = len(shape)
    pad = tuple(2 * s for s in shape)
    rng = np.random.default_rng(seed)
    noise = rng.normal(size=pad)
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(p, d=h) for p in pad], indexing='ij')
    k2 = sum(k * k for k in ks)
    filt = (ell ** -2 + k2) ** (-(nu + d / 2.0) / 2.0)
    f = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    f = f[tuple(slice(0, s) for s in shape)]
    f = f - f.mean()
    return sigma * f / f.std()


def rough_state(n, faces, seed, lo=-1.0, hi=1.0, ncomp=1):
    """Uniform values on the DoFs, 0 on Dirichlet nodes."""
    rng = np.random.default_rng(seed)
    shape = node_shape(n) if ncomp == 1 else (ncomp,) + node_shape(n)
    u = rng.uniform(lo, hi, shape)
    m = boundary_mask(n, faces)
    if ncomp == 1:
        u[m] = 0.0
    else:
        u[:, m] = 0.0
    return u


def normal_vector(n, faces, seed, ncomp=1):
    """N(0, 1) values on the DoFs, 0 on Dirichlet nodes."""
    rng = np.random.default_rng(seed)
    shape = node_shape(n) if ncomp == 1 else (ncomp,) + node_shape(n)
    v = rng.normal(size=shape)
    m = boundary_mask(n, faces)
    if ncomp == 1:
        v[m] = 0.0
    else:
        v[:, m] = 0.0
    return v


def dirichlet_state(w):
    """Start state of a preset: its Dirichlet data on the boundary nodes, 0 elsewhere.

    'minsurf': u = x(1 - x) on the faces y = 0 and y = 1, 0 on x = 0 and x = 1
    (Sec. 3, minimal surface); presets without boundary data start from 0.
    """
    n, h = w['n'], w['h']
    shape = node_shape(n)
    u = np.zeros(shape) if w['kind'] != 'neohooke' else np.zeros((3,) + shape)
    if w.get('dirichlet_data') == 'minsurf':
        x = np.arange(n[0] + 1) * h
        u[0, :] = x * (1.0 - x)
        u[-1, :] = x * (1.0 - x)
    if w.get('dirichlet_data') == 'rotation':
        # the end face x = n_x h of the beam (Sec. 3, hyperelasticity): half the
        # displacement of a pi/6 rotation of (y, z) about (1/2, 1/2)
        c, s = np.cos(np.pi / 6), np.sin(np.pi / 6)
        y = (np.arange(n[1] + 1) * h)[None, :]
        z = (np.arange(n[2] + 1) * h)[:, None]
        u[1, :, :, -1] = 0.5 * (0.5 + (y - 0.5) * c - (z - 0.5) * s - y)
        u[2, :, :, -1] = 0.5 * (0.5 + (y - 0.5) * s + (z - 0.5) * c - z)
    return u


# ---- presets --------------------------------------------------------------------------
# The paper's solver settings (Sec. 3, setup): CG-MG outer solver, V(5, 5)
# cycles, power method <= 30 iterations or 1e-2 change, the paper's FD step,
# coarse CG-QN with 20 pairs and shift gamma = 5 stopped at ||r|| <= 1e-12,
# forcing min(0.5, ||F||), stop at ||F|| <= 1e-6, FP64 levels.
PAPER_OPTIONS = dict(nu_pre=5, nu_post=5, power_maxit=30, power_rtol=1e-2, eps_mode=1, coarse_atol=1e-12,
                     coarse_rtol=0.0, coarse_qn=20, shift_gamma=5.0, outer_krylov=1, forcing=1,
                     newton_rtol=0.0, newton_atol=1e-6, vcycle_prec=0)

WORKLOADS = {
    'bratu2d-32': dict(kind='bratu', n=(32, 32), h=1 / 32, faces=ALL2, params=(5.0,), nlevels=3,
                       options=dict(nu_pre=3, nu_post=3, power_fixed=1, power_maxit=10, vcycle_prec=0,
                                    coarse_rtol=1e-6)),
    'plap3d-128': dict(kind='plap', n=(128, 128, 128), h=1 / 128, faces=ALL3, params=(3.0, 1e-2), nlevels=5,
                       load_seed=1, options=dict(nu_pre=4, nu_post=4, vcycle_prec=0, coarse_rtol=1e-6)),
    'plap3d-256': dict(kind='plap', n=(256, 256, 256), h=1 / 256, faces=ALL3, params=(3.0, 1e-2), nlevels=6,
                       load_seed=1, options=dict(nu_pre=4, nu_post=4, vcycle_prec=1, coarse_rtol=1e-3)),
    'neohooke-256x64': dict(kind='neohooke', n=(256, 64, 64), h=1 / 64, faces=[(0, 0)], params=(1.0, 0.3),
                            nlevels=5, traction_seed=2, load_steps=10,
                            options=dict(nu_pre=4, nu_post=4, vcycle_prec=1, coarse_rtol=1e-3)),
    'invcoef3d-128': dict(kind='invcoef', n=(128, 128, 128), h=1 / 128, faces=ALL3, params=(), nlevels=5,
                          load_seed=1, m_seed=3, obs_seed=4,
                          options=dict(nu_pre=4, nu_post=4, vcycle_prec=0, coarse_rtol=1e-6)),
    'bratu2d-800': dict(kind='bratu', n=(800, 800), h=1 / 800, faces=ALL2, params=(5.0,), nlevels=6,
                        options=dict(PAPER_OPTIONS)),
    'minsurf2d-800': dict(kind='plap', n=(800, 800), h=1 / 800, faces=ALL2, params=(1.0, 1.0), nlevels=6,
                          dirichlet_data='minsurf', options=dict(PAPER_OPTIONS)),
    'beam3d-160x16x16': dict(kind='neohooke', n=(160, 16, 16), h=1 / 16, faces=[(0, 0), (0, 1)],
                             params=(10.0, 0.3), nlevels=5, dirichlet_data='rotation',
                             options=dict(PAPER_OPTIONS)),
}


def scaled(name, n, nlevels=None, **over):
    """A preset with another grid size (same physics and options)."""
    w = dict(WORKLOADS[name])
    w['n'] = tuple(n)
    w['h'] = w['h'] * WORKLOADS[name]['n'][0] / n[0]
    if nlevels is not None:
        w['nlevels'] = nlevels
    opts = dict(w['options'])
    opts.update(over)
    w['options'] = opts
    return w
