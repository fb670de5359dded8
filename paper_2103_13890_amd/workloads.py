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


# ---- presets --------------------------------------------------------------------------
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
