"""Transfer operators between nested grids (oracle; test infrastructure).

Sec. 2 (transfer operators): the interpolation I maps a coarse correction
to the next finer level, the restriction is R = I^T, and the Newton
iterate is carried to the coarse level by the projection P = 2^-d I^T,
whose scaling keeps constant functions constant.

Here I is multilinear interpolation on nested Q1 grids, built as the
Kronecker product of 1D interpolation matrices over all nodes (boundary
included).  Readings where the paper is silent:

* R: I^T r, then zero at coarse Dirichlet nodes (Dirichlet rows of the
  coarse system vanish).
* P at coarse nodes off Dirichlet faces: (I^T x)_i / (I^T 1)_i.  At coarse
  interior nodes (I^T 1)_i = 2^d exactly, so this is the paper's
  2^-d I^T; at nodes on natural-boundary faces it is the same operator
  normalised so that constants are still preserved, which is the property
  the paper states for its scaling.
* P at coarse Dirichlet nodes: the fine value at the coincident node, so
  the boundary data are carried exactly.

Pins: I reproduces multilinear functions exactly; I^T K_fine I equals the
coarse Q1 stiffness; P maps constants to constants
(tests/test_oracle_transfer.py).
"""
import numpy as np
import scipy.sparse as sp


def interp_1d(n_coarse):
    """(2 n_c + 1) x (n_c + 1) linear interpolation between nested 1D grids."""
    rows, cols, vals = [], [], []
    for i in range(n_coarse + 1):
        rows.append(2 * i)
        cols.append(i)
        vals.append(1.0)
    for i in range(n_coarse):
        rows += [2 * i + 1, 2 * i + 1]
        cols += [i, i + 1]
        vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * n_coarse + 1, n_coarse + 1))


def interpolation(coarse):
    """Sparse I acting on C-order flattened node arrays (x fastest)."""
    mats = [interp_1d(k) for k in coarse.n]       # x, y, z
    out = mats[0]
    for M in mats[1:]:
        out = sp.kron(M, out, format='csr')       # slower axes on the left
    return out


def _apply(M, v, in_shape, out_shape):
    if v.ndim == len(in_shape):
        return (M @ v.reshape(-1)).reshape(out_shape)
    return np.stack([(M @ c.reshape(-1)).reshape(out_shape) for c in v])


def prolong(coarse, fine, c):
    """I c (corrections vanish on Dirichlet nodes, so the result does too)."""
    out = _apply(interpolation(coarse), c, coarse.node_shape, fine.node_shape)
    m = fine.dirichlet_mask()
    if out.ndim == fine.dim:
        out[m] = 0.0
    else:
        out[:, m] = 0.0
    return out


def restrict(coarse, fine, r):
    """R r = I^T r, zero at coarse Dirichlet nodes."""
    out = _apply(interpolation(coarse).T.tocsr(), r, fine.node_shape, coarse.node_shape)
    m = coarse.dirichlet_mask()
    if out.ndim == coarse.dim:
        out[m] = 0.0
    else:
        out[:, m] = 0.0
    return out


def project(coarse, fine, x):
    """P x: normalised I^T x off Dirichlet faces, injection on them."""
    IT = interpolation(coarse).T.tocsr()
    wsum = (IT @ np.ones(fine.n_nodes)).reshape(coarse.node_shape)
    inj = tuple(slice(0, None, 2) for _ in range(fine.dim))
    m = coarse.dirichlet_mask()

    def one(xc):
        out = (IT @ xc.reshape(-1)).reshape(coarse.node_shape) / wsum
        out[m] = xc[inj][m]
        return out
    if x.ndim == fine.dim:
        return one(x)
    return np.stack([one(c) for c in x])
