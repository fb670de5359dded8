"""Structured Q1 finite-element grids (oracle; test infrastructure only).

The paper discretises with first-order finite elements (Sec. 3, "discretize
then optimize") on nested meshes {T_l} (Sec. 2).  Here every level is a
uniform box grid of n_x x n_y (x n_z) square/cubic elements of edge h,
nodes stored as a C-order array of shape (n_z+1, n_y+1, n_x+1): x varies
fastest.  Vector fields carry a leading component axis.

Element corners are numbered a = a_x + 2 a_y + 4 a_z with a_k in {0, 1}.
The Q1 basis on the reference cell [0,1]^d is the tensor product of
phi_0(t) = 1 - t and phi_1(t) = t.

Pins: the assembled stiffness matches the closed-form Q1 stencils and the
sine-mode eigenvalues (tests/test_oracle_fe.py).
"""
import itertools

import numpy as np

# Two-point Gauss rule on [0, 1]: nodes 1/2 -+ 1/(2 sqrt 3), weights 1/2.
GAUSS_T = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
GAUSS_W = (0.5, 0.5)


def _phi1(a, t):
    return 1.0 - t if a == 0 else t


def _dphi1(a):
    return -1.0 if a == 0 else 1.0


def corners(dim):
    """Corner bit tuples (a_x, a_y, a_z) in local order a = sum a_k 2^k."""
    return [tuple((a >> k) & 1 for k in range(dim)) for a in range(2 ** dim)]


def reference_rule(dim, points=None):
    """Q1 basis values and reference gradients at quadrature points.

    Returns (phi[q, a], dphi[q, a, k], w[q], xi[q, k]) on [0,1]^dim; the
    weights sum to 1.  Default points: the 2^dim tensor Gauss points.
    """
    if points is None:
        pts = list(itertools.product(range(2), repeat=dim))
        xi = np.array([[GAUSS_T[p[k]] for k in range(dim)] for p in pts])
        w = np.array([np.prod([GAUSS_W[p[k]] for k in range(dim)]) for p in pts])
    else:
        xi = np.atleast_2d(np.asarray(points, dtype=float))
        w = np.full(len(xi), np.nan)
    cs = corners(dim)
    nq = len(xi)
    phi = np.zeros((nq, len(cs)))
    dphi = np.zeros((nq, len(cs), dim))
    for q in range(nq):
        for a, bits in enumerate(cs):
            vals = [_phi1(bits[k], xi[q, k]) for k in range(dim)]
            phi[q, a] = np.prod(vals)
            for k in range(dim):
                g = _dphi1(bits[k])
                for j in range(dim):
                    if j != k:
                        g *= vals[j]
                dphi[q, a, k] = g
    return phi, dphi, w, xi


def element_stiffness(dim, h):
    """K_e[a, b] = int_e grad phi_a . grad phi_b on a cube of edge h.

    Integrated with the 2^d Gauss rule, which is exact for Q1 products.
    """
    _, dphi, w, _ = reference_rule(dim)
    # physical gradient = dphi / h, physical weight = w h^d
    return np.einsum('q,qak,qbk->ab', w, dphi, dphi) * h ** (dim - 2)


def element_mass(dim, h):
    """M_e[a, b] = int_e phi_a phi_b (exact with the 2^d Gauss rule)."""
    phi, _, w, _ = reference_rule(dim)
    return np.einsum('q,qa,qb->ab', w, phi, phi) * h ** dim


class Grid:
    """A uniform structured grid with Dirichlet data on selected faces.

    n: elements per axis (x, y[, z]); h: element edge; dirichlet: iterable
    of (axis, side) with side 0 for the low face and 1 for the high face.
    """

    def __init__(self, n, h, dirichlet):
        self.n = tuple(int(k) for k in n)
        self.dim = len(self.n)
        self.h = float(h)
        self.dirichlet = tuple(sorted(set((int(a), int(s)) for a, s in dirichlet)))
        self.node_shape = tuple(k + 1 for k in reversed(self.n))
        self.elem_shape = tuple(reversed(self.n))

    # ---- geometry -------------------------------------------------------
    def coarsen(self):
        if any(k % 2 for k in self.n):
            raise ValueError('grid with an odd element count cannot be coarsened')
        return Grid([k // 2 for k in self.n], 2.0 * self.h, self.dirichlet)

    def node_coords(self):
        """Coordinate arrays (x, y[, z]) of every node, each of node_shape."""
        axes = [np.arange(k + 1) * self.h for k in self.n]
        mesh = np.meshgrid(*reversed(axes), indexing='ij')
        return tuple(reversed(mesh))

    def elem_origins(self):
        axes = [np.arange(k) * self.h for k in self.n]
        mesh = np.meshgrid(*reversed(axes), indexing='ij')
        return tuple(reversed(mesh))

    @property
    def n_nodes(self):
        return int(np.prod(self.node_shape))

    # ---- boundary -------------------------------------------------------
    def dirichlet_mask(self):
        m = np.zeros(self.node_shape, dtype=bool)
        for axis, side in self.dirichlet:
            idx = [slice(None)] * self.dim
            idx[self.dim - 1 - axis] = 0 if side == 0 else self.n[axis]
            m[tuple(idx)] = True
        return m

    def dof_mask(self):
        return ~self.dirichlet_mask()

    def n_dof(self, ncomp=1):
        return int(self.dof_mask().sum()) * ncomp

    # ---- element gather / scatter ---------------------------------------
    def corner_slices(self):
        out = []
        for bits in corners(self.dim):
            sl = [slice(bits[k], bits[k] + self.n[k]) for k in range(self.dim)]
            out.append(tuple(reversed(sl)))
        return out

    def gather(self, u):
        """Corner values per element: shape (2^d,) + elem_shape (scalar u)
        or (ncomp, 2^d) + elem_shape (u with a leading component axis)."""
        lead = u.shape[: u.ndim - self.dim]
        pre = tuple(slice(None) for _ in lead)
        return np.stack([u[pre + s] for s in self.corner_slices()], axis=len(lead))

    def scatter(self, re, ncomp_axes=0):
        """Sum element corner vectors into nodes (inverse layout of gather)."""
        lead = re.shape[:ncomp_axes]
        out = np.zeros(lead + self.node_shape)
        pre = tuple(slice(None) for _ in lead)
        for a, s in enumerate(self.corner_slices()):
            out[pre + s] += re[pre + (a,)]
        return out

    def quad_points(self, xi):
        """Physical coordinates of reference point xi in every element."""
        org = self.elem_origins()
        return tuple(org[k] + self.h * xi[k] for k in range(self.dim))
