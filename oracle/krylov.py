"""Flexible GMRES(m) (oracle; test infrastructure).

The outer Krylov solver of the Newton step.  The paper uses CG with the
multigrid preconditioner (Sec. 3, setup); the finite-difference V-cycle is
a variable preconditioner, so this implementation uses right-preconditioned
flexible GMRES (Saad, SIAM J. Sci. Comput. 14, 1993) with restart m = 30:

    r = b - A x,  v_1 = r / ||r||
    z_j = M(v_j),  w = A z_j
    two passes of classical Gram-Schmidt against v_1..v_j (CGS2)
    Givens rotations on the Hessenberg matrix; |g_{j+1}| is ||b - A x_j||
    x = x + Z y after the cycle, restart while the estimate exceeds tol.

The paper's own outer solver, CG with the multigrid preconditioner
(Sec. 3, setup), is ``pcg``: preconditioned conjugate gradients in the
Hestenes-Stiefel form from x = 0, stopped when the recursive residual
reaches tol, or at a direction of non-positive curvature.

Pins: on small dense systems the result matches numpy.linalg.solve, and
the estimate matches the true residual; PCG with the identity is plain CG,
with the exact inverse it takes one step (tests/test_oracle_krylov.py).
"""
import numpy as np


def _dot(a, b):
    return float(np.sum(a * b))


def fgmres(A, b, M, tol, restart=30, max_cycles=50, x0=None):
    """Solve A x = b to ||b - A x|| <= tol.  Returns (x, iterations, resid_est, ok)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    total = 0
    est = np.inf
    for cycle in range(max_cycles):
        r = b - A(x) if (cycle > 0 or x0 is not None) else b.copy()
        beta = np.sqrt(_dot(r, r))
        est = beta
        if beta <= tol:
            return x, total, est, True
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            w = A(z)
            total += 1
            h = np.array([_dot(v, w) for v in V])
            w = w - sum(hi * v for hi, v in zip(h, V))
            h2 = np.array([_dot(v, w) for v in V])
            w = w - sum(hi * v for hi, v in zip(h2, V))
            H[: j + 1, j] = h + h2
            H[j + 1, j] = np.sqrt(_dot(w, w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V.append(w / H[j + 1, j])
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rad = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / rad, H[j + 1, j] / rad
            H[j, j] = rad
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            est = abs(g[j + 1])
            if est <= tol or breakdown:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + sum(yi * z for yi, z in zip(y, Z))
        if est <= tol:
            return x, total, est, True
    return x, total, est, False


def pcg(A, b, M, tol, maxit):
    """Preconditioned CG on A x = b from x = 0 to ||r|| <= tol (recursive
    residual), M(r) the preconditioner.  Returns (x, iterations, ||r||, ok);
    ok is False at non-positive curvature p^T A p <= 0 or after maxit steps
    (x is then the last iterate; at non-positive curvature on the first
    direction it is that direction, the preconditioned residual M(b))."""
    x = np.zeros_like(b)
    r = b.copy()
    rn = np.sqrt(_dot(r, r))
    if rn <= tol:
        return x, 0, rn, True
    z = M(r)
    p = z.copy()
    rz = _dot(r, z)
    for it in range(1, maxit + 1):
        q = A(p)
        pq = _dot(p, q)
        if pq <= 0.0:
            # truncated Newton-CG (Nocedal and Wright, Alg. 7.1): a first
            # direction of non-positive curvature is returned itself
            return (p.copy() if it == 1 else x), it, rn, False
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rn = np.sqrt(_dot(r, r))
        if rn <= tol:
            return x, it, rn, True
        z = M(r)
        rz_new = _dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, rn, False
