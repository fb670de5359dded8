"""Pins of the oracle's flexible GMRES and preconditioned CG against dense
linear algebra; CG also against its finite termination on an SPD system."""
import numpy as np

from oracle.krylov import fgmres, pcg


def _system(n, seed):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) / np.sqrt(n)
    b = rng.normal(size=n)
    return A, b


def test_fgmres_matches_dense_solve():
    A, b = _system(60, 0)
    D = np.diag(A)
    x, its, est, ok = fgmres(lambda v: A @ v, b, lambda v: v / D, 1e-12 * np.linalg.norm(b))
    assert ok
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)
    assert abs(np.linalg.norm(b - A @ x) - est) < 1e-10 * np.linalg.norm(b)


def test_fgmres_restarts_and_variable_preconditioner():
    A, b = _system(80, 1)
    count = [0]

    def M(v):        # a preconditioner that changes every call (flexible variant needed)
        count[0] += 1
        return v * (1.0 + 0.1 * np.sin(count[0])) / np.diag(A)
    x, its, est, ok = fgmres(lambda v: A @ v, b, M, 1e-11 * np.linalg.norm(b), restart=5)
    assert ok and its > 5
    assert np.linalg.norm(b - A @ x) <= 1.01e-11 * np.linalg.norm(b) + 1e-15


def test_fgmres_happy_breakdown():
    A = np.diag([1.0, 2.0, 3.0])
    b = np.array([1.0, 0.0, 0.0])
    x, its, est, ok = fgmres(lambda v: A @ v, b, lambda v: v, 1e-14)
    assert ok and its == 1 and np.allclose(x, [1, 0, 0])


def test_fgmres_zero_rhs():
    x, its, est, ok = fgmres(lambda v: v, np.zeros(5), lambda v: v, 0.0)
    assert ok and its == 0 and not np.any(x)


def _spd(n, seed, cond):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T, rng.normal(size=n)


def test_pcg_matches_dense_solve():
    A, b = _spd(50, 2, 1e3)
    D = np.diag(A)
    x, its, rn, ok = pcg(lambda v: A @ v, b, lambda v: v / D, 1e-12 * np.linalg.norm(b), 500)
    assert ok
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) < 1e-9 * np.linalg.norm(ref)
    # the recursive residual tracks the true one
    assert abs(np.linalg.norm(b - A @ x) - rn) < 1e-10 * np.linalg.norm(b)


def test_pcg_finite_termination_and_exact_preconditioner():
    # 6 distinct eigenvalues: unpreconditioned CG ends in at most 6 steps
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    A = (Q * np.repeat([1.0, 2.0, 3.0, 5.0, 8.0, 13.0], 5)) @ Q.T
    b = rng.normal(size=30)
    x, its, rn, ok = pcg(lambda v: A @ v, b, lambda v: v, 1e-10 * np.linalg.norm(b), 100)
    assert ok and its <= 6
    x, its, rn, ok = pcg(lambda v: A @ v, b, lambda v: np.linalg.solve(A, v), 1e-10 * np.linalg.norm(b), 100)
    assert ok and its == 1


def test_pcg_negative_curvature_stop():
    A = np.diag([2.0, -1.0, 3.0])
    b = np.array([0.0, 1.0, 0.0])
    x, its, rn, ok = pcg(lambda v: A @ v, b, lambda v: v, 1e-12, 10)
    assert not ok and its == 1 and np.array_equal(x, b)     # the first direction itself
