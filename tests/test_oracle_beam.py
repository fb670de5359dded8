"""The paper's hyperelastic beam in the oracle (Sec. 3, hyperelasticity;
Table 3).

* Frame indifference: a rigid rotation (here 60 degrees about the x axis)
  plus a translation has deformation gradient R, so C = I, J = 1, the
  Neo-Hookean energy is 0 and the first Piola stress mu (R - R^-T) +
  lam ln(J) R^-T vanishes: Psi_h = 0 and F = 0 at every node, whatever the
  rotation angle.  A linearised strain or a sign slip in the stress fails
  this at large angles.
* The rotational Dirichlet data: on the face x = 10 the preset holds half
  the displacement of a pi/6 rotation of (y, z) about (1/2, 1/2), computed
  here with a rotation matrix; 0 on x = 0 and inside.
* The preset is the paper's beam: (0, 10) x (0, 1)^2, E = 10, nu = 0.3,
  the 10 x 1 x 1 coarse mesh refined four times.
* L1 with the paper's settings (CG-MG, shifted coarse CG): converges to
  ||F|| <= 1e-6 with the boundary data kept, and the coarse solver meets
  negative curvature and shifts (the non-convexity Table 3 is about).
"""
import numpy as np
import pytest

from oracle import newton as ON
from oracle.fe import Grid
from oracle.mg import MGOptions
from oracle.problems import Problem, apply_A, energy
from paper_2103_13890_amd import workloads as W

BEAM = Problem('neohooke', {'E': 10.0, 'nu': 0.3})


def test_rigid_rotation_is_stress_free():
    g = Grid([6, 3, 3], 1.0 / 3, [(0, 0)])
    X = np.stack(g.node_coords())                  # (3, nz+1, ny+1, nx+1), x first
    t = np.pi / 3
    R = np.array([[1, 0, 0], [0, np.cos(t), -np.sin(t)], [0, np.sin(t), np.cos(t)]])
    c = np.array([0.0, 0.5, 0.5])[:, None, None, None]
    u = np.einsum('ij,j...->i...', R - np.eye(3), X - c) + np.array([0.3, -0.2, 0.1])[:, None, None, None]
    zero = np.zeros_like(u)
    assert abs(energy(BEAM, g, u, zero)) < 1e-12
    assert np.max(np.abs(apply_A(BEAM, g, u))) < 1e-12
    # a stretch is not stress-free
    assert np.max(np.abs(apply_A(BEAM, g, 0.05 * X))) > 1e-3


def test_rotational_dirichlet_data():
    w = W.scaled('beam3d-160x16x16', (20, 2, 2), nlevels=2)
    u = W.dirichlet_state(w)
    g = Grid(w['n'], w['h'], w['faces'])
    assert u.shape == (3,) + g.node_shape
    t = np.pi / 6
    R = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    for iz in range(3):
        for iy in range(3):
            yz = np.array([iy * w['h'], iz * w['h']])
            ref = 0.5 * (R @ (yz - 0.5) + 0.5 - yz)
            assert u[0, iz, iy, -1] == 0.0
            assert np.allclose(u[1:, iz, iy, -1], ref, rtol=0, atol=1e-15)
    assert not np.any(u[:, :, :, :-1])


def test_beam_preset_is_the_papers():
    w = W.WORKLOADS['beam3d-160x16x16']
    assert w['kind'] == 'neohooke' and w['params'] == (10.0, 0.3)
    assert [k * w['h'] for k in w['n']] == [10.0, 1.0, 1.0]
    assert [k >> (w['nlevels'] - 1) for k in w['n']] == [10, 1, 1]
    assert sorted(w['faces']) == [(0, 0), (0, 1)]


@pytest.mark.slow
def test_beam_l1_paper_settings():
    w = W.scaled('beam3d-160x16x16', (20, 2, 2), nlevels=2)
    g = Grid(w['n'], w['h'], w['faces'])
    u0 = W.dirichlet_state(w)
    mo = MGOptions(nu_pre=5, nu_post=5, eps_mode='paper', coarse_atol=1e-12, coarse_rtol=0.0, shift_gamma=5.0)
    u, rep = ON.solve(BEAM, g, 2, u0, np.zeros_like(u0), None, mo,
                      ON.NewtonOptions(rtol=0.0, atol=1e-6, forcing='paper', outer='cg'))
    assert rep.status == 'ok' and rep.fnorm[-1] <= 1e-6
    m = g.dirichlet_mask()
    assert np.array_equal(u[:, m], u0[:, m])
    assert rep.stats.neg_curv > 0 and min(rep.stats.shifts) < 0
    assert 3 <= rep.newton_iters <= 12
