"""Pins of the particle oracle (Section 2.3) against the paper's printed
settling times, the fixed point of the scheme, the defining implicit-Euler
equation and closed forms of the interpolation."""
import os

import numpy as np

from oracle import particles as P

NU, RHO_P, RHO_F, G = 1.6e-5, 1000.0, 1.225, 9.81
HERE = os.path.dirname(os.path.abspath(__file__))


def test_settling_times_match_paper():
    rows = np.loadtxt(os.path.join(HERE, "golden", "particle_settling.txt"))
    for diam, minutes in rows:
        v = P.terminal_speed(diam, NU, RHO_P, RHO_F, G)
        t_s = 1.5 / v / 60.0
        # the paper prints whole minutes
        assert abs(t_s - minutes) <= 0.5, (diam, t_s, minutes)


def test_small_particle_terminal_speed_is_g_tau():
    d = 2e-6
    v = P.terminal_speed(d, NU, RHO_P, RHO_F, G)
    tp = RHO_P * d * d / (18 * RHO_F * NU)
    assert abs(v / (G * tp) - 1) < 1e-3


def still_air(n=(8, 6, 4)):
    nx, ny, nz = n
    return [np.zeros((nz, ny, nx)) for _ in range(3)], (0.1, 0.1, 0.1), (nx * 0.1, ny * 0.1, nz * 0.1)


def test_fixed_point_is_terminal_velocity():
    """In still air the implicit-Euler iteration settles exactly on v = g tau_p / C_d(v)."""
    u, d, box = still_air()
    diam = np.array([5e-6, 10e-6, 30e-6])
    pos = np.tile(np.array([[0.3], [0.2], [0.25]]), (1, 3))
    vel = np.zeros((3, 3))
    for _ in range(400):
        pos, vel = P.step(pos, vel, diam, u, d, box, NU, RHO_P, RHO_F, (0, 0, -G), 0.01)
    for q in range(3):
        v = P.terminal_speed(diam[q], NU, RHO_P, RHO_F, G)
        assert abs(-vel[2, q] / v - 1) < 1e-9
        assert abs(vel[0, q]) == 0 and abs(vel[1, q]) == 0


def test_step_solves_implicit_euler_equation():
    """The new velocity satisfies u' = u + dt [(C_d/tau_p)(u_f - u') + g] with
    C_d from the old velocities (residual at round-off), and x' = x + dt u'."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 7, 5, 6
    d = (0.05, 0.07, 0.04)
    box = (nx * d[0], ny * d[1], nz * d[2])
    u = [rng.standard_normal((nz, ny, nx)) for _ in range(3)]
    n = 50
    pos = np.stack([rng.uniform(0, box[a], n) for a in range(3)])
    vel = rng.standard_normal((3, n)) * 0.3
    diam = rng.uniform(1e-6, 80e-6, n)
    g = (0.1, -0.2, -9.81)
    dt = 0.003
    p2, v2 = P.step(pos, vel, diam, u, d, box, NU, RHO_P, RHO_F, g, dt)
    uf = np.stack([P.interp(u[a], pos, d) for a in range(3)])
    rel = np.linalg.norm(uf - vel, axis=0)
    cd = 1 + (rel * diam / NU) ** (2 / 3) / 6
    k = cd / (RHO_P * diam ** 2 / (18 * RHO_F * NU))
    resid = v2 - vel - dt * (k * (uf - v2) + np.array(g)[:, None])
    assert np.abs(resid).max() < 1e-12 * max(1.0, np.abs(k * dt).max())
    moved = np.stack([np.mod(pos[a] + dt * v2[a], box[a]) for a in range(3)])
    assert np.allclose(p2, moved, rtol=0, atol=1e-15)


def test_interpolation_exact_on_nodes_and_linear_fields():
    rng = np.random.default_rng(4)
    nx, ny, nz = 6, 5, 4
    d = (0.2, 0.3, 0.5)
    f = rng.standard_normal((nz, ny, nx))
    # at the nodes: the node values
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pos = np.stack([I.ravel() * d[0], J.ravel() * d[1], K.ravel() * d[2]])
    np.testing.assert_allclose(P.interp(f, pos, d), f[K.ravel(), J.ravel(), I.ravel()], rtol=0, atol=1e-14)
    # a field linear in x, y, z away from the periodic seam is reproduced exactly
    a, b, c, e = 0.7, -1.3, 2.1, 0.4
    X, Y, Z = np.arange(nx) * d[0], np.arange(ny) * d[1], np.arange(nz) * d[2]
    lin = e + a * X[None, None, :] + b * Y[None, :, None] + c * Z[:, None, None]
    q = np.stack([rng.uniform(0, (nx - 1) * d[0], 100), rng.uniform(0, (ny - 1) * d[1], 100),
                  rng.uniform(0, (nz - 1) * d[2], 100)])
    np.testing.assert_allclose(P.interp(lin, q, d), e + a * q[0] + b * q[1] + c * q[2], rtol=0, atol=1e-13)
    # across the seam: halfway between the last and the first cell
    s = np.array([[(nx - 0.5) * d[0]], [0.0], [0.0]])
    assert abs(P.interp(f, s, d)[0] - 0.5 * (f[0, 0, nx - 1] + f[0, 0, 0])) < 1e-15


def test_tiny_particles_follow_uniform_flow():
    nx, ny, nz = 8, 8, 8
    d = (0.1, 0.1, 0.1)
    box = (0.8, 0.8, 0.8)
    U = (0.3, -0.2, 0.1)
    u = [np.full((nz, ny, nx), U[a]) for a in range(3)]
    pos = np.array([[0.05], [0.31], [0.77]])
    vel = np.array([[0.3], [-0.2], [0.1]])
    diam = np.array([1e-7])
    dt, n = 0.01, 50
    for _ in range(n):
        pos, vel = P.step(pos, vel, diam, u, d, box, NU, RHO_P, RHO_F, (0, 0, 0), dt)
    want = np.mod(np.array([[0.05], [0.31], [0.77]]) + n * dt * np.array(U)[:, None], 0.8)
    np.testing.assert_allclose(pos, want, rtol=0, atol=1e-12)


def test_drag_law_worked_values():
    """C_d = 1 + Re_p^(2/3)/6 at Reynolds numbers with exact cube roots:
    Re_p = 0, 1, 8, 27 give 1, 7/6, 5/3, 5/2."""
    nu, d = 1.6e-5, 1e-4
    for re, cd in ((0.0, 1.0), (1.0, 7 / 6), (8.0, 5 / 3), (27.0, 5 / 2)):
        rel = re * nu / d
        assert abs(P.drag_coefficient(rel, d, nu) - cd) < 1e-14


def test_relaxation_time_worked_value():
    """tau_p = rho_p d^2 / (18 rho_f nu): 10 um, water-density particle in air
    (rho_f = 1.2, nu = 1.5e-5): 1000 * 1e-10 / (18 * 1.2 * 1.5e-5) = 3.0864... e-4 s."""
    assert abs(P.tau_p(10e-6, 1.5e-5, 1000.0, 1.2) - 1e-7 / 3.24e-4) < 1e-18
