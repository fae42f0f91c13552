"""Lagrangian particles of Section 2.3, written out plainly in float64.

Test infrastructure (see the package docstring).

The equations of motion: du_p/dt = (C_d / tau_p)(u_f - u_p) + g with
tau_p = rho_p d^2 / (18 rho_f nu), Re_p = |u_f - u_p| d / nu and
C_d = 1 + Re_p^(2/3) / 6, advanced by implicit Euler.  Readings where the
text is silent or at odds with itself:

- ``d`` is the particle diameter (Stokes' relaxation time uses it; the settling
  times the paper prints for 5, 10 and 30 um particles come out only with it),
  with rho_p = 1000 kg/m^3 and rho_f = 1.225 kg/m^3 (not stated; these give the
  printed 36 / 9 / 1 min);
- the fluid velocity at a particle is the trilinear interpolation of the
  collocated cell values, cell (i, j, k) sitting at (i dx, j dy, k dz) in the
  periodic box;
- implicit Euler with C_d taken from the velocities at the start of the step,
  so each step solves a linear equation per particle:
  u_p' = u_p + dt [(C_d / tau_p)(u_f - u_p') + g], then x_p' = x_p + dt u_p',
  wrapped into the periodic box;
- one-way coupling: the particles feel the fluid, not the reverse.

Parity status: pinned by ``tests/test_oracle_particles.py`` (the paper's
settling times, the terminal velocity as the scheme's fixed point, the
residual of the implicit Euler equation, exact interpolation of grid values and
of linear fields, uniform-flow advection).
"""
from __future__ import annotations

import numpy as np


def interp(f: np.ndarray, pos: np.ndarray, d) -> np.ndarray:
    """Trilinear interpolation of the cell field f (shape (nz, ny, nx)) at the
    positions pos (shape (3, n): x, y, z), periodic."""
    nz, ny, nx = f.shape
    n_ax = (nx, ny, nz)
    i0, w1 = [], []
    for a in range(3):
        s = pos[a] / d[a]
        fl = np.floor(s)
        i0.append(fl.astype(np.int64) % n_ax[a])
        w1.append(s - fl)
    out = np.zeros(pos.shape[1])
    for cz in (0, 1):
        wz = w1[2] if cz else 1.0 - w1[2]
        kz = (i0[2] + cz) % nz
        for cy in (0, 1):
            wy = w1[1] if cy else 1.0 - w1[1]
            jy = (i0[1] + cy) % ny
            for cx in (0, 1):
                wx = w1[0] if cx else 1.0 - w1[0]
                ix = (i0[0] + cx) % nx
                out += (wx * wy * wz) * f[kz, jy, ix]
    return out


def tau_p(diam, nu, rho_p, rho_f):
    """Particle relaxation time (Section 2.3)."""
    return rho_p * diam ** 2 / (18.0 * rho_f * nu)


def drag_coefficient(rel_speed, diam, nu):
    """C_d = 1 + Re_p^(2/3) / 6 with Re_p = |u_f - u_p| d / nu (Section 2.3)."""
    re = rel_speed * diam / nu
    return 1.0 + re ** (2.0 / 3.0) / 6.0


def step(pos, vel, diam, u, d, box, nu, rho_p, rho_f, g, dt):
    """One implicit-Euler step of all particles in the velocity field u = (u, v, w).

    pos, vel: arrays of shape (3, n); diam: shape (n,); box: (Lx, Ly, Lz);
    g: gravity vector.  Returns the new (pos, vel)."""
    uf = np.stack([interp(u[a], pos, d) for a in range(3)])
    rel = np.sqrt(np.sum((uf - vel) ** 2, axis=0))
    k = drag_coefficient(rel, diam, nu) / tau_p(diam, nu, rho_p, rho_f)     # C_d / tau_p
    g = np.asarray(g, dtype=np.float64)[:, None]
    vel_new = (vel + dt * k * uf + dt * g) / (1.0 + dt * k)
    pos_new = pos + dt * vel_new
    for a in range(3):
        pos_new[a] = np.mod(pos_new[a], box[a])
    return pos_new, vel_new


def terminal_speed(diam, nu, rho_p, rho_f, g, iters=200):
    """Settling speed in still air: the fixed point of v = g tau_p / C_d(v)."""
    tp = tau_p(diam, nu, rho_p, rho_f)
    v = g * tp
    for _ in range(iters):
        v = g * tp / drag_coefficient(v, diam, nu)
    return v
