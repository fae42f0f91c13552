"""Discrete operators of the scheme, written out plainly in float64.

Test infrastructure (see the package docstring).  Section 2.1 states the
discretisation: second-order central differences, skew-symmetric convection
for momentum, a sixth-order explicit filter, and a pressure equation solved in
Fourier space (Section 2.2).  Where the text leaves a choice open the reading
taken is stated at the function.

Array layout: shape (nz, ny, nx); axis a in {0, 1, 2} = {x, y, z} maps to the
numpy axis 2 - a.  ``d`` is the spacing triple (dx, dy, dz).
"""
from __future__ import annotations

import numpy as np


def shift(f: np.ndarray, a: int, m: int) -> np.ndarray:
    """Periodic shift: value of f at x + m e_a (the periodic box of Section 2.1)."""
    return np.roll(f, -m, axis=2 - a)


def ddx(f, a, d):
    """Central first difference along axis a (Section 2.1: 2nd-order central)."""
    return (shift(f, a, 1) - shift(f, a, -1)) / (2.0 * d[a])


def div(v, d):
    """Divergence of a vector field with central differences (Section 2.2)."""
    return ddx(v[0], 0, d) + ddx(v[1], 1, d) + ddx(v[2], 2, d)


def grad(p, d):
    """Central-difference gradient (Section 2.2, the velocity correction)."""
    return [ddx(p, 0, d), ddx(p, 1, d), ddx(p, 2, d)]


def lap(f, d):
    """Compact three-point second difference summed over axes (the viscous term
    of the momentum equation, Section 2.1)."""
    out = np.zeros_like(f)
    for a in range(3):
        out += (shift(f, a, 1) - 2.0 * f + shift(f, a, -1)) / (d[a] * d[a])
    return out


def conv_skew(u, d):
    """Skew-symmetric convection C_i(u) = 1/2 sum_a [D_a(u_a u_i) + u_a D_a u_i]
    (Section 2.1: central differences in the energy-conserving skew form)."""
    out = []
    for i in range(3):
        acc = np.zeros_like(u[i])
        for a in range(3):
            acc += ddx(u[a] * u[i], a, d) + u[a] * ddx(u[i], a, d)
        out.append(0.5 * acc)
    return out


def conv_scalar(u, c, d):
    """Flux-form scalar convection sum_a D_a(u_a c) (Section 2.1, the transport
    equation is written in divergence form)."""
    return ddx(u[0] * c, 0, d) + ddx(u[1] * c, 1, d) + ddx(u[2] * c, 2, d)


def lap_masked(c, beta, d):
    """Masked diffusion div(beta grad c) (Section 2.1, scalar equation and its
    zero-flux condition at solids).  Reading: the face between two cells
    conducts only when both cells are fluid, beta_{a+} = beta * s_a^{+1} beta.
    """
    b = beta.astype(np.float64)
    out = np.zeros_like(c)
    for a in range(3):
        bp = b * shift(b, a, 1)
        bm = b * shift(b, a, -1)
        out += (bp * (shift(c, a, 1) - c) - bm * (c - shift(c, a, -1))) / (d[a] * d[a])
    return out


def delta6(f, a):
    """Undivided seven-point sixth difference along axis a (binomial weights
    1, -6, 15, -20, 15, -6, 1)."""
    return (shift(f, a, -3) - 6.0 * shift(f, a, -2) + 15.0 * shift(f, a, -1) - 20.0 * f
            + 15.0 * shift(f, a, 1) - 6.0 * shift(f, a, 2) + shift(f, a, 3))


def filter6(f, d):
    """Sixth-order explicit filter of Section 2.1: f + sum_a gamma_a d^6 f/dx_a^6
    with gamma_a = dx_a^6/pi^6.  Reading: the sixth derivative is the discrete
    undivided difference over dx_a^6, so the filter is f + pi^-6 sum_a delta6_a f.
    """
    acc = np.zeros_like(f)
    for a in range(3):
        gamma = d[a] ** 6 / np.pi ** 6
        acc += gamma * delta6(f, a) / d[a] ** 6
    return f + acc


def _sin2_table(n: int, m: np.ndarray, h: float) -> np.ndarray:
    """sin^2(2 pi m / n) / h^2, exactly 0 where 2m is a multiple of n."""
    s = np.sin(2.0 * np.pi * m / n) ** 2 / (h * h)
    s[(2 * m) % n == 0] = 0.0
    return s


def poisson_symbol(shape, d):
    """Eigenvalues of div(grad .) with central differences on the rfftn grid.

    Section 2.2 solves the pressure equation by FFT with the operator whose
    right-hand side uses central differences; the matching symbol is
    lambda(m) = -sum_a sin^2(2 pi m_a / N_a) / dx_a^2.  Returns (lam, null)
    with ``null`` true where every m_a is 0 or N_a/2 (lambda = 0 there).
    """
    nz, ny, nx = shape
    mx = np.arange(nx // 2 + 1)
    my = np.arange(ny)
    mz = np.arange(nz)
    sx = _sin2_table(nx, mx, d[0])
    sy = _sin2_table(ny, my, d[1])
    sz = _sin2_table(nz, mz, d[2])
    lam = -(sz[:, None, None] + sy[None, :, None] + sx[None, None, :])
    nullx = (2 * mx) % nx == 0
    nully = (2 * my) % ny == 0
    nullz = (2 * mz) % nz == 0
    null = nullz[:, None, None] & nully[None, :, None] & nullx[None, None, :]
    return lam, null


def poisson_solve(r, d):
    """p = irfftn(rfftn(r) / lambda) with p_hat = 0 on the null modes
    (Section 2.2, pressure equation diagonalised in Fourier space)."""
    lam, null = poisson_symbol(r.shape, d)
    rh = np.fft.rfftn(r)
    safe = np.where(null, 1.0, lam)
    ph = np.where(null, 0.0, rh / safe)
    return np.fft.irfftn(ph, s=r.shape, axes=(0, 1, 2))


def ib_rhs(r0, p, beta, d):
    """Right-hand side of the immersed-boundary pressure iteration (Section 2.2):
    r0 + div((1 - beta) grad p), with central differences and (1 - beta) taken at
    cell centres."""
    omb = 1.0 - beta.astype(np.float64)
    g = grad(p, d)
    return r0 + div([omb * g[0], omb * g[1], omb * g[2]], d)
