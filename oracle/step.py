"""One explicit projection time step, in the paper's order (test infrastructure).

Section 2.1: classical explicit RK4 for the momentum equation without the
pressure gradient, one projection per time step (not per stage), a passive
scalar advanced by RK4 with the projected velocity, and the sixth-order filter
at the end of the step.  Section 2.2: the immersed-boundary pressure iteration
with n = 4 FFT solves warm-started from the previous pressure, then the
velocity correction u = u* - grad p.  Section 2.4: the time step follows from a
user-given maximum Courant number.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository):
  * collocated grid, central differences everywhere, Poisson symbol of
    div(grad .) with central differences;
  * forcing, body force and viscous terms are multiplied by beta every stage;
    u and c are multiplied by beta after the projection and after the filter;
  * the scalar uses the projected velocity u^{n+1}, frozen over its RK4;
  * Courant number sum_a |u_a| dt / dx_a, its denominator floored at
    u_ref / min(dx);
  * pressure null modes (every m_a in {0, N_a/2}) are set to zero.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import ops


@dataclass
class OracleParams:
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    nu: float
    alpha_c: float
    tau_f: float
    body: Sequence[float]
    cfl: float
    dt_fixed: float
    u_ref: float
    n_piter: int = 4
    filter: bool = True

    @property
    def d(self):
        return (self.lx / self.nx, self.ly / self.ny, self.lz / self.nz)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


@dataclass
class OracleState:
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    p: np.ndarray
    c: np.ndarray
    t: float = 0.0
    step: int = 0

    def copy(self):
        return OracleState(self.u.copy(), self.v.copy(), self.w.copy(), self.p.copy(),
                           self.c.copy(), self.t, self.step)


def momentum_rhs(u, beta, S, uset, body, nu, tau_f, d):
    """F(u)_i = beta [ -C_i(u) + nu L u_i + S (u_set,i - u_i)/tau_f + b_i ]
    (momentum equation of Section 2.1 without the pressure gradient; the
    boundary conditions multiply by beta)."""
    b = beta.astype(np.float64)
    C = ops.conv_skew(u, d)
    out = []
    for i in range(3):
        f = -C[i] + nu * ops.lap(u[i], d) + S * (uset[i] - u[i]) / tau_f + body[i]
        out.append(b * f)
    return out


def scalar_rhs(c, u, beta, S, cset, alpha_c, tau_f, d):
    """G(c; u) = beta [ -div(u c) + alpha_c div(beta grad c) + S (c_set - c)/tau_f ]
    (scalar transport equation of Section 2.1)."""
    b = beta.astype(np.float64)
    g = (-ops.conv_scalar(u, c, d) + alpha_c * ops.lap_masked(c, beta, d)
         + S * (cset - c) / tau_f)
    return b * g


def courant_rate(u, d):
    """max over cells of |u|/dx + |v|/dy + |w|/dz (summed left to right)."""
    return float(np.max(np.abs(u[0]) / d[0] + np.abs(u[1]) / d[1] + np.abs(u[2]) / d[2]))


class Oracle:
    """Holds the static inputs (mask, forcing) and advances a state."""

    def __init__(self, params: OracleParams, beta, forced_idx, forced_S, forced_uset,
                 forced_cset, room_mask=None):
        self.P = params
        shape = params.shape
        self.beta = np.asarray(beta, np.uint8).reshape(shape)
        n = int(np.prod(shape))
        S = np.zeros(n)
        us = np.zeros((3, n))
        cs = np.zeros(n)
        S[forced_idx] = forced_S
        for i in range(3):
            us[i, forced_idx] = np.asarray(forced_uset)[:, i]
        cs[forced_idx] = forced_cset
        self.S = S.reshape(shape)
        self.uset = [us[i].reshape(shape) for i in range(3)]
        self.cset = cs.reshape(shape)
        self.room = None if room_mask is None else np.asarray(room_mask, np.uint8).reshape(shape)

    @classmethod
    def from_scenario(cls, sc):
        P = OracleParams(sc.nx, sc.ny, sc.nz, sc.lx, sc.ly, sc.lz, sc.nu, sc.alpha_c,
                         sc.tau_f, tuple(sc.body), sc.cfl, sc.dt_fixed, sc.u_ref,
                         sc.n_piter, bool(sc.filter))
        return cls(P, sc.beta, sc.forced_idx, sc.forced_S, sc.forced_uset,
                   sc.forced_cset, sc.room_mask)

    @staticmethod
    def state_from_scenario(sc) -> OracleState:
        return OracleState(sc.u.copy(), sc.v.copy(), sc.w.copy(), sc.p.copy(), sc.c.copy())

    # -- pieces ------------------------------------------------------------
    def F(self, u):
        P = self.P
        return momentum_rhs(u, self.beta, self.S, self.uset, P.body, P.nu, P.tau_f, P.d)

    def G(self, c, u):
        P = self.P
        return scalar_rhs(c, u, self.beta, self.S, self.cset, P.alpha_c, P.tau_f, P.d)

    def dt_for(self, u):
        """Time step (Section 2.4, dynamic time stepping from a maximum Courant
        number); a positive dt_fixed overrides it."""
        P = self.P
        if P.dt_fixed > 0:
            return float(P.dt_fixed)
        d = P.d
        rate = max(courant_rate(u, d), P.u_ref / min(d))
        return P.cfl / rate

    def rk4_momentum(self, u, dt):
        """Classical RK4 without pressure (Section 2.1)."""
        k1 = self.F(u)
        u1 = [u[i] + 0.5 * dt * k1[i] for i in range(3)]
        k2 = self.F(u1)
        u2 = [u[i] + 0.5 * dt * k2[i] for i in range(3)]
        k3 = self.F(u2)
        u3 = [u[i] + dt * k3[i] for i in range(3)]
        k4 = self.F(u3)
        return [u[i] + (dt / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) for i in range(3)]

    def pressure(self, ustar, p_prev, n_iter=None):
        """Immersed-boundary pressure iteration of Section 2.2: n FFT solves of
        Delta p^{k+1} = div u* + div((1 - beta) grad p^k), warm-started from the
        previous pressure.  Returns the list of iterates p^1..p^n."""
        P = self.P
        n = P.n_piter if n_iter is None else n_iter
        d = P.d
        r0 = ops.div(ustar, d)
        p = p_prev
        its = []
        for _ in range(n):
            p = ops.poisson_solve(ops.ib_rhs(r0, p, self.beta, d), d)
            its.append(p)
        return its

    def project(self, ustar, p_prev, n_iter=None):
        """u = beta (u* - grad p^n) (Section 2.2 correction; beta re-applied as
        the no-slip condition of Section 2.1).  Returns (u, p)."""
        its = self.pressure(ustar, p_prev, n_iter)
        p = its[-1] if its else p_prev
        g = ops.grad(p, self.P.d)
        b = self.beta.astype(np.float64)
        return [b * (ustar[i] - g[i]) for i in range(3)], p

    def rk4_scalar(self, c, u, dt):
        """Classical RK4 of the scalar with the velocity frozen (Section 2.1)."""
        k1 = self.G(c, u)
        k2 = self.G(c + 0.5 * dt * k1, u)
        k3 = self.G(c + 0.5 * dt * k2, u)
        k4 = self.G(c + dt * k3, u)
        return c + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    def filter_all(self, u, c):
        """Sixth-order filter of velocity and scalar at the end of the step
        (Section 2.1), then the mask."""
        b = self.beta.astype(np.float64)
        d = self.P.d
        return [b * ops.filter6(u[i], d) for i in range(3)], b * ops.filter6(c, d)

    # -- the step ----------------------------------------------------------
    def step(self, s: OracleState, project_each_stage: bool = False):
        """Advance one time step; returns (new_state, diagnostics dict)."""
        P = self.P
        d = P.d
        u = [s.u, s.v, s.w]
        rate = courant_rate(u, d)
        dt = self.dt_for(u)
        if project_each_stage:
            ustar, p = self._rk4_projected(u, s.p, dt)
            unew = ustar
        else:
            ustar = self.rk4_momentum(u, dt)
            unew, p = self.project(ustar, s.p)
        divu = ops.div(unew, d)
        b = self.beta.astype(np.float64)
        cstar = self.rk4_scalar(s.c, unew, dt)
        cnew = b * cstar
        if P.filter:
            unew, cnew = self.filter_all(unew, cnew)
        dv = d[0] * d[1] * d[2]
        ke = 0.5 * float(np.sum(b * (unew[0] ** 2 + unew[1] ** 2 + unew[2] ** 2))) * dv
        mass = float(np.sum(b * cnew)) * dv
        if self.room is not None:
            rb = self.room.astype(np.float64) * b
            mean = float(np.sum(rb * cnew) / np.sum(rb))
        else:
            mean = float(np.sum(b * cnew) / np.sum(b))
        diag = {
            "t": s.t + dt, "dt": dt, "ke": ke,
            "div_l2": float(np.sqrt(np.sum(divu * divu) * dv)),
            "co2_mass": mass, "co2_room_mean": mean, "cfl_max": dt * rate,
            "step": s.step + 1,
        }
        ns = OracleState(unew[0], unew[1], unew[2], p, cnew, s.t + dt, s.step + 1)
        return ns, diag

    def _rk4_projected(self, u, p_prev, dt):
        """Variant with a projection after every RK4 stage: the alternative the
        paper's Section 2.1 mentions and skips for speed.  Used only for
        temporal-accuracy pins."""
        p = p_prev
        proj = self.project
        k1 = self.F(u)
        u1, p = proj([u[i] + 0.5 * dt * k1[i] for i in range(3)], p)
        k2 = self.F(u1)
        u2, p = proj([u[i] + 0.5 * dt * k2[i] for i in range(3)], p)
        k3 = self.F(u2)
        u3, p = proj([u[i] + dt * k3[i] for i in range(3)], p)
        k4 = self.F(u3)
        us = [u[i] + (dt / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) for i in range(3)]
        return proj(us, p)

    def run(self, s: OracleState, nsteps: int, project_each_stage=False):
        diags = []
        for _ in range(nsteps):
            s, dg = self.step(s, project_each_stage)
            diags.append(dg)
        return s, diags
