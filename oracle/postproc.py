"""Post-processing of Section 3.3-3.4, written out plainly (test infrastructure).

- The CO2 distribution function f(CO2) over the room (Section 3.3): counts of
  fluid cells of the room region per concentration bin.  Reading: bins of equal
  width over [lo, hi), bin index floor((c - lo) / (hi - lo) * nbins) evaluated
  in float64, values outside clamped into the end bins.
- Time averages of the fields: plain running sums (divided by the count when
  read).
- The air-change rate fitted to the mean CO2 decay (Section 3.3, Table 4):
  the paper's three-parameter fit C0 exp(-ACH t) + C1 (least squares, all
  three free), and, for short records where C1 cannot be told apart from C0
  (ACH t << 1), the same model with the outdoor level C1 = c_out known: least
  squares of log(<c> - c_out) against t.  ACH in 1/h.
- Theoretical ACH = volume flow / room volume (Section 3.3).
- Wells-Riley risk with decaying quanta (Section 3.4):
  P = 1 - exp(-Q), Q(t) = (C0 p / ACH) (1 - exp(-ACH t)), and Q = C0 p t
  without ventilation (the ACH -> 0 limit).

- The force of the fluid on an obstacle (Section 3.1.1, Table 2: drag
  coefficient and Strouhal number of the obstacle in the channel), per unit
  density.  Readings: the obstacle is the set of solid cells inside an index
  box.  Pressure part: every face of an obstacle cell carries the force
  -P_face n A with P_face the mean of the two cells' kinematic pressures (n
  the outward face normal, A the face area; faces between two obstacle cells
  cancel).  This is the share of the obstacle in the momentum the central
  pressure gradient removes from the fluid: summed over all cells that
  gradient vanishes, so what the fluid loses is what the solid cells hold.
  Viscous part: every face between an obstacle cell and a fluid cell adds
  nu u_f A / dx_a, the flux of the masked second difference into the solid
  cell (velocity zero there).  The solver's p absorbs the time step (the
  correction is u = u* - grad p), so P = p / dt with the step's dt.
- The shedding frequency of a periodic signal sampled at arbitrary times:
  upward crossings of its mean, located by linear interpolation; the
  frequency is (crossings - 1) over the time between the first and the last.

Parity status: pinned by ``tests/test_oracle_postproc.py`` (the paper's
theoretical ACH values and printed infection risks, brute-force bin counts,
exact recovery of synthetic exponential decays (with the asymptote known,
and free at a level other than the outdoor one), closed-form forces of a
linear pressure field (buoyancy: minus the gradient times the obstacle's
volume) and of a uniform stream on a rectangular obstacle, the frequency of
synthetic sinusoids).
"""
from __future__ import annotations

import numpy as np


def co2_histogram(c, beta, room, nbins, lo, hi):
    """Counts per bin of c over the cells with beta = 1 inside the room region."""
    sel = (beta == 1) if room is None else ((beta == 1) & (room != 0))
    vals = np.asarray(c, dtype=np.float64)[sel]
    idx = np.floor((vals - lo) / (hi - lo) * nbins)
    idx = np.clip(idx, 0, nbins - 1).astype(np.int64)
    return np.bincount(idx, minlength=nbins).astype(np.int64)


def ach_fit(t_s, mean_c, c_out=400.0):
    """Air changes per hour from <c>(t) = c_out + A exp(-ACH t) with the
    outdoor level c_out known: least squares of log(<c> - c_out) in t.
    Undefined (ValueError) once <c> <= c_out."""
    t = np.asarray(t_s, dtype=np.float64)
    c = np.asarray(mean_c, dtype=np.float64)
    if np.any(c <= c_out):
        raise ValueError("mean CO2 at or below the outdoor level: log fit undefined")
    y = np.log(c - c_out)
    A = np.vstack([t, np.ones_like(t)]).T
    slope = np.linalg.lstsq(A, y, rcond=None)[0][0]
    return -slope * 3600.0


def ach_fit3(t_s, mean_c):
    """Air changes per hour from the three-parameter fit of Section 3.3,
    <c>(t) = C0 exp(-ACH t) + C1 with C0, ACH and C1 all free, least squares.
    For a fixed rate the model is linear in (C0, C1) and numpy's lstsq solves
    it; the rate with the smallest residual is found on a log-spaced scan over
    1e-3 .. 1e3 decays per record length, then refined with scipy's bounded
    scalar minimiser between the scan's neighbours of the best point."""
    from scipy.optimize import minimize_scalar
    t = np.asarray(t_s, dtype=np.float64)
    t = t - t[0]
    y = np.asarray(mean_c, dtype=np.float64)
    span = t[-1]

    def sse(logk):
        A = np.vstack([np.exp(-np.exp(logk) * t), np.ones_like(t)]).T
        coef = np.linalg.lstsq(A, y, rcond=None)[0]
        r = A @ coef - y
        return float(r @ r)

    grid = np.linspace(np.log(1e-3 / span), np.log(1e3 / span), 601)
    vals = [sse(g) for g in grid]
    i = int(np.argmin(vals))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    best = minimize_scalar(sse, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12})
    return float(np.exp(best.x)) * 3600.0


def theoretical_ach(flow_area_m2, speed_m_s, volume_m3):
    """Volume flow over room volume, per hour."""
    return flow_area_m2 * speed_m_s / volume_m3 * 3600.0


def wells_riley(c0, p, ach, t_h):
    """Infection probability after t_h hours (C0 quanta/m^3, p m^3/h, ACH 1/h)."""
    if ach == 0:
        q = c0 * p * t_h
    else:
        q = c0 * p / ach * -np.expm1(-ach * t_h)
    return 1.0 - np.exp(-q)


def body_force(p, u, v, w, beta, box, spacing, nu, dt):
    """(pressure force, viscous force) on the solid cells of box = (i0, i1,
    j0, j1, k0, k1), each a 3-vector, per unit density."""
    nz, ny, nx = beta.shape
    i0, i1, j0, j1, k0, k1 = box
    dv = spacing[0] * spacing[1] * spacing[2]
    vel = (u, v, w)
    n = (nx, ny, nz)
    fp = np.zeros(3)
    fv = np.zeros(3)
    for k in range(k0, k1):
        for j in range(j0, j1):
            for i in range(i0, i1):
                if beta[k, j, i] != 0:
                    continue
                for a in range(3):
                    area = dv / spacing[a]
                    for sgn in (1, -1):
                        c = [i, j, k]
                        c[a] = (c[a] + sgn) % n[a]
                        p_face = 0.5 * (p[k, j, i] + p[c[2], c[1], c[0]]) / dt
                        fp[a] -= p_face * sgn * area
                        if beta[c[2], c[1], c[0]] == 0:
                            continue
                        for comp in range(3):
                            fv[comp] += nu * vel[comp][c[2], c[1], c[0]] * area / spacing[a]
    return fp, fv


def shedding_frequency(t, sig):
    """Frequency of a periodic signal from its upward mean crossings."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(sig, dtype=np.float64)
    y = y - y.mean()
    cross = []
    for q in range(len(y) - 1):
        if y[q] < 0.0 <= y[q + 1]:
            frac = -y[q] / (y[q + 1] - y[q])
            cross.append(t[q] + frac * (t[q + 1] - t[q]))
    if len(cross) < 2:
        return 0.0
    return (len(cross) - 1) / (cross[-1] - cross[0])
