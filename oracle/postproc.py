"""Post-processing of Section 3.3-3.4, written out plainly (test infrastructure).

- The CO2 distribution function f(CO2) over the room (Section 3.3): counts of
  fluid cells of the room region per concentration bin.  Reading: bins of equal
  width over [lo, hi), bin index floor((c - lo) / (hi - lo) * nbins) evaluated
  in float64, values outside clamped into the end bins.
- Time averages of the fields: plain running sums (divided by the count when
  read).
- The air-change rate fitted to the mean CO2 decay (Section 3.3, Table 4):
  reading: least squares of log(<c> - c_out) against t with the outdoor level
  c_out = 400 ppm known (the paper fits C0 exp(-ACH t) + C1); ACH in 1/h.
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
exact recovery of a synthetic exponential decay, closed-form forces of a
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
    """Air changes per hour from <c>(t) = c_out + A exp(-ACH t)."""
    t = np.asarray(t_s, dtype=np.float64)
    y = np.log(np.asarray(mean_c, dtype=np.float64) - c_out)
    A = np.vstack([t, np.ones_like(t)]).T
    slope = np.linalg.lstsq(A, y, rcond=None)[0][0]
    return -slope * 3600.0


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
