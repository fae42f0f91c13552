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

Parity status: pinned by ``tests/test_oracle_postproc.py`` (the paper's
theoretical ACH values and printed infection risks, brute-force bin counts,
exact recovery of a synthetic exponential decay).
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
