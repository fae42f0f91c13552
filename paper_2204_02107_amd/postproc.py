"""Host side of the post-processing of Sections 3.3-3.4.

The heavy parts run on the device (``Solver.co2_histogram``,
``Solver.accumulate``); these functions turn their results and the per-step
diagnostics into the quantities the paper reports.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def pdf(counts, lo, hi):
    """Normalised distribution function f(CO2) from bin counts over [lo, hi)."""
    counts = np.asarray(counts, dtype=np.float64)
    width = (hi - lo) / len(counts)
    total = counts.sum()
    return counts / (total * width) if total > 0 else counts


def fitted_ach(diags: Sequence[dict], c_out: float = 400.0) -> float:
    """Air changes per hour from the room-mean CO2 of a run of diagnostics:
    the decay rate of <c> - c_out, least squares in log space (Section 3.3)."""
    t = np.array([d["t"] for d in diags])
    y = np.log(np.array([d["co2_room_mean"] for d in diags]) - c_out)
    tm, ym = t.mean(), y.mean()
    slope = np.sum((t - tm) * (y - ym)) / np.sum((t - tm) ** 2)
    return -slope * 3600.0


def infection_risk(quanta_per_m3: float, breathing_m3_per_h: float, ach_per_h: float, hours: float) -> float:
    """Wells-Riley probability with the quanta concentration decaying at the
    air-change rate (Section 3.4): 1 - exp(-Q), Q = C0 p (1 - e^{-ACH t}) / ACH."""
    if ach_per_h == 0.0:
        dose = quanta_per_m3 * breathing_m3_per_h * hours
    else:
        dose = quanta_per_m3 * breathing_m3_per_h * (-math.expm1(-ach_per_h * hours)) / ach_per_h
    return -math.expm1(-dose)
