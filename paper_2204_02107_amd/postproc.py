"""Host side of the post-processing of Sections 3.1.1 and 3.3-3.4.

The heavy parts run on the device (``Solver.body_force``,
``Solver.co2_histogram``, ``Solver.accumulate``); these functions turn their
results and the per-step diagnostics into the quantities the paper reports.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np


def pdf(counts, lo, hi):
    """Normalised distribution function f(CO2) from bin counts over [lo, hi)."""
    counts = np.asarray(counts, dtype=np.float64)
    width = (hi - lo) / len(counts)
    total = counts.sum()
    return counts / (total * width) if total > 0 else counts


def fitted_ach(diags: Sequence[dict], c_out: Optional[float] = None) -> float:
    """Air changes per hour from the room-mean CO2 of a run of diagnostics
    (Section 3.3, Table 4).

    c_out None: the paper's fit <c>(t) = C0 exp(-ACH t) + C1 with all three
    parameters free.  For a given rate k the best C0 and C1 are a straight
    line fit of <c> on e = exp(-k t), whose residual is n (var c - cov(e, c)^2
    / var e); k maximises cov(e, c)^2 / var e, found on a coarse log scan and
    refined by golden-section search.

    c_out given: the asymptote is the known outdoor level and the rate is the
    least-squares slope of log(<c> - c_out) against t; this suits records much
    shorter than 1/ACH, where C0 and C1 cannot be told apart.  ValueError if
    <c> reaches c_out (the logarithm is undefined)."""
    t = np.array([d["t"] for d in diags], dtype=np.float64)
    c = np.array([d["co2_room_mean"] for d in diags], dtype=np.float64)
    if c_out is not None:
        if np.any(c <= c_out):
            raise ValueError("room-mean CO2 at or below c_out: the log-linear ACH fit is undefined")
        y = np.log(c - c_out)
        tm, ym = t.mean(), y.mean()
        slope = np.sum((t - tm) * (y - ym)) / np.sum((t - tm) ** 2)
        return float(-slope * 3600.0)
    tr = t - t[0]
    cc = c - c.mean()

    def score(lk):
        e = np.exp(-math.exp(lk) * tr)
        e = e - e.mean()
        ve = float(e @ e)
        return float(e @ cc) ** 2 / ve if ve > 0 else 0.0

    lo, hi = math.log(1e-3 / tr[-1]), math.log(1e3 / tr[-1])
    scan = np.linspace(lo, hi, 241)
    i = int(np.argmax([score(q) for q in scan]))
    a, b = scan[max(i - 1, 0)], scan[min(i + 1, scan.size - 1)]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = b - g * (b - a), a + g * (b - a)
    f1, f2 = score(x1), score(x2)
    while b - a > 1e-13 * max(1.0, abs(a)):
        if f1 >= f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - g * (b - a)
            f1 = score(x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + g * (b - a)
            f2 = score(x2)
    return float(math.exp(0.5 * (a + b)) * 3600.0)


def infection_risk(quanta_per_m3: float, breathing_m3_per_h: float, ach_per_h: float, hours: float) -> float:
    """Wells-Riley probability with the quanta concentration decaying at the
    air-change rate (Section 3.4): 1 - exp(-Q), Q = C0 p (1 - e^{-ACH t}) / ACH."""
    if ach_per_h == 0.0:
        dose = quanta_per_m3 * breathing_m3_per_h * hours
    else:
        dose = quanta_per_m3 * breathing_m3_per_h * (-math.expm1(-ach_per_h * hours)) / ach_per_h
    return -math.expm1(-dose)


def shedding_frequency(t, signal) -> float:
    """Frequency of a periodic signal sampled at increasing times t: the number
    of periods between its first and last upward crossing of the mean,
    crossings placed by linear interpolation between samples."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(signal, dtype=np.float64)
    y = y - np.mean(y)
    up = np.nonzero((y[:-1] < 0.0) & (y[1:] >= 0.0))[0]
    if up.size < 2:
        return 0.0
    tc = t[up] - y[up] * (t[up + 1] - t[up]) / (y[up + 1] - y[up])
    return float((up.size - 1) / (tc[-1] - tc[0]))


def obstacle_coefficients(records, h: float, u_b: float, depth: float, start_frac: float = 0.5) -> dict:
    """Drag and lift coefficients and Strouhal number of an obstacle (Section
    3.1.1, Table 2) from ``Solver.body_force`` records (rows: pressure force,
    viscous force, t, dt), over the records after ``start_frac`` of the run:
    C_D = mean F_x / (U_b^2 h depth / 2), C_L' = rms of the lift coefficient,
    St = f h / U_b with f the frequency of the lift."""
    r = np.asarray(records, dtype=np.float64)
    r = r[int(len(r) * start_frac):]
    fx = r[:, 0] + r[:, 3]
    fy = r[:, 1] + r[:, 4]
    q = 0.5 * u_b ** 2 * h * depth
    cl = fy / q
    f = shedding_frequency(r[:, 6], fy)
    return {"C_D": float(np.mean(fx) / q), "C_D_pressure": float(np.mean(r[:, 0]) / q),
            "C_L_rms": float(np.sqrt(np.mean((cl - cl.mean()) ** 2))), "St": f * h / u_b,
            "t0": float(r[0, 6]), "t1": float(r[-1, 6]), "samples": int(len(r))}