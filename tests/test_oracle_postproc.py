"""Pins of the post-processing oracle against the paper's printed values."""
import os

import numpy as np

from oracle import postproc as PP

HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "wells_riley_table4.txt")):
        line = line.split("#")[0].split()
        if line:
            out[line[0]] = [float(v) for v in line[1:]]
    return out


def test_theoretical_ach_values():
    g = golden()
    assert abs(PP.theoretical_ach(2 * 1.2, 1.0, 8 * 8 * 3) - g["theory"][0]) < 1e-12
    assert abs(PP.theoretical_ach(2 * 1.2, 0.1, 8 * 8 * 3) - g["theory"][1]) < 1e-12


def risks(quanta, achs):
    c0 = quanta / (8 * 8 * 3)
    return [100 * PP.wells_riley(c0, 1.2, a, 0.5) for a in achs]


def test_wells_riley_matches_printed_ranges():
    """The printed ranges are read to about a percentage point (values quoted
    to two digits); the formula evaluated at Table 4's ACH values must fall in
    them to that precision."""
    g = golden()
    r = risks(100, g["ach_high"])
    assert g["risk100_high"][0] - 0.1 <= min(r) and max(r) <= g["risk100_high"][1] + 0.1, r
    r = risks(100, g["ach_low"])
    assert g["risk100_low"][0] - 1 <= min(r) and max(r) <= g["risk100_low"][1] + 1, r
    r = risks(500, g["ach_low"])
    assert g["risk500_low"][0] - 1 <= min(r) and max(r) <= g["risk500_low"][1] + 1, r
    r = risks(500, [0.0])[0]
    assert abs(r - g["risk500_off"][0]) <= 1.5, r


def test_wells_riley_limits():
    # no ventilation is the ACH -> 0 limit; long exposures saturate at C0 p / ACH
    assert abs(PP.wells_riley(0.5, 1.2, 1e-9, 0.5) - PP.wells_riley(0.5, 1.2, 0.0, 0.5)) < 1e-9
    assert abs(PP.wells_riley(0.5, 1.2, 10.0, 100.0) - (1 - np.exp(-0.06))) < 1e-15


def test_ach_fit_recovers_exponential():
    t = np.linspace(0, 120, 200)
    ach = 37.5
    c = 400 + 600 * np.exp(-ach / 3600 * t)
    assert abs(PP.ach_fit(t, c) - ach) < 1e-9


def test_histogram_brute_force():
    rng = np.random.default_rng(3)
    shape = (4, 5, 6)
    c = rng.uniform(350, 1050, shape)
    beta = (rng.random(shape) > 0.2).astype(np.uint8)
    room = (rng.random(shape) > 0.3).astype(np.uint8)
    nb, lo, hi = 7, 400.0, 1000.0
    want = np.zeros(nb, np.int64)
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                if beta[k, j, i] == 1 and room[k, j, i]:
                    b = int(np.floor((c[k, j, i] - lo) / (hi - lo) * nb))
                    want[min(max(b, 0), nb - 1)] += 1
    assert np.array_equal(PP.co2_histogram(c, beta, room, nb, lo, hi), want)
