"""Pins of the post-processing oracle against the paper's printed values."""
import os

import numpy as np
import pytest

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


@pytest.mark.parametrize("c0,ach,c1", [(600.0, 12.0, 550.0), (450.0, 36.9, 350.0), (-200.0, 4.5, 900.0)])
def test_ach_fit3_recovers_free_asymptote(c0, ach, c1):
    """The three-parameter fit C0 exp(-ACH t) + C1 of Section 3.3 recovers the
    rate of a synthetic decay whose asymptote is not the 400 ppm outdoor
    level (also below it, and a rising curve), over a record of about two
    decay times, irregularly sampled."""
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0.0, 2.0 * 3600.0 / ach, 400))
    c = c0 * np.exp(-ach / 3600.0 * t) + c1
    assert abs(PP.ach_fit3(t, c) / ach - 1) < 1e-7


def test_ach_fit_known_level_refuses_values_below_it():
    t = np.linspace(0, 3600, 50)
    c = 400 * np.exp(-t / 1800) + 300       # crosses 400 ppm
    with pytest.raises(ValueError):
        PP.ach_fit(t, c)


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


def _block_case(nx=20, ny=16, nz=1, box=(6, 11, 5, 9, 0, 1), d=(0.1, 0.2, 0.3)):
    beta = np.ones((nz, ny, nx), np.uint8)
    i0, i1, j0, j1, k0, k1 = box
    beta[k0:k1, j0:j1, i0:i1] = 0
    return beta


def test_body_force_linear_pressure_closed_form():
    """Kinematic pressure G x (p = G x dt): the force on the obstacle is
    minus G times its volume (the buoyancy law), whatever the box around it;
    no y force, no viscous force at rest."""
    d = (0.1, 0.2, 0.3)
    box = (6, 11, 5, 9, 0, 1)
    beta = _block_case(box=box, d=d)
    nz, ny, nx = beta.shape
    G, dt = 2.5, 0.04
    x = np.arange(nx) * d[0]
    p = np.broadcast_to(G * dt * x[None, None, :], beta.shape).copy()
    z = np.zeros(beta.shape)
    fp, fv = PP.body_force(p, z, z, z, beta, (5, 12, 4, 10, 0, 1), d, nu=0.7, dt=dt)
    i0, i1, j0, j1, _, _ = box
    expect = -G * (i1 - i0) * d[0] * (j1 - j0) * d[1] * d[2]
    assert abs(fp[0] - expect) < 1e-12 * abs(expect)
    fp2, _ = PP.body_force(p, z, z, z, beta, box, d, nu=0.7, dt=dt)
    assert abs(fp2[0] - expect) < 1e-12 * abs(expect)
    assert abs(fp[1]) < 1e-12 and fp[2] == 0.0 and np.all(fv == 0.0)
    # uniform pressure: a closed body feels nothing
    fp0, _ = PP.body_force(np.full(beta.shape, 3.0), z, z, z, beta, (5, 12, 4, 10, 0, 1), d, nu=0.7, dt=dt)
    assert np.all(np.abs(fp0) < 1e-12)


def test_body_force_uniform_stream_closed_form():
    """u = U everywhere in the fluid, p = 0: the viscous force is nu U times
    the sum over the faces of area / spacing: 2 (j1 - j0) dy dz / dx over the
    x faces and 2 (i1 - i0) dx dz / dy over the y faces (nz = 1: the z
    neighbours are the cell itself, solid); a box that also holds fluid cells
    and misses none of the obstacle gives the same."""
    d = (0.1, 0.2, 0.3)
    box = (6, 11, 5, 9, 0, 1)
    beta = _block_case(box=box, d=d)
    U, nu = 1.7, 0.05
    u = U * beta.astype(np.float64)
    z = np.zeros(beta.shape)
    i0, i1, j0, j1, _, _ = box
    expect = nu * U * (2 * (j1 - j0) * d[1] * d[2] / d[0] + 2 * (i1 - i0) * d[0] * d[2] / d[1])
    for b in (box, (0, 20, 0, 16, 0, 1)):
        fp, fv = PP.body_force(z, u, z, z, beta, b, d, nu=nu, dt=0.1)
        assert abs(fv[0] - expect) < 1e-12 * expect
        assert fv[1] == 0.0 and fv[2] == 0.0 and np.all(fp == 0.0)


def test_shedding_frequency_of_sinusoids():
    """Known frequency recovered from irregularly spaced samples, with an
    offset and a second harmonic (upward crossings of the mean stay one per
    period when the harmonic is small)."""
    rng = np.random.default_rng(3)
    for f in (0.21, 1.0, 3.7):
        t = np.cumsum(rng.uniform(0.5, 1.5, 20000)) * (0.002 / f)
        y = 4.0 + np.sin(2 * np.pi * f * t + 0.3) + 0.2 * np.sin(4 * np.pi * f * t)
        est = PP.shedding_frequency(t, y)
        assert abs(est / f - 1) < 1e-4, (f, est)
    assert PP.shedding_frequency(np.arange(10.0), np.ones(10)) == 0.0


def test_body_force_is_what_the_pressure_gradient_takes_from_the_fluid():
    """Reading of the obstacle force: over the whole periodic grid the central
    pressure gradient sums to zero, so the pressure force on all solid cells
    equals dV times the sum of grad P over the fluid cells (what the
    correction u = u* - dt grad P removes from the fluid), for any p and any
    mask (the central differences written out with np.roll)."""
    rng = np.random.default_rng(8)
    shape = (6, 10, 12)
    d = (0.3, 0.2, 0.1)
    beta = np.ones(shape, np.uint8)
    beta[1:3, 2:5, 3:7] = 0
    beta[4:6, 6:9, 8:11] = 0
    p = rng.standard_normal(shape)
    dt = 0.05
    z = np.zeros(shape)
    fp, _ = PP.body_force(p, z, z, z, beta, (0, 12, 0, 10, 0, 6), d, nu=0.0, dt=dt)
    P = p / dt
    dv = d[0] * d[1] * d[2]
    fluid = beta == 1
    for a, ax in ((0, 2), (1, 1), (2, 0)):
        grad = (np.roll(P, -1, axis=ax) - np.roll(P, 1, axis=ax)) / (2 * d[a])
        want = dv * grad[fluid].sum()
        assert abs(fp[a] - want) < 1e-10 * np.abs(grad).sum() * dv, (a, fp[a], want)
