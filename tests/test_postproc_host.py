"""Host-side post-processing of the package against the oracle and against
synthetic records with known answers (no GPU)."""
import numpy as np
import pytest

from oracle import postproc as PP
from paper_2204_02107_amd import postproc


def test_shedding_frequency_matches_oracle():
    rng = np.random.default_rng(11)
    for f in (0.05, 0.2094, 2.0):
        t = np.cumsum(rng.uniform(0.2, 1.8, 5000)) * (0.01 / f)
        y = -1.0 + 0.3 * np.sin(2 * np.pi * f * t + 1.0) + 1e-3 * rng.standard_normal(t.size)
        a, b = postproc.shedding_frequency(t, y), PP.shedding_frequency(t, y)
        assert abs(a - b) <= 1e-12 * b and abs(a / f - 1) < 1e-3


def test_obstacle_coefficients_of_synthetic_records():
    """Records with a known mean drag, lift amplitude and frequency: C_D,
    C_L' = amplitude / sqrt(2) / q and St = f h / U_b come back."""
    h, u_b, depth = 1.3, 0.8, 0.05
    q = 0.5 * u_b ** 2 * h * depth
    f = 0.2 * u_b / h
    t = np.linspace(0.0, 400.0, 40001)
    rec = np.zeros((t.size, 8))
    rec[:, 0] = 2.9 * q + 0.01 * q * np.sin(4 * np.pi * f * t)     # pressure drag, second harmonic
    rec[:, 3] = 0.1 * q                                           # friction drag
    rec[:, 1] = 0.5 * q * np.sin(2 * np.pi * f * t)               # lift
    rec[:, 6] = t
    rec[:, 7] = t[1] - t[0]
    c = postproc.obstacle_coefficients(rec, h, u_b, depth)
    assert abs(c["C_D"] - 3.0) < 1e-3 and abs(c["C_D_pressure"] - 2.9) < 1e-3
    assert abs(c["C_L_rms"] - 0.5 / np.sqrt(2)) < 1e-3
    assert abs(c["St"] - 0.2) < 1e-4
    assert c["samples"] == t.size - t.size // 2


@pytest.mark.parametrize("c0,ach,c1", [(600.0, 12.0, 550.0), (450.0, 36.9, 350.0), (30.0, 2.1, 1000.0)])
def test_fitted_ach_three_parameters_matches_oracle(c0, ach, c1):
    """The package's three-parameter ACH fit (golden-section search) against
    the oracle's (scan + scipy bounded minimiser) and the exact rate, on
    synthetic decays whose asymptote is not the outdoor level; with a little
    noise both land on the same least-squares rate."""
    rng = np.random.default_rng(8)
    t = np.sort(rng.uniform(0.0, 1.5 * 3600.0 / ach, 300))
    c = c0 * np.exp(-ach / 3600.0 * t) + c1
    diags = [{"t": a, "co2_room_mean": b} for a, b in zip(t, c)]
    assert abs(postproc.fitted_ach(diags) / ach - 1) < 1e-7
    noisy = c + 0.01 * abs(c0) * rng.standard_normal(t.size)
    nd = [{"t": a, "co2_room_mean": b} for a, b in zip(t, noisy)]
    assert abs(postproc.fitted_ach(nd) / PP.ach_fit3(t, noisy) - 1) < 1e-6


def test_fitted_ach_known_level():
    t = np.linspace(0.0, 60.0, 100)
    c = 400.0 + 600.0 * np.exp(-2.0 / 3600.0 * t)
    diags = [{"t": a, "co2_room_mean": b} for a, b in zip(t, c)]
    assert abs(postproc.fitted_ach(diags, c_out=400.0) - PP.ach_fit(t, c)) < 1e-9
    with pytest.raises(ValueError):
        postproc.fitted_ach([{"t": 0.0, "co2_room_mean": 399.0}, {"t": 1.0, "co2_room_mean": 398.0}], c_out=400.0)
