"""RK4 stages two per pass (momentum and scalar stage pairs) against the FP64
oracle and against one kernel per stage, forced on small rooms through
dnslab_set_stage_pairs (by default the FP64 momentum pairs run where a launch
has a block per CU or more, the others where each block's z chunk is long:
the 3.1M-, 25M- and 134M-cell grids of the full-size tests).  Ragged z chunks: nz = 36 and 54 are not multiples of the pair
kernels' chunk length.

Tolerances: FP64 whole steps 1e-10 against the oracle (the stated bar); the
two GPU paths evaluate the same expressions, so FP64 pairs and single stages
agree to 1e-12 (rounding only where the compiler contracts differently);
FP32 form: field rel L2 1e-4 against the oracle after 50 steps, and the two
GPU paths within 1e-5 of each other.
"""
import numpy as np
import pytest

from oracle.step import Oracle
import scenarios
from gpu_util import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "w", "p", "c")


def rel_l2(got, ref, mask):
    return float(np.sqrt(np.sum((got[mask] - ref[mask]) ** 2) / max(np.sum(ref[mask] ** 2), 1e-300)))


def run(sc, nsteps, prec, mode):
    torch, m = need_gpu()
    S = m.Solver(sc, precision=prec)
    S.set_stage_pairs(mode)
    d = S.step(nsteps)
    got = S.state()
    S.close()
    return got, d


@pytest.mark.parametrize("grid", [(64, 48, 36), (128, 32, 54)])
def test_fp64_pairs_match_oracle_and_single_stages(grid):
    torch, m = need_gpu()
    sc = scenarios.room(*grid, dx=0.0390625, n_boxes=3, seed=2204)
    announce(f"stage pairs fp64 room {grid} x12")
    got, d = run(sc, 12, m.FP64, 1)
    ref_gpu, d1 = run(sc, 12, m.FP64, 0)
    O = Oracle.from_scenario(sc)
    st, diags = O.run(Oracle.state_from_scenario(sc), 12)
    errs = {k: rel_err(got[k], getattr(st, k)) for k in FIELDS}
    same = {k: rel_err(got[k], ref_gpu[k]) for k in FIELDS}
    print(f"[pairs] fp64 {grid}: vs oracle {errs}; vs single stages {same}", flush=True)
    for k in FIELDS:
        assert errs[k] < 1e-10, (k, errs)
        assert same[k] < 1e-12, (k, same)
    ref = diags[-1]
    for k in ("t", "dt", "ke", "co2_mass", "co2_room_mean", "cfl_max"):
        assert abs(d[k] - ref[k]) <= 1e-10 * abs(ref[k]), (k, d[k], ref[k])
    floor = 1e-12 * np.sqrt(2 * ref["ke"]) / min(sc.spacing)
    assert abs(d["div_l2"] - ref["div_l2"]) <= 1e-10 * ref["div_l2"] + floor
    assert abs(d["co2_mass"] - d1["co2_mass"]) <= 1e-12 * abs(d1["co2_mass"])


def test_fp32_pairs_match_oracle_and_single_stages():
    torch, m = need_gpu()
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("stage pairs fp32 room 64x48x36 x50")
    got, d = run(sc, 50, m.FP32_REFINE, 1)
    ref_gpu, _ = run(sc, 50, m.FP32_REFINE, 0)
    O = Oracle.from_scenario(sc)
    st, diags = O.run(Oracle.state_from_scenario(sc), 50)
    fluid = sc.beta == 1
    errs = {k: rel_l2(got[k], getattr(st, k), fluid) for k in ("u", "v", "w", "c")}
    same = {k: rel_l2(got[k], ref_gpu[k], fluid) for k in ("u", "v", "w", "c")}
    print(f"[pairs] fp32: vs oracle {errs}; vs single stages {same}", flush=True)
    for k in errs:
        assert errs[k] < 1e-4, (k, errs)
        assert same[k] < 1e-5, (k, same)
    excess = (d["div_l2"] - diags[-1]["div_l2"]) * min(sc.spacing) / np.sqrt(2 * diags[-1]["ke"])
    assert excess < 1e-7, excess
    assert abs(d["co2_room_mean"] / diags[-1]["co2_room_mean"] - 1) < 1e-6


def test_pairs_need_a_dividing_tile():
    """nx = 48 is no multiple of the 64-wide tile: forcing the pairs on leaves
    the single-stage kernels in place (same results as mode 0, bit for bit)."""
    torch, m = need_gpu()
    sc = scenarios.room(48, 32, 24, dx=0.0390625, n_boxes=2, seed=5)
    announce("stage pairs on an undividable grid")
    a, _ = run(sc, 4, m.FP64, 1)
    b, _ = run(sc, 4, m.FP64, 0)
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def test_stage_pairs_mode_is_validated():
    torch, m = need_gpu()
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=1, seed=1)
    S = m.Solver(sc)
    with pytest.raises(Exception):
        S.set_stage_pairs(2)
    S.close()
