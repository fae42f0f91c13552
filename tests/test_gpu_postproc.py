"""On-device post-processing against the oracle: CO2 distribution counts,
running sums for time averages, and the fitted ACH / infection risk chain."""
import numpy as np
import pytest

from oracle import postproc as PP
import scenarios
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_histogram_equals_oracle(precision):
    torch, m = need_gpu()
    prec = m.FP64 if precision == "fp64" else m.FP32_REFINE
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce(f"co2 histogram {precision}")
    S = m.Solver(sc, precision=prec)
    S.step(30, diag=False)
    c = S.c.double().cpu().numpy()
    for nb, lo, hi in ((60, 400.0, 1000.0), (4096, 990.0, 1000.5), (1, 0.0, 1.0), (17, 500.0, 900.0)):
        got = S.co2_histogram(nb, lo, hi)
        want = PP.co2_histogram(c, sc.beta, sc.room_mask, nb, lo, hi)
        assert np.array_equal(got, want), (nb, lo, hi)
    S.close()


def test_accumulate_equals_sums():
    torch, m = need_gpu()
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=7)
    announce("accumulate")
    S = m.Solver(sc)
    sums = torch.zeros((5,) + sc.shape, dtype=torch.float64, device=S.device)
    ref = np.zeros((5,) + sc.shape)
    for _ in range(4):
        S.step(3, diag=False)
        S.accumulate(sums)
        st = S.state()
        for f, k in enumerate(("u", "v", "w", "p", "c")):
            ref[f] += st[k]
    assert np.array_equal(sums.cpu().numpy(), ref)
    S.close()


def test_fitted_ach_and_risk_chain():
    torch, m = need_gpu()
    from paper_2204_02107_amd import postproc
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=2, seed=9)
    announce("ach fit chain")
    S = m.Solver(sc)
    S.step(200, diag=False)
    diags = S.read_diags(200)
    S.close()
    t = [d["t"] for d in diags]
    cm = [d["co2_room_mean"] for d in diags]
    ach = postproc.fitted_ach(diags, c_out=400.0)
    assert abs(ach - PP.ach_fit(t, cm)) < 1e-9 * abs(ach)
    assert ach > 0
    c0 = 100 / (sc.lx * sc.ly * sc.lz)
    assert abs(postproc.infection_risk(c0, 1.2, ach, 0.5) - PP.wells_riley(c0, 1.2, ach, 0.5)) < 1e-15


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_body_force_equals_oracle(precision):
    """Obstacle force of the channel case: the kernel against the oracle's
    face sum on the same (device) fields, for the obstacle box, a box that
    also holds wall cells, and the whole grid; t and dt in the record are the
    step's."""
    torch, m = need_gpu()
    prec = m.FP64 if precision == "fp64" else m.FP32_REFINE
    sc = scenarios.cube_channel(8)
    announce(f"body force {precision}")
    S = m.Solver(sc, precision=prec)
    dg = S.step(25)
    st = S.state()
    i0, i1, j0, j1, _, _ = sc.meta["obstacle_cells"]
    boxes = [(i0 - 1, i1 + 1, j0 - 1, j1 + 1, 0, 1), (i0, i1, 0, j1, 0, 1), (0, sc.nx, 0, sc.ny, 0, 1)]
    out = torch.full((len(boxes), 8), float("nan"), dtype=torch.float64, device=S.device)
    for r, b in enumerate(boxes):
        S.body_force(b, out, r)
    got = out.cpu().numpy()
    for r, b in enumerate(boxes):
        fp, fv = PP.body_force(st["p"], st["u"], st["v"], st["w"], sc.beta, b, sc.spacing, sc.nu, dg["dt"])
        want = np.concatenate([fp, fv])
        scale = np.abs(want).max()
        # summation order differs; the whole-grid box sums many cancelling faces
        tol = 1e-12 if r < 2 else 1e-9
        assert np.all(np.abs(got[r, :6] - want) <= tol * scale), (b, got[r, :6], want)
        assert got[r, 6] == dg["t"] and got[r, 7] == dg["dt"]
    # the obstacle feels a drag along the flow and both parts contribute
    assert got[0, 0] > 0 and got[0, 3] > 0
    with pytest.raises(m.DnslabError):
        S.body_force((0, 0, 0, 1, 0, 1), out, 0)
    with pytest.raises(m.DnslabError):
        S.body_force((0, sc.nx + 1, 0, 1, 0, 1), out, 0)
    S.close()


def test_cube_channel_steps_equal_oracle():
    """The obstacle-in-channel case (2D, forced parabolic inflow, masked
    obstacle and walls) stepped on the device and by the oracle."""
    torch, m = need_gpu()
    from oracle.step import Oracle
    sc = scenarios.cube_channel(8)
    announce("cube channel 432x54 x30 vs oracle")
    S = m.Solver(sc)
    dg = S.step(30)
    got = S.state()
    S.close()
    O = Oracle.from_scenario(sc)
    st, diags = O.run(Oracle.state_from_scenario(sc), 30)
    for k in ("u", "v", "p"):
        ref = getattr(st, k)
        assert np.sqrt(np.sum((got[k] - ref) ** 2) / np.sum(ref ** 2)) < 1e-10, k
    for k in ("t", "dt", "ke"):
        assert abs(dg[k] - diags[-1][k]) <= 1e-10 * abs(diags[-1][k]), k
