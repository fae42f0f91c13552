"""FP32 form with FP64 refinement of the last pressure solve, against the FP64
oracle.

Bars: operators in FP32 arithmetic agree with the FP64 oracle to a few FP32
ulps (1e-5 relative); whole steps over a 50-step horizon to a relative L2
error <= 1e-4 per field over fluid cells; the divergence of the projected
velocity, ||div u||_2 min(dx) / ||u||_2, <= 1e-7 for unmasked flow, and in
masked flow exceeds the oracle's own immersed-boundary residual by <= 1e-7.
"""
import numpy as np
import pytest

from oracle import ops
from oracle.step import Oracle
import scenarios
from gpu_util import announce, need_gpu, rel_err, to_np
from test_gpu_parity import make_case

pytestmark = pytest.mark.gpu


def rel_l2(got, ref, mask=None):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is not None:
        got = got[mask]
        ref = ref[mask]
    den = np.sqrt(np.sum(ref * ref))
    return float(np.sqrt(np.sum((got - ref) ** 2)) / max(den, 1e-300))


@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 36, 24), (12, 1, 6)])
def test_fp32_operators(shape):
    torch, m = need_gpu()
    sc = make_case(shape, 21)
    announce(f"fp32 operators {shape}")
    S = m.Solver(sc, precision=m.FP32_REFINE)
    O = Oracle.from_scenario(sc)
    got = [to_np(t) for t in S.momentum_rhs(sc.u, sc.v, sc.w)]
    ref = O.F([sc.u, sc.v, sc.w])
    for a in range(3):
        assert rel_err(got[a], ref[a]) < 1e-5
    assert rel_err(to_np(S.scalar_rhs(sc.c, sc.u, sc.v, sc.w)), O.G(sc.c, [sc.u, sc.v, sc.w])) < 1e-5
    assert rel_err(to_np(S.filter(sc.c)), sc.beta * ops.filter6(sc.c, sc.spacing)) < 1e-5
    r = np.random.default_rng(2).standard_normal(shape)
    assert rel_err(to_np(S.poisson(r)), ops.poisson_solve(r, sc.spacing)) < 1e-5


@pytest.mark.parametrize("shape", [(2, 2, 8192), (4096, 2, 4), (2, 4096, 4)])
def test_fp32_poisson_longest_lines(shape):
    """FP32 lines at the length limits (x 8192, y and z 4096)."""
    torch, m = need_gpu()
    sc = make_case(shape, 23, masked=False, forced=False, filt=False)
    announce(f"fp32 poisson long lines {shape}")
    S = m.Solver(sc, precision=m.FP32_REFINE)
    r = np.random.default_rng(3).standard_normal(shape)
    assert rel_err(to_np(S.poisson(r)), ops.poisson_solve(r, sc.spacing)) < 1e-5


@pytest.mark.parametrize("shape", [(64, 64, 8), (96, 64, 8), (96, 128, 8), (128, 128, 4), (144, 96, 4)])
def test_fp32_poisson_fused_plane_sizes(shape):
    """Planes of 4096, 6144, 12288, 16384 and 13824 (960-thread block) FP32
    values: each instance of the fused y/z pass, up to the largest plane."""
    torch, m = need_gpu()
    sc = make_case(shape, 24, masked=False, forced=False, filt=False)
    announce(f"fp32 poisson fused planes {shape}")
    S = m.Solver(sc, precision=m.FP32_REFINE)
    r = np.random.default_rng(4).standard_normal(shape)
    assert rel_err(to_np(S.poisson(r)), ops.poisson_solve(r, sc.spacing)) < 1e-5


@pytest.mark.parametrize("masked", [False, True])
def test_fp32_project_refined(masked):
    """The refined projection matches the FP64 projection to FP32 storage
    precision, well below the error of an unrefined FP32 solve."""
    torch, m = need_gpu()
    sc = make_case((32, 48, 64), 22, masked=masked)
    announce(f"fp32 project masked={masked}")
    S = m.Solver(sc, precision=m.FP32_REFINE)
    us = [S._dev(a) for a in (sc.u, sc.v, sc.w)]
    S.project(*us)
    O = Oracle.from_scenario(sc)
    ref_u, ref_p = O.project([sc.u, sc.v, sc.w], sc.p)
    for a in range(3):
        assert rel_err(to_np(us[a]), ref_u[a]) < 2e-6
    assert rel_err(to_np(S.p), ref_p) < 2e-6
    if not masked:
        u64 = [to_np(t) for t in us]
        d = ops.div(u64, sc.spacing)
        ratio = np.sqrt(np.sum(d * d)) * min(sc.spacing) / np.sqrt(sum(np.sum(x * x) for x in u64))
        assert ratio < 1e-7, ratio


def run_both(sc, nsteps):
    torch, m = need_gpu()
    S = m.Solver(sc, precision=m.FP32_REFINE)
    dg = S.step(nsteps)
    got = S.state()
    O = Oracle.from_scenario(sc)
    st, diags = O.run(Oracle.state_from_scenario(sc), nsteps)
    S.close()
    return got, dg, st, diags


def test_fp32_taylor_green_50_steps():
    sc = scenarios.taylor_green(32)
    announce("fp32 tgv32 x50")
    got, dg, st, diags = run_both(sc, 50)
    for k in ("u", "v", "w", "c"):
        assert rel_l2(got[k], getattr(st, k)) < 1e-4, k
    ratio = dg["div_l2"] * min(sc.spacing) / np.sqrt(2 * dg["ke"])
    assert ratio < 1e-7, ratio
    assert abs(dg["ke"] / diags[-1]["ke"] - 1) < 1e-5


def test_fp32_room_50_steps():
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("fp32 room 64x48x36 x50")
    got, dg, st, diags = run_both(sc, 50)
    fluid = sc.beta == 1
    for k in ("u", "v", "w", "c"):
        assert rel_l2(got[k], getattr(st, k), fluid) < 1e-4, (k, rel_l2(got[k], getattr(st, k), fluid))
    unorm = np.sqrt(2 * diags[-1]["ke"])
    excess = (dg["div_l2"] - diags[-1]["div_l2"]) * min(sc.spacing) / unorm
    assert excess < 1e-7, excess
    assert abs(dg["co2_room_mean"] / diags[-1]["co2_room_mean"] - 1) < 1e-6
    assert abs(dg["t"] / diags[-1]["t"] - 1) < 1e-6


def test_fp32_channel_case_close_to_oracle():
    """FP32 form on the obstacle-in-channel case (2D, masked walls and
    obstacle, forced inflow) against the FP64 oracle over 30 steps: fluid-cell
    fields to FP32 rounding level."""
    torch, m = need_gpu()
    sc = scenarios.cube_channel(8)
    announce("fp32 channel case x30 vs oracle")
    S = m.Solver(sc, precision=m.FP32_REFINE)
    S.step(30, diag=False)
    got = S.state()
    S.close()
    O = Oracle.from_scenario(sc)
    st, _ = O.run(Oracle.state_from_scenario(sc), 30)
    fluid = sc.beta == 1
    for k in ("u", "v"):
        a, b = got[k][fluid], getattr(st, k)[fluid]
        assert np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)) < 1e-4, k
