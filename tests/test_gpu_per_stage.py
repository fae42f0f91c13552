"""The per-stage projection variant (a projection after every RK4 stage, the
alternative that Section 2.1 mentions and skips for speed) against the oracle's
same variant, and against the closed form it makes exact on the 2D
Taylor-Green vortex."""
import numpy as np
import pytest

from oracle.step import Oracle
import scenarios
from gpu_util import announce, need_gpu, rel_err
from test_gpu_parity import make_case

pytestmark = pytest.mark.gpu


def R4(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def run_both(sc, nsteps, precision=None):
    torch, m = need_gpu()
    S = m.Solver(sc, precision=m.FP64 if precision is None else precision, project_each_stage=True)
    dg = S.step(nsteps)
    got = S.state()
    S.close()
    O = Oracle.from_scenario(sc)
    st, diags = O.run(Oracle.state_from_scenario(sc), nsteps, project_each_stage=True)
    return got, dg, st, diags


def test_per_stage_tgv2d_exact():
    """2D Taylor-Green, 16 x 16: the step reduces to RK4 of the viscous decay,
    u(t_n) = u0 R(z)^n with z the discrete viscous eigenvalue times dt."""
    torch, m = need_gpu()
    n = 16
    h = 2 * np.pi / n
    x = np.arange(n) * h
    Y, X = np.meshgrid(x, x, indexing="ij")
    z0 = np.zeros((1, n, n))
    sc = scenarios.Scenario(
        name="tgv2d", nx=n, ny=n, nz=1, lx=2 * np.pi, ly=2 * np.pi, lz=1.0, nu=0.05, alpha_c=0.0, tau_f=1.0,
        body=(0.0, 0.0, 0.0), cfl=0.3, dt_fixed=0.05, u_ref=1.0, n_piter=4, filter=False,
        beta=np.ones((1, n, n), np.uint8), forced_idx=np.zeros(0, np.int64), forced_S=np.zeros(0),
        forced_uset=np.zeros((0, 3)), forced_cset=np.zeros(0), room_mask=None,
        u=(np.sin(X) * np.cos(Y))[None].copy(), v=(-np.cos(X) * np.sin(Y))[None].copy(), w=z0.copy(),
        p=z0.copy(), c=z0.copy())
    announce("per-stage tgv2d")
    S = m.Solver(sc, project_each_stage=True)
    nst = 5
    S.step(nst)
    got = S.state()
    S.close()
    z = -0.05 * 0.05 * 2 * 4 * np.sin(h / 2) ** 2 / h ** 2
    np.testing.assert_allclose(got["u"], sc.u * R4(z) ** nst, atol=1e-14)
    np.testing.assert_allclose(got["v"], sc.v * R4(z) ** nst, atol=1e-14)


def test_per_stage_tgv3d_vs_oracle():
    sc = scenarios.taylor_green(32)
    announce("per-stage tgv32 x20")
    got, dg, st, diags = run_both(sc, 20)
    for k in ("u", "v", "w", "p"):
        assert rel_err(got[k], getattr(st, k)) < 1e-10, k
    assert abs(dg["ke"] - diags[-1]["ke"]) < 1e-10 * diags[-1]["ke"]


@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 36, 24)])
def test_per_stage_masked_vs_oracle(shape):
    sc = make_case(shape, 23)
    for k in ("u", "v", "w"):
        setattr(sc, k, getattr(sc, k) * 0.1)
    announce(f"per-stage masked {shape}")
    got, dg, st, diags = run_both(sc, 4)
    for k in ("u", "v", "w", "p", "c"):
        assert rel_err(got[k], getattr(st, k)) < 1e-10, k


def test_per_stage_room_vs_oracle():
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("per-stage room 64x48x36 x5")
    got, dg, st, diags = run_both(sc, 5)
    for k in ("u", "v", "w", "p", "c"):
        assert rel_err(got[k], getattr(st, k)) < 1e-10, k
    for k in ("t", "dt", "ke", "co2_room_mean"):
        assert abs(dg[k] - diags[-1][k]) <= 1e-10 * abs(diags[-1][k]), k


def test_per_stage_fp32_refine_close_to_fp64():
    """FP32 form with the per-stage variant (each projection refined in FP64)
    against the FP64 oracle's per-stage run: FP32 rounding level."""
    torch, m = need_gpu()
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("per-stage fp32 room 64x48x36 x5")
    got, dg, st, diags = run_both(sc, 5, precision=m.FP32_REFINE)
    fluid = sc.beta == 1
    for k in ("u", "v", "w", "c"):
        a, b = got[k][fluid], getattr(st, k)[fluid]
        assert np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)) < 1e-4, k
