"""Parity at the benchmark sizes, whole steps, through the C ABI.

* The ventilated room 256x128x96, FP64, 100 steps against the FP64 oracle:
  every field and every step's diagnostics to 1e-10 relative (the stated bar
  of the FP64 path on the scheme of Sections 2.1-2.2).
* The large room 512x256x192, FP64, 3 steps against the oracle, to 1e-10.
* The hall 1024x512x256: the FP32 form with FP64 refinement against the FP64
  path over 500 steps (field rel L2 <= 1e-4 at 50 steps, divergence excess
  <= 1e-7 of the velocity-gradient scale at every step, mean CO2 and its
  decrease within 1%).

The oracle takes seconds to a minute per step at these sizes, so its results
are stored under tests/golden/ (sampled cells, plane norms and every step's
diagnostics), written by tests/golden/make_fullsize_refs.py, which calls only
the oracle and the scenario generator.
"""
import os

import numpy as np
import pytest

import scenarios
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

DIAG_KEYS = ("t", "dt", "ke", "co2_mass", "co2_room_mean", "cfl_max")
FIELDS = ("u", "v", "w", "p", "c")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_l2(a, b, mask):
    a = a[mask]
    b = b[mask]
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b * b), 1e-300)))


def load_ref(case):
    path = os.path.join(GOLDEN, f"fullsize_{case}.npz")
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: run tests/golden/make_fullsize_refs.py {case}")
    z = np.load(path)
    keys = [str(k) for k in z["keys"]]
    diags = [dict(zip(keys, row)) for row in z["diags"]]
    for d in diags:
        d["step"] = int(d["step"])
    return z, diags


def compare_with_ref(sc, case, tol):
    """Run the FP64 path from the scenario's initial state for the stored
    number of steps and compare it with the oracle's stored results:
    sampled cells (max error over the sample relative to the field's max),
    the L2 norm of every z-plane and x-plane (bounded by the same max-norm
    bar: |norm_got - norm_ref| <= ||got - ref||_2 <= sqrt(n_plane) tol max|ref|),
    and every step's diagnostics."""
    torch, m = need_gpu()
    z, ref_diags = load_ref(case)
    nsteps = int(z["steps"])
    assert tuple(z["shape"]) == sc.shape
    S = m.Solver(sc)
    S.step(nsteps, diag=False)
    hist = S.read_diags(nsteps)
    got = S.state()
    S.close()
    torch.cuda.empty_cache()
    idx = z["idx"]
    errs = {}
    for k in FIELDS:
        g = np.asarray(got[k], dtype=np.float64)
        scale = float(z[k + "_max"])
        errs[k] = float(np.abs(g.reshape(-1)[idx] - z[k + "_samp"]).max() / scale)
        for ax, key, n_plane in (((1, 2), "_zl2", sc.nx * sc.ny), ((0, 1), "_xl2", sc.ny * sc.nz)):
            nrm = np.sqrt(np.sum(g * g, axis=ax))
            bound = np.sqrt(n_plane) * tol * scale
            worst = float(np.abs(nrm - z[k + key]).max())
            assert worst <= bound, (k, key, worst, bound)
    print(f"[full-size] {sc.name} {nsteps} steps: sampled field errors {errs}", flush=True)
    for k, e in errs.items():
        assert e < tol, (k, errs)
    floor_scale = 1e-12 / min(sc.spacing)
    worst = {}
    assert len(hist) == len(ref_diags)
    for h, r in zip(hist, ref_diags):
        assert h["step"] == r["step"]
        for k in DIAG_KEYS:
            e = abs(h[k] - r[k]) / max(abs(r[k]), 1e-300)
            worst[k] = max(worst.get(k, 0.0), e)
            assert abs(h[k] - r[k]) <= tol * max(abs(r[k]), 1e-300), (h["step"], k, h[k], r[k])
        floor = floor_scale * np.sqrt(2 * r["ke"])
        assert abs(h["div_l2"] - r["div_l2"]) <= tol * r["div_l2"] + floor, (h["step"], h["div_l2"], r["div_l2"])
    print(f"[full-size] {sc.name} worst diagnostic errors {worst}", flush=True)


def test_room_fp64_100_steps_vs_oracle():
    """256x128x96 room (duct forcing, 8 boxes, filter, CFL dt): 100 steps."""
    need_gpu()
    sc = scenarios.room()
    announce("full-size room 256x128x96 x100 vs oracle")
    compare_with_ref(sc, "room100", 1e-10)


def test_large_room_fp64_3_steps_vs_oracle():
    """512x256x192 room: 3 whole steps of the FP64 path against the oracle."""
    need_gpu()
    sc = scenarios.room(512, 256, 192, dx=10.0 / 512)
    announce("full-size large room 512x256x192 x3 vs oracle")
    compare_with_ref(sc, "large3", 1e-10)


def test_hall_fp32_refine_vs_fp64_500_steps():
    """1024x512x256 hall: the FP32 form against the FP64 path."""
    torch, m = need_gpu()
    sc = scenarios.hall()
    announce("hall 1024x512x256 fp32 vs fp64 x500")
    fluid = sc.beta == 1
    res = {}
    for prec in (m.FP64, m.FP32_REFINE):
        S = m.Solver(sc, precision=prec)
        S.step(50, diag=False)
        st50 = S.state()
        S.step(450, diag=False)
        hist = S.read_diags(500)
        S.close()
        torch.cuda.empty_cache()
        res[prec] = (st50, hist)
        print(f"[full-size] hall precision {prec}: 500 steps, t = {hist[-1]['t']:.4f} s", flush=True)
    s64, h64 = res[m.FP64]
    s32, h32 = res[m.FP32_REFINE]
    errs = {k: rel_l2(s32[k], s64[k], fluid) for k in ("u", "v", "w", "p", "c")}
    print(f"[full-size] hall rel L2 at 50 steps: {errs}", flush=True)
    for k, e in errs.items():
        assert e < 1e-4, (k, errs)
    dmin = min(sc.spacing)
    excess = max((a["div_l2"] - b["div_l2"]) * dmin / np.sqrt(2 * b["ke"]) for a, b in zip(h32, h64))
    print(f"[full-size] hall divergence excess {excess:.3e}", flush=True)
    assert excess < 1e-7
    c64 = np.array([h["co2_room_mean"] for h in h64])
    c32 = np.array([h["co2_room_mean"] for h in h32])
    assert np.max(np.abs(c32 / c64 - 1)) < 0.01
    c_init = float(np.sum(sc.c * sc.beta * sc.room_mask) / np.sum(sc.beta * sc.room_mask))
    drop64, drop32 = c_init - c64[-1], c_init - c32[-1]
    print(f"[full-size] hall mean CO2 drop over 500 steps: FP64 {drop64:.6f} ppm, FP32 {drop32:.6f} ppm", flush=True)
    assert drop64 > 0
    assert abs(drop32 / drop64 - 1) < 0.01
