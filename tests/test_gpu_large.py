"""Parity and accuracy at the full sizes of the large room (512x256x192,
25M cells) and the hall (1024x512x256, 134M cells).

The oracle cannot run whole steps at these sizes in a test, so:
  * the local operators (momentum and scalar right-hand sides, filter) are
    compared at sampled cells, the oracle evaluating its own operators on the
    periodic neighbourhood patch of each sampled cell;
  * the FFT Poisson solve is checked through its residual at sampled cells:
    div grad p must equal the right-hand side minus its null-mode part;
  * the FP32 form is checked against the FP64 GPU path (itself pinned to the
    oracle by the parity tests) over a 50-step horizon and, for the mean CO2
    decay and the air-change rate it implies, over 1000 steps.
"""
import numpy as np
import pytest

from oracle import ops
from oracle.step import momentum_rhs, scalar_rhs
import scenarios
from gpu_util import announce, need_gpu, to_np

pytestmark = pytest.mark.gpu


def sample_cells(sc, n, seed):
    rng = np.random.default_rng(seed)
    shape = sc.shape
    near = np.zeros(shape, bool)
    b = sc.beta == 0
    for ax in range(3):
        near |= np.roll(b, 1, axis=ax) | np.roll(b, -1, axis=ax)
    pick = [rng.integers(0, sc.ncells, n)]
    nz = np.flatnonzero(near.ravel())
    pick.append(rng.choice(nz, min(n // 4, len(nz)), replace=False))
    if len(sc.forced_idx):
        pick.append(rng.choice(sc.forced_idx, min(n // 8, len(sc.forced_idx)), replace=False))
    flat = np.unique(np.concatenate(pick))
    return np.stack(np.unravel_index(flat, shape), axis=1)      # (ns, 3) as (k, j, i)


def patch(arr, kji, r):
    nz, ny, nx = arr.shape
    off = np.arange(-r, r + 1)
    K = (kji[:, 0, None] + off) % nz
    J = (kji[:, 1, None] + off) % ny
    I = (kji[:, 2, None] + off) % nx
    return arr[K[:, :, None, None], J[:, None, :, None], I[:, None, None, :]]


def dense_forcing(sc):
    n = sc.ncells
    S = np.zeros(n)
    S[sc.forced_idx] = sc.forced_S
    us = np.zeros((3, n))
    for a in range(3):
        us[a, sc.forced_idx] = sc.forced_uset[:, a]
    cs = np.zeros(n)
    cs[sc.forced_idx] = sc.forced_cset
    return S.reshape(sc.shape), [x.reshape(sc.shape) for x in us], cs.reshape(sc.shape)


def random_state(sc, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    b = sc.beta.astype(np.float64)
    u = [rng.standard_normal(sc.shape) * scale * b for _ in range(3)]
    c = (400 + 600 * rng.random(sc.shape)) * b
    return u, c


@pytest.mark.parametrize("which", ["large", "hall"])
def test_local_operators_sampled_full_size(which):
    torch, m = need_gpu()
    sc = scenarios.room(512, 256, 192, dx=10.0 / 512) if which == "large" else scenarios.hall()
    announce(f"sampled operators {which} {sc.shape}")
    u, c = random_state(sc, 3)
    S = m.Solver(sc)
    fu = [to_np(t) for t in S.momentum_rhs(*u)]
    gc = to_np(S.scalar_rhs(c, *u))
    fc = to_np(S.filter(c))
    S.close()
    torch.cuda.empty_cache()
    kji = sample_cells(sc, 1200, 5)
    Sd, usd, csd = dense_forcing(sc)
    d = sc.spacing
    P1 = lambda a: patch(a, kji, 1)
    up, bp, Sp, cp = [P1(x) for x in u], P1(sc.beta), P1(Sd), P1(c)
    usp, csp = [P1(x) for x in usd], P1(csd)
    cp3, bp3 = patch(c, kji, 3), patch(sc.beta, kji, 3)
    err_f = err_g = err_filt = 0.0
    scale_f = max(np.abs(x).max() for x in fu)
    scale_g = np.abs(gc).max()
    for s in range(len(kji)):
        k, j, i = kji[s]
        F = momentum_rhs([up[a][s] for a in range(3)], bp[s], Sp[s], [usp[a][s] for a in range(3)],
                         sc.body, sc.nu, sc.tau_f, d)
        for a in range(3):
            err_f = max(err_f, abs(F[a][1, 1, 1] - fu[a][k, j, i]))
        G = scalar_rhs(cp[s], [up[a][s] for a in range(3)], bp[s], Sp[s], csp[s], sc.alpha_c, sc.tau_f, d)
        err_g = max(err_g, abs(G[1, 1, 1] - gc[k, j, i]))
        Fc = bp3[s][3, 3, 3] * ops.filter6(cp3[s], d)[3, 3, 3]
        err_filt = max(err_filt, abs(Fc - fc[k, j, i]))
    assert err_f < 1e-12 * scale_f, err_f / scale_f
    assert err_g < 1e-12 * scale_g, err_g / scale_g
    assert err_filt < 1e-13 * np.abs(c).max()


def null_part(r):
    """Component of r on the modes every m_a of which is 0 or N_a/2."""
    nz, ny, nx = r.shape
    out = np.zeros_like(r)
    axes_modes = []
    for n in (nz, ny, nx):
        axes_modes.append([np.ones(n)] + ([(-1.0) ** np.arange(n)] if n % 2 == 0 and n > 1 else []))
    for pz in axes_modes[0]:
        for py in axes_modes[1]:
            for px in axes_modes[2]:
                pat = pz[:, None, None] * py[None, :, None] * px[None, None, :]
                out += pat * (np.sum(r * pat) / r.size)
    return out


@pytest.mark.parametrize("which", ["hall", "large"])
def test_poisson_residual_full_size(which):
    """FP64 solve: div grad p equals the right-hand side less its null-mode
    part at sampled cells (the residual of a random right-hand side is
    amplified by at most the symbol's range, ~0.1 N^2, times FP64 rounding)."""
    torch, m = need_gpu()
    sc = scenarios.room(512, 256, 192, dx=10.0 / 512) if which == "large" else scenarios.hall()
    announce(f"poisson residual {which}")
    S = m.Solver(sc)
    r = np.random.default_rng(9).standard_normal(sc.shape)
    p = to_np(S.poisson(r))
    S.close()
    torch.cuda.empty_cache()
    rr = r - null_part(r)
    kji = sample_cells(sc, 4000, 7)
    pp = patch(p, kji, 2)
    d = sc.spacing
    lap = ((pp[:, 2, 2, 4] - 2 * pp[:, 2, 2, 2] + pp[:, 2, 2, 0]) / (4 * d[0] ** 2)
           + (pp[:, 2, 4, 2] - 2 * pp[:, 2, 2, 2] + pp[:, 2, 0, 2]) / (4 * d[1] ** 2)
           + (pp[:, 4, 2, 2] - 2 * pp[:, 2, 2, 2] + pp[:, 0, 2, 2]) / (4 * d[2] ** 2))
    target = rr[kji[:, 0], kji[:, 1], kji[:, 2]]
    assert np.abs(lap - target).max() < 1e-10 * np.abs(rr).max()


def test_poisson_fp32_vs_fp64_large():
    """The FP32 solve against the FP64 one at full large-room size."""
    torch, m = need_gpu()
    sc = scenarios.room(512, 256, 192, dx=10.0 / 512)
    announce("poisson fp32 vs fp64 large")
    r = np.random.default_rng(10).standard_normal(sc.shape)
    out = {}
    for prec in (m.FP64, m.FP32_REFINE):
        S = m.Solver(sc, precision=prec)
        out[prec] = to_np(S.poisson(r))
        S.close()
        torch.cuda.empty_cache()
    err = np.abs(out[m.FP32_REFINE] - out[m.FP64]).max() / np.abs(out[m.FP64]).max()
    assert err < 1e-5, err


def rel_l2(a, b, mask):
    a = a[mask]
    b = b[mask]
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b * b), 1e-300)))


@pytest.mark.parametrize("u_in", [1.0, 0.1])
def test_large_room_fp32_vs_fp64(u_in):
    """512x256x192 room: FP32 with FP64 refinement against the FP64 path.
    50-step horizon: rel L2 <= 1e-4 per field over fluid cells, divergence
    excess <= 1e-7; 1000 steps: mean CO2 and the implied air-change rate
    within 1%."""
    torch, m = need_gpu()
    sc = scenarios.room(512, 256, 192, dx=10.0 / 512, u_in=u_in)
    announce(f"large fp32 vs fp64 u_in={u_in}")
    res = {}
    for prec in (m.FP64, m.FP32_REFINE):
        S = m.Solver(sc, precision=prec)
        d50 = S.step(50)
        st50 = S.state()
        S.step(950, diag=False)
        hist = S.read_diags(1000)
        S.close()
        torch.cuda.empty_cache()
        res[prec] = (d50, st50, hist)
    fluid = sc.beta == 1
    d64, s64, h64 = res[m.FP64]
    d32, s32, h32 = res[m.FP32_REFINE]
    for k in ("u", "v", "w", "c"):
        assert rel_l2(s32[k], s64[k], fluid) < 1e-4, k
    unorm = np.sqrt(2 * d64["ke"])
    assert (d32["div_l2"] - d64["div_l2"]) * min(sc.spacing) / unorm < 1e-7
    c64 = np.array([h["co2_room_mean"] for h in h64])
    c32 = np.array([h["co2_room_mean"] for h in h32])
    t64 = np.array([h["t"] for h in h64])
    assert np.max(np.abs(c32 / c64 - 1)) < 0.01

    def ach(cm, t):
        # decay rate of (<c> - 400 ppm) fitted over the run, per hour
        y = np.log(cm - 400.0)
        A = np.vstack([t, np.ones_like(t)]).T
        return -np.linalg.lstsq(A, y, rcond=None)[0][0] * 3600.0

    a64, a32 = ach(c64, t64), ach(c32, np.array([h["t"] for h in h32]))
    assert a64 > 0
    assert abs(a32 / a64 - 1) < 0.01, (a32, a64)
