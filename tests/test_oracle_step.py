"""Pins of the oracle's time step against closed forms and invariants.

Each case has an exact answer that follows from the mathematics of the scheme
(RK4 amplification factors, exact discrete steady states, conservation laws),
so a dropped term, a wrong sign or coefficient, or a misplaced mask fails one.
"""
import numpy as np
import pytest

import oracle
from oracle import ops
from oracle.step import Oracle, OracleParams, OracleState
import scenarios


def R4(z):
    """Classical RK4 amplification polynomial."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def make(shape, lengths, **kw):
    nz, ny, nx = shape
    base = dict(nx=nx, ny=ny, nz=nz, lx=lengths[0], ly=lengths[1], lz=lengths[2], nu=0.01,
                alpha_c=0.01, tau_f=1.0, body=(0.0, 0.0, 0.0), cfl=0.5, dt_fixed=0.01,
                u_ref=1.0, n_piter=4, filter=False)
    beta = kw.pop("beta", np.ones(shape, np.uint8))
    forced = kw.pop("forced", (np.zeros(0, np.int64), np.zeros(0), np.zeros((0, 3)), np.zeros(0)))
    base.update(kw)
    return Oracle(OracleParams(**base), beta, *forced)


def zeros(shape):
    return np.zeros(shape)


@pytest.mark.parametrize("filt", [False, True])
def test_shear_mode_rk4_amplification(filt):
    """v = A sin(k x): convection vanishes identically and the field is
    divergence-free, so the step is the RK4 of the discrete viscous decay,
    times the filter gain when the filter is on."""
    shape = (4, 6, 16)
    L = (2 * np.pi, 1.0, 1.0)
    O = make(shape, L, nu=0.05, dt_fixed=0.02, filter=filt)
    dx = L[0] / shape[2]
    x = np.arange(shape[2]) * dx
    kx = 3
    v0 = np.broadcast_to(2.0 * np.sin(kx * x), shape).copy()
    s = OracleState(zeros(shape), v0.copy(), zeros(shape), zeros(shape), zeros(shape))
    n = 7
    s, _ = O.run(s, n)
    th = kx * dx
    z = -0.05 * 0.02 * 4 * np.sin(th / 2) ** 2 / dx ** 2
    g = (1 - 64 * np.sin(th / 2) ** 6 / np.pi ** 6) if filt else 1.0
    np.testing.assert_allclose(s.v, v0 * (R4(z) * g) ** n, rtol=0, atol=1e-14)
    assert np.all(s.u == 0) and np.all(s.w == 0)


def test_uniform_forcing_relaxation():
    """Uniform fields forced everywhere with S = 1 relax as
    u = u_set + (u0 - u_set) R4(-dt/tau)^n, likewise c."""
    shape = (3, 4, 5)
    n = int(np.prod(shape))
    uset = np.array([0.3, -0.2, 0.7])
    forced = (np.arange(n, dtype=np.int64), np.ones(n), np.tile(uset, (n, 1)), np.full(n, 400.0))
    O = make(shape, (1.0, 1.0, 1.0), tau_f=0.05, dt_fixed=0.02, forced=forced)
    u0 = np.array([1.0, 2.0, -1.0])
    s = OracleState(*(np.full(shape, u0[i]) for i in range(3)), zeros(shape), np.full(shape, 1000.0))
    nst = 5
    s, _ = O.run(s, nst)
    r = R4(-0.02 / 0.05) ** nst
    for i, f in enumerate((s.u, s.v, s.w)):
        np.testing.assert_allclose(f, uset[i] + (u0[i] - uset[i]) * r, rtol=1e-14)
    np.testing.assert_allclose(s.c, 400 + 600 * r, rtol=1e-14)


def test_constant_body_force_is_exact():
    shape = (3, 4, 5)
    b = (0.1, -0.3, 0.25)
    O = make(shape, (1.0, 1.0, 1.0), body=b, dt_fixed=0.1)
    s = OracleState(zeros(shape), zeros(shape), zeros(shape), zeros(shape), zeros(shape))
    s, _ = O.run(s, 4)
    for i, f in enumerate((s.u, s.v, s.w)):
        np.testing.assert_allclose(f, 4 * 0.1 * b[i], rtol=1e-14)


def test_channel_poiseuille_fixed_point():
    """The discrete parabola U_j = b/(2 nu) y_j (D - y_j) (y from the last solid
    cell centre, D = (fluid cells + 1) dy) is an exact steady state of the
    masked, body-force-driven step (Section 3.1.1 channel)."""
    sc = scenarios.channel2d(ny_fluid=14, nx=6, wall=2, nu=0.02, bx=3e-3, dt=0.05)
    O = Oracle.from_scenario(sc)
    wall = sc.meta["wall"]
    nf = sc.ny - wall
    dy = sc.ly / sc.ny
    D = (nf + 1) * dy
    j = np.arange(sc.ny)
    y = (j - (wall - 1)) * dy
    U = np.where(j >= wall, sc.body[0] / (2 * sc.nu) * y * (D - y), 0.0)
    u0 = np.broadcast_to(U[None, :, None], sc.shape).copy()
    s = OracleState(u0.copy(), zeros(sc.shape), zeros(sc.shape), zeros(sc.shape), zeros(sc.shape))
    s, dg = O.run(s, 3)
    np.testing.assert_allclose(s.u, u0, rtol=0, atol=1e-14 * U.max())
    assert np.all(s.v == 0) and np.all(s.w == 0)
    # bulk velocity of the discrete profile tends to U_b = b D^2 / (12 nu)
    ub = U[wall:].mean()
    assert abs(ub / (sc.body[0] * D ** 2 / (12 * sc.nu)) - (nf + 2) / (nf + 1)) < 1e-13


def test_scalar_sine_mode_under_uniform_flow():
    """c = Re(A e^{i k x}) advected by uniform U and diffused: exact RK4 with the
    complex symbol z = dt(-i U sin(th)/dx - 4 alpha sin^2(th/2)/dx^2)."""
    shape = (2, 3, 12)
    L = (3.0, 1.0, 1.0)
    O = make(shape, L, alpha_c=0.02, dt_fixed=0.03)
    dx = L[0] / shape[2]
    x = np.arange(shape[2]) * dx
    m = 2
    th = 2 * np.pi * m / shape[2]
    kx = th / dx
    U = 0.8
    c0 = np.broadcast_to(np.cos(kx * x), shape).copy()
    s = OracleState(np.full(shape, U), zeros(shape), zeros(shape), zeros(shape), c0.copy())
    nst = 6
    s, _ = O.run(s, nst)
    z = 0.03 * (-1j * U * np.sin(th) / dx - 0.02 * 4 * np.sin(th / 2) ** 2 / dx ** 2)
    ref = np.real(np.exp(1j * kx * x) * R4(z) ** nst)
    np.testing.assert_allclose(s.c[0, 0], ref, atol=1e-14)
    np.testing.assert_allclose(s.u, U, rtol=1e-15)


def test_scalar_conservation_masked_no_source():
    """With u = 0 and no source the masked diffusion conserves sum(beta c)."""
    shape = (6, 7, 8)
    beta = scenarios.random_beta(shape, 5, n_boxes=3, max_size=3)
    O = make(shape, (1.0, 1.2, 0.9), beta=beta, alpha_c=0.01, dt_fixed=0.01)
    c = np.random.default_rng(2).random(shape) * beta
    s = OracleState(zeros(shape), zeros(shape), zeros(shape), zeros(shape), c.copy())
    s, _ = O.run(s, 5)
    assert abs(np.sum(s.c) - np.sum(c)) < 1e-13 * np.sum(c)


def test_projection_unmasked_divergence_free_and_idempotent():
    shape = (8, 10, 12)
    d = (0.3, 0.25, 0.4)
    O = make(shape, (12 * d[0], 10 * d[1], 8 * d[2]))
    rng = np.random.default_rng(9)
    us = [rng.standard_normal(shape) for _ in range(3)]
    u, p = O.project(us, zeros(shape))
    du = ops.div(u, d)
    scale = np.sqrt(sum(np.sum(ops.ddx(us[a], a, d) ** 2) for a in range(3)))
    assert np.sqrt(np.sum(du ** 2)) / scale < 1e-14
    u2, _ = O.project(u, zeros(shape))
    for a in range(3):
        np.testing.assert_allclose(u2[a], u[a], atol=1e-13)
    # orthogonal projection: energy does not increase; gradients are removed
    assert sum(np.sum(x * x) for x in u) <= sum(np.sum(x * x) for x in us)
    q = rng.standard_normal(shape)
    g, _ = O.project(ops.grad(q, d), zeros(shape))
    assert max(np.abs(x).max() for x in g) < 1e-12


def test_ib_iteration_unmasked_iterates_identical():
    shape = (6, 8, 10)
    O = make(shape, (1.0, 1.0, 1.0))
    rng = np.random.default_rng(3)
    us = [rng.standard_normal(shape) for _ in range(3)]
    its = O.pressure(us, rng.standard_normal(shape))
    for k in range(1, 4):
        assert np.array_equal(its[k], its[0])


def _masked_dense_solution(O, ustar):
    """Solve div(beta grad p) = div u* by dense least squares (tiny grid) and
    remove the null-mode components."""
    shape = O.P.shape
    d = O.P.d
    b = O.beta.astype(np.float64)
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1
        g = ops.grad(e.reshape(shape), d)
        A[:, col] = ops.div([b * g[0], b * g[1], b * g[2]], d).ravel()
    r0 = ops.div(ustar, d).ravel()
    p = np.linalg.lstsq(A, r0, rcond=None)[0].reshape(shape)
    assert np.abs(A @ p.ravel() - r0).max() < 1e-9 * np.abs(r0).max()
    ph = np.fft.rfftn(p)
    _, null = ops.poisson_symbol(shape, d)
    ph[null] = 0
    return np.fft.irfftn(ph, s=shape, axes=(0, 1, 2))


def test_ib_iteration_fixed_point_and_monotone_error():
    """Section 2.2: the fixed point of the iteration solves div(beta grad p) =
    div u*.  The exact solution (dense) is left unchanged by an iteration, and
    from a cold start the error in grad p never grows."""
    shape = (4, 6, 8)
    beta = scenarios.random_beta(shape, 11, n_boxes=2, max_size=2)
    O = make(shape, (1.0, 1.5, 0.8), beta=beta)
    rng = np.random.default_rng(4)
    us = [rng.standard_normal(shape) * beta for _ in range(3)]
    pfp = _masked_dense_solution(O, us)
    its = O.pressure(us, pfp, n_iter=1)
    np.testing.assert_allclose(its[0], pfp, atol=1e-10 * np.abs(pfp).max())
    d = O.P.d
    its = O.pressure(us, zeros(shape), n_iter=30)
    errs = [np.sqrt(sum(np.sum(g * g) for g in ops.grad(p - pfp, d))) for p in its]
    assert all(errs[k + 1] <= errs[k] * (1 + 1e-12) for k in range(len(errs) - 1))
    # the velocity correction in the fluid converges to the exact one
    bg = [beta * g for g in ops.grad(its[-1] - pfp, d)]
    e0 = np.sqrt(sum(np.sum((beta * g) ** 2) for g in ops.grad(pfp, d)))
    assert np.sqrt(sum(np.sum(x * x) for x in bg)) < 0.05 * e0


def _central_difference_matrices(shape, d):
    """Periodic central first differences (p[i+1] - p[i-1]) / (2 d_a) along x, y
    and z as dense matrices, entry by entry from the cell indices (no use of
    the oracle's stencils)."""
    nz, ny, nx = shape
    n = nx * ny * nz
    mats = []
    for a, (na, da) in enumerate(zip((nx, ny, nz), d)):
        G = np.zeros((n, n))
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    row = (k * ny + j) * nx + i
                    c = [i, j, k]
                    for sgn in (1, -1):
                        q = list(c)
                        q[a] = (q[a] + sgn) % na
                        G[row, (q[2] * ny + q[1]) * nx + q[0]] += sgn / (2.0 * da)
        mats.append(G)
    return mats


@pytest.mark.parametrize("n_iter", [1, 4])
def test_ib_iterates_equal_dense_iteration(n_iter):
    """Section 2.2: each iterate is the minimum-norm solution of
    Div Grad p^{k+1} = Div u* + Div((1 - beta) Grad p^k).  With Div, Grad and
    the pseudo-inverse written as dense matrices on a tiny masked grid, the
    oracle's n iterates from a random warm start must match one by one (the
    null modes of Div Grad carry no pressure in either)."""
    shape = (4, 5, 6)
    d = (0.3, 0.45, 0.7)
    beta = scenarios.random_beta(shape, 21, n_boxes=2, max_size=2)
    O = make(shape, (d[0] * shape[2], d[1] * shape[1], d[2] * shape[0]), beta=beta)
    assert np.allclose(O.P.d, d)
    rng = np.random.default_rng(22)
    us = [rng.standard_normal(shape) * beta for _ in range(3)]
    p = rng.standard_normal(shape).ravel()
    G = _central_difference_matrices(shape, d)
    omb = np.diag(1.0 - beta.astype(np.float64).ravel())
    A = sum(Ga @ Ga for Ga in G)
    M = sum(Ga @ omb @ Ga for Ga in G)
    r0 = sum(Ga @ u.ravel() for Ga, u in zip(G, us))
    Ainv = np.linalg.pinv(A)
    its = O.pressure(us, p.reshape(shape), n_iter=n_iter)
    assert len(its) == n_iter
    for got in its:
        p = Ainv @ (r0 + M @ p)
        np.testing.assert_allclose(got.ravel(), p, atol=1e-11 * np.abs(p).max())


def test_tgv3d_early_decay():
    """3D Taylor-Green, 32^3, Re = 100: kinetic energy follows the viscous
    decay of the discrete Laplacian to within 1e-3 at t = 0.1 (convection
    starts the cascade only at later times)."""
    sc = scenarios.taylor_green(32)
    O = Oracle.from_scenario(sc)
    s = Oracle.state_from_scenario(sc)
    h = 2 * np.pi / 32
    e0 = 0.5 * np.sum(sc.u ** 2 + sc.v ** 2) * h ** 3
    s, dg = O.run(s, 10)
    rate = 3 * 4 * np.sin(h / 2) ** 2 / h ** 2       # discrete eigenvalue of the mode
    ref = e0 * np.exp(-2 * sc.nu * rate * 0.1)
    assert abs(dg[-1]["ke"] / ref - 1) < 1e-3
    assert dg[-1]["div_l2"] < 1e-12


def test_tgv2d_per_stage_projection_exact():
    """2D Taylor-Green: with a projection after every stage the convection
    (a discrete gradient on an isotropic grid) is removed exactly and the
    step is the RK4 of the viscous decay (the 4th-order variant of Section 2.1)."""
    n = 16
    h = 2 * np.pi / n
    shape = (1, n, n)
    O = make(shape, (2 * np.pi, 2 * np.pi, 1.0), nu=0.05, dt_fixed=0.05)
    x = np.arange(n) * h
    Y, X = np.meshgrid(x, x, indexing="ij")
    u0 = (np.sin(X) * np.cos(Y))[None]
    v0 = (-np.cos(X) * np.sin(Y))[None]
    s = OracleState(u0.copy(), v0.copy(), zeros(shape), zeros(shape), zeros(shape))
    nst = 5
    s, _ = O.run(s, nst, project_each_stage=True)
    z = -0.05 * 0.05 * 2 * 4 * np.sin(h / 2) ** 2 / h ** 2
    np.testing.assert_allclose(s.u, u0 * R4(z) ** nst, atol=1e-14)
    np.testing.assert_allclose(s.v, v0 * R4(z) ** nst, atol=1e-14)


def test_courant_time_step():
    shape = (3, 4, 5)
    O = make(shape, (1.0, 2.0, 0.5), dt_fixed=0.0, cfl=0.3, u_ref=0.1)
    u = [np.zeros(shape) for _ in range(3)]
    d = O.P.d
    # at rest the floor u_ref/min(dx) sets dt
    assert O.dt_for(u) == 0.3 / (0.1 / min(d))
    u[0][1, 2, 3] = 2.0
    u[2][1, 2, 3] = -1.0
    u[1][0, 0, 0] = 5.0
    rate = max(2.0 / d[0] + 1.0 / d[2], 5.0 / d[1])
    assert O.dt_for(u) == 0.3 / rate


def _golden(name):
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if len(line) == 2:
                vals[line[0]] = float(line[1])
    return vals


def test_channel_at_table1_resolution():
    """Table 1 channel (D = 2 pi, walls 0.05 D, Ly = 1.1 D, 198 cells across,
    Re = 500 from Re = b D^3 / (12 nu^2)): the discrete parabola between the
    solid cells is an exact steady state of the oracle step, and its bulk
    velocity matches U_b = b D^2/(12 nu) up to the (n+2)/(n+1) factor of the
    cell-centred profile."""
    g = _golden("channel_table1.txt")
    D = g["channel_width_D"]
    ny = int(g["grid_y"])
    dy = g["Ly_over_D"] * D / ny
    nwall = int(round(2 * g["wall_width_over_D"] * D / dy))   # the two walls meet across the seam
    nf = ny - nwall
    nu = 0.01
    bx = g["Re"] * 12 * nu ** 2 / D ** 3
    sc = scenarios.channel2d(ny_fluid=nf, nx=4, wall=nwall, nu=nu, bx=bx, dt=0.02)
    sc.ly = ny * dy
    sc.lx = 4 * dy
    O = Oracle.from_scenario(sc)
    j = np.arange(ny)
    y = (j - (nwall - 1)) * dy
    De = (nf + 1) * dy
    U = np.where(j >= nwall, bx / (2 * nu) * y * (De - y), 0.0)
    u0 = np.broadcast_to(U[None, :, None], sc.shape).copy()
    s = OracleState(u0.copy(), zeros(sc.shape), zeros(sc.shape), zeros(sc.shape), zeros(sc.shape))
    s, _ = O.run(s, 2)
    np.testing.assert_allclose(s.u, u0, rtol=0, atol=1e-13 * U.max())
    ub = U[nwall:].mean()
    assert nf == 180
    assert abs(ub / (bx * De ** 2 / (12 * nu)) - (nf + 2) / (nf + 1)) < 1e-13
    # and the bulk Reynolds number on the printed width is the printed one
    assert abs(bx * D ** 3 / (12 * nu ** 2) - g["Re"]) < 1e-9


def test_projection_masks_solids():
    shape = (4, 6, 8)
    beta = scenarios.random_beta(shape, 21, n_boxes=2, max_size=3)
    O = make(shape, (1.0, 1.0, 1.0), beta=beta)
    rng = np.random.default_rng(5)
    us = [rng.standard_normal(shape) * beta for _ in range(3)]
    u, p = O.project(us, rng.standard_normal(shape))
    for a in range(3):
        assert np.all(u[a][beta == 0] == 0)
        g = ops.grad(p, O.P.d)[a]
        np.testing.assert_allclose(u[a][beta == 1], (us[a] - g)[beta == 1], rtol=1e-15, atol=1e-15)


def test_scalar_is_advected_by_projected_velocity():
    """Uniform velocity relaxing under S = 1 forcing, plus a scalar sine mode:
    the scalar RK4 sees the end-of-step velocity u^{n+1} (frozen), and its mean
    relaxes to c_set.  Exact affine RK4 per step."""
    shape = (2, 2, 12)
    n = int(np.prod(shape))
    L = (3.0, 1.0, 1.0)
    tau, dt, alpha = 0.2, 0.03, 0.02
    uset = np.array([0.5, 0.0, 0.0])
    forced = (np.arange(n, dtype=np.int64), np.ones(n), np.tile(uset, (n, 1)), np.full(n, 2.0))
    O = make(shape, L, tau_f=tau, dt_fixed=dt, alpha_c=alpha, forced=forced)
    dx = L[0] / shape[2]
    x = np.arange(shape[2]) * dx
    th = 2 * np.pi * 1 / shape[2]
    kx = th / dx
    U0 = 1.5
    cbar0 = 1.0
    c0 = np.broadcast_to(cbar0 + np.cos(kx * x), shape).copy()
    s = OracleState(np.full(shape, U0), zeros(shape), zeros(shape), zeros(shape), c0.copy())
    amp = 1.0 + 0j
    U = U0
    cbar = cbar0
    for _ in range(3):
        s, _ = O.run(s, 1)
        U = uset[0] + (U - uset[0]) * R4(-dt / tau)
        z = dt * (-1j * U * np.sin(th) / dx - alpha * 4 * np.sin(th / 2) ** 2 / dx ** 2 - 1 / tau)
        amp *= R4(z)
        cbar = 2.0 + (cbar - 2.0) * R4(-dt / tau)
        np.testing.assert_allclose(s.u, U, rtol=1e-14)
        np.testing.assert_allclose(s.c[0, 0], cbar + np.real(np.exp(1j * kx * x) * amp), atol=1e-13)


def test_step_diagnostics_definitions():
    shape = (4, 6, 16)
    L = (2 * np.pi, 1.0, 1.0)
    beta = np.ones(shape, np.uint8)
    beta[:, 0, :] = 0
    room = np.zeros(shape, np.uint8)
    room[:, 2:4, :] = 1
    O = Oracle(OracleParams(16, 6, 4, *L, 0.05, 0.05, 1.0, (0, 0, 0), 0.5, 0.02, 1.0, 4, False),
               beta, np.zeros(0, np.int64), np.zeros(0), np.zeros((0, 3)), np.zeros(0), room)
    x = np.arange(16) * L[0] / 16
    v0 = np.broadcast_to(np.sin(3 * x), shape) * beta
    c0 = np.random.default_rng(1).random(shape) * beta
    s = OracleState(zeros(shape), v0.copy(), zeros(shape), zeros(shape), c0)
    s, dg = O.step(s)
    dv = (L[0] / 16) * (L[1] / 6) * (L[2] / 4)
    assert dg["ke"] == pytest.approx(0.5 * np.sum(s.u ** 2 + s.v ** 2 + s.w ** 2) * dv, rel=1e-14)
    assert dg["co2_mass"] == pytest.approx(np.sum(s.c) * dv, rel=1e-14)
    assert dg["co2_room_mean"] == pytest.approx(np.mean(s.c[:, 2:4, :]), rel=1e-14)
    assert dg["dt"] == 0.02 and dg["step"] == 1 and dg["t"] == 0.02
    rate = np.max(np.abs(v0)) / (L[1] / 6)
    assert dg["cfl_max"] == pytest.approx(0.02 * rate, rel=1e-14)


def test_div_l2_definition_masked():
    """div_l2 of the diagnostics is sqrt(sum (div u)^2 dV) of the projected
    velocity.  With solids the projected field keeps a divergence at the
    walls (the immersed-boundary iteration is not exact after n solves), so
    the norm is O(1) here, not round-off; the central differences are written
    out with np.roll in this test, independently of the oracle's operators.
    The spacing makes dV far from 1 and the norm far from its square, so a
    dropped dV or square root fails."""
    shape = (6, 8, 10)
    L = (0.7, 1.9, 0.45)
    rng = np.random.default_rng(42)
    beta = np.ones(shape, np.uint8)
    beta[1:3, 2:6, 3:7] = 0
    beta[:, 0, :] = 0
    u0 = [5.0 * rng.standard_normal(shape) * beta for _ in range(3)]
    O = make(shape, L, beta=beta, n_piter=2, dt_fixed=1e-3, nu=1e-3)
    s = OracleState(u0[0].copy(), u0[1].copy(), u0[2].copy(), zeros(shape), zeros(shape))
    s, dg = O.step(s)
    dx, dy, dz = L[0] / shape[2], L[1] / shape[1], L[2] / shape[0]
    div = ((np.roll(s.u, -1, axis=2) - np.roll(s.u, 1, axis=2)) / (2 * dx)
           + (np.roll(s.v, -1, axis=1) - np.roll(s.v, 1, axis=1)) / (2 * dy)
           + (np.roll(s.w, -1, axis=0) - np.roll(s.w, 1, axis=0)) / (2 * dz))
    dv = dx * dy * dz
    expected = np.sqrt(np.sum(div ** 2) * dv)
    assert expected > 1e-2                     # a real divergence, not round-off
    assert abs(dv - 1) > 0.9 and abs(expected - expected ** 2) > 0.1 * expected
    assert dg["div_l2"] == pytest.approx(expected, rel=1e-13)


def test_momentum_shear_mode_advected_by_uniform_flow():
    """u = (U, A cos(k x), 0): C_y = U D_x v and C_x = 0 exactly, the field is
    divergence-free, so v is advected and diffused with the exact complex RK4
    factor z = dt(-i U sin(th)/dx - 4 nu sin^2(th/2)/dx^2).  Pins the sign and
    weight of the momentum convection."""
    shape = (2, 3, 12)
    L = (3.0, 1.0, 1.0)
    nu, dt = 0.02, 0.03
    O = make(shape, L, nu=nu, dt_fixed=dt)
    dx = L[0] / shape[2]
    x = np.arange(shape[2]) * dx
    th = 2 * np.pi * 2 / shape[2]
    kx = th / dx
    U = 0.8
    v0 = np.broadcast_to(np.cos(kx * x), shape).copy()
    s = OracleState(np.full(shape, U), v0.copy(), zeros(shape), zeros(shape), zeros(shape))
    nst = 5
    s, _ = O.run(s, nst)
    z = dt * (-1j * U * np.sin(th) / dx - nu * 4 * np.sin(th / 2) ** 2 / dx ** 2)
    np.testing.assert_allclose(s.v[0, 0], np.real(np.exp(1j * kx * x) * R4(z) ** nst), atol=1e-14)
    np.testing.assert_allclose(s.u, U, rtol=1e-15)
