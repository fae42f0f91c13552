"""Seeded synthetic scenarios: the inputs of one projection time step.

This module is shared by the CPU oracle (test infrastructure) and by the
GPU library's callers.  It holds no arithmetic of the solver itself: it only
lays out the problem the solver is given, the way the paper's case-setup
scripts do (Section 2.4: fluid properties and grid, the solid mask beta built
from primitive blocks, the source regions S, the initial fields).

Conventions (shared by every consumer):

* The grid is uniform and periodic, ``(nx, ny, nz)`` cells of size
  ``dx = lx/nx`` etc.  Cell ``(i, j, k)`` sits at ``(i*dx, j*dy, k*dz)``.
* Arrays are numpy arrays of shape ``(nz, ny, nx)`` (x fastest), so the flat
  index of cell ``(i, j, k)`` is ``i + nx*(j + ny*k)``.
* ``beta`` is ``uint8``: 1 for fluid, 0 for solid (Section 2.1, the binary
  mask of the boundary conditions).
* The source term ``S (u_set - u)/tau_f`` (Section 2.1, momentum and scalar
  equations) is nonzero only in a few duct cells, so it is carried as a
  sparse list: sorted flat indices, the mask value ``S`` in (0, 1], the target
  velocity ``u_set`` (n, 3) and the target concentration ``c_set``.
* ``room_mask`` marks the region over which the mean CO2 concentration is
  monitored (Section 3.3.2); ``None`` means the whole domain.

Workload recipes follow the shapes of the paper's cases: air viscosity
1.6e-5 m^2/s (Table 3), CO2 initially 1000 ppm with 400 ppm supply air
(Section 3.3.2), inflow 0.1 or 1 m/s (Section 3.1.2), block obstacles
(Section 2.5), grid spacing of a few centimetres (Table 3), periodic
inflow/outflow arrangements A (opposite wall) and B (extra passage around the
room) of Section 2.1.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

NU_AIR = 1.6e-5          # m^2/s, Table 3 (printed with wrong units there)
CO2_STALE = 1000.0       # ppm, Section 3.3.2
CO2_FRESH = 400.0        # ppm, Section 3.3.2
TANH_B = 5.0             # smoothness B_a of the source mask (not given by the paper)


@dataclass
class Scenario:
    """Everything one solver instance needs, in host memory."""

    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    nu: float
    alpha_c: float
    tau_f: float
    body: Tuple[float, float, float]
    cfl: float
    dt_fixed: float          # > 0: fixed time step; otherwise CFL-adaptive
    u_ref: float             # floor velocity of the Courant denominator
    n_piter: int             # immersed-boundary pressure iterations per step
    filter: bool             # sixth-order explicit filter at the end of a step
    beta: np.ndarray         # uint8 (nz, ny, nx)
    forced_idx: np.ndarray   # int64 (n,), sorted, unique
    forced_S: np.ndarray     # float64 (n,)
    forced_uset: np.ndarray  # float64 (n, 3)
    forced_cset: np.ndarray  # float64 (n,)
    room_mask: Optional[np.ndarray]  # uint8 (nz, ny, nx) or None
    u: np.ndarray            # float64 (nz, ny, nx) initial fields
    v: np.ndarray
    w: np.ndarray
    p: np.ndarray
    c: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def spacing(self) -> Tuple[float, float, float]:
        return (self.lx / self.nx, self.ly / self.ny, self.lz / self.nz)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def copy(self) -> "Scenario":
        arrays = {k: getattr(self, k).copy() for k in
                  ("beta", "forced_idx", "forced_S", "forced_uset", "forced_cset",
                   "u", "v", "w", "p", "c")}
        rm = None if self.room_mask is None else self.room_mask.copy()
        return replace(self, room_mask=rm, meta=dict(self.meta), **arrays)


def _no_forcing():
    return (np.zeros(0, np.int64), np.zeros(0), np.zeros((0, 3)), np.zeros(0))


# --------------------------------------------------------------------------
# Source mask (Section 2.1, eq. tanh): product of three smoothed top-hats.
# --------------------------------------------------------------------------
def tanh_factor(r: np.ndarray, half_width: float, b: float) -> np.ndarray:
    """One factor of the source-mask product for distances ``r >= 0``.

    0.5 * (1 - tanh(b * (r/h - h/r))) with h = W/2; at r = 0 the bracket tends
    to -inf and the factor to 1 (taken explicitly).
    """
    r = np.asarray(r, dtype=np.float64)
    out = np.ones_like(r)
    nz = r > 0
    arg = b * (r[nz] / half_width - half_width / r[nz])
    out[nz] = 0.5 * (1.0 - np.tanh(arg))
    return out


def periodic_distance(x: np.ndarray, xc: float, length: float) -> np.ndarray:
    d = np.abs(np.asarray(x, dtype=np.float64) - xc) % length
    return np.minimum(d, length - d)


def source_mask(shape, spacing, lengths, centre, widths, b=TANH_B) -> np.ndarray:
    """Dense S on the grid for one source region (periodic distances)."""
    nz, ny, nx = shape
    dx, dy, dz = spacing
    fx = tanh_factor(periodic_distance(np.arange(nx) * dx, centre[0], lengths[0]), widths[0] / 2, b)
    fy = tanh_factor(periodic_distance(np.arange(ny) * dy, centre[1], lengths[1]), widths[1] / 2, b)
    fz = tanh_factor(periodic_distance(np.arange(nz) * dz, centre[2], lengths[2]), widths[2] / 2, b)
    return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]


def forced_list(S: np.ndarray, beta: np.ndarray, uset, cset, threshold=1e-6):
    """Sparse forced-cell list from dense S fields (fluid cells with S > threshold)."""
    sel = np.flatnonzero((S.ravel() > threshold) & (beta.ravel() == 1))
    n = sel.size
    return (sel.astype(np.int64), S.ravel()[sel].astype(np.float64),
            np.broadcast_to(np.asarray(uset, np.float64), (n, 3)).copy(),
            np.full(n, float(cset)))


def merge_forced(*lists):
    """Union of several forced-cell lists; later lists win on overlapping cells."""
    idx = np.concatenate([l[0] for l in lists])
    S = np.concatenate([l[1] for l in lists])
    us = np.concatenate([l[2] for l in lists])
    cs = np.concatenate([l[3] for l in lists])
    order = np.argsort(idx, kind="stable")
    idx, S, us, cs = idx[order], S[order], us[order], cs[order]
    keep = np.ones(idx.size, bool)
    keep[:-1] = idx[1:] != idx[:-1]
    return idx[keep], S[keep], us[keep], cs[keep]


# --------------------------------------------------------------------------
# Geometry helpers (Section 2.4: obstacles are blocks; box rounding rule).
# --------------------------------------------------------------------------
def box_cells(x0: float, x1: float, d: float, n: int) -> slice:
    """Cells i with round(x0/d) <= i < round(x1/d), clipped to the grid."""
    a = int(np.clip(np.rint(x0 / d), 0, n))
    b = int(np.clip(np.rint(x1 / d), 0, n))
    return slice(a, max(a, b))


def wall_slabs(shape, t=2) -> np.ndarray:
    """beta with 2-cell solid slabs on all six faces of the periodic box."""
    nz, ny, nx = shape
    beta = np.ones(shape, np.uint8)
    for ax, n in ((2, nx), (1, ny), (0, nz)):
        if n > 2 * t:
            idx = [slice(None)] * 3
            idx[ax] = np.r_[0:t, n - t:n]
            beta[tuple(idx)] = 0
    return beta


def draw_boxes(rng, n_boxes, lengths, spacing, z_floor, size_lo=0.4, size_hi=1.2,
               max_frac=None, x_margin=0.5):
    """Seeded obstacle boxes standing on the floor: list of (x0,x1,y0,y1,z0,z1).

    Draw order per box: sx, sy, sz ~ U(lo, hi); x0; y0; z0 = floor.
    """
    lx, ly, lz = lengths
    dx, dy, dz = spacing
    boxes = []
    for _ in range(n_boxes):
        sx, sy, sz = rng.uniform(size_lo, size_hi, 3)
        if max_frac is not None:
            room = (lx - 4 * dx, ly - 4 * dy, lz - 4 * dz)
            sx = min(sx, max_frac * room[0])
            sy = min(sy, max_frac * room[1])
            sz = min(sz, max_frac * room[2])
        xlo, xhi = 2 * dx + x_margin, lx - 2 * dx - x_margin - sx
        if xhi < xlo:
            xlo, xhi = 2 * dx, max(2 * dx, lx - 2 * dx - sx)
        x0 = rng.uniform(xlo, xhi)
        y0 = rng.uniform(2 * dy, max(2 * dy, ly - 2 * dy - sy))
        z0 = z_floor
        boxes.append((x0, x0 + sx, y0, y0 + sy, z0, z0 + sz))
    return boxes


def carve_boxes(beta, boxes, spacing):
    nz, ny, nx = beta.shape
    dx, dy, dz = spacing
    for (x0, x1, y0, y1, z0, z1) in boxes:
        beta[box_cells(z0, z1, dz, nz), box_cells(y0, y1, dy, ny), box_cells(x0, x1, dx, nx)] = 0
    return beta


# --------------------------------------------------------------------------
# Recipes
# --------------------------------------------------------------------------
def taylor_green(n: int = 32, nu: float = 0.01, dt: float = 0.01, with_scalar: bool = True,
                 n_piter: int = 4) -> Scenario:
    """3D Taylor-Green vortex in the periodic cube of side 2*pi, unmasked.

    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0, sampled at x_i = i*dx;
    optional scalar c = 1 + 0.5 sin x with diffusivity nu.  Fixed dt, no filter.
    """
    L = 2 * np.pi
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    c = 1.0 + 0.5 * np.sin(X) if with_scalar else np.zeros_like(u)
    idx, S, us, cs = _no_forcing()
    return Scenario(
        name=f"tgv{n}", nx=n, ny=n, nz=n, lx=L, ly=L, lz=L, nu=nu, alpha_c=nu,
        tau_f=1.0, body=(0.0, 0.0, 0.0), cfl=0.5, dt_fixed=dt, u_ref=1.0,
        n_piter=n_piter, filter=False, beta=np.ones(u.shape, np.uint8),
        forced_idx=idx, forced_S=S, forced_uset=us, forced_cset=cs, room_mask=None,
        u=u, v=v, w=w, p=np.zeros_like(u), c=c,
        meta={"kind": "tgv"})


def room(nx=256, ny=128, nz=96, dx=10.0 / 256, u_in=1.0, n_boxes=8, seed=2204,
         cfl=0.3, filter=True, duct=0.3, n_piter=4, box_max_frac=None) -> Scenario:
    """Ventilated room, periodic arrangement A (Section 2.1, inlet and outlet on
    opposite walls joined through the periodic seam).

    2-cell solid slabs on all faces; a square duct of round(duct/dx) cells at the
    top of the x-walls, cut through both x-slabs so that the seam x = 0 forms a
    4-cell passage; forcing from the tanh mask centred on the seam with
    W_x = 4 dx, W_y = W_z = duct width; obstacles drawn from
    ``numpy.random.default_rng(seed)``.  u = 0, p = 0, c = 1000 ppm in the fluid.
    """
    shape = (nz, ny, nx)
    dy = dz = dx
    lx, ly, lz = nx * dx, ny * dy, nz * dz
    beta = wall_slabs(shape)
    nd = int(np.rint(duct / dx))
    j0 = (ny - nd) // 2
    k0 = nz - 2 - nd
    # duct through both x-slabs (the periodic seam)
    beta[k0:k0 + nd, j0:j0 + nd, 0:2] = 1
    beta[k0:k0 + nd, j0:j0 + nd, nx - 2:nx] = 1
    rng = np.random.default_rng(seed)
    boxes = draw_boxes(rng, n_boxes, (lx, ly, lz), (dx, dy, dz), z_floor=2 * dz,
                       max_frac=box_max_frac)
    carve_boxes(beta, boxes, (dx, dy, dz))
    # keep the duct and its mouth clear of obstacles
    beta[k0:k0 + nd, j0:j0 + nd, 0:2] = 1
    beta[k0:k0 + nd, j0:j0 + nd, nx - 2:nx] = 1
    centre = (lx - 0.5 * dx, (j0 + 0.5 * (nd - 1)) * dy, (k0 + 0.5 * (nd - 1)) * dz)
    widths = (4 * dx, nd * dy, nd * dz)
    S = source_mask(shape, (dx, dy, dz), (lx, ly, lz), centre, widths)
    forced = forced_list(S, beta, (u_in, 0.0, 0.0), CO2_FRESH)
    rm = np.zeros(shape, np.uint8)
    rm[2:nz - 2, 2:ny - 2, 2:nx - 2] = 1
    z = np.zeros(shape)
    tau_f = 2.0 * cfl * dx / u_in
    return Scenario(
        name=f"room{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz,
        nu=NU_AIR, alpha_c=NU_AIR, tau_f=tau_f, body=(0.0, 0.0, 0.0), cfl=cfl,
        dt_fixed=0.0, u_ref=u_in, n_piter=n_piter, filter=filter, beta=beta,
        forced_idx=forced[0], forced_S=forced[1], forced_uset=forced[2],
        forced_cset=forced[3], room_mask=rm, u=z.copy(), v=z.copy(), w=z.copy(),
        p=z.copy(), c=CO2_STALE * beta.astype(np.float64),
        meta={"kind": "room", "boxes": boxes, "duct_cells": nd, "u_in": u_in, "seed": seed})


def hall(nx=1024, ny=512, nz=256, dx=40.0 / 1024, u_in=1.0, n_boxes=64, seed=2204,
         cfl=0.3, filter=True, vent=0.6, plenum=16, n_piter=4) -> Scenario:
    """Hall with ceiling vents, periodic arrangement B (Section 2.1: an extra air
    passage, here a return plenum above a 2-cell ceiling slab).

    Four forced inlet holes (vent x vent m) in the ceiling slab blow downwards
    with u_set = (0, 0, -u_in), c_set = 400 ppm; two unforced outlet holes let
    the air back into the plenum.  Obstacles from ``default_rng(seed)``.
    """
    shape = (nz, ny, nx)
    dy = dz = dx
    lx, ly, lz = nx * dx, ny * dy, nz * dz
    beta = wall_slabs(shape)
    kc0 = nz - 2 - plenum - 2            # ceiling slab cells kc0, kc0+1
    beta[kc0:kc0 + 2, :, :] = 0
    nv = int(np.rint(vent / dx))
    inlets = [(0.25, 0.25), (0.75, 0.25), (0.25, 0.75), (0.75, 0.75)]
    outlets = [(0.5, 0.1), (0.5, 0.9)]
    holes = []
    for (fx, fy) in inlets + outlets:
        i0 = int(np.rint(fx * nx)) - nv // 2
        j0 = int(np.rint(fy * ny)) - nv // 2
        beta[kc0:kc0 + 2, j0:j0 + nv, i0:i0 + nv] = 1
        holes.append((i0, j0))
    rng = np.random.default_rng(seed)
    boxes = draw_boxes(rng, n_boxes, (lx, ly, kc0 * dz), (dx, dy, dz), z_floor=2 * dz)
    carve_boxes(beta, boxes, (dx, dy, dz))
    lists = []
    for (i0, j0) in holes[:4]:
        centre = ((i0 + 0.5 * (nv - 1)) * dx, (j0 + 0.5 * (nv - 1)) * dy, (kc0 + 0.5) * dz)
        S = source_mask(shape, (dx, dy, dz), (lx, ly, lz), centre, (nv * dx, nv * dy, 2 * dz))
        lists.append(forced_list(S, beta, (0.0, 0.0, -u_in), CO2_FRESH))
    forced = merge_forced(*lists)
    rm = np.zeros(shape, np.uint8)
    rm[2:kc0, 2:ny - 2, 2:nx - 2] = 1
    c = CO2_STALE * beta.astype(np.float64)
    c[kc0 + 2:, :, :] = CO2_FRESH * beta[kc0 + 2:, :, :]
    z = np.zeros(shape)
    tau_f = 2.0 * cfl * dx / u_in
    return Scenario(
        name=f"hall{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz,
        nu=NU_AIR, alpha_c=NU_AIR, tau_f=tau_f, body=(0.0, 0.0, 0.0), cfl=cfl,
        dt_fixed=0.0, u_ref=u_in, n_piter=n_piter, filter=filter, beta=beta,
        forced_idx=forced[0], forced_S=forced[1], forced_uset=forced[2],
        forced_cset=forced[3], room_mask=rm, u=z.copy(), v=z.copy(), w=z.copy(),
        p=z.copy(), c=c, meta={"kind": "hall", "boxes": boxes, "u_in": u_in, "seed": seed})


def channel2d(ny_fluid=16, nx=8, wall=2, nu=0.01, bx=1e-3, dt=0.01) -> Scenario:
    """2D laminar channel driven by a body force (Section 3.1.1, Table 1):
    solid walls of ``wall`` cells at the bottom of the periodic y-direction,
    ``ny_fluid`` fluid cells between them, nz = 1."""
    ny = ny_fluid + wall
    dy = 1.0
    shape = (1, ny, nx)
    beta = np.ones(shape, np.uint8)
    beta[:, :wall, :] = 0
    z = np.zeros(shape)
    idx, S, us, cs = _no_forcing()
    return Scenario(
        name="channel2d", nx=nx, ny=ny, nz=1, lx=nx * dy, ly=ny * dy, lz=1.0,
        nu=nu, alpha_c=nu, tau_f=1.0, body=(bx, 0.0, 0.0), cfl=0.5, dt_fixed=dt,
        u_ref=1.0, n_piter=4, filter=False, beta=beta, forced_idx=idx, forced_S=S,
        forced_uset=us, forced_cset=cs, room_mask=None, u=z.copy(), v=z.copy(),
        w=z.copy(), p=z.copy(), c=z.copy(), meta={"kind": "channel", "wall": wall})


def _fft_size_at_least(n: int) -> int:
    """Smallest 2^a 3^b >= n (the FFT lengths the solver accepts)."""
    m = max(1, int(n))
    while True:
        r = m
        for f in (2, 3):
            while r % f == 0:
                r //= f
        if r == 1:
            return m
        m += 1


def cube_channel(n_h=30, re_ob=84.0, u_max=1.5, cfl=0.3, filter=True, n_piter=4,
                 perturb=0.01, seed=2204, length_d=8.8, band_h=1.0) -> Scenario:
    """Square obstacle in a 2D channel with a forced parabolic inflow
    (Section 3.1.1, Tables 1 and 2): channel width D = 2 pi between solid
    walls, obstacle edge h = D/6 resolved by n_h cells, obstacle centred at
    (1.2 D, D/2) downstream of the inflow, Re_ob = U_b h / nu with the bulk
    velocity U_b = 2/3 U_max.

    Grid (nz = 1, dx = dy = h/n_h): ny = 6 n_h fluid cells plus two equal
    solid wall slabs of at least 2 cells (the paper's 0.05 D walls, thinner
    here: a solid slab's thickness does not enter the flow), nx about
    length_d D (the paper's 8.8 D by default); both are FFT lengths 2^a 3^b,
    nx even.  The inflow is the source term of Section 2.1 across the whole
    channel in a band of width band_h h centred on the periodic seam x = 0,
    with u_set the parabola U_max 4 y (D' - y) / D'^2, where y is
    measured from the centre of the last wall cell and D' = (6 n_h + 1) dx
    (where the masked central-difference operators put the no-slip wall).
    Initial state: the same parabola in every fluid cell plus a small seeded
    cross-stream perturbation that breaks the symmetry; c = 0."""
    D = 2.0 * np.pi
    h = D / 6.0
    d = h / n_h
    nf = 6 * n_h
    ny = _fft_size_at_least(nf + 4)
    while (ny - nf) % 2:
        ny = _fft_size_at_least(ny + 1)
    wall = (ny - nf) // 2
    target = length_d * nf
    cands = [_fft_size_at_least(int(np.floor(target * 0.9)))]
    while cands[-1] < 1.1 * target:
        cands.append(_fft_size_at_least(cands[-1] + 1))
    nx = min((n for n in cands if n % 2 == 0), key=lambda n: abs(n - target))
    shape = (1, ny, nx)
    u_b = 2.0 * u_max / 3.0
    nu = u_b * h / re_ob
    beta = np.ones(shape, np.uint8)
    beta[:, :wall, :] = 0
    beta[:, wall + nf:, :] = 0
    xc = 1.2 * nf                      # obstacle centre, in cells from the seam
    i0, i1 = int(np.rint(xc - n_h / 2)), int(np.rint(xc + n_h / 2))
    j0, j1 = wall + (nf - n_h) // 2, wall + (nf - n_h) // 2 + n_h
    beta[:, j0:j1, i0:i1] = 0
    # parabolic profile from the centre of the last wall cell
    y = (np.arange(ny) - wall + 1) * d
    dp = (nf + 1) * d
    prof = np.where((np.arange(ny) >= wall) & (np.arange(ny) < wall + nf), u_max * 4.0 * y * (dp - y) / dp ** 2, 0.0)
    fx = tanh_factor(periodic_distance(np.arange(nx) * d, 0.0, nx * d), band_h * h / 2, TANH_B)
    S = np.broadcast_to(fx[None, None, :], shape)
    sel = np.flatnonzero((S.ravel() > 1e-6) & (beta.ravel() == 1))
    jj = (sel // nx) % ny
    uset = np.zeros((sel.size, 3))
    uset[:, 0] = prof[jj]
    rng = np.random.default_rng(seed)
    b = beta.astype(np.float64)
    u = prof[None, :, None] * b
    x = np.arange(nx) * d
    v = perturb * u_max * np.sin(2 * np.pi * x / (nx * d))[None, None, :] * rng.uniform(0.5, 1.5) * b
    v = np.broadcast_to(v, shape).copy()
    z = np.zeros(shape)
    return Scenario(
        name=f"cube_channel{n_h}", nx=nx, ny=ny, nz=1, lx=nx * d, ly=ny * d, lz=d,
        nu=nu, alpha_c=nu, tau_f=2.0 * cfl * d / u_max, body=(0.0, 0.0, 0.0), cfl=cfl,
        dt_fixed=0.0, u_ref=u_max, n_piter=n_piter, filter=filter, beta=beta,
        forced_idx=sel.astype(np.int64), forced_S=S.ravel()[sel].astype(np.float64),
        forced_uset=uset, forced_cset=np.zeros(sel.size), room_mask=None,
        u=u, v=v, w=z.copy(), p=z.copy(), c=z.copy(),
        meta={"kind": "cube_channel", "n_h": n_h, "h": h, "D": D, "u_b": u_b, "u_max": u_max,
              "wall": wall, "obstacle_cells": (i0, i1, j0, j1, 0, 1)})


def random_fields(shape, seed, scale=1.0, beta=None):
    """Smooth-ish random periodic fields (u, v, w, p, c) for operator tests."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(5):
        f = rng.standard_normal(shape) * scale
        out.append(f)
    if beta is not None:
        b = beta.astype(np.float64)
        out = [out[0] * b, out[1] * b, out[2] * b, out[3], out[4] * b]
    return out


def random_beta(shape, seed, n_boxes=3, max_size=None):
    """A mask with a few random solid boxes (periodic grid, arbitrary placement)."""
    rng = np.random.default_rng(seed)
    beta = np.ones(shape, np.uint8)
    nz, ny, nx = shape
    for _ in range(n_boxes):
        sz = []
        for n in (nz, ny, nx):
            hi = min(n, max_size) if max_size else max(1, n // 2)
            sz.append(int(rng.integers(1, hi + 1)) if n > 1 else 1)
        o = [int(rng.integers(0, n)) for n in (nz, ny, nx)]
        kk = (np.arange(sz[0]) + o[0]) % nz
        jj = (np.arange(sz[1]) + o[1]) % ny
        ii = (np.arange(sz[2]) + o[2]) % nx
        beta[np.ix_(kk, jj, ii)] = 0
    return beta


def serving_requests(n=64, seed=7, mean_gap=0.5, n_steps=2000):
    """The serving stream: Poisson arrivals and per-request room draws.

    Returns a list of dicts: arrival time, grid, inflow, box count, seed.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap, n)
    t = np.cumsum(gaps) - gaps[0]
    grids = [(64, 64, 64), (128, 64, 64), (192, 96, 64), (256, 128, 96)]
    reqs = []
    for i in range(n):
        ri = np.random.default_rng(1000 + i)
        g = grids[int(ri.integers(0, len(grids)))]
        u_in = float(ri.choice([0.1, 1.0]))
        nb = int(ri.integers(0, 13))
        reqs.append({"id": i, "arrival": float(t[i]), "grid": g, "u_in": u_in,
                     "n_boxes": nb, "seed": 1000 + i, "n_steps": n_steps})
    return reqs


def serving_scenario(req, dx=10.0 / 256) -> Scenario:
    nx, ny, nz = req["grid"]
    return room(nx=nx, ny=ny, nz=nz, dx=dx, u_in=req["u_in"], n_boxes=req["n_boxes"],
                seed=req["seed"], box_max_frac=0.4)
