"""MI355X (gfx950) library for one explicit projection time step of the
incompressible Navier-Stokes equations with a passive CO2 scalar and a binary
immersed-boundary mask (Korhonen et al., arXiv 2204.02107, Sections 2.1-2.4).

The compute path is the HIP library ``libdnslab.so`` (C ABI in
``include/dnslab.h``).  This module only marshals arguments: PyTorch provides
device memory and the stream.  There is no CPU fallback; without the built
library every call raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import _lib
from ._lib import Diag, DnslabError, Params, FP64, FP32_REFINE

__all__ = ["Solver", "Diag", "DnslabError", "Params", "FP64", "FP32_REFINE", "workspace_bytes", "load"]

load = _lib.load


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def make_params(case, precision=FP64, stream=None, project_each_stage=False) -> Params:
    P = Params()
    P.nx, P.ny, P.nz = int(case.nx), int(case.ny), int(case.nz)
    P.lx, P.ly, P.lz = float(case.lx), float(case.ly), float(case.lz)
    P.nu, P.alpha_c, P.tau_f = float(case.nu), float(case.alpha_c), float(case.tau_f)
    for i in range(3):
        P.body[i] = float(case.body[i])
    P.cfl, P.dt_fixed, P.u_ref = float(case.cfl), float(case.dt_fixed), float(case.u_ref)
    P.n_piter, P.filter, P.precision = int(case.n_piter), int(bool(case.filter)), int(precision)
    P.stream = stream
    P.project_each_stage = int(bool(project_each_stage))
    return P


def workspace_bytes(case, precision=FP64) -> int:
    out = ctypes.c_size_t()
    lib = load()
    _lib.check(lib.dnslab_workspace_bytes(ctypes.byref(make_params(case, precision)), ctypes.byref(out)))
    return int(out.value)


class Solver:
    """One context of the library bound to resident torch state tensors.

    ``case`` is any object with the attributes of a scenario: grid and
    parameters, ``beta`` (uint8, shape (nz, ny, nx)), the sparse forcing list
    (``forced_idx``, ``forced_S``, ``forced_uset``, ``forced_cset``),
    ``room_mask`` and the initial fields ``u, v, w, p, c``.
    """

    def __init__(self, case, precision=FP64, device="cuda:0", stream=None, project_each_stage=False,
                 graph_steps=0):
        torch = _torch()
        self.lib = load()
        self.device = torch.device(device)
        self.precision = precision
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        self.shape = (int(case.nz), int(case.ny), int(case.nx))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
            if graph_steps and stream.cuda_stream == 0:
                stream = torch.cuda.Stream(self.device)   # graphs need a stream other than the legacy default
        self.stream = stream
        dev = self.device

        def field(a):
            return torch.as_tensor(a, dtype=self.dtype).reshape(self.shape).to(dev).contiguous()

        self.u, self.v, self.w = field(case.u), field(case.v), field(case.w)
        self.p, self.c = field(case.p), field(case.c)
        beta = torch.as_tensor(case.beta, dtype=torch.uint8).reshape(self.shape).to(dev).contiguous()
        n = int(len(case.forced_idx))
        fidx = torch.as_tensor(case.forced_idx, dtype=torch.int64).to(dev).contiguous()
        fS = torch.as_tensor(case.forced_S, dtype=torch.float64).to(dev).contiguous()
        fus = torch.as_tensor(case.forced_uset, dtype=torch.float64).reshape(-1).to(dev).contiguous()
        fcs = torch.as_tensor(case.forced_cset, dtype=torch.float64).to(dev).contiguous()
        room = None
        if getattr(case, "room_mask", None) is not None:
            room = torch.as_tensor(case.room_mask, dtype=torch.uint8).reshape(self.shape).to(dev).contiguous()
        self.params = make_params(case, precision, ctypes.c_void_p(stream.cuda_stream), project_each_stage)
        # the context's workspace comes from torch's caching allocator, so that
        # torch and the library see one pool of HBM
        self._alloc = _lib.TorchAllocator(dev.index if dev.index is not None else torch.cuda.current_device(),
                                          stream.cuda_stream)
        self._alloc.fill(self.params)
        ctx = ctypes.c_void_p()
        rc = self.lib.dnslab_init(
            ctypes.byref(self.params), _ptr(beta), n,
            _ptr(fidx) if n else None, _ptr(fS) if n else None,
            _ptr(fus) if n else None, _ptr(fcs) if n else None,
            _ptr(room) if room is not None else None,
            _ptr(self.u), _ptr(self.v), _ptr(self.w), _ptr(self.p), _ptr(self.c),
            ctypes.byref(ctx))
        _lib.check(rc, None)
        self.ctx = ctx
        if graph_steps:
            self._check(self.lib.dnslab_set_graph_steps(self.ctx, int(graph_steps)))

    # -- life cycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dnslab_destroy(self.ctx)
            self.ctx = None
        if getattr(self, "_alloc", None) is not None:
            self._alloc.close()
            self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        return _lib.check(rc, self.ctx)

    def _call(self, fn, *args):
        """Run a library call on the solver's stream, ordered after the work
        torch has queued on its current stream and before what comes next."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        same = cur.cuda_stream == self.stream.cuda_stream
        if not same:
            self.stream.wait_stream(cur)
        rc = fn(*args)
        if not same:
            cur.wait_stream(self.stream)
        return self._check(rc)

    # -- the step ------------------------------------------------------------
    def step(self, nsteps: int = 1, diag: bool = True) -> Optional[dict]:
        d = Diag() if diag else None
        self._call(self.lib.dnslab_step, self.ctx, int(nsteps), ctypes.byref(d) if diag else None)
        return d.as_dict() if diag else None

    def read_diags(self, n: int):
        arr = (Diag * n)()
        self._check(self.lib.dnslab_read_diags(self.ctx, int(n), arr))
        return [a.as_dict() for a in arr]

    def set_time(self, t: float = 0.0, step: int = 0):
        self._check(self.lib.dnslab_set_time(self.ctx, float(t), int(step)))

    # -- pieces of the step --------------------------------------------------
    def poisson(self, rhs, out=None):
        out = self._empty() if out is None else out
        self._call(self.lib.dnslab_poisson, self.ctx, _ptr(self._dev(rhs)), _ptr(out))
        return out

    def project(self, u, v, w):
        self._call(self.lib.dnslab_project, self.ctx, _ptr(u), _ptr(v), _ptr(w))

    def scalar_step(self, dt: float):
        self._call(self.lib.dnslab_scalar_step, self.ctx, float(dt))

    def momentum_rhs(self, u, v, w):
        u, v, w = self._dev(u), self._dev(v), self._dev(w)
        out = [self._empty() for _ in range(3)]
        self._call(self.lib.dnslab_momentum_rhs, self.ctx, _ptr(u), _ptr(v), _ptr(w), *map(_ptr, out))
        return out

    def scalar_rhs(self, c, u, v, w):
        c, u, v, w = map(self._dev, (c, u, v, w))
        out = self._empty()
        self._call(self.lib.dnslab_scalar_rhs, self.ctx, _ptr(c), _ptr(u), _ptr(v), _ptr(w), _ptr(out))
        return out

    def filter(self, f):
        f = self._dev(f)
        out = self._empty()
        self._call(self.lib.dnslab_filter, self.ctx, _ptr(f), _ptr(out))
        return out

    # -- Lagrangian particles (Section 2.3) ----------------------------------
    def particles_step(self, pos, vel, diam, rho_p=1000.0, rho_f=1.225, g=(0.0, 0.0, -9.81), dt=0.0):
        """Advance particles in place: pos, vel are FP64 device tensors of shape
        (3, n) (x, y, z rows), diam of shape (n,).  dt <= 0 uses the last step's dt."""
        n = int(diam.numel())
        for t in (pos, vel, diam):
            if t.dtype != _torch().float64 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("particle arrays must be contiguous float64 tensors on the solver's device")
        if tuple(pos.shape) != (3, n) or tuple(vel.shape) != (3, n):
            raise ValueError("pos and vel must have shape (3, n)")
        pp = _lib.ParticleParams(float(rho_p), float(rho_f), (ctypes.c_double * 3)(*map(float, g)))
        self._call(self.lib.dnslab_particles_step, self.ctx, n, _ptr(pos), _ptr(vel), _ptr(diam),
                   ctypes.byref(pp), float(dt))

    def particles_sort(self, pos, vel, diam):
        """Reorder the particles in place by the cell holding each one (stable),
        so that the step kernel's velocity gathers are coalesced."""
        n = int(diam.numel())
        for t in (pos, vel, diam):
            if t.dtype != _torch().float64 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("particle arrays must be contiguous float64 tensors on the solver's device")
        if tuple(pos.shape) != (3, n) or tuple(vel.shape) != (3, n):
            raise ValueError("pos and vel must have shape (3, n)")
        self._call(self.lib.dnslab_particles_sort, self.ctx, n, _ptr(pos), _ptr(vel), _ptr(diam))

    # -- post-processing (Sections 3.3-3.4) ----------------------------------
    def co2_histogram(self, nbins=60, lo=400.0, hi=1000.0):
        """Counts of room fluid cells per CO2 bin (numpy int64, nbins values)."""
        import numpy as np
        out = np.zeros(int(nbins), dtype=np.int64)
        self._call(self.lib.dnslab_co2_histogram, self.ctx, int(nbins), float(lo), float(hi),
                   out.ctypes.data_as(ctypes.c_void_p))
        return out

    def accumulate(self, sums):
        """sums (FP64 device tensor of shape (5,) + grid shape) += (u, v, w, p, c)."""
        if sums.dtype != _torch().float64 or not sums.is_contiguous() or tuple(sums.shape) != (5,) + self.shape:
            raise ValueError("sums must be a contiguous float64 tensor of shape (5, nz, ny, nx)")
        self._call(self.lib.dnslab_accumulate, self.ctx, _ptr(sums))

    def body_force(self, box, out, row=0):
        """Force on the solid cells of box = (i0, i1, j0, j1, k0, k1) into
        out[row] (FP64 device tensor of shape (rows, 8): pressure force,
        viscous force, t, dt), asynchronously, so that a run can sample it
        every few steps without a host round trip."""
        if out.dtype != _torch().float64 or not out.is_contiguous() or out.dim() != 2 or out.shape[1] != 8:
            raise ValueError("out must be a contiguous float64 tensor of shape (rows, 8)")
        if not 0 <= row < out.shape[0]:
            raise IndexError("row out of range")
        b = (ctypes.c_int32 * 6)(*[int(q) for q in box])
        self._call(self.lib.dnslab_body_force, self.ctx, b, ctypes.c_void_p(out.data_ptr() + 64 * int(row)))

    def set_overlap(self, enable: bool):
        """True (the default): the scalar half of a step runs on a second
        stream beside the next step's velocity work; False: one stream, every
        kernel alone (same results)."""
        self._check(self.lib.dnslab_set_overlap(self.ctx, int(bool(enable))))

    def set_stage_pairs(self, mode: int):
        """RK4 stages two per pass: -1 by grid size (the default), 0 never,
        1 wherever the 64 x 8 tile divides the grid."""
        self._check(self.lib.dnslab_set_stage_pairs(self.ctx, int(mode)))

    def set_fft_pipeline(self, mode: int):
        """Pipelined column passes of the FFT solve: -1 by tile count (the
        default), 0 never, 1 wherever they apply."""
        self._check(self.lib.dnslab_set_fft_pipeline(self.ctx, int(mode)))

    # -- kernel timing -------------------------------------------------------
    def profile(self, kernel: Optional[str]):
        self._check(self.lib.dnslab_profile_enable(self.ctx, kernel.encode() if kernel else None))

    def profile_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.dnslab_profile_read(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # -- helpers -------------------------------------------------------------
    def _empty(self):
        return _torch().empty(self.shape, dtype=self.dtype, device=self.device)

    def _dev(self, a):
        torch = _torch()
        t = torch.as_tensor(a, dtype=self.dtype, device=self.device).reshape(self.shape)
        return t.contiguous()

    def state(self):
        """Host copies (numpy) of the bound fields (synchronises)."""
        self.stream.synchronize()
        return {k: getattr(self, k).double().cpu().numpy() for k in ("u", "v", "w", "p", "c")}
