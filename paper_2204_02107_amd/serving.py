"""Serving: continuous batching of ventilation scenarios on one GPU.

``Pool`` wraps the library's pool (``dnslab_pool_*`` in ``include/dnslab.h``):
scenarios are admitted against an HBM budget, stay resident, and are advanced
together by batched launches.  ``serve`` is the host request loop: requests
arrive over wall-clock time, are admitted as soon as memory is free, run their
steps interleaved with everything else on the GPU, and are retired (memory
returned) when done.  ``fifo`` is the baseline: the same stream served one
request at a time with the plain per-scenario loop.

Host logic only: every step of every scenario runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from typing import List, Optional

import numpy as np

from . import _lib
from ._lib import Diag, DnslabError, FP32_REFINE, FP64, Params


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _params(case, precision):
    from . import make_params
    return make_params(case, precision, None)


class Pool:
    def __init__(self, hbm_budget: int, precision=FP32_REFINE, stream=None, graph=False):
        import torch
        self.lib = _lib.load()
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        # every device block of the pool comes from torch's caching allocator
        self._alloc = _lib.TorchAllocator(torch.cuda.current_device(), stream.cuda_stream)
        _lib.check_pool(self.lib.dnslab_pool_create(int(hbm_budget), int(precision),
                                                   ctypes.c_void_p(stream.cuda_stream), *self._alloc.triple(),
                                                   ctypes.byref(h)))
        self.h = h
        self._keep = {}
        if graph:
            self._check(self.lib.dnslab_pool_set_graph(self.h, 1))

    def _check(self, rc):
        return _lib.check_pool(rc, self.h)

    def admit(self, case, target_steps: int) -> Optional[int]:
        """Admit a scenario; None when the budget has no room right now."""
        P = _params(case, self.precision)
        shape = (int(case.nz), int(case.ny), int(case.nx))
        beta = np.ascontiguousarray(case.beta, dtype=np.uint8).reshape(shape)
        fidx = np.ascontiguousarray(case.forced_idx, dtype=np.int64)
        fS = np.ascontiguousarray(case.forced_S, dtype=np.float64)
        fus = np.ascontiguousarray(case.forced_uset, dtype=np.float64).reshape(-1)
        fcs = np.ascontiguousarray(case.forced_cset, dtype=np.float64)
        room = None if case.room_mask is None else np.ascontiguousarray(case.room_mask, dtype=np.uint8)
        fields = [np.ascontiguousarray(getattr(case, k), dtype=np.float64) for k in ("u", "v", "w", "p", "c")]
        n = len(fidx)
        slot = ctypes.c_int32()
        rc = self.lib.dnslab_pool_admit(
            self.h, ctypes.byref(P), int(target_steps), _ptr(beta), n,
            _ptr(fidx) if n else None, _ptr(fS) if n else None, _ptr(fus) if n else None,
            _ptr(fcs) if n else None, _ptr(room), *[_ptr(f) for f in fields], ctypes.byref(slot))
        if rc == -6:   # DNSLAB_EAGAIN
            return None
        self._check(rc)
        return int(slot.value)

    def step(self, nsteps: int):
        self._check(self.lib.dnslab_pool_step(self.h, int(nsteps)))

    def query(self, slot: int):
        d = Diag()
        done_steps = ctypes.c_int64()
        done = ctypes.c_int32()
        self._check(self.lib.dnslab_pool_query(self.h, int(slot), ctypes.byref(d), ctypes.byref(done_steps),
                                               ctypes.byref(done)))
        return d.as_dict(), int(done_steps.value), bool(done.value)

    def read_field(self, slot: int, field: int, shape):
        out = np.empty(shape, dtype=np.float64)
        self._check(self.lib.dnslab_pool_read_field(self.h, int(slot), int(field), _ptr(out)))
        return out

    def state(self, slot: int, shape):
        return {k: self.read_field(slot, i, shape) for i, k in enumerate(("u", "v", "w", "p", "c"))}

    def release(self, slot: int):
        self._check(self.lib.dnslab_pool_release(self.h, int(slot)))

    def usage(self):
        b = ctypes.c_size_t()
        a = ctypes.c_int32()
        r = ctypes.c_int32()
        self._check(self.lib.dnslab_pool_usage(self.h, ctypes.byref(b), ctypes.byref(a), ctypes.byref(r)))
        return int(b.value), int(a.value), int(r.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.dnslab_pool_destroy(self.h)
            self.h = None
        if getattr(self, "_alloc", None) is not None:
            self._alloc.close()
            self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(requests, cases, hbm_budget: int, precision=FP32_REFINE, chunk: int = 25, log=None,
          graph: bool = True) -> List[dict]:
    """Run a request stream with continuous batching.

    ``requests``: dicts with ``id``, ``arrival`` (s from stream start) and
    ``n_steps``; ``cases[id]``: the scenario.  Returns per-request records with
    arrival, admission and completion times (s) and the final diagnostics.

    The pool works on its own non-blocking stream.  The loop keeps one chunk of
    steps in flight: while the GPU runs it, the host admits the requests that
    have arrived (their set-up runs on the pool's admission stream), then waits
    for the chunk, retires the scenarios it completed and enqueues the next.
    """
    import torch
    stream = torch.cuda.Stream()
    pool = Pool(hbm_budget, precision, stream=stream, graph=graph)
    pending = deque(sorted(requests, key=lambda r: r["arrival"]))
    waiting = deque()
    running = {}
    out = []
    t0 = time.perf_counter()
    cell_steps = 0
    inflight = None          # (event, slots finishing in that chunk)
    while pending or waiting or running or inflight:
        now = time.perf_counter() - t0
        while pending and pending[0]["arrival"] <= now:
            waiting.append(pending.popleft())
        while waiting:
            r = waiting[0]
            slot = pool.admit(cases[r["id"]], r["n_steps"])
            if slot is None:
                break
            waiting.popleft()
            running[slot] = dict(r, admitted=time.perf_counter() - t0, slot=slot, left=r["n_steps"])
        if inflight is not None:
            ev, finishing = inflight
            ev.synchronize()
            tdone = time.perf_counter() - t0
            for slot in finishing:
                r = running.pop(slot)
                diag, nsteps, done = pool.query(slot)
                r["finished"] = tdone
                r["diag"] = diag
                c = cases[r["id"]]
                cell_steps += c.nx * c.ny * c.nz * nsteps
                pool.release(slot)
                out.append(r)
                if log:
                    log(f"done id={r['id']} ttr={r['finished'] - r['arrival']:.3f}s")
            inflight = None
        if running:
            # every scenario stops at its own target inside the pool
            pool.step(chunk)
            finishing = []
            for slot, r in running.items():
                r["left"] = max(0, r["left"] - chunk)
                if r["left"] == 0:
                    finishing.append(slot)
            ev = torch.cuda.Event()
            ev.record(stream)
            inflight = (ev, finishing)
        elif pending:
            time.sleep(max(0.0, min(0.005, pending[0]["arrival"] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    pool.close()
    for r in out:
        r["wall"] = wall
        r["cell_steps_total"] = cell_steps
    return out


def fifo(requests, cases, precision=FP64, log=None) -> List[dict]:
    """Baseline: one request at a time, in arrival order, with the plain
    per-scenario loop (``dnslab_step``)."""
    import torch
    from . import Solver
    out = []
    t0 = time.perf_counter()
    cell_steps = 0
    for r in sorted(requests, key=lambda r: r["arrival"]):
        now = time.perf_counter() - t0
        if r["arrival"] > now:
            time.sleep(r["arrival"] - now)
        start = time.perf_counter() - t0
        c = cases[r["id"]]
        S = Solver(c, precision=precision)
        d = S.step(r["n_steps"])
        S.close()
        torch.cuda.synchronize()
        fin = time.perf_counter() - t0
        cell_steps += c.nx * c.ny * c.nz * r["n_steps"]
        out.append(dict(r, admitted=start, finished=fin, diag=d))
        if log:
            log(f"fifo id={r['id']} ttr={fin - r['arrival']:.3f}s")
    wall = time.perf_counter() - t0
    for r in out:
        r["wall"] = wall
        r["cell_steps_total"] = cell_steps
    return out


def summarize(records) -> dict:
    ttr = np.array([r["finished"] - r["arrival"] for r in records])
    wall = records[0]["wall"] if records else 0.0
    cs = records[0]["cell_steps_total"] if records else 0
    return {
        "requests": len(records),
        "p50_s": float(np.percentile(ttr, 50)) if len(ttr) else None,
        "p99_s": float(np.percentile(ttr, 99)) if len(ttr) else None,
        "max_s": float(ttr.max()) if len(ttr) else None,
        "wall_s": wall,
        "throughput_Gcell_steps_s": cs / wall / 1e9 if wall else None,
    }
