"""Write the sampled FP64 oracle references of the full-size parity tests.

The FP64 oracle takes seconds (256x128x96) to about a minute (512x256x192)
per step, too long to recompute inside a GPU test run, so its results at
these sizes are stored here, written by this script and nothing else: it
imports only ``oracle`` (the plain numpy implementation of Sections 2.1-2.2
and 2.4) and ``scenarios`` (the seeded input generator).

For each case the file ``fullsize_<case>.npz`` holds, after the stated number
of whole steps from the scenario's initial state:

* ``idx``: flat cell indices (x fastest) of the sample: 8192 cells drawn
  uniformly with a fixed seed, plus for each field the 512 cells where its
  magnitude is largest;
* ``<f>_samp`` for f in u, v, w, p, c: the oracle's values at ``idx``;
* ``<f>_max``: max |f| over the whole grid (the scale of the relative error);
* ``<f>_zl2``, ``<f>_xl2``: the L2 norm of f over each z-plane and each
  x-plane (every cell enters one of each);
* ``diags`` (steps x len(keys)) with ``keys``: every step's diagnostics.

Usage: ``python tests/golden/make_fullsize_refs.py [room100] [large3]``.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

CASES = {
    # case: (scenario recipe, steps)
    "room100": ("room 256x128x96, 8 seeded boxes, 1 m/s duct, CFL 0.3, filter on", 100),
    "large3": ("large room 512x256x192, 8 seeded boxes, 1 m/s duct, CFL 0.3, filter on", 3),
}
FIELDS = ("u", "v", "w", "p", "c")
DIAG_KEYS = ("t", "dt", "ke", "div_l2", "co2_mass", "co2_room_mean", "cfl_max", "step")
N_UNIFORM = 8192
N_PEAK = 512
SAMPLE_SEED = 20220405


def scenario(case):
    import scenarios
    if case == "room100":
        return scenarios.room()
    if case == "large3":
        return scenarios.room(512, 256, 192, dx=10.0 / 512)
    raise ValueError(case)


def sample_indices(ncells, fields):
    """Uniform sample plus the largest-magnitude cells of every field."""
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = [rng.choice(ncells, size=min(N_UNIFORM, ncells), replace=False)]
    for f in fields:
        flat = np.abs(f.reshape(-1))
        idx.append(np.argpartition(flat, -N_PEAK)[-N_PEAK:])
    return np.unique(np.concatenate(idx)).astype(np.int64)


def write(case, out_dir=HERE):
    from oracle.step import Oracle
    sc = scenario(case)
    steps = CASES[case][1]
    O = Oracle.from_scenario(sc)
    st = Oracle.state_from_scenario(sc)
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        st, d = O.step(st)
        hist.append([d[k] for k in DIAG_KEYS])
        print(f"[golden] {case} step {s + 1}/{steps} {time.perf_counter() - t0:.1f} s", flush=True)
    fields = {f: getattr(st, f) for f in FIELDS}
    idx = sample_indices(sc.ncells, fields.values())
    out = {"idx": idx, "diags": np.array(hist), "keys": np.array(DIAG_KEYS),
           "shape": np.array(sc.shape), "steps": np.array(steps)}
    for f, a in fields.items():
        out[f + "_samp"] = a.reshape(-1)[idx]
        out[f + "_max"] = np.array(np.abs(a).max())
        out[f + "_zl2"] = np.sqrt(np.sum(a * a, axis=(1, 2)))
        out[f + "_xl2"] = np.sqrt(np.sum(a * a, axis=(0, 1)))
    path = os.path.join(out_dir, f"fullsize_{case}.npz")
    np.savez_compressed(path, **out)
    print(f"[golden] wrote {path} ({os.path.getsize(path)} bytes)", flush=True)
    return path


if __name__ == "__main__":
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    for case in sys.argv[1:] or list(CASES):
        write(case)
