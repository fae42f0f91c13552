"""Oracle reference runs for the full-size parity tests (test infrastructure).

The FP64 oracle takes seconds to minutes per step at the benchmark grid sizes,
so these runs are started in child processes as soon as pytest has collected
the GPU tests that need them (``conftest.pytest_collection_finish``) and run
beside the other GPU tests.  Each run writes its final state and per-step
diagnostics to ``<out_dir>/<case>.npz`` (written to a temporary name, then
renamed, so a reader never sees a partial file).

Run directly: ``python tests/oracle_refs.py CASE OUT_DIR``.
"""
from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# case -> (scenario recipe, number of steps)
CASES = {
    "room100": ("room 256x128x96", 100),
    "large3": ("large room 512x256x192", 3),
}


def scenario(case):
    import scenarios
    if case == "room100":
        return scenarios.room()
    if case == "large3":
        return scenarios.room(512, 256, 192, dx=10.0 / 512)
    raise ValueError(case)


def run(case: str, out_dir: str) -> str:
    import numpy as np
    from oracle.step import Oracle
    sc = scenario(case)
    steps = CASES[case][1]
    O = Oracle.from_scenario(sc)
    st = Oracle.state_from_scenario(sc)
    keys = ("t", "dt", "ke", "div_l2", "co2_mass", "co2_room_mean", "cfl_max", "step")
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        st, d = O.step(st)
        hist.append([d[k] for k in keys])
        print(f"[oracle-ref] {case} step {s + 1}/{steps} {time.perf_counter() - t0:.1f} s", flush=True)
    path = os.path.join(out_dir, case + ".npz")
    tmp = os.path.join(out_dir, case + ".partial.npz")
    np.savez(tmp, u=st.u, v=st.v, w=st.w, p=st.p, c=st.c, diags=np.array(hist), keys=np.array(keys))
    os.replace(tmp, path)
    return path


if __name__ == "__main__":
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    print(run(sys.argv[1], sys.argv[2]), flush=True)
