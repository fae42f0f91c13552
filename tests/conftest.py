import os
import subprocess
import sys
import tempfile
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Oracle reference runs started in child processes (see tests/oracle_refs.py):
# case -> (Popen, output directory, log path)
_REF_RUNS = {}


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "oracle_ref(case): uses a full-size oracle run computed in a child process")


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def pytest_collection_finish(session):
    """Start the oracle runs the selected tests need, before any test runs, so
    that they overlap the other GPU tests (the oracle is single-threaded)."""
    cases = []
    for item in session.items:
        for mk in item.iter_markers("oracle_ref"):
            if mk.args and mk.args[0] not in cases:
                cases.append(mk.args[0])
    if not cases or not _gpu_present():
        return
    out = tempfile.mkdtemp(prefix="dnslab_oracle_refs_")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    for case in cases:
        log = os.path.join(out, case + ".log")
        with open(log, "w") as lf:
            p = subprocess.Popen([sys.executable, os.path.join(ROOT, "tests", "oracle_refs.py"), case, out],
                                 stdout=lf, stderr=subprocess.STDOUT, cwd=ROOT, env=env)
        _REF_RUNS[case] = (p, out, log)
        print(f"[oracle-ref] started {case} (pid {p.pid}) -> {out}", file=sys.stderr, flush=True)


def pytest_sessionfinish(session, exitstatus):
    for case, (p, out, log) in list(_REF_RUNS.items()):
        if p.poll() is None:
            p.kill()
            p.wait()
        for name in os.listdir(out):
            try:
                os.remove(os.path.join(out, name))
            except OSError:
                pass
        try:
            os.rmdir(out)
        except OSError:
            pass
    _REF_RUNS.clear()


@pytest.fixture
def oracle_ref():
    """wait(case, timeout) -> dict of the oracle's final fields and its
    per-step diagnostics (list of dicts), waiting for the child run."""
    import numpy as np

    def wait(case, timeout=900.0):
        if case not in _REF_RUNS:
            pytest.fail(f"oracle reference {case} was not started (mark the test oracle_ref('{case}'))")
        p, out, log = _REF_RUNS[case]
        path = os.path.join(out, case + ".npz")
        t0 = time.time()
        last = t0
        while not os.path.exists(path):
            if p.poll() is not None and not os.path.exists(path):
                with open(log) as f:
                    tail = f.read()[-2000:]
                pytest.fail(f"oracle reference {case} exited with {p.returncode}:\n{tail}")
            if time.time() - t0 > timeout:
                pytest.fail(f"oracle reference {case} not ready after {timeout} s")
            if time.time() - last > 30:
                last = time.time()
                with open(log) as f:
                    lines = f.read().strip().splitlines()
                print(f"[oracle-ref] waiting for {case}: {lines[-1] if lines else 'starting'}", flush=True)
            time.sleep(1.0)
        p.wait()
        z = np.load(path)
        keys = [str(k) for k in z["keys"]]
        diags = [dict(zip(keys, row)) for row in z["diags"]]
        for d in diags:
            d["step"] = int(d["step"])
        return {"u": z["u"], "v": z["v"], "w": z["w"], "p": z["p"], "c": z["c"], "diags": diags}

    return wait
