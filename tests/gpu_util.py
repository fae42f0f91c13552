"""Helpers shared by the GPU parity tests (not collected: no test_ prefix)."""
import sys

import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_02107_amd as m
    m.load()            # raises if the HIP library is not built: no fallback
    return torch, m


def announce(msg):
    """Name the case before a GPU step, flushed, so a crash still shows it."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        return float(np.abs(got).max())
    return float(np.abs(got - ref).max() / scale)


def to_np(t):
    return t.detach().double().cpu().numpy()
