"""The allocation-free Poisson solve (dnslab_poisson_noalloc) against the
context's solve (dnslab_poisson), through the C ABI: the same grid, the same
right-hand side, FP64 and FP32.  Two calls in a row, the second on a smaller
grid, so that the second finds the shared scratch holding the first call's
spectrum and tables; an aliased call (p in place of rhs); no device memory
taken from torch's allocator by the calls; and a grid too large for the
scratch rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import scenarios
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

# (nx, ny, nz, mask boxes): the second grid is smaller than the first; the
# first (192 x 96 planes) takes the three column passes in both precisions,
# the second the fused y/z pass
GRIDS = [(64, 192, 96, 2), (48, 32, 24, 1)]
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _noalloc(lib, m, sc, prec, stream, rhs, out):
    P = m.make_params(sc, prec, ctypes.c_void_p(stream.cuda_stream))
    return lib.dnslab_poisson_noalloc(ctypes.byref(P), ctypes.c_void_p(rhs.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_noalloc_poisson_matches_context_solve(form):
    torch, m = need_gpu()
    lib = m.load()
    prec = m.FP64 if form == "fp64" else m.FP32_REFINE
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for call, (nx, ny, nz, nb) in enumerate(GRIDS):
        sc = scenarios.room(nx, ny, nz, dx=0.05, n_boxes=nb, seed=2204)
        announce(f"no-alloc poisson {form} call {call + 1}: {nx}x{ny}x{nz}")
        S = m.Solver(sc, precision=prec, device=dev)
        rng = np.random.default_rng(100 + call)
        rhs = S._dev(rng.standard_normal(sc.shape))
        ref = S.poisson(rhs)
        torch.cuda.synchronize()
        out = torch.full_like(rhs, float("nan"))
        alias = rhs.clone()
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        rc = _noalloc(lib, m, sc, prec, stream, rhs, out)
        assert rc == 0, lib.dnslab_last_error(None)
        rc = _noalloc(lib, m, sc, prec, stream, alias, alias)
        assert rc == 0, lib.dnslab_last_error(None)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        r = ref.double().cpu().numpy()
        scale = np.abs(r).max()
        assert scale > 0
        for got in (out, alias):
            g = got.double().cpu().numpy()
            assert np.isfinite(g).all()
            err = np.abs(g - r).max() / scale
            print(f"[no-alloc] {form} {nx}x{ny}x{nz}: max error {err:.3e} of max |p|", flush=True)
            assert err <= TOL[form], err
        S.close()


def test_noalloc_rejects_grid_beyond_scratch():
    torch, m = need_gpu()
    lib = m.load()
    sc = scenarios.room(48, 32, 24, dx=0.05, n_boxes=1, seed=2204)
    big = sc.copy()
    big.nx, big.ny, big.nz = 512, 256, 192          # FP64 spectrum 16 * 272 * 256 * 192 B > 64 MiB
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    x = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    announce("no-alloc poisson: oversized grid rejected on the host")
    rc = _noalloc(lib, m, big, m.FP64, stream, x, x)
    assert rc == -1
    assert b"bytes of scratch" in lib.dnslab_last_error(None)
    torch.cuda.synchronize()
    assert float(x.abs().sum()) == 0.0
