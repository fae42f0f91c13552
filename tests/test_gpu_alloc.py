"""Device memory through the caller's allocator (the dnslab_params alloc /
free_ callbacks): with the binding's default, the context's workspace comes
from torch's caching allocator and goes back to it on destroy; the plain
hipMalloc path (callbacks NULL) gives the same results."""
import ctypes

import numpy as np
import pytest

import scenarios
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def test_workspace_comes_from_torch_allocator():
    torch, m = need_gpu()
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("allocator: workspace from torch")
    ws = m.workspace_bytes(sc)
    torch.cuda.synchronize()
    S = m.Solver(sc)            # state tensors and workspace from torch
    torch.cuda.synchronize()
    state = 5 * sc.ncells * 8
    with_ctx = torch.cuda.memory_allocated()
    S.step(3, diag=False)
    S.particles_sort(*[torch.zeros((3, 64), dtype=torch.float64, device=S.device) for _ in range(2)],
                     torch.full((64,), 1e-5, dtype=torch.float64, device=S.device))
    S.co2_histogram(16, 400.0, 1000.0)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated()
    lib = S.lib
    S.lib.dnslab_destroy(S.ctx)
    S.ctx = None
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated()
    # destroying the context returns the workspace, the list of cells next to
    # a solid, the sort scratch and the histogram counters to torch; the
    # state tensors stay with the Solver
    assert with_ctx >= ws + state
    assert grown - after >= ws
    assert after <= with_ctx - ws
    S.close()
    del S


def test_hipmalloc_path_matches_torch_path():
    torch, m = need_gpu()
    from paper_2204_02107_amd import _lib
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("allocator: NULL callbacks (hipMalloc)")
    S = m.Solver(sc)
    S.step(5, diag=False)
    ref = S.state()
    S.close()
    # a second context on the same inputs with the callbacks cleared
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    shape = sc.shape
    f = [torch.as_tensor(getattr(sc, k), dtype=torch.float64).reshape(shape).to(dev).contiguous()
         for k in ("u", "v", "w", "p", "c")]
    beta = torch.as_tensor(sc.beta, dtype=torch.uint8).to(dev).contiguous()
    n = len(sc.forced_idx)
    fidx = torch.as_tensor(sc.forced_idx, dtype=torch.int64).to(dev)
    fS = torch.as_tensor(sc.forced_S, dtype=torch.float64).to(dev)
    fus = torch.as_tensor(sc.forced_uset, dtype=torch.float64).reshape(-1).to(dev).contiguous()
    fcs = torch.as_tensor(sc.forced_cset, dtype=torch.float64).to(dev)
    room = torch.as_tensor(sc.room_mask, dtype=torch.uint8).to(dev).contiguous()
    P = m.make_params(sc, m.FP64, ctypes.c_void_p(stream.cuda_stream))
    assert not P.alloc and not P.free_
    ctx = ctypes.c_void_p()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    lib = _lib.load()
    _lib.check(lib.dnslab_init(ctypes.byref(P), p(beta), n, p(fidx), p(fS), p(fus), p(fcs), p(room),
                               *[p(t) for t in f], ctypes.byref(ctx)))
    _lib.check(lib.dnslab_step(ctx, 5, None), ctx)
    lib.dnslab_destroy(ctx)
    for k, t in zip(("u", "v", "w", "p", "c"), f):
        assert np.array_equal(t.cpu().numpy(), ref[k]), k


def test_pool_memory_from_torch_and_budget_counts_staging():
    torch, m = need_gpu()
    from paper_2204_02107_amd import serving
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=2204)
    announce("allocator: pool")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    pool = serving.Pool(1 << 30, m.FP64)
    slot = pool.admit(sc, 4)
    assert slot is not None
    used, active, resident = pool.usage()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    requested = pool._alloc.bytes_held()
    # state, workspace, list of cells next to a solid and the staging buffer,
    # all requested through torch's allocator (which rounds blocks up)
    assert held >= requested >= m.workspace_bytes(sc) + 5 * sc.ncells * 8
    assert used >= requested        # the budget counts everything the pool holds (plus table reserve)
    pool.step(4)
    pool.release(slot)
    pool.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
