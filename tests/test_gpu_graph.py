"""Graph replay (whole steps captured into a HIP graph) gives the same results,
bit for bit, as issuing the same steps launch by launch; each replay is
checked against the eager run, with eager work and synchronisation between
replays."""
import numpy as np
import pytest

import scenarios
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def same_state(a, b):
    for k in ("u", "v", "w", "p", "c"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("per_stage,precision", [(False, "fp64"), (True, "fp64"), (False, "fp32")])
def test_graph_steps_equal_eager(per_stage, precision):
    torch, m = need_gpu()
    prec = m.FP64 if precision == "fp64" else m.FP32_REFINE
    sc = scenarios.room(64, 48, 36, dx=0.0390625, n_boxes=3, seed=5)
    announce(f"graph vs eager per_stage={per_stage} {precision}")
    E = m.Solver(sc, precision=prec, project_each_stage=per_stage)
    G = m.Solver(sc, precision=prec, project_each_stage=per_stage, graph_steps=4)
    for call in range(3):
        n = 10 + call            # 2 replays of 4 steps + 2..4 steps launch by launch
        de = E.step(n)
        dg = G.step(n)
        assert de == dg, call
        same_state(E.state(), G.state())
    assert E.read_diags(33) == G.read_diags(33)
    E.close()
    G.close()


def test_graph_tgv_small_grid():
    torch, m = need_gpu()
    sc = scenarios.taylor_green(32)
    announce("graph tgv32")
    E = m.Solver(sc)
    G = m.Solver(sc, graph_steps=16)
    E.step(64, diag=False)
    G.step(64, diag=False)
    same_state(E.state(), G.state())
    E.close()
    G.close()


def test_graph_steps_rejects_bad_arguments():
    torch, m = need_gpu()
    from paper_2204_02107_amd import _lib
    sc = scenarios.taylor_green(8)
    S = m.Solver(sc)
    lib = _lib.load()
    assert lib.dnslab_set_graph_steps(S.ctx, -1) == -1
    assert lib.dnslab_set_graph_steps(S.ctx, 5000) == -1
    if S.stream.cuda_stream == 0:
        assert lib.dnslab_set_graph_steps(S.ctx, 4) == -1    # legacy default stream
    S.close()


def test_pool_graph_equals_launches():
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    from test_gpu_serving import cases, run_mixed
    cs = cases()
    announce("pool graph vs launches")
    out = []
    for graph in (False, True):
        pool = Pool(8 << 30, m.FP32_REFINE, stream=torch.cuda.Stream(), graph=graph)
        slots = run_mixed(pool, cs, 9, stagger=(0, 2, 5))
        out.append([pool.state(s, c.shape) for s, c in zip(slots, cs)])
        pool.close()
    for a, b in zip(*out):
        same_state(a, b)


def test_graph_and_early_fork_on_a_large_grid():
    """2^23 cells: the scalar half forks before the momentum stages; graph
    replay and eager issue agree bit for bit, and both agree with the same
    scenario run through a pool of one (a direct group there, on the pool's
    own streams)."""
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    sc = scenarios.room(256, 256, 128, dx=10.0 / 256, n_boxes=4, seed=6)
    assert sc.ncells == 1 << 23
    announce("graph vs eager vs pool, 256x256x128")
    E = m.Solver(sc)
    G = m.Solver(sc, graph_steps=3)
    E.step(7, diag=False)
    G.step(7, diag=False)
    se, sg = E.state(), G.state()
    same_state(se, sg)
    E.close()
    G.close()
    pool = Pool(8 << 30, m.FP64)
    s = pool.admit(sc, 7)
    pool.step(7)
    same_state(se, pool.state(s, sc.shape))
    pool.close()
