"""Serving pool: admission by HBM budget, continuous batching, and results that
are the same alone and in the mix.

Scenarios of different grid sizes are admitted at different times into one
pool and advanced by batched launches; each must end bitwise equal to the same
scenario run alone (plain dnslab_step in FP64, a pool of one in FP32), and a
pooled FP64 scenario must match the oracle like a plain one.
"""
import numpy as np
import pytest

from oracle.step import Oracle
import scenarios
from gpu_util import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu

DX = 0.0390625


def cases():
    return [
        scenarios.room(64, 64, 64, dx=DX, u_in=1.0, n_boxes=3, seed=11, box_max_frac=0.4),
        scenarios.room(128, 64, 64, dx=DX, u_in=0.1, n_boxes=5, seed=12, box_max_frac=0.4),
        scenarios.room(96, 48, 32, dx=DX, u_in=1.0, n_boxes=0, seed=13, box_max_frac=0.4),
    ]


def run_mixed(pool, cs, steps, stagger=(0, 3, 7)):
    """Admit scenario q after stagger[q] pool steps; every scenario runs `steps`."""
    slots = [None] * len(cs)
    t = 0
    while True:
        for q, c in enumerate(cs):
            if slots[q] is None and t >= stagger[q]:
                slots[q] = pool.admit(c, steps)
                assert slots[q] is not None
        if all(s is not None for s in slots):
            _, active, _ = pool.usage()
            if active == 0:
                break
        pool.step(1)
        t += 1
    return slots


def test_pool_fp64_mix_equals_plain_step():
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    cs = cases()
    steps = 12
    announce("pool fp64 mix vs plain")
    alone = []
    for c in cs:
        S = m.Solver(c)
        S.step(steps, diag=False)
        alone.append(S.state())
        S.close()
    pool = Pool(8 << 30, m.FP64)
    slots = run_mixed(pool, cs, steps)
    for q, c in enumerate(cs):
        got = pool.state(slots[q], c.shape)
        d, nst, done = pool.query(slots[q])
        assert done and nst == steps and d["step"] == steps
        for k in ("u", "v", "w", "p", "c"):
            assert np.array_equal(got[k], alone[q][k]), (q, k)
    pool.close()


def test_pool_fp32_mix_equals_alone():
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    cs = cases()
    steps = 10
    announce("pool fp32 mix vs alone")
    alone = []
    for c in cs:
        pool = Pool(8 << 30, m.FP32_REFINE)
        s = pool.admit(c, steps)
        pool.step(steps)
        alone.append(pool.state(s, c.shape))
        pool.close()
    pool = Pool(8 << 30, m.FP32_REFINE)
    slots = run_mixed(pool, cs, steps, stagger=(5, 0, 2))
    for q, c in enumerate(cs):
        got = pool.state(slots[q], c.shape)
        for k in ("u", "v", "w", "p", "c"):
            assert np.array_equal(got[k], alone[q][k]), (q, k)
    pool.close()


def test_pool_budget_admission_and_release():
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    c0, c1, _ = cases()
    announce("pool budget")
    probe = Pool(1 << 40, m.FP32_REFINE)
    s = probe.admit(c1, 1)
    need1, _, _ = probe.usage()
    probe.close()
    pool = Pool(int(need1 * 1.5), m.FP32_REFINE)
    a = pool.admit(c1, 3)
    assert a is not None
    assert pool.admit(c1, 3) is None          # no room for a second one
    used, active, resident = pool.usage()
    assert used == need1 and active == 1 and resident == 1
    pool.step(3)
    _, _, done = pool.query(a)
    assert done
    pool.release(a)
    # the scenario's bytes return to the budget; the pool keeps (and counts)
    # its staging buffer for admission inputs, a small part of a scenario
    left = pool.usage()[0]
    assert 0 < left < 0.1 * need1
    b = pool.admit(c1, 2)                     # memory returned to the budget
    assert b is not None
    pool.close()


def test_pooled_scenario_matches_oracle():
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    cs = cases()
    target = scenarios.room(64, 48, 36, dx=DX, n_boxes=3, seed=2204)
    announce("pool vs oracle")
    pool = Pool(8 << 30, m.FP64)
    other = pool.admit(cs[1], 6)
    slot = pool.admit(target, 6)
    pool.step(6)
    got = pool.state(slot, target.shape)
    O = Oracle.from_scenario(target)
    st, diags = O.run(Oracle.state_from_scenario(target), 6)
    for k in ("u", "v", "w", "p", "c"):
        assert rel_err(got[k], getattr(st, k)) < 1e-10, k
    d, _, _ = pool.query(slot)
    assert abs(d["co2_room_mean"] - diags[-1]["co2_room_mean"]) < 1e-10 * diags[-1]["co2_room_mean"]
    pool.close()


def test_pool_large_scenarios_direct_equal_plain():
    """Scenarios of at least 2^20 cells run their own plain step inside the pool
    (with the scalar half deferred onto a second stream across pool steps);
    two of them plus a small one, admitted at different times, must end bitwise
    equal to plain runs."""
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    big = [scenarios.room(128, 128, 64, dx=DX, u_in=1.0, n_boxes=4, seed=21, box_max_frac=0.4),
           scenarios.room(128, 128, 64, dx=DX, u_in=0.1, n_boxes=2, seed=22, box_max_frac=0.4)]
    cs = big + [cases()[0]]
    steps = 7
    announce("pool direct large vs plain")
    alone = []
    for c in cs:
        S = m.Solver(c)
        S.step(steps, diag=False)
        alone.append(S.state())
        S.close()
    pool = Pool(8 << 30, m.FP64, stream=torch.cuda.Stream())
    slots = [None] * len(cs)
    t = 0
    while True:
        for q, c in enumerate(cs):
            if slots[q] is None and t >= (0, 2, 1)[q]:
                slots[q] = pool.admit(c, steps)
        if all(s is not None for s in slots) and pool.usage()[1] == 0:
            break
        pool.step(3)           # several steps per call: the deferred scalar half crosses steps
        t += 1
    for q, c in enumerate(cs):
        got = pool.state(slots[q], c.shape)
        for k in ("u", "v", "w", "p", "c"):
            assert np.array_equal(got[k], alone[q][k]), (q, k)
    pool.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pool_mix_with_channel_case(precision):
    """A 2D obstacle-in-channel scenario (nz = 1) pooled with two small rooms
    whose (ky, kz) planes take the fused y/z FFT pass and one larger room
    (column passes): each ends bitwise equal to its pool of one."""
    torch, m = need_gpu()
    from paper_2204_02107_amd.serving import Pool
    prec = m.FP64 if precision == "fp64" else m.FP32_REFINE
    cs = [scenarios.cube_channel(8), cases()[0], cases()[1],
          scenarios.room(96, 96, 64, dx=DX, u_in=1.0, n_boxes=2, seed=14, box_max_frac=0.4)]
    steps = 8
    announce(f"pool {precision} mix with channel case")
    alone = []
    for c in cs:
        pool = Pool(8 << 30, prec)
        s = pool.admit(c, steps)
        pool.step(steps)
        alone.append(pool.state(s, c.shape))
        pool.close()
    pool = Pool(8 << 30, prec)
    slots = run_mixed(pool, cs, steps, stagger=(0, 2, 1, 4))
    for q, c in enumerate(cs):
        got = pool.state(slots[q], c.shape)
        for k in ("u", "v", "w", "p", "c"):
            assert np.array_equal(got[k], alone[q][k]), (q, k)
    pool.close()
