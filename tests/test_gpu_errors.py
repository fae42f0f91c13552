"""Error paths through the C ABI on the GPU: argument errors leave nothing
enqueued and the state untouched, and a non-finite value in the fields is
reported by the next synchronising step.  Every condition comes from the host
(an argument or a value in the input); every kernel runs to its normal end."""
import ctypes

import numpy as np
import pytest

import scenarios
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def test_argument_errors_enqueue_nothing():
    torch, m = need_gpu()
    from paper_2204_02107_amd import _lib
    sc = scenarios.room(32, 32, 24, dx=0.05, n_boxes=2, seed=3)
    announce("argument errors")
    S = m.Solver(sc)
    S.step(2, diag=False)
    before = S.state()
    lib = _lib.load()
    assert lib.dnslab_step(S.ctx, -1, None) == -1
    assert lib.dnslab_poisson(S.ctx, None, None) == -1
    assert lib.dnslab_project(S.ctx, None, None, None) == -1
    assert lib.dnslab_read_diags(S.ctx, -1, None) == -1
    assert lib.dnslab_read_diags(S.ctx, 5000, None) == -1
    assert lib.dnslab_profile_enable(S.ctx, b"no_such_kernel") == -1
    assert b"kernel" in lib.dnslab_last_error(S.ctx)
    box = (ctypes.c_int32 * 6)(0, 0, 0, 1, 0, 1)
    assert lib.dnslab_body_force(S.ctx, box, None) == -1
    assert lib.dnslab_particles_sort(S.ctx, -1, None, None, None) == -1
    assert lib.dnslab_co2_histogram(S.ctx, 0, 0.0, 1.0, None) == -1
    after = S.state()
    for k in ("u", "v", "w", "p", "c"):
        assert np.array_equal(after[k], before[k]), k
    # the context still works
    d = S.step(1)
    assert d["step"] == 3
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonfinite_field_is_reported(precision):
    """A NaN in one fluid cell of u spreads through the step; the step that
    returns diagnostics reports DNSLAB_ENONFINITE, and read_diags shows the
    NaN."""
    torch, m = need_gpu()
    prec = m.FP64 if precision == "fp64" else m.FP32_REFINE
    sc = scenarios.room(32, 32, 24, dx=0.05, n_boxes=2, seed=3)
    k, j, i = np.argwhere(sc.beta == 1)[len(np.argwhere(sc.beta == 1)) // 2]
    sc.u[k, j, i] = np.nan
    announce(f"non-finite field {precision}")
    S = m.Solver(sc, precision=prec)
    with pytest.raises(m.DnslabError) as e:
        S.step(2)
    assert e.value.code == -7
    d = S.read_diags(1)[0]
    assert not np.isfinite(d["ke"])
    S.close()
