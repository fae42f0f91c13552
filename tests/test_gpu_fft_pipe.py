"""The pipelined column passes of the FFT solve (each block walks several
tiles, the next tile's asynchronous global -> LDS load in flight while the
current one is transformed) against the one-tile-per-block passes and the
oracle's Poisson solve (Section 2.2), forced on through
dnslab_set_fft_pipeline on grids where the default would not pick them.

The two GPU paths evaluate the same transforms in the same order, so their
results must agree bit for bit; against the oracle the FFT-solve bar of the
parity tests applies (1e-11 in FP64, 1e-5 in FP32).  The shapes (nz, ny, nx)
cover ragged kx tiles (nx/2 not a multiple of the tile width), the Nyquist
column tiles, both precisions, an odd nx/2 (FP64 only: the FP32 pipeline
loads two columns per lane and needs nx/2 even), lengths of mixed radix,
a 128 x 128 plane that the FP32 form gives to the fused plane pass
(the switch then changes nothing), and the longest compile-time transform
lengths (z 384 and 768, y 1024).
"""
import numpy as np
import pytest

from oracle import ops
import scenarios
from gpu_util import announce, need_gpu, rel_err, to_np

pytestmark = pytest.mark.gpu

# (ky, kz) planes above 16384 values, so that the column passes (not the
# fused plane pass) run in both precisions
SHAPES = [(128, 192, 32), (192, 128, 48), (256, 96, 36), (96, 256, 54), (256, 128, 24), (128, 128, 64),
          (768, 64, 32), (64, 1024, 16), (384, 96, 24)]


def case(shape, seed):
    nz, ny, nx = shape
    beta = np.ones(shape, np.uint8)
    z = np.zeros(shape)
    return scenarios.Scenario(
        name="pipe", nx=nx, ny=ny, nz=nz, lx=nx * 0.05, ly=ny * 0.045, lz=nz * 0.055,
        nu=1e-3, alpha_c=1e-3, tau_f=0.1, body=(0.0, 0.0, 0.0), cfl=0.3, dt_fixed=0.01, u_ref=1.0,
        n_piter=4, filter=False, beta=beta, forced_idx=np.zeros(0, np.int64), forced_S=np.zeros(0),
        forced_uset=np.zeros((0, 3)), forced_cset=np.zeros(0), room_mask=None,
        u=z.copy(), v=z.copy(), w=z.copy(), p=z.copy(), c=z.copy())


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_pipelined_column_passes(shape, form):
    torch, m = need_gpu()
    prec = m.FP64 if form == "fp64" else m.FP32_REFINE
    sc = case(shape, 3)
    announce(f"fft pipeline {form} shape={shape}")
    S = m.Solver(sc, precision=prec)
    r = np.random.default_rng(21).standard_normal(shape)
    S.set_fft_pipeline(0)
    plain = to_np(S.poisson(r))
    S.set_fft_pipeline(1)
    piped = to_np(S.poisson(r))
    S.close()
    assert np.array_equal(plain, piped), np.abs(plain - piped).max()
    ref = ops.poisson_solve(r, sc.spacing)
    err = rel_err(piped, ref)
    assert err < (1e-11 if form == "fp64" else 1e-5), err
