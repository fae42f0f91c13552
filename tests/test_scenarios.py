"""Checks of the seeded input recipes (geometry, source mask of Section 2.1)."""
import numpy as np

import scenarios


def test_tanh_factor_shape():
    h = 0.4
    r = np.array([0.0, 1e-9, h, 10 * h])
    f = scenarios.tanh_factor(r, h, 5.0)
    assert f[0] == 1.0 and f[1] == 1.0
    assert abs(f[2] - 0.5) < 1e-15             # bracket vanishes at r = W/2
    assert f[3] < 1e-20
    rr = np.linspace(0, 3 * h, 200)
    ff = scenarios.tanh_factor(rr, h, 5.0)
    assert np.all(np.diff(ff) <= 0) and ff.min() >= 0 and ff.max() <= 1


def test_room_geometry():
    sc = scenarios.room(64, 48, 40, dx=0.05, n_boxes=3, seed=1)
    b = sc.beta
    assert b.dtype == np.uint8 and set(np.unique(b)) <= {0, 1}
    nd = sc.meta["duct_cells"]
    # slabs closed except for the duct cut through the x walls
    assert b[:2].max() == 0 and b[:, :2].max() == 0
    assert b[:, :, :2].sum() == 2 * nd * nd
    # forced cells are fluid, sorted, unique, S in (0, 1]
    idx = sc.forced_idx
    assert np.all(np.diff(idx) > 0)
    assert np.all(b.ravel()[idx] == 1)
    assert sc.forced_S.min() > 1e-6 and sc.forced_S.max() <= 1.0
    assert np.all(sc.forced_uset[:, 0] == 1.0) and np.all(sc.forced_cset == 400.0)
    assert np.all(sc.c[b == 1] == 1000.0) and np.all(sc.c[b == 0] == 0.0)
    # same seed, same scenario
    sc2 = scenarios.room(64, 48, 40, dx=0.05, n_boxes=3, seed=1)
    assert np.array_equal(sc.beta, sc2.beta) and np.array_equal(sc.forced_S, sc2.forced_S)


def test_serving_stream_is_seeded():
    a = scenarios.serving_requests(8)
    b = scenarios.serving_requests(8)
    assert a == b
    assert all(r["grid"] in [(64, 64, 64), (128, 64, 64), (192, 96, 64), (256, 128, 96)] for r in a)
    assert all(0 <= r["n_boxes"] <= 12 for r in a)


def _is_fft_size(n):
    for f in (2, 3):
        while n % f == 0:
            n //= f
    return n == 1


def test_cube_channel_geometry():
    """Obstacle in a channel (Tables 1-2): FFT grid sizes, the channel of
    6 n_h fluid cells between equal walls, an n_h x n_h obstacle centred on the
    channel 1.2 D from the seam, the parabolic inflow peaking at about U_max
    with the bulk velocity 2/3 U_max, Re_ob from nu."""
    for n_h in (8, 30):
        sc = scenarios.cube_channel(n_h)
        m = sc.meta
        assert sc.nz == 1 and sc.nx % 2 == 0 and _is_fft_size(sc.nx) and _is_fft_size(sc.ny)
        nf, w = 6 * n_h, m["wall"]
        assert sc.ny == nf + 2 * w and w >= 2
        b = sc.beta[0]
        assert b[:w].max() == 0 and b[w + nf:].max() == 0
        i0, i1, j0, j1, _, _ = m["obstacle_cells"]
        assert i1 - i0 == n_h and j1 - j0 == n_h
        assert b[j0:j1, i0:i1].max() == 0 and b[w:w + nf].sum() == nf * sc.nx - n_h * n_h
        assert (j0 - w) == (w + nf - j1)                       # centred across the channel
        assert abs((i0 + i1) / 2 - 1.2 * nf) <= 0.5            # 1.2 D downstream of the seam
        assert abs(sc.nx / nf - 8.8) < 0.6
        d = sc.spacing[0]
        assert abs(d - m["h"] / n_h) < 1e-15 and abs(sc.spacing[1] - d) < 1e-15
        assert abs(m["u_b"] * m["h"] / sc.nu - 84.0) < 1e-9
        # inflow: sorted fluid cells around the seam, u_set a parabola across the channel
        idx = sc.forced_idx
        assert np.all(np.diff(idx) > 0) and np.all(sc.beta.ravel()[idx] == 1)
        prof = sc.u[0, w:w + nf, 0]
        assert abs(prof.max() / m["u_max"] - 1) < 2.0 / nf
        assert abs(prof.mean() / m["u_b"] - 1) < 2.0 / nf
        assert np.allclose(prof, prof[::-1], rtol=0, atol=1e-14)
        assert np.all(sc.forced_uset[:, 1:] == 0) and sc.forced_uset[:, 0].max() <= m["u_max"]
