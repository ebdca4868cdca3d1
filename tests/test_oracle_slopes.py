"""Pins of the oracle's slope step and the end-to-end IM (paper Sec. 2.2).

Central differences are exact on quadratics, so the subaperture mean of a
quadratic phase is an exact linear function of the subaperture's pupil-pixel
centroid; a linear IF gives exactly constant slopes A^T g through any affine
warp; per-pixel loops re-derive the vectorised sums.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import geometry, im, slopes, warp


def haloed_grid(H, W):
    Y, X = np.meshgrid(np.arange(-1, H + 1, dtype=np.float64),
                       np.arange(-1, W + 1, dtype=np.float64), indexing="ij")
    return X, Y


def test_linear_phase_gives_constant_slopes_on_any_mask():
    cfg = wl.scao_small()
    X, Y = haloed_grid(80, 80)
    phase = (0.25 * X - 0.6 * Y + 3.0)[None]
    s = slopes.slopes(phase, cfg.pupil, 10, cfg.valid)
    nv = cfg.n_valid
    assert np.max(np.abs(s[0, :nv] - 0.25)) < 1e-14
    assert np.max(np.abs(s[0, nv:] + 0.6)) < 1e-14


def test_quadratic_phase_gives_exact_centroid_slopes():
    cfg = wl.scao_elt(0)
    H = W = cfg.n_out
    X, Y = haloed_grid(H, W)
    al, be, ga, de, ep = 1e-3, -2e-3, 5e-4, 0.1, -0.05
    phase = (al * X ** 2 + be * Y ** 2 + ga * X * Y + de * X + ep * Y)[None]
    s = slopes.slopes(phase, cfg.pupil, cfg.p, cfg.valid)
    nv = cfg.n_valid
    P = cfg.pupil.astype(np.float64)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    p = cfg.p
    for kk in range(0, nv, 97):
        v, u = divmod(int(cfg.valid[kk]), cfg.n_sub)
        m = P[v * p:(v + 1) * p, u * p:(u + 1) * p]
        xb = (xx[v * p:(v + 1) * p, u * p:(u + 1) * p] * m).sum() / m.sum()
        yb = (yy[v * p:(v + 1) * p, u * p:(u + 1) * p] * m).sum() / m.sum()
        assert abs(s[0, kk] - (2 * al * xb + ga * yb + de)) < 1e-13
        assert abs(s[0, nv + kk] - (2 * be * yb + ga * xb + ep)) < 1e-13


def test_slopes_vectorised_matches_loops():
    rng = np.random.default_rng(5)
    pupil = wl.pupil_mask(24, 24.0, 0.3)
    valid = wl.valid_subapertures(pupil, 4)
    phase = rng.standard_normal((2, 26, 26))
    assert np.max(np.abs(slopes.slopes(phase, pupil, 4, valid) -
                         slopes.slopes_loops(phase, pupil, 4, valid))) < 1e-15


def test_partial_subaperture_uses_pupil_pixel_count():
    # one subaperture of 2x2 with a single pupil pixel: the mean is that pixel's g
    pupil = np.array([[1, 0], [0, 0]], np.uint8)
    phase = np.zeros((1, 4, 4))
    phase[0, 1, 2] = 2.0      # phi at (x=1, y=0)
    phase[0, 1, 0] = -2.0     # phi at (x=-1, y=0)
    s = slopes.slopes(phase, pupil, 2, np.array([0]))
    assert s[0, 0] == 2.0 and s[0, 1] == 0.0


@pytest.mark.parametrize("theta", [(0.3, -0.2, math.radians(0.5), 1.01),
                                   (-0.9, 0.4, math.radians(-1.0), 0.98),
                                   (2.5, 1.5, math.radians(30.0), 1.1)])
def test_linear_if_gives_exactly_AT_g(theta):
    cfg = wl.scao_small()
    g = np.array([0.013, -0.021])
    yy, xx = np.mgrid[0:96, 0:96].astype(np.float64)
    F = (g[0] * xx + g[1] * yy + 1.0)[None]
    A, b = geometry.inverse_from_misreg(theta, 96, 96, 80, 80)
    s = im.im_build(F, A, b, cfg.pupil, 10, cfg.valid)
    expect = A.T @ g
    nv = cfg.n_valid
    assert np.max(np.abs(s[0, :nv] - expect[0])) < 1e-15
    assert np.max(np.abs(s[0, nv:] - expect[1])) < 1e-15


def test_im_is_linear_in_the_if_stack():
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    A, b = geometry.inverse_from_misreg(cfg.theta, 96, 96, 80, 80)
    I = im.im_build(F, A, b, cfg.pupil, 10, cfg.valid)
    F64 = F.astype(np.float64)
    combo = (0.7 * F64[3] - 1.3 * F64[40])[None]
    Ic = im.im_build(combo, A, b, cfg.pupil, 10, cfg.valid)
    assert np.max(np.abs(Ic[0] - (0.7 * I[3] - 1.3 * I[40]))) < 1e-12 * np.abs(I).max()


def test_mirror_symmetry_of_identity_geometry():
    # theta = identity on the symmetric 8x8 geometry: the actuator mirrored in x
    # gives slopes mirrored in x with s_x negated and s_y unchanged
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    A, b = geometry.inverse_from_misreg((0, 0, 0, 1), 96, 96, 80, 80)
    I = im.im_build(F, A, b, cfg.pupil, 10, cfg.valid)
    nv = cfg.n_valid
    pos = {int(k): i for i, k in enumerate(cfg.valid)}
    for a in (0, 12, 30):
        r, c = divmod(a, 9)
        am = r * 9 + (8 - c)
        for k, i in pos.items():
            v, u = divmod(k, 8)
            im_ = pos[v * 8 + (7 - u)]
            assert abs(I[a, i] + I[am, im_]) < 1e-15
            assert abs(I[a, nv + i] - I[am, nv + im_]) < 1e-15


def test_warp_then_slopes_matches_im_build_loops_tiny():
    rng = np.random.default_rng(9)
    F = rng.standard_normal((2, 14, 14)).astype(np.float32)
    pupil = wl.pupil_mask(8, 8.0)
    valid = wl.valid_subapertures(pupil, 4)
    theta = (0.21, -0.33, 0.05, 1.04)
    A, b = geometry.inverse_from_misreg(theta, 14, 14, 8, 8)
    loops = slopes.slopes_loops(warp.warp_loops(F, A, b, 8, 8, 1), pupil, 4, valid)
    assert np.max(np.abs(im.im_build(F, A, b, pupil, 4, valid) - loops)) < 1e-14


def test_workload_counts():
    # the valid-subaperture and actuator counts implied by the stated readings
    assert wl.scao_small().n_valid == 52
    e = wl.scao_elt(0)
    assert e.n_valid == 4632 and e.grid.n_act == 5257
    m = wl.mcao(0)
    assert [g.n_act for g in m.grids] == [5257, 1789, 1125]
    assert len(m.pairs) == 18
    nv = [v.size for v in m.valids]
    assert len(set(nv)) > 1            # uneven valid-subaperture counts
