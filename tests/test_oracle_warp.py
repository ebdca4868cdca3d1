"""Pins of the oracle's composite-affine bilinear warp (paper Sec. 2.1, 2.2).

Each check fixes the warp against something other than itself: exact crops and
translations, an exact 90-degree permutation, reproduction of affine functions
(bilinear interpolation is exact on them), explicit per-pixel loops, and the
composite 3x3 matrix chain.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import geometry, warp


def rng_stack(n, H, W, seed=1):
    return np.random.default_rng(seed).standard_normal((n, H, W)).astype(np.float32)


def test_identity_is_exact_centred_crop():
    F = rng_stack(3, 96, 96)
    A, b = geometry.inverse_from_misreg((0, 0, 0, 1), 96, 96, 80, 80)
    out = warp.warp(F, A, b, 80, 80, halo=1)
    # output pixel x maps to source x + 8; the halo window -1..80 -> 7..88
    assert np.array_equal(out, F[:, 7:89, 7:89].astype(np.float64))


@pytest.mark.parametrize("t", [(3, -2), (-5, 7), (1, 1)])
def test_integer_shift_is_exact_translation(t):
    F = rng_stack(2, 96, 96, seed=2)
    A, b = geometry.inverse_from_misreg((t[0], t[1], 0, 1), 96, 96, 80, 80)
    out = warp.warp(F, A, b, 80, 80, halo=1)
    # p_s = p_o + 8 - t
    r0, c0 = 7 - t[1], 7 - t[0]
    assert np.array_equal(out, F[:, r0:r0 + 82, c0:c0 + 82].astype(np.float64))


def test_quarter_turn_is_exact_permutation():
    F = rng_stack(2, 40, 40, seed=3)
    A, b = geometry.inverse_from_misreg((0, 0, math.pi / 2, 1), 40, 40, 40, 40)
    out = warp.warp(F, A, b, 40, 40, halo=0)
    # forward map rotates +90 deg in the (x=col, y=row) frame: out = rot90(in, -1)
    assert np.array_equal(out, np.rot90(F, -1, axes=(1, 2)).astype(np.float64))


def test_quarter_turn_direction_matches_forward_map():
    # a single bright IF pixel at source (x=30, y=20) must land where the forward
    # map p_o = c + R(+90deg)(p_s - c) sends it: (x, y) -> (c - (y - c), c + (x - c))
    F = np.zeros((1, 40, 40), np.float32)
    F[0, 20, 30] = 1.0
    A, b = geometry.inverse_from_misreg((0, 0, math.pi / 2, 1), 40, 40, 40, 40)
    out = warp.warp(F, A, b, 40, 40, halo=0)
    c = 19.5
    xo, yo = c - (20 - c), c + (30 - c)
    assert out[0, int(yo), int(xo)] == 1.0 and out.sum() == 1.0


def test_affine_function_reproduced_exactly():
    # bilinear interpolation is exact on affine functions: F = g.p_s + c
    H = W = 64
    g = np.array([0.37, -1.21])
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    F = (g[0] * xx + g[1] * yy + 0.5)[None]
    theta = (0.31, -0.77, math.radians(0.7), 1.013)
    A, b = geometry.inverse_from_misreg(theta, H, W, 40, 40)
    out = warp.warp(F, A, b, 40, 40, halo=1)
    xs, ys = warp.source_coords(A, b, 40, 40, 1)
    expect = g[0] * xs + g[1] * ys + 0.5
    assert np.max(np.abs(out[0] - expect)) < 1e-12


def test_zero_fill_outside_grid():
    F = np.ones((1, 20, 20), np.float32)
    A, b = geometry.inverse_from_misreg((15, 0, 0, 1), 20, 20, 20, 20)
    out, n_oob = warp.warp(F, A, b, 20, 20, halo=0, count_oob=True)
    # shift 15 px right: output columns 0..14 sample x_s = x_o - 15 < 0 -> zero
    assert np.all(out[0, :, :15] == 0.0) and np.all(out[0, :, 15:] == 1.0)
    assert n_oob == 20 * 15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vectorised_matches_per_pixel_loops(seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((2, 7, 7)).astype(np.float32)
    theta = (rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-0.4, 0.4), rng.uniform(0.8, 1.2))
    A, b = geometry.inverse_from_misreg(theta, 7, 7, 4, 4)
    v = warp.warp(F, A, b, 4, 4, halo=1)
    lp = warp.warp_loops(F, A, b, 4, 4, halo=1)
    assert np.max(np.abs(v - lp)) <= 1e-14


def test_inverse_map_inverts_forward_map():
    theta = (0.4, -0.3, math.radians(0.8), 1.02)
    A, b = geometry.inverse_from_misreg(theta, 96, 96, 80, 80, kappa=1.2)
    # forward: p_o = c_o + t + (m/kappa) R(rho)(p_s - c_s)
    rng = np.random.default_rng(0)
    po = rng.uniform(0, 80, size=(2, 10))
    ps = A @ po + b[:, None]
    back = np.array([39.5, 39.5])[:, None] + np.array([[0.4], [-0.3]]) + \
        (1.02 / 1.2) * geometry.rot(math.radians(0.8)) @ (ps - 47.5)
    assert np.max(np.abs(back - po)) < 1e-12


def test_composite_chain_reduces_to_misreg_form():
    theta = (0.3, -0.2, math.radians(0.5), 1.01)
    g = wl.misreg_geometry(theta)
    A1, b1 = geometry.inverse_from_misreg(theta, 96, 96, 80, 80)
    A2, b2 = geometry.inverse_from_geometry(g, 96, 96, 80, 80)
    assert np.max(np.abs(A1 - A2)) < 1e-14 and np.max(np.abs(b1 - b2)) < 1e-12


def test_composite_chain_cone_and_footprint():
    # an LGS pair: pupil pixel w maps to the DM at cone*w + footprint (DM px)
    g = wl.Geometry(cone_scale=0.8, footprint_x=10.0, footprint_y=-4.0)
    A, b = geometry.inverse_from_geometry(g, 512, 512, 476, 476)
    po = np.array([100.0, 300.0])
    ps = A @ po + b
    expect = 255.5 + 0.8 * (po - 237.5) + np.array([10.0, -4.0])
    assert np.max(np.abs(ps - expect)) < 1e-12


def test_derivative_maps_match_finite_differences_of_the_map():
    theta = np.array([0.3, -0.2, math.radians(0.5), 1.01])
    po = np.array([[13.0, 70.0, 41.5], [2.0, 55.0, 79.0]])
    dm = geometry.derivative_maps(theta, 96, 96, 80, 80)
    for j in range(4):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        Ap, bp = geometry.inverse_from_misreg(tp, 96, 96, 80, 80)
        Am, bm = geometry.inverse_from_misreg(tm, 96, 96, 80, 80)
        fd = ((Ap @ po + bp[:, None]) - (Am @ po + bm[:, None])) / (2 * h)
        an = dm[j][0] @ po + dm[j][1][:, None]
        assert np.max(np.abs(fd - an)) < 1e-6 * max(1.0, np.abs(an).max())


# --- WFS side of the composite chain (Sec. 2.1: the WFS transform, anamorphosis
# included, is multiplied into the same matrix as the DM and the LGS perspective).
# Each pin below is a point or a permutation worked out by hand, not a re-evaluation
# of the product.

def _ps(g, po, H_in=512, W_in=512, H_out=476, W_out=476):
    A, b = geometry.inverse_from_geometry(g, H_in, W_in, H_out, W_out)
    return A @ np.asarray(po, dtype=np.float64) + b


def test_wfs_rotation_quarter_turn_point():
    # WFS pixel (100, 300) on the 476 grid is (-137.5, 62.5) from its centre 237.5.
    # The forward map turns DM offsets by +90 deg, (x, y) -> (-y, x); undoing it sends
    # (-137.5, 62.5) to (62.5, 137.5), i.e. IF pixel 255.5 + (62.5, 137.5).
    g = wl.Geometry(wfs_rot=math.pi / 2)
    assert np.max(np.abs(_ps(g, (100.0, 300.0)) - np.array([318.0, 393.0]))) < 1e-12


def test_wfs_rotation_quarter_turn_is_exact_permutation():
    # same-size grids: a +90 deg WFS clocking permutes pixels exactly as rot90(in, -1)
    F = rng_stack(2, 40, 40, seed=5)
    A, b = geometry.inverse_from_geometry(wl.Geometry(wfs_rot=math.pi / 2), 40, 40, 40, 40)
    out = warp.warp(F, A, b, 40, 40, halo=0)
    assert np.array_equal(out, np.rot90(F, -1, axes=(1, 2)).astype(np.float64))


def test_wfs_anamorphic_magnification_point():
    # forward scales x offsets by 1.05 and y offsets by 0.97 (WFS axes), so the
    # offset (-137.5, 62.5) comes from (-130.952380952381, 64.43298969072166)
    g = wl.Geometry(wfs_mag_x=1.05, wfs_mag_y=0.97)
    expect = 255.5 + np.array([-130.95238095238095, 64.43298969072165])
    assert np.max(np.abs(_ps(g, (100.0, 300.0)) - expect)) < 1e-11


def test_wfs_anamorphic_half_scale_is_exact_decimation():
    # WFS x magnification 0.5 on an 81-wide IF grid and a 41-wide WFS grid (centres
    # 40 and 20): x_s = 40 + (x_o - 20) / 0.5 = 2 x_o, y unchanged: out = F[:, :, ::2]
    F = rng_stack(2, 41, 81, seed=6)
    A, b = geometry.inverse_from_geometry(wl.Geometry(wfs_mag_x=0.5), 41, 81, 41, 41)
    out = warp.warp(F, A, b, 41, 41, halo=0)
    assert np.array_equal(out, F[:, :, 0::2].astype(np.float64))


@pytest.mark.parametrize("s", [(3, -2), (-5, 7)])
def test_wfs_shift_is_exact_translation(s):
    # a WFS shift moves the image by exactly that many WFS pixels: p_s = p_o + 8 - s
    F = rng_stack(2, 96, 96, seed=7)
    A, b = geometry.inverse_from_geometry(wl.Geometry(wfs_shift_x=s[0], wfs_shift_y=s[1]),
                                          96, 96, 80, 80)
    out = warp.warp(F, A, b, 80, 80, halo=1)
    r0, c0 = 7 - s[1], 7 - s[0]
    assert np.array_equal(out, F[:, r0:r0 + 82, c0:c0 + 82].astype(np.float64))


def test_wfs_rotation_then_anamorphosis_order():
    # forward WFS part = diag(mx, my) R(rot): the clocking turns the footprint first and
    # the anamorphosis scales along the WFS's own axes.  With rot = 90 deg, mx = 1.25,
    # my = 0.8: undo diag -> (-137.5/1.25, 62.5/0.8) = (-110, 78.125); undo R(+90) ->
    # (78.125, 110).  (The other order would give (50, 171.875).)
    g = wl.Geometry(wfs_rot=math.pi / 2, wfs_mag_x=1.25, wfs_mag_y=0.8)
    expect = 255.5 + np.array([78.125, 110.0])
    assert np.max(np.abs(_ps(g, (100.0, 300.0)) - expect)) < 1e-12


def test_chain_order_dm_then_footprint_then_wfs():
    # cone 0.8, footprint (10, -4) DM px, WFS clocking +90 deg, documented order
    # DM placement -> LGS footprint -> WFS.  Undo the WFS: (-137.5, 62.5) -> (62.5, 137.5);
    # undo the footprint: 0.8 * (62.5, 137.5) + (10, -4) = (60, 106); IF pixel
    # 255.5 + (60, 106).  (Footprint applied after the clocking would give (46, 100).)
    g = wl.Geometry(cone_scale=0.8, footprint_x=10.0, footprint_y=-4.0, wfs_rot=math.pi / 2)
    expect = np.array([315.5, 361.5])
    assert np.max(np.abs(_ps(g, (100.0, 300.0)) - expect)) < 1e-12


def test_chain_full_worked_point():
    # every stage at once, worked by hand on WFS offset w = (-137.5, 62.5):
    #   undo WFS shift (2, -1):          (-139.5, 63.5)
    #   undo diag(1.25, 0.8):            (-111.6, 79.375)
    #   undo R(+90):  (x, y) -> (y, -x): (79.375, 111.6)
    #   undo footprint, cone 0.8:        0.8*(79.375, 111.6) + (10, -4) = (73.5, 85.28)
    #   undo DM shift (1, 2):            (72.5, 83.28)
    #   undo DM mag 2 and R(+90):        (x, y)/2 -> (y, -x): (41.64, -36.25)
    #   IF pixel:                        255.5 + (41.64, -36.25) = (297.14, 219.25)
    g = wl.Geometry(dm_shift_x=1.0, dm_shift_y=2.0, dm_rot=math.pi / 2, dm_mag=2.0,
                    cone_scale=0.8, footprint_x=10.0, footprint_y=-4.0,
                    wfs_shift_x=2.0, wfs_shift_y=-1.0, wfs_rot=math.pi / 2,
                    wfs_mag_x=1.25, wfs_mag_y=0.8)
    assert np.max(np.abs(_ps(g, (100.0, 300.0)) - np.array([297.14, 219.25]))) < 1e-11


def test_kappa_scales_wfs_offsets_into_dm_pixels():
    # kappa DM pixels per WFS pixel: with kappa = 2 and nothing else, a WFS offset w maps
    # to the DM offset 2 w.  WFS pixel (100, 300) on 476 -> 255.5 + (-275, 125).
    g = wl.Geometry(kappa=2.0)
    assert np.max(np.abs(_ps(g, (100.0, 300.0)) - np.array([-19.5, 380.5]))) < 1e-12


def test_oob_count_single_subaperture_by_hand():
    # one 4x4 subaperture, full pupil, identity map onto a 4x4 IF grid: the central
    # differences read columns {-1, 0, 3, 4} of rows 0..3 (c_x) and rows {-1, 0, 3, 4} of
    # columns 0..3 (c_y), 28 samples; the 16 in column -1 or 4, or in row -1 or 4, lie
    # outside the IF grid.
    from oracle import im as oim
    pupil = np.ones((4, 4), np.uint8)
    A, b = geometry.inverse_from_misreg((0, 0, 0, 1), 4, 4, 4, 4)
    assert oim.oob_count(A, b, pupil, 4, [0], 4, 4) == 16
    # on a 6x6 IF grid the same samples all lie inside (centred: source = sample + 1)
    A, b = geometry.inverse_from_misreg((0, 0, 0, 1), 6, 6, 4, 4)
    assert oim.oob_count(A, b, pupil, 4, [0], 6, 6) == 0
    # shifted one pixel right (t_x = 1): source x = sample x, so column -1 (4 samples) is
    # outside; columns 0..4 and rows -1..4 map to 0..4 and 0..5: inside
    A, b = geometry.inverse_from_misreg((1, 0, 0, 1), 6, 6, 4, 4)
    assert oim.oob_count(A, b, pupil, 4, [0], 6, 6) == 4


def test_oob_count_matches_warp_zero_fill():
    # every sample the count names is one the warp zero-fills: with a constant IF of 1,
    # the warped value at those samples is exactly 0 (inside: 1, or a partial edge cell)
    from oracle import im as oim
    pupil = wl.pupil_mask(40, 40.0)
    valid = wl.valid_subapertures(pupil, 5)
    A, b = geometry.inverse_from_misreg((9.5, -7.25, math.radians(2.0), 0.95), 50, 50, 40, 40)
    n = oim.oob_count(A, b, pupil, 5, valid, 50, 50)
    assert n > 0
    xs, ys = warp.source_coords(A, b, 40, 40, 1)
    phi = warp.warp(np.ones((1, 50, 50), np.float32), A, b, 40, 40, halo=1)[0]
    far = (xs < -1) | (xs > 50) | (ys < -1) | (ys > 50)
    assert np.all(phi[far] == 0.0)
