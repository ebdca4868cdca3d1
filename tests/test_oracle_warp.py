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
