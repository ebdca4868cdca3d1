"""Pins of the oracle's edge repair (paper Sec. 2.3: strict binarisation and
clearing, edge identification by binary dilation, four-direction extrapolation
2 P1 - P2 or P1, averaged over the valid directions).

Tiny masks are worked out by hand; a linear phase on a rectangular core is
restored exactly (linear extrapolation is exact on it); the threshold is
inclusive; and, end to end, a pre-masked linear IF whose mask edge falls on the
WFS window's outer ring gives the exact slopes A^T g again, which it does not
without the repair.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import geometry, im as oim, repair


def rnd(H, W, seed=0):
    return np.random.default_rng(seed).standard_normal((H, W))


def test_single_pixel_core():
    S = np.zeros((5, 5), bool)
    S[2, 2] = True
    phi = rnd(5, 5)
    out = repair.repair(phi, S)
    # the four cross neighbours each see the core in one direction, one pixel deep
    for y, x in ((1, 2), (3, 2), (2, 1), (2, 3)):
        assert out[y, x] == phi[2, 2]
    mask = np.zeros((5, 5), bool)
    mask[2, 2] = True
    for y, x in ((1, 2), (3, 2), (2, 1), (2, 3)):
        mask[y, x] = True
    assert np.all(out[~mask] == 0.0) and out[2, 2] == phi[2, 2]


def test_two_pixel_core_by_hand():
    # core (x=1, y=2) and (x=2, y=2): a = phi(1,2), b = phi(2,2)
    S = np.zeros((5, 5), bool)
    S[2, 1] = S[2, 2] = True
    phi = rnd(5, 5, 1)
    a, b = phi[2, 1], phi[2, 2]
    out = repair.repair(phi, S)
    assert out[2, 0] == 2 * a - b          # +x: P1 = a, P2 = b
    assert out[2, 3] == 2 * b - a          # -x: P1 = b, P2 = a
    assert out[1, 1] == a and out[3, 1] == a   # +-y: P1 only
    assert out[1, 2] == b and out[3, 2] == b
    assert np.count_nonzero(out) == 8


def test_l_shaped_core_averages_two_directions():
    # core (1,1), (2,1), (1,2) [as (x, y)]; edge pixel (2,2) sees P1 = (1,2) going -x and
    # P1 = (2,1) going -y, neither with a second pixel: mean of the two
    S = np.zeros((5, 5), bool)
    S[1, 1] = S[1, 2] = S[2, 1] = True
    phi = rnd(5, 5, 2)
    out = repair.repair(phi, S)
    assert out[2, 2] == (phi[2, 1] + phi[1, 2]) / 2
    # (0,1) [x=0, y=1]: +x gives 2 phi(1,1) - phi(2,1); +y: P1 (0,2) not in S
    assert out[1, 0] == 2 * phi[1, 1] - phi[1, 2]


def test_linear_phase_on_rectangle_is_restored_exactly():
    H, W = 20, 24
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    phi = 0.37 * xx - 1.1 * yy + 2.0
    S = np.zeros((H, W), bool)
    S[4:15, 3:19] = True
    out = repair.repair(phi, S)
    E = repair.edge_ring(S)
    assert E.sum() == 2 * (11 + 16)          # the four sides, no corners (cross dilation)
    assert np.max(np.abs(out[E] - phi[E])) < 1e-12
    assert np.all(out[~(S | E)] == 0.0)


def test_threshold_is_inclusive_and_strict():
    m = np.array([[1.0, 0.999999, 0.9999989, 0.5]])
    assert repair.strict_core(m).tolist() == [[True, True, False, False]]


def test_warped_mask_core_shrinks_by_the_soft_edge():
    # binary mask, half-pixel shift in x: the columns whose bilinear cell straddles
    # the mask edge get m = 0.5 and leave the core
    M = np.zeros((40, 40))
    M[10:30, 10:30] = 1.0
    A, b = geometry.inverse_from_misreg((0.5, 0, 0, 1), 40, 40, 40, 40)
    from oracle import warp
    m = warp.warp(M[None], A, b, 40, 40, halo=0)[0]
    S = repair.strict_core(m)
    assert S.sum() == 20 * 19
    assert set(np.unique(m).tolist()) == {0.0, 0.5, 1.0}


def _linear_if(g, H, W, c=0.25):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    return g[0] * xx + g[1] * yy + c


def test_repair_restores_exact_slopes_of_a_linear_if():
    # WFS: 6x6 subapertures of 5 px, full square pupil (30x30).  IF grid 40x40, map
    # near the identity (source = p_o + 5 + small shift/rotation).  The DM mask
    # covers the WFS window except its outermost haloed ring, so that ring comes out
    # of the core and must be restored for the central differences at the pupil edge.
    p, n = 5, 6
    pupil = np.ones((n * p, n * p), np.uint8)
    valid = wl.valid_subapertures(pupil, p)
    theta = (0.21, -0.13, math.radians(0.3), 1.0)
    A, b = geometry.inverse_from_misreg(theta, 40, 40, 30, 30)
    g = np.array([0.8, -0.45])
    F = _linear_if(g, 40, 40)
    # source x = x_o + 4.71..4.87, y = y_o + 5.05..5.21 over the window (shift plus the
    # rotation about the centre): with the mask on IF columns 4..34 and rows 5..35, the
    # haloed ring (x_o or y_o = -1 or 30) straddles the mask edge (m < 1, edge ring) and
    # the samples 0..29 lie in the core
    M = np.zeros((40, 40))
    M[5:36, 4:35] = 1.0
    Fm = (F * M)[None]
    from oracle import warp
    m = warp.warp(M[None], A, b, 30, 30, halo=1)[0]
    S = repair.strict_core(m)
    assert S[1:-1, 1:-1].all() and not (S[0].any() or S[-1].any() or S[:, 0].any() or S[:, -1].any())
    exact = np.array([A[0, 0] * g[0] + A[1, 0] * g[1], A[0, 1] * g[0] + A[1, 1] * g[1]])
    got = repair.im_build_repaired(Fm, M, A, b, pupil, p, valid)[0]
    N = valid.size
    assert np.max(np.abs(got[:N] - exact[0])) < 1e-11
    assert np.max(np.abs(got[N:] - exact[1])) < 1e-11
    # without the repair the pupil-edge subapertures see the collapse
    plain = oim.im_build(Fm, A, b, pupil, p, valid)[0]
    assert np.max(np.abs(plain[:N] - exact[0])) > 1e-2
