"""Pins of the oracle's tomographic projection (paper Sec. 2.5).

* on axis at zero altitude, with the pupil and component grids of one size and
  pixel, every sample lands on a pixel centre: P's columns are the basis
  functions read at the pupil pixels, exactly;
* a footprint shift h theta / s of whole pixels reads the basis shifted by
  exactly those pixels, and rows are ordered direction-major;
* 2x2 binning of a linear function inside the mask gives its value at the
  block centre;
* P_opt with P_Layer = P_DM and lambda = 0 is the identity; for lambda > 0 it
  equals the least-squares solution of the stacked system
  [P_DM; sqrt(lambda) I] X = [P_Layer; 0] (numpy's lstsq, an SVD-based
  minimiser, not the normal equations).
"""
import numpy as np

import workloads as wl
from oracle import projection as pj


def _stack(rng, n, H, W):
    return rng.standard_normal((n, H, W))


def test_on_axis_samples_are_exact():
    rng = np.random.default_rng(1)
    F = _stack(rng, 4, 20, 20)
    mask = wl.pupil_mask(20, 18.0)
    P = pj.projection_matrix([(F, 0.0, 0.5)], [(0.0, 0.0)], mask, 0.5)
    assert P.shape == (int(mask.sum()), 4)
    for a in range(4):
        assert np.array_equal(P[:, a], F[a][mask > 0])


def test_integer_footprint_shift_and_direction_order():
    rng = np.random.default_rng(2)
    F = _stack(rng, 3, 30, 30)
    mask = wl.pupil_mask(20, 18.0)
    h, s = 5000.0, 0.5
    th = (2 * s / h, -3 * s / h)                       # +2 px in x, -3 px in y
    P = pj.projection_matrix([(F, h, s)], [(0.0, 0.0), th], mask, s)
    n = int(mask.sum())
    ys, xs = np.nonzero(mask)
    # component grid 30x30 centred at 14.5, pupil 20x20 centred at 9.5: offset 5 px
    assert np.allclose(P[:n], F[:, ys + 5, xs + 5].T, rtol=0, atol=1e-12)
    assert np.allclose(P[n:], F[:, ys + 5 - 3, xs + 5 + 2].T, rtol=0, atol=1e-12)


def test_binning_of_linear_function():
    H = 24
    yy, xx = np.mgrid[0:H, 0:H].astype(np.float64)
    F = (0.3 * xx - 0.7 * yy + 2.0)[None]
    mask = np.ones((16, 16), bool)
    P = pj.projection_matrix([(F, 0.0, 1.0)], [(0.0, 0.0)], mask, 1.0, b=2)
    blocks = pj.pupil_blocks(mask, 2)
    assert len(blocks) == 64 and P.shape == (64, 1)
    for r, (by, bx, _) in enumerate(blocks):
        # block centre on the pupil grid, offset 4 px onto the 24-px component grid
        cx, cy = 2 * bx + 0.5 + 4, 2 * by + 0.5 + 4
        assert abs(P[r, 0] - (0.3 * cx - 0.7 * cy + 2.0)) < 1e-12


def test_popt_identity_and_stacked_least_squares():
    rng = np.random.default_rng(3)
    P_dm = rng.standard_normal((120, 15))
    X = pj.p_opt(P_dm, P_dm, 0.0)
    assert np.max(np.abs(X - np.eye(15))) < 1e-10
    P_l = rng.standard_normal((120, 7))
    lam = 0.37
    X = pj.p_opt(P_dm, P_l, lam)
    Aug = np.vstack([P_dm, np.sqrt(lam) * np.eye(15)])
    Rhs = np.vstack([P_l, np.zeros((15, 7))])
    ref = np.linalg.lstsq(Aug, Rhs, rcond=None)[0]
    assert np.max(np.abs(X - ref)) < 1e-10 * np.abs(ref).max()
