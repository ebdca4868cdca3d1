"""Pins of the oracle's telescoping-sum (G-tilt) engine and of the exact G-tilt
of a continuous Gaussian used by the engine ablation.

* a full subaperture has one left and one right boundary point per row and
  column; a partial one follows its pupil runs (worked by hand);
* a linear IF gives exactly A^T g on every subaperture, full or partial,
  under any map (bilinear interpolation reproduces affine functions and each
  row's boundary difference is the gradient times the run length);
* on a map with an integer shift and no rotation or magnification every
  boundary point falls half-way between two IF pixel centres, so its bilinear
  value is their mean and the telescoping sum equals the central-difference
  slopes exactly;
* the segment integral of the Gaussian matches the closed form with erf;
* the telescoping engine on a well-sampled Gaussian converges to the exact
  G-tilt as the Gaussian widens.
"""
import math

import numpy as np

import workloads as wl
from oracle import geometry, im as oim, tsum


def test_edge_points_full_and_partial_by_hand():
    p = 3
    pupil = np.ones((3, 6), np.uint8)
    pupil[0, 3] = 0            # subaperture 1 (columns 3..5): its top-left pixel is dark
    px, py = tsum.edge_points(pupil, p, 0, 2)
    assert sorted(px) == sorted([(-0.5, y, -1) for y in (0.0, 1.0, 2.0)] +
                                [(2.5, y, 1) for y in (0.0, 1.0, 2.0)])
    assert sorted(py) == sorted([(x, -0.5, -1) for x in (0.0, 1.0, 2.0)] +
                                [(x, 2.5, 1) for x in (0.0, 1.0, 2.0)])
    px, py = tsum.edge_points(pupil, p, 1, 2)
    # row 0: run [4, 5] -> left boundary at 3.5
    assert (3.5, 0.0, -1) in px and (2.5, 0.0, -1) not in px
    assert (2.5, 1.0, -1) in px and (5.5, 0.0, 1) in px
    # column 3: run [1, 2] -> top boundary at 0.5
    assert (3.0, 0.5, -1) in py and (3.0, -0.5, -1) not in py


def _linear(g, H, W, c=0.3):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    return (g[0] * xx + g[1] * yy + c)[None]


def test_linear_if_exact_any_geometry():
    pupil = wl.pupil_mask(48, 46.0, 0.3, (0.7, -0.4))
    valid = wl.valid_subapertures(pupil, 6)
    g = np.array([0.61, -1.3])
    for theta in [(0.3, -0.2, math.radians(0.5), 1.01), (-1.7, 2.2, math.radians(17.0), 0.93)]:
        A, b = geometry.inverse_from_misreg(theta, 64, 64, 48, 48)
        s = tsum.im_build_tsum(_linear(g, 64, 64), A, b, pupil, 6, valid)[0]
        N = valid.size
        ex = A[0, 0] * g[0] + A[1, 0] * g[1]
        ey = A[0, 1] * g[0] + A[1, 1] * g[1]
        assert np.max(np.abs(s[:N] - ex)) < 1e-12
        assert np.max(np.abs(s[N:] - ey)) < 1e-12


def test_integer_shift_equals_central_differences():
    rng = np.random.default_rng(4)
    pupil = wl.pupil_mask(40, 38.0, 0.2, (0.3, 0.1))
    valid = wl.valid_subapertures(pupil, 5)
    F = rng.standard_normal((3, 48, 48))
    A, b = geometry.inverse_from_misreg((2.0, -1.0, 0.0, 1.0), 48, 48, 40, 40)
    t = tsum.im_build_tsum(F, A, b, pupil, 5, valid)
    c = oim.im_build(F, A, b, pupil, 5, valid)
    assert np.max(np.abs(t - c)) < 1e-13 * np.abs(F).max()
    # a sub-pixel shift breaks the equality (the engines differ)
    A, b = geometry.inverse_from_misreg((0.3, -0.2, 0.0, 1.0), 48, 48, 40, 40)
    t = tsum.im_build_tsum(F, A, b, pupil, 5, valid)
    c = oim.im_build(F, A, b, pupil, 5, valid)
    assert np.max(np.abs(t - c)) > 1e-2


def test_segment_integral_matches_erf():
    A, b = np.eye(2), np.zeros(2)
    amp, cx, cy, s = 1.7, 3.2, -1.1, 0.8
    # segment x = 2.5, y from -2 to 1 (vertical): closed form
    got = tsum._line_integral_gaussian(amp, cx, cy, s, A, b, (2.5, -2.0), (2.5, 1.0)) * 3.0
    d = 2.5 - cx
    ref = amp * math.exp(-d * d / (2 * s * s)) * s * math.sqrt(math.pi / 2) * (
        math.erf((1.0 - cy) / (math.sqrt(2) * s)) - math.erf((-2.0 - cy) / (math.sqrt(2) * s)))
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_exact_gtilt_of_wide_gaussian_and_convergence():
    pupil = wl.pupil_mask(30, 30.0)
    valid = wl.valid_subapertures(pupil, 5)
    A, b = geometry.inverse_from_misreg((0.4, -0.3, math.radians(3.0), 1.02), 40, 40, 30, 30)
    # sigma = 6 IF px over 5-px subapertures: the telescoping engine (midpoint
    # rule on bilinear values) is within 1e-2 of the exact G-tilt (RMS relative)
    G = tsum.gaussian_if(1.0, 18.3, 21.1, 6.0, 40, 40)[None]
    ex = tsum.gtilt_exact_gaussian(1.0, 18.3, 21.1, 6.0, A, b, pupil, 5, valid)
    est = tsum.im_build_tsum(G, A, b, pupil, 5, valid)[0]
    e6 = tsum.rel_rms(est, ex)
    assert e6 < 1e-2
    # twice as wide: the interpolation and midpoint errors, relative to the
    # gradient, shrink about twofold
    G = tsum.gaussian_if(1.0, 18.3, 21.1, 12.0, 40, 40)[None]
    ex = tsum.gtilt_exact_gaussian(1.0, 18.3, 21.1, 12.0, A, b, pupil, 5, valid)
    e12 = tsum.rel_rms(tsum.im_build_tsum(G, A, b, pupil, 5, valid)[0], ex)
    assert e12 < e6 / 2
