"""GPU parity of the edge-repaired build (paper Sec. 2.3) against the FP64
oracle, through the C ABI (synim_im_build_repaired).

Cases (max|dIM| <= 1e-5 max|IM|):
* the 8x8 SCAO geometry with its Gaussian IFs pre-masked by a DM-side circular
  mask whose edge falls inside the WFS pupil, so the pupil-edge subapertures
  read repaired samples (the repair changes the IM there, which the test
  checks against the unrepaired build);
* a ragged 13x13 WFS of 5-px subapertures with random IFs under a shifted,
  rotated, magnified map and an off-centre mask;
* the oracle's exact case: a pre-masked linear IF whose mask edge runs through
  the haloed window's outer ring, whose repaired slopes are A^T g everywhere.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import geometry as og, im as oim, repair as orep

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def cases():
    out = []
    cfg = wl.scao_small()
    M = wl.pupil_mask(96, 74.0)                      # edge inside the 80-px pupil
    F = wl.if_stack(cfg.grid) * M
    out.append(("scao_8x8_mask74", cfg.pupil, cfg.p, cfg.valid, F.astype(np.float32), M,
                (96, 96, 80, 80), cfg.theta))
    rng = np.random.default_rng(17)
    P = wl.pupil_mask(65, 60.0, 0.3, (1.3, -0.7))
    v = wl.valid_subapertures(P, 5)
    M = wl.pupil_mask(72, 58.0, 0.25, (0.6, 0.9))[:, :71]
    F = (rng.standard_normal((6, 72, 71)) * M).astype(np.float32)
    out.append(("ragged_13x13_p5", P, 5, v, F, M, (72, 71, 65, 65),
                (0.37, -0.81, math.radians(1.2), 1.03)))
    return out


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
def test_repaired_build_parity(gpu_lib, case):
    S = gpu_lib
    name, P, p, v, F, M, dims, theta = case
    say("[case] repair", name)
    Hi, Wi, Ho, Wo = dims
    A, _ = S.affine_from_misreg(theta, Hi, Wi, Ho, Wo)
    wfs = S.Wfs.from_numpy(P, p, v)
    Md = to_dev(M.astype(np.uint8))
    got = S.im_build_repaired(to_dev(F), Md, A, wfs).cpu().numpy()
    ref = orep.im_build_repaired(F, M, A[:, :2], A[:, 2], P, p, v)
    e = rel_err(got, ref)
    plain = oim.im_build(F, A[:, :2], A[:, 2], P, p, v)
    say(f"  rel err {e:.2e}; repair moves the IM by {rel_err(plain, ref):.2e} of its max")
    assert e <= IM_TOL, e
    assert rel_err(plain, ref) > 1e-3          # the repair is not a no-op here


def test_repaired_linear_if_is_exact(gpu_lib):
    S = gpu_lib
    say("[case] repair linear IF")
    p, n = 5, 6
    pupil = np.ones((n * p, n * p), np.uint8)
    valid = wl.valid_subapertures(pupil, p)
    theta = (0.21, -0.13, math.radians(0.3), 1.0)
    A, _ = S.affine_from_misreg(theta, 40, 40, 30, 30)
    g = np.array([0.8, -0.45])
    yy, xx = np.mgrid[0:40, 0:40].astype(np.float64)
    M = np.zeros((40, 40), np.uint8)
    M[5:36, 4:35] = 1
    Fm = ((g[0] * xx + g[1] * yy + 0.25) * M).astype(np.float32)[None]
    wfs = S.Wfs.from_numpy(pupil, p, valid)
    got = S.im_build_repaired(to_dev(Fm), to_dev(M), A, wfs).cpu().numpy()[0]
    ref = orep.im_build_repaired(Fm, M, A[:, :2], A[:, 2], pupil, p, valid)[0]
    N = valid.size
    exact = np.array([A[0, 0] * g[0] + A[1, 0] * g[1], A[0, 1] * g[0] + A[1, 1] * g[1]])
    assert rel_err(got, ref) <= IM_TOL
    # FP32 IF values of magnitude ~30 round at ~2e-6; the slopes stay within 1e-5 of A^T g
    assert np.max(np.abs(got[:N] - exact[0])) <= 1e-5 * 40 * abs(exact).max()
    assert np.max(np.abs(got[N:] - exact[1])) <= 1e-5 * 40 * abs(exact).max()
