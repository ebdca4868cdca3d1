"""The telescoping-sum (G-tilt) slope engine on the GPU (synim_im_build_tsum)
against the FP64 oracle, and the engine ablation of Sec. 2.2.

Parity (max|dIM| <= 1e-5 max|IM|): the 8x8 SCAO build, a ragged 13x13 WFS,
a 30 deg turn, and the anamorphic composite; a linear IF gives A^T g; on an
integer shift the two engines agree.

Ablation: Gaussian IFs of shrinking width on the 8x8 SCAO geometry (10-px
subapertures, the adjoint workload's map), both engines' IMs from the GPU
against the exact G-tilt of the continuous Gaussians (oracle, quadrature of
the boundary integrals).  The paper's claim that the numerical-derivative
engine follows a diffractive sensor better cannot be tested without a
diffractive model; what is checked is the geometric side: both engines
converge to the G-tilt as the IFs widen, and the telescoping sum, which reads
the boundary values directly, stays the closer of the two to the exact
geometric gradient at every width tried.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import geometry as og, im as oim, tsum as otsum

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def cases(S):
    out = []
    cfg = wl.scao_small()
    A, _ = S.affine_from_misreg(cfg.theta, 96, 96, 80, 80)
    out.append(("scao_8x8", cfg.pupil, cfg.p, cfg.valid, wl.if_stack(cfg.grid), A))
    rng = np.random.default_rng(23)
    P = wl.pupil_mask(65, 60.0, 0.3, (1.3, -0.7))
    v = wl.valid_subapertures(P, 5)
    F = rng.standard_normal((7, 70, 71)).astype(np.float32)
    A, _ = S.affine_from_misreg((0.37, -0.81, 0.12, 1.03), 70, 71, 65, 65)
    out.append(("ragged_13x13_p5", P, 5, v, F, A))
    P = wl.pupil_mask(48, 48.0, 0.2)
    v = wl.valid_subapertures(P, 4)
    F = rng.standard_normal((3, 52, 52)).astype(np.float32)
    A, _ = S.affine_from_misreg((0.2, 0.1, math.radians(30.0), 1.1), 52, 52, 48, 48)
    out.append(("rot30_p4", P, 4, v, F, A))
    P = wl.pupil_mask(48, 48.0, 0.25, (0.6, -0.4))
    v = wl.valid_subapertures(P, 6)
    F = rng.standard_normal((5, 64, 64)).astype(np.float32)
    g = wl.Geometry(dm_shift_x=0.7, dm_shift_y=-1.1, dm_rot=math.radians(1.5), dm_mag=1.01,
                    cone_scale=0.93, footprint_x=1.8, footprint_y=-2.4, wfs_shift_x=0.35,
                    wfs_shift_y=-0.45, wfs_rot=math.radians(20.0), wfs_mag_x=1.05,
                    wfs_mag_y=0.97)
    out.append(("anamorphic", P, 6, v, F, S.affine_from_geometry(g, 64, 64, 48, 48)))
    return out


def test_tsum_parity(gpu_lib):
    S = gpu_lib
    for name, P, p, v, F, A in cases(S):
        say("[case] tsum", name)
        wfs = S.Wfs.from_numpy(P, p, v)
        got = S.im_build_tsum(to_dev(F), A, wfs).cpu().numpy()
        ref = otsum.im_build_tsum(F, A[:, :2], A[:, 2], P, p, v)
        e = rel_err(got, ref)
        say(f"  rel err {e:.2e}")
        assert e <= IM_TOL, (name, e)


def test_tsum_linear_and_integer_shift(gpu_lib):
    S = gpu_lib
    say("[case] tsum linear / integer shift")
    P = wl.pupil_mask(48, 46.0, 0.3, (0.7, -0.4))
    v = wl.valid_subapertures(P, 6)
    wfs = S.Wfs.from_numpy(P, 6, v)
    A, _ = S.affine_from_misreg((-1.7, 2.2, math.radians(17.0), 0.93), 64, 64, 48, 48)
    g = np.array([0.61, -1.3])
    yy, xx = np.mgrid[0:64, 0:64].astype(np.float64)
    F = (g[0] * (xx - 31.5) + g[1] * (yy - 31.5) + 0.3).astype(np.float32)[None]
    got = S.im_build_tsum(to_dev(F), A, wfs).cpu().numpy()[0]
    N = v.size
    ex = np.array([A[0, 0] * g[0] + A[1, 0] * g[1], A[0, 1] * g[0] + A[1, 1] * g[1]])
    assert np.max(np.abs(got[:N] - ex[0])) <= 1e-5 * 32 * np.abs(ex).max()
    assert np.max(np.abs(got[N:] - ex[1])) <= 1e-5 * 32 * np.abs(ex).max()
    rng = np.random.default_rng(4)
    F = rng.standard_normal((3, 56, 56)).astype(np.float32)
    A, _ = S.affine_from_misreg((2.0, -1.0, 0.0, 1.0), 56, 56, 48, 48)
    t = S.im_build_tsum(to_dev(F), A, wfs).cpu().numpy()
    c = S.im_build(to_dev(F), A, wfs).cpu().numpy()
    assert np.max(np.abs(t - c)) <= IM_TOL * np.abs(c).max()


def test_engine_ablation_against_exact_gtilt(gpu_lib):
    S = gpu_lib
    cfg = wl.scao_small()
    A, _ = S.affine_from_misreg(cfg.theta, 96, 96, 80, 80)
    wfs = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid)
    grid = cfg.grid
    acts = list(range(0, grid.n_act, 4))          # 21 of the 81 actuators
    rows = []
    for sigma in (8.0, 5.134, 3.0, 2.0, 1.5, 1.0):
        say(f"[case] engine ablation sigma {sigma}")
        F = np.stack([otsum.gaussian_if(grid.amp[a], grid.x[a], grid.y[a], sigma, 96, 96)
                      for a in acts]).astype(np.float32)
        ex = np.stack([otsum.gtilt_exact_gaussian(grid.amp[a], grid.x[a], grid.y[a], sigma,
                                                  A[:, :2], A[:, 2], cfg.pupil, cfg.p, cfg.valid)
                       for a in acts])
        Fd = to_dev(F)
        cd = S.im_build(Fd, A, wfs).cpu().numpy()
        ts = S.im_build_tsum(Fd, A, wfs).cpu().numpy()
        e_cd, e_ts = otsum.rel_rms(cd, ex), otsum.rel_rms(ts, ex)
        e_engines = otsum.rel_rms(cd, ts)
        rows.append((sigma, e_cd, e_ts, e_engines))
        say(f"  sigma {sigma:5.3f} px: rel RMS vs exact G-tilt: central differences {e_cd:.3e}, "
            f"telescoping sum {e_ts:.3e}; between the engines {e_engines:.3e}")
    for sigma, e_cd, e_ts, _ in rows:
        assert e_ts < e_cd, sigma
    assert rows[0][1] < 0.02 and rows[0][2] < 0.02
    assert rows[-1][1] > rows[0][1] and rows[-1][2] > rows[0][2]
