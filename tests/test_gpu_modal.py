"""Modal interaction matrices under the full composite map, and the
sequential-resampling ablation (paper Sec. 2.1: the DM and WFS transforms are
multiplied into one matrix and the grid is interpolated exactly once;
resampling them one after the other acts as a low-pass filter).

Workload: one LGS WFS of the MCAO system (68x68 subapertures of 7 px, clocked
15 deg) with an anamorphic WFS magnification (1.00 x 0.97), the 4-km DM's
512^2 grid at that LGS's cone and footprint, misregistered by (0.37, -0.23) px,
0.3 deg and 1.003, and a Fourier modal
basis on the IF grid (period = the 480-px meta-pupil; 4519 modes up to 38
cycles per pupil, of which every 71st is taken here, spanning every
frequency).

* parity: the GPU's modal IM (one composite interpolation) against the FP64
  oracle, max|dIM| <= 1e-5 max|IM|;
* ablation: against the slopes of the exact warped modes (each mode evaluated
  analytically at the composite map's source point of every haloed WFS
  sample, slopes by the oracle), the composite build's error is compared with
  a sequential build on the GPU (DM placement and LGS footprint resampled onto
  an intermediate grid, then the WFS transform resampled from it, then the
  slopes).  The composite error is the single interpolation's floor; the
  second interpolation of the sequential build about doubles it at every
  order (1.9x over the high orders here).
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import im as oim, slopes as osl

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def setup(S):
    cfg = wl.mcao(0)
    n_out = cfg.n_sub * cfg.p
    g = cfg.pairs[4].geometry            # WFS 1 (15 deg clocking), the 4-km DM
    g.wfs_mag_x, g.wfs_mag_y = 1.0, 0.97
    # the DM's own misregistration (shift, rotation, magnification)
    g.dm_shift_x, g.dm_shift_y, g.dm_rot, g.dm_mag = 0.37, -0.23, math.radians(0.3), 1.003
    modes = wl.fourier_modes(4519)[::71]
    return cfg, n_out, g, modes


def split_maps(S, g, n_out, n_mid):
    """(A1, A2): intermediate <- IF (DM placement and LGS footprint) and
    WFS <- intermediate (the WFS transform), each about its grid centre."""
    g1 = wl.Geometry(dm_shift_x=g.dm_shift_x, dm_shift_y=g.dm_shift_y, dm_rot=g.dm_rot,
                     dm_mag=g.dm_mag, cone_scale=g.cone_scale, footprint_x=g.footprint_x,
                     footprint_y=g.footprint_y, kappa=g.kappa)
    g2 = wl.Geometry(wfs_shift_x=g.wfs_shift_x, wfs_shift_y=g.wfs_shift_y, wfs_rot=g.wfs_rot,
                     wfs_mag_x=g.wfs_mag_x, wfs_mag_y=g.wfs_mag_y)
    A1 = S.affine_from_geometry(g1, 512, 512, n_mid, n_mid)
    A2 = S.affine_from_geometry(g2, n_mid, n_mid, n_out, n_out)
    return A1, A2


def test_modal_im_parity_and_sequential_ablation(gpu_lib):
    S = gpu_lib
    cfg, n_out, g, modes = setup(S)
    P, v = cfg.pupils[1], cfg.valids[1]
    wfs = S.Wfs.from_numpy(P, cfg.p, v)
    A = S.affine_from_geometry(g, 512, 512, n_out, n_out)
    period = 480.0
    F = wl.fourier_stack(modes, 512, period)
    say("[case] modal IM", len(modes), "Fourier modes, composite with anamorphosis")
    Fd = to_dev(F)
    comp = S.im_build(Fd, A, wfs).cpu().numpy()
    ref = oim.im_build(F, A[:, :2], A[:, 2], P, cfg.p, v)
    e = rel_err(comp, ref)
    say(f"  composite build vs oracle: {e:.2e}")
    assert e <= IM_TOL
    # the composite map is the product of the two stages
    n_mid = n_out + 24
    A1, A2 = split_maps(S, g, n_out, n_mid)
    Ac = A1[:, :2] @ A2[:, :2]
    bc = A1[:, :2] @ A2[:, 2] + A1[:, 2]
    assert np.max(np.abs(Ac - A[:, :2])) < 1e-12 and np.max(np.abs(bc - A[:, 2])) < 1e-9
    say("[case] sequential resampling")
    mid = S.affine_warp(Fd, A1, n_mid, n_mid, halo=0)
    phi = S.affine_warp(mid, A2, n_out, n_out, halo=1)
    seq = S.sa_slopes(phi, wfs).cpu().numpy()
    # exact warped modes at the haloed WFS samples, slopes by the oracle
    ys, xs = np.mgrid[-1:n_out + 1, -1:n_out + 1].astype(np.float64)
    sx = A[0, 0] * xs + A[0, 1] * ys + A[0, 2]
    sy = A[1, 0] * xs + A[1, 1] * ys + A[1, 2]
    c = (512 - 1) / 2.0
    exact_phi = np.stack([wl.fourier_mode_values(m, sx, sy, period, c, c) for m in modes])
    exact = osl.slopes(exact_phi, P, cfg.p, v)
    rows = []
    for i, m in enumerate(modes):
        nrm = np.sqrt(np.mean(exact[i] ** 2))
        rows.append((math.hypot(m.kx, m.ky), np.sqrt(np.mean((comp[i] - exact[i]) ** 2)) / nrm,
                     np.sqrt(np.mean((seq[i] - exact[i]) ** 2)) / nrm))
    rows = np.array(rows)
    for lo, hi in ((0, 10), (10, 20), (20, 30), (30, 40)):
        sel = (rows[:, 0] >= lo) & (rows[:, 0] < hi)
        if sel.any():
            say(f"  |k| in [{lo},{hi}) cycles/pupil: rel RMS error vs exact slopes: composite "
                f"{rows[sel, 1].mean():.3e}, sequential {rows[sel, 2].mean():.3e}")
    hi = rows[:, 0] >= 20
    assert rows[hi, 2].mean() > 1.5 * rows[hi, 1].mean()
    assert np.all(rows[:, 2] >= rows[:, 1] * 0.9)
