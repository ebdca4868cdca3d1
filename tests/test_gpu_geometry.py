"""GPU parity of the fused build on geometries the workloads do not reach, and
the boundary's error conventions.

Geometries (each against the FP64 oracle, max|dIM| <= 1e-5 max|IM|):
* a non-square WFS (12 x 9 subapertures) on a non-square IF grid, so any
  confusion of n_sub_x with n_sub_y in the subaperture indexing shows;
* kappa = 2 (two IF pixels per WFS pixel);
* a general anamorphic composite (DM rotation and magnification, LGS cone and
  footprint, WFS clocking and unequal x/y magnification);
* an exact quarter turn and an integer shift (every sample on the IF grid).

Conventions:
* the out-of-grid count of the plan equals the oracle's count, and the strict
  check reports SYNIM_E_OOB exactly when it is non-zero;
* synim_batch_set_maps with maps whose weight patches outgrow the batch's
  kernel variant returns SYNIM_E_UNSUPPORTED; maps whose tiles outgrow their
  staged-box bound re-bind and still build the oracle's IM with a clean
  status.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import im as oim

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def ellipse_pupil(h, w, ry, rx):
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    cy, cx = (h - 1) / 2, (w - 1) / 2
    return ((((x - cx) / rx) ** 2 + ((y - cy) / ry) ** 2) <= 1.0).astype(np.uint8)


def cases(S):
    rng = np.random.default_rng(21)
    out = []
    P = ellipse_pupil(45, 60, 22.0, 29.5)           # 9 rows x 12 columns of 5 px
    v = wl.valid_subapertures(P, 5)
    F = rng.standard_normal((9, 58, 73)).astype(np.float32)
    A, _ = S.affine_from_misreg((0.4, -0.3, math.radians(0.7), 1.02), 58, 73, 45, 60)
    out.append(("nonsquare_12x9", P, 5, v, F, A))
    P = wl.pupil_mask(40, 40.0, 0.2)
    v = wl.valid_subapertures(P, 5)
    F = rng.standard_normal((6, 100, 100)).astype(np.float32)
    A, _ = S.affine_from_misreg((0.25, 0.6, math.radians(-0.8), 0.99), 100, 100, 40, 40,
                                kappa=2.0)
    out.append(("kappa2", P, 5, v, F, A))
    P = wl.pupil_mask(48, 48.0, 0.25, (0.6, -0.4))
    v = wl.valid_subapertures(P, 6)
    F = rng.standard_normal((5, 64, 64)).astype(np.float32)
    g = wl.Geometry(dm_shift_x=0.7, dm_shift_y=-1.1, dm_rot=math.radians(1.5), dm_mag=1.01,
                    cone_scale=0.93, footprint_x=1.8, footprint_y=-2.4,
                    wfs_shift_x=0.35, wfs_shift_y=-0.45, wfs_rot=math.radians(20.0),
                    wfs_mag_x=1.05, wfs_mag_y=0.97)
    A = S.affine_from_geometry(g, 64, 64, 48, 48)
    out.append(("anamorphic", P, 6, v, F, A))
    P = wl.pupil_mask(40, 40.0, 0.0)
    v = wl.valid_subapertures(P, 5)
    F = rng.standard_normal((4, 44, 44)).astype(np.float32)
    A, _ = S.affine_from_misreg((0.0, 0.0, math.pi / 2, 1.0), 44, 44, 40, 40)
    out.append(("quarter_turn", P, 5, v, F, A))
    A, _ = S.affine_from_misreg((1.0, -1.0, 0.0, 1.0), 44, 44, 40, 40)
    out.append(("integer_shift", P, 5, v, F, A))
    A, _ = S.affine_from_misreg((4.0, 3.0, 0.0, 1.0), 44, 44, 40, 40)
    out.append(("shift_out_of_grid", P, 5, v, F, A))
    return out


def test_geometries_and_oob_count(gpu_lib):
    S = gpu_lib
    for name, P, p, v, F, A in cases(S):
        say("[case] geometry", name)
        Hi, Wi = F.shape[1:]
        wfs = S.Wfs.from_numpy(P, p, v)
        ws = S.im_plan(wfs, A, grid=(Hi, Wi))
        assert S.plan_status(ws) == 0, name
        got = S.im_apply(to_dev(F), A, wfs, ws).cpu().numpy()
        ref = oim.im_build(F, A[:, :2], A[:, 2], P, p, v)
        e = rel_err(got, ref)
        assert e <= IM_TOL, (name, e)
        n_ref = oim.oob_count(A[:, :2], A[:, 2], P, p, v, Hi, Wi)
        assert S.plan_oob(ws) == n_ref, name
        if name == "shift_out_of_grid":
            assert n_ref > 0
        else:
            assert n_ref == 0, name
        say(f"  rel err {e:.2e}, out-of-grid samples {n_ref}")


def test_strict_check_status_code(gpu_lib):
    import ctypes as C
    S = gpu_lib
    lib = S.load()
    name, P, p, v, F, A = cases(S)[-1]
    wfs = S.Wfs.from_numpy(P, p, v)
    ws = S.im_plan(wfs, A, grid=F.shape[1:])
    n = C.c_int64(-1)
    assert lib.synim_plan_oob(ws.data_ptr(), C.byref(n), None) == S.STATUS_OOB
    assert n.value == oim.oob_count(A[:, :2], A[:, 2], P, p, v, *F.shape[1:])
    ws = S.im_plan(wfs, cases(S)[-2][5], ws=ws, grid=F.shape[1:])
    assert lib.synim_plan_oob(ws.data_ptr(), C.byref(n), None) == 0 and n.value == 0


def _small_batch(S):
    rng = wl.rng_for(3)
    wfs_np = []
    for w in range(2):
        off = (float(rng.uniform(-2, 2)), float(rng.uniform(-2, 2)))
        Pw = wl.pupil_mask(60, 60.0, 0.25, off)
        wfs_np.append((Pw, wl.valid_subapertures(Pw, 5)))
    grid = wl.actuator_grid(9, 7.5, 80, keep_radius=37.0)
    F = wl.if_stack(grid)
    return wfs_np, F


def test_batch_set_maps_bounds(gpu_lib):
    import torch
    S = gpu_lib
    wfs_np, F = _small_batch(S)
    wfs = [S.Wfs.from_numpy(P, 5, v) for P, v in wfs_np]
    geos = [wl.Geometry(wfs_rot=math.radians(2.0 * w)) for w in range(2)]
    maps = [S.affine_from_geometry(g, 80, 80, 60, 60) for g in geos]
    B = S.Batch(wfs, [to_dev(F)], [(w, 0, maps[w]) for w in range(2)])
    B.run()
    torch.cuda.synchronize()
    assert B.status() == 0
    # a 4 deg turn widens every tile's staged box: the pair tables re-bind
    geos2 = [wl.Geometry(wfs_rot=math.radians(2.0 * w + 4.0), footprint_x=0.4) for w in range(2)]
    maps2 = [S.affine_from_geometry(g, 80, 80, 60, 60) for g in geos2]
    try:
        B.set_maps(maps2)
    except S.SynimError as e:
        # only a patch that outgrows the kernel variant may refuse the maps
        assert e.status == -8, e
        say("  set_maps refused the turned maps (patch outgrew the variant)")
    else:
        B.run_graph()
        torch.cuda.synchronize()
        assert B.status() == 0
        for w in range(2):
            P, v = wfs_np[w]
            A = maps2[w]
            ref = oim.im_build(F, A[:, :2], A[:, 2], P, 5, v)
            assert rel_err(B.outs[w].cpu().numpy(), ref) <= IM_TOL, w
    # half the magnification doubles the patch every subaperture needs
    geos3 = [wl.Geometry(dm_mag=0.5) for _ in range(2)]
    maps3 = [S.affine_from_geometry(g, 80, 80, 60, 60) for g in geos3]
    with pytest.raises(S.SynimError) as ei:
        B.set_maps(maps3)
    assert ei.value.status == -8
    B.close()
