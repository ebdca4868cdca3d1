"""Every stream-kernel configuration the autotuner may pick gives the same IM.

The configurations differ in kernel variant, tile shape and schedule (short
chunks dealt round-robin to the XCDs; one chunk per XCD; one chunk per XCD
with the bounded-lag sync of the XCD's tiles).  Each one is pinned with
synim_im_set_config and checked against the FP64 oracle (max|dIM| <= 1e-5
max|IM|); configurations that share variant and tile shape and differ only in
schedule must agree bit for bit (the per-actuator arithmetic is the same).
"""
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


def _run_all(S, F, A, wfs, cols, ref, label):
    import torch
    cands = S.im_candidates(wfs, A)
    assert any(c["schedule"] != 0 for c in cands), "no XCD schedule offered"
    by_shape = {}
    worst = 0.0
    for c in cands:
        S.im_set_config(wfs, A, c)
        assert S.im_config(wfs, A) == c
        ws = S.im_plan(wfs, A, device=F.device)
        out = S.im_apply(F, A, wfs, ws)
        torch.cuda.synchronize()
        assert S.plan_status(ws) == 0, c
        got = out[cols].cpu().numpy()
        e = rel_err(got, ref)
        worst = max(worst, e)
        assert e <= IM_TOL, (label, c, e)
        key = tuple(c[k] for k in ("block", "lanes_per_subap", "patch_rows", "patch_cols",
                                    "tile_x", "tile_y", "stages"))
        if key in by_shape:
            assert torch.equal(out, by_shape[key]), (label, c)
        else:
            by_shape[key] = out
    S.autotune_clear()
    by_shape.clear()
    say(f"{label}: {len(cands)} configurations, worst rel err {worst:.2e}")


def test_every_configuration_small(gpu_lib):
    import torch
    S = gpu_lib
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    A, _ = S.affine_from_misreg(cfg.theta, 96, 96, 80, 80)
    wfs = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device="cuda:0")
    ref = oim.im_build(F, A[:, :2], A[:, 2], cfg.pupil, cfg.p, cfg.valid)
    say("[case] all configurations, 8x8 SCAO")
    _run_all(S, torch.from_numpy(F).cuda(), A, wfs, np.arange(F.shape[0]), ref, "scao_8x8")


def test_every_configuration_single_actuator(gpu_lib):
    """Fewer actuators than XCDs: most XCDs get no chunk."""
    import torch
    S = gpu_lib
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)[40:43]
    A, _ = S.affine_from_misreg(cfg.theta, 96, 96, 80, 80)
    wfs = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device="cuda:0")
    ref = oim.im_build(F, A[:, :2], A[:, 2], cfg.pupil, cfg.p, cfg.valid)
    say("[case] all configurations, 3 actuators")
    _run_all(S, torch.from_numpy(np.ascontiguousarray(F)).cuda(), A, wfs, np.arange(3), ref,
             "scao_8x8_3act")


def test_every_configuration_elt_sampled(gpu_lib):
    import torch
    S = gpu_lib
    cfg = wl.scao_elt(0)
    say("[case] all configurations, ELT SCAO (generating the IF stack)")
    F = wl.if_stack_torch(cfg.grid, "cuda:0")
    A, _ = S.affine_from_misreg(cfg.theta, 512, 512, 480, 480)
    wfs = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device="cuda:0")
    cols = np.array([0, 1311, 2628, 2629, 4100, cfg.grid.n_act - 1])
    Fs = np.stack([wl.if_single(cfg.grid, int(a)) for a in cols])
    ref = oim.im_build(Fs, A[:, :2], A[:, 2], cfg.pupil, cfg.p, cfg.valid)
    _run_all(S, F, A, wfs, cols, ref, "scao_elt")
    del F
    torch.cuda.empty_cache()
