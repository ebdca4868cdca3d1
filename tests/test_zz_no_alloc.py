"""The build entry point that allocates nothing (synim_im_build_noalloc),
called through the C ABI and checked against synim_im_build on the same
inputs (max|dIM| <= 1e-5 max|IM|, and identical here since both run the same
plan and kernels): two calls in a row on one GPU, the second with a smaller
WFS and fewer IFs, so the shared fixed array is re-planned; and the limit:
a plan larger than SYNIM_NOALLOC_WS_BYTES is refused before any device work.
"""
import ctypes as C
import math
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _noalloc(S, F, A, wfs):
    import torch
    lib = S.load()
    n, Hi, Wi = F.shape
    out = torch.full((n, 2 * wfs.n_valid), float("nan"), dtype=torch.float32, device=F.device)
    s = wfs.struct()
    a = S._affine_struct(A)
    rc = lib.synim_im_build_noalloc(F.data_ptr(), n, Hi, Wi, C.byref(a), C.byref(s),
                                    out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return rc, out


def test_noalloc_matches_build_twice(gpu_lib):
    import torch
    S = gpu_lib
    cfg = wl.scao_small()
    F1 = torch.from_numpy(wl.if_stack(cfg.grid)).cuda()
    A1, _ = S.affine_from_misreg(cfg.theta, 96, 96, 80, 80)
    w1 = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid)
    rng = np.random.default_rng(31)
    P2 = wl.pupil_mask(40, 40.0, 0.2, (0.4, -0.3))
    v2 = wl.valid_subapertures(P2, 5)
    F2 = torch.from_numpy(rng.standard_normal((7, 47, 45)).astype(np.float32)).cuda()
    A2, _ = S.affine_from_misreg((0.3, -0.45, math.radians(-0.6), 1.015), 47, 45, 40, 40)
    w2 = S.Wfs.from_numpy(P2, 5, v2)
    for name, F, A, w in (("scao 8x8, 81 IFs", F1, A1, w1), ("10x10 WFS, 7 IFs", F2, A2, w2)):
        say("[case] noalloc", name)
        rc, got = _noalloc(S, F, A, w)
        assert rc == 0, rc
        ref = S.im_build(F, A, w)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(g))
        assert np.max(np.abs(g - r)) <= IM_TOL * np.abs(r).max(), name
        assert np.array_equal(g, r), name


def test_noalloc_refuses_plans_beyond_its_array(gpu_lib):
    import torch
    S = gpu_lib
    lib = S.load()
    say("[case] noalloc limit")
    P = wl.pupil_mask(1200, 1200.0, 0.0)          # 200 x 200 subapertures of 6 px
    v = wl.valid_subapertures(P, 6)
    w = S.Wfs.from_numpy(P, 6, v)
    A, _ = S.affine_from_misreg((0.2, 0.1, 0.0, 1.0), 1232, 1232, 1200, 1200)
    ws_bytes = S.im_workspace_bytes(w, A, 1)
    assert ws_bytes > lib_limit()
    F = torch.zeros((1, 1232, 1232), dtype=torch.float32, device="cuda")
    rc, _ = _noalloc(S, F, A, w)
    assert rc == -5   # SYNIM_E_WORKSPACE


def lib_limit():
    return 16 << 20
