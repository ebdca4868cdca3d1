"""C-ABI contract checks that need no GPU.

* the library builds/loads and exports every function declared in include/*.h;
* the host-side FP64 geometry (composite map, derivative maps) agrees with the
  oracle's independent implementation;
* argument errors are reported before any device work (null pointers, bad
  shapes, bad parameters, too-small workspaces);
* the binding fails loudly when the library is missing (no CPU fallback).
"""
import ctypes as C
import glob
import math
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle import geometry as og

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_07759_amd import _abi, build
    if not os.path.exists(_abi.LIB_PATH):
        build.build(verbose=False)
    return _abi.load_library()


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(synim_\w+)\s*\(", txt)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_declares_every_symbol():
    from paper_2606_07759_amd import _abi
    assert set(declared_functions()) <= set(_abi.SIGNATURES)


def test_missing_library_raises():
    from paper_2606_07759_amd import _abi
    with pytest.raises(RuntimeError):
        _abi.load_library("/nonexistent/libsynim.so")


def test_status_strings(lib):
    assert lib.synim_status_str(0) == b"ok"
    assert lib.synim_status_str(-5).startswith(b"workspace")
    assert lib.synim_version() >= 10000


@pytest.mark.parametrize("theta", [(0.3, -0.2, math.radians(0.5), 1.01),
                                   (-0.9, 0.4, math.radians(-1.0), 0.98),
                                   (1.5, 2.5, math.pi / 2, 1.2)])
def test_host_misreg_map_matches_oracle(lib, theta):
    import paper_2606_07759_amd as S
    for kappa in (1.0, 1.3):
        A, dA = S.affine_from_misreg(theta, 96, 96, 80, 80, kappa)
        Ao, bo = og.inverse_from_misreg(theta, 96, 96, 80, 80, kappa)
        assert np.max(np.abs(A[:, :2] - Ao)) < 1e-15 and np.max(np.abs(A[:, 2] - bo)) < 1e-12
        for j, (dAo, dbo) in enumerate(og.derivative_maps(theta, 96, 96, 80, 80, kappa)):
            assert np.max(np.abs(dA[j][:, :2] - dAo)) < 1e-15
            assert np.max(np.abs(dA[j][:, 2] - dbo)) < 1e-12


def test_host_quarter_turn_is_exact(lib):
    import paper_2606_07759_amd as S
    A, _ = S.affine_from_misreg((0, 0, math.pi / 2, 1), 40, 40, 40, 40)
    assert np.array_equal(A[:, :2], np.array([[0.0, 1.0], [-1.0, 0.0]]))


def test_host_composite_geometry_matches_oracle(lib):
    import paper_2606_07759_amd as S
    cfg = wl.mcao(0)
    for pr in cfg.pairs[::4]:
        A = S.affine_from_geometry(pr.geometry, 512, 512, 476, 476)
        Ao, bo = og.inverse_from_geometry(pr.geometry, 512, 512, 476, 476)
        assert np.max(np.abs(A[:, :2] - Ao)) < 1e-14 and np.max(np.abs(A[:, 2] - bo)) < 1e-10
    g = wl.Geometry(dm_shift_x=0.4, dm_rot=0.01, dm_mag=1.02, cone_scale=0.9, footprint_x=3.0,
                    wfs_rot=0.3, wfs_mag_x=1.05, wfs_mag_y=0.97, wfs_shift_y=-0.6, kappa=1.1)
    A = S.affine_from_geometry(g, 128, 128, 80, 80)
    Ao, bo = og.inverse_from_geometry(g, 128, 128, 80, 80)
    assert np.max(np.abs(A[:, :2] - Ao)) < 1e-14 and np.max(np.abs(A[:, 2] - bo)) < 1e-12


def test_host_geometry_errors(lib):
    from paper_2606_07759_amd import _abi
    th = _abi.SynimMisreg(0, 0, 0, 0.0)
    A = _abi.SynimAffine()
    assert lib.synim_affine_from_misreg(C.byref(th), 8, 8, 8, 8, 1.0, C.byref(A), None) == -3
    assert lib.synim_affine_from_misreg(None, 8, 8, 8, 8, 1.0, C.byref(A), None) == -1
    g = _abi.SynimGeometry(cone_scale=1.0, dm_mag=1.0, wfs_mag_x=0.0, wfs_mag_y=1.0, kappa=1.0)
    assert lib.synim_affine_from_geometry(C.byref(g), 8, 8, 8, 8, C.byref(A)) == -3


def _fake_wfs(n_sub=8, p=10, nv=52):
    from paper_2606_07759_amd import _abi
    # non-null dummy device pointers: only host-side validation runs
    return _abi.SynimWfs(n_sub, n_sub, p, nv, 0x1000, 0x2000)


def test_argument_validation_before_device_work(lib):
    from paper_2606_07759_amd import _abi
    A = _abi.SynimAffine()
    A.A[0][0] = A.A[1][1] = 1.0
    w = _fake_wfs()
    n = C.c_size_t(0)
    assert lib.synim_im_workspace(C.byref(w), C.byref(A), 1, C.byref(n)) == 0 and n.value > 0
    n5 = C.c_size_t(0)
    assert lib.synim_im_workspace(C.byref(w), C.byref(A), 5, C.byref(n5)) == 0
    assert n5.value > n.value
    assert lib.synim_im_workspace(C.byref(w), C.byref(A), 3, C.byref(n)) == -3
    bad = _fake_wfs(nv=65)              # more valid subapertures than exist
    assert lib.synim_im_workspace(C.byref(bad), C.byref(A), 1, C.byref(n)) == -2
    nul = _abi.SynimWfs(8, 8, 10, 52, None, 0x2000)
    assert lib.synim_im_workspace(C.byref(nul), C.byref(A), 1, C.byref(n)) == -1
    # a map that magnifies the IF grid 4x needs patches no kernel variant has
    big = _abi.SynimAffine()
    big.A[0][0] = big.A[1][1] = 4.0
    assert lib.synim_im_workspace(C.byref(w), C.byref(big), 1, C.byref(n)) == -8
    # null / shape errors of the compute entry points return before launching
    assert lib.synim_affine_warp(None, 1, 8, 8, C.byref(A), 8, 8, 1, 0x10, None, None) == -1
    assert lib.synim_affine_warp(0x10, 0, 8, 8, C.byref(A), 8, 8, 1, 0x10, None, None) == -2
    assert lib.synim_affine_warp(0x10, 1, 8, 8, C.byref(A), 8, 8, 9, 0x10, None, None) == -2
    assert lib.synim_sa_slopes(0x10, 1, C.byref(bad), 0x20, None) == -2
    assert lib.synim_im_build(0x10, 4, 96, 96, C.byref(A), C.byref(w), 0x20, None, 0, None) == -5
    assert lib.synim_im_build(0x10, 4, 96, 96, C.byref(A), C.byref(w), 0x20, 0x30, 16, None) == -5
    assert lib.synim_im_build(0x10, 0, 96, 96, C.byref(A), C.byref(w), 0x20, 0x30, 16, None) == -2
    assert lib.synim_im_jacobian(0x10, 4, 96, 96, C.byref(A), None, C.byref(w), None, 0x20,
                                 0x30, 1 << 20, None) == -1
    assert lib.synim_im_apply(0x10, 4, 96, 96, C.byref(A), C.byref(w), 1, 1, 0x20, 0x30,
                              1 << 20, None) == -3


def test_autotune_cache_round_trip(lib, tmp_path):
    """The autotune cache leaves the process as a record / JSON file and comes
    back: a pinned configuration survives clear + load; a record of another
    variant table, a malformed one, or one measured on another device is not
    taken."""
    import paper_2606_07759_amd as S
    from paper_2606_07759_amd import _abi
    A = _abi.SynimAffine()
    A.A[0][0] = A.A[1][1] = 1.0
    A.A[0][1] = 0.01
    w = _fake_wfs()
    S.autotune_clear()
    rec = S.autotune_export()
    assert len(rec) == 3 and rec[0] == 1 and rec[2] == 0
    NC = 10
    cands = (C.c_int * (256 * NC))()
    n = C.c_int(0)
    assert lib.synim_im_candidates(C.byref(w), C.byref(A), cands, 256, C.byref(n)) == 0
    assert n.value >= 2
    first = list(cands[0:NC])
    last = list(cands[(n.value - 1) * NC:n.value * NC])
    assert first != last
    assert lib.synim_im_set_config(C.byref(w), C.byref(A), (C.c_int * NC)(*last)) == 0
    cfg = (C.c_int * NC)()

    def current():
        assert lib.synim_im_config(C.byref(w), C.byref(A), cfg) == 0
        return list(cfg)

    assert current() == last
    rec = S.autotune_export()
    assert len(rec) == 3 + 18 and rec[2] == 1
    path = str(tmp_path / "tune.json")
    S.autotune_save(path, "device A")
    S.autotune_clear()
    assert current() == first
    assert not S.autotune_load(path, "device B")
    assert current() == first
    assert S.autotune_load(path, "device A")
    assert current() == last
    S.autotune_clear()
    bad = list(rec)
    bad[1] ^= 1                              # another variant table
    with pytest.raises(S.SynimError) as e:
        S.autotune_import(bad)
    assert e.value.status == -8
    with pytest.raises(S.SynimError) as e:
        S.autotune_import(rec[:-1])          # truncated
    assert e.value.status == -2
    bad = list(rec)
    bad[3 + 12] = 10 ** 6                    # no such variant
    with pytest.raises(S.SynimError) as e:
        S.autotune_import(bad)
    assert e.value.status == -3
    assert current() == first
