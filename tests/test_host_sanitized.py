"""The library's host geometry code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

`host_sanitize_driver.cpp` and the host sources of the composite map
(`csrc/geometry.cpp`) are built with both sanitizers (host code only: every
sanitizer flag applies to the host compilation), run on misregistration and
composite-geometry cases, on error cases (non-positive magnification, a
singular chain, null pointers) and on every status string; the run must end
cleanly, with no sanitizer report, and its maps must equal the FP64 oracle's
to the tolerances of the unsanitized ABI tests (Sec. 2.1: the DM and WFS
transforms composed into one map, inverted in FP64)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as wl
from oracle import geometry as og

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("san") / "geometry_san")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", *san, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "paper_2606_07759_amd", "csrc", "geometry.cpp"),
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and ("asan" in r.stderr.lower() or "ubsan" in r.stderr.lower()):
        pytest.skip("sanitizer runtimes not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def run(driver, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       timeout=120, env=env)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    return r.stdout.strip().splitlines()


def nums(line):
    v = line.split()
    return int(v[0]), np.array([float(x) for x in v[1:]])


def as_map(v):
    """[A00 A01 A10 A11 b0 b1] (the driver's order) as the 2 x 3 map [A | b]."""
    return np.array([[v[0], v[1], v[4]], [v[2], v[3], v[5]]])


THETAS = [(0.3, -0.2, math.radians(0.5), 1.01), (-0.9, 0.4, math.radians(-1.0), 0.98),
          (1.5, 2.5, math.pi / 2, 1.2), (0.0, 0.0, math.pi, 1.0), (0.2, 0.1, -math.pi / 2, 0.9)]


def test_misreg_maps_under_sanitizers(driver):
    cases = [(th, k) for th in THETAS for k in (1.0, 1.3)]
    out = run(driver, [f"M {th[0]!r} {th[1]!r} {th[2]!r} {th[3]!r} 96 96 80 80 {k!r} 1"
                       for th, k in cases])
    assert len(out) == len(cases)
    for (th, k), line in zip(cases, out):
        rc, v = nums(line)
        assert rc == 0
        Ao, bo = og.inverse_from_misreg(th, 96, 96, 80, 80, k)
        A = as_map(v[:6])
        assert np.max(np.abs(A[:, :2] - Ao)) < 1e-15 and np.max(np.abs(A[:, 2] - bo)) < 1e-12
        for j, (dAo, dbo) in enumerate(og.derivative_maps(th, 96, 96, 80, 80, k)):
            d = as_map(v[6 + 6 * j:12 + 6 * j])
            assert np.max(np.abs(d[:, :2] - dAo)) < 1e-15 and np.max(np.abs(d[:, 2] - dbo)) < 1e-12


def test_composite_maps_under_sanitizers(driver):
    geos = [pr.geometry for pr in wl.mcao(0).pairs[::3]]
    geos.append(wl.Geometry(dm_shift_x=0.4, dm_rot=0.01, dm_mag=1.02, cone_scale=0.9,
                            footprint_x=3.0, wfs_rot=0.3, wfs_mag_x=1.05, wfs_mag_y=0.97,
                            wfs_shift_y=-0.6, kappa=1.1))
    fields = ("dm_shift_x", "dm_shift_y", "dm_rot", "dm_mag", "cone_scale", "footprint_x",
              "footprint_y", "wfs_shift_x", "wfs_shift_y", "wfs_rot", "wfs_mag_x", "wfs_mag_y",
              "kappa")
    lines = ["G " + " ".join(repr(float(getattr(g, f))) for f in fields) + " 512 512 476 476"
             for g in geos]
    out = run(driver, lines)
    assert len(out) == len(geos)
    for g, line in zip(geos, out):
        rc, v = nums(line)
        assert rc == 0
        Ao, bo = og.inverse_from_geometry(g, 512, 512, 476, 476)
        A = as_map(v)
        assert np.max(np.abs(A[:, :2] - Ao)) < 1e-14 and np.max(np.abs(A[:, 2] - bo)) < 1e-10


def test_error_paths_under_sanitizers(driver):
    out = run(driver, ["M 0 0 0 0 8 8 8 8 1 0",        # zero magnification
                       "M 0 0 0 1 8 8 8 8 0 0",        # zero kappa
                       "M 0 0 0 1 0 8 8 8 1 1",        # empty grid
                       "G 0 0 0 1 1 0 0 0 0 0 0 1 1 8 8 8 8",   # wfs_mag_x = 0: singular
                       "N"] + [f"S {s}" for s in range(-10, 2)])
    assert nums(out[0])[0] == -3 and nums(out[1])[0] == -3 and nums(out[2])[0] == -3
    assert nums(out[3])[0] == -3
    assert [int(x) for x in out[4].split()] == [-1, -1, -1, -1]
    assert out[5 + 10] == "ok"   # status 0
    assert all(len(s) > 0 for s in out[5:])
