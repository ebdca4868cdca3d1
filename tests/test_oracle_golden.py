"""The oracle reproduces its committed regression fixtures (tests/golden)."""
import os

import numpy as np

import workloads as wl
from oracle import im

G = os.path.join(os.path.dirname(__file__), "golden")


def test_im_columns_fixture():
    ref = np.loadtxt(os.path.join(G, "scao_8x8_im_columns.txt"))
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    I = im.im_build_misreg(F[[0, 10, 40, 44, 80]], cfg.theta, cfg.pupil, cfg.p, cfg.valid)
    assert np.max(np.abs(I.T - ref)) <= 1e-15 * np.abs(ref).max()


def test_jacobian_fixture():
    ref = np.loadtxt(os.path.join(G, "scao_8x8_jacobian_act40.txt"))
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    J = im.jacobian(F[[40]], cfg.theta, cfg.pupil, cfg.p, cfg.valid)
    assert np.max(np.abs(J[:, 0, :].T - ref)) <= 1e-15 * np.abs(ref).max()
