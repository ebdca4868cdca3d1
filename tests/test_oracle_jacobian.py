"""Pins of the oracle's misregistration Jacobian and vector-Jacobian product.

* Closed forms for a linear IF: dS/dt = 0, dS/dm = -S/m,
  dS/drho = -(kappa/m) J^T R(-rho)^T g.
* FP64 central differences of the oracle IM itself at a small step agree with
  the analytic Jacobian on a Gaussian-IF geometry (bilinear kinks are avoided
  by the step being far below the smallest distance to a cell edge).
* At the coarse steps of the adjoint workload (1e-3 px, 1e-4 rad, 1e-4), entries
  whose stencil crosses a cell edge within the step are excluded and the rest
  agree (the kink protocol).
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import geometry, im, warp


def test_linear_if_closed_forms():
    cfg = wl.scao_small()
    g = np.array([0.013, -0.021])
    yy, xx = np.mgrid[0:96, 0:96].astype(np.float64)
    F = (g[0] * xx + g[1] * yy + 1.0)[None]
    theta = (0.3, -0.2, math.radians(0.5), 1.01)
    J = im.jacobian(F, theta, cfg.pupil, 10, cfg.valid)
    S = im.im_build_misreg(F, theta, cfg.pupil, 10, cfg.valid)
    nv = cfg.n_valid
    assert np.max(np.abs(J[0])) < 1e-15 and np.max(np.abs(J[1])) < 1e-15
    assert np.max(np.abs(J[3] + S / 1.01)) < 1e-15
    R = geometry.rot(-theta[2])
    Jm = np.array([[0.0, -1.0], [1.0, 0.0]])
    drho = -(1.0 / 1.01) * Jm.T @ R.T @ g
    assert np.max(np.abs(J[2][0, :nv] - drho[0])) < 1e-15
    assert np.max(np.abs(J[2][0, nv:] - drho[1])) < 1e-15


def _fd(F, theta, j, h, cfg):
    tp = np.array(theta, dtype=np.float64)
    tm = tp.copy()
    tp[j] += h
    tm[j] -= h
    return (im.im_build_misreg(F, tp, cfg.pupil, 10, cfg.valid) -
            im.im_build_misreg(F, tm, cfg.pupil, 10, cfg.valid)) / (2 * h)


def test_jacobian_matches_fine_central_differences():
    # each step is sized so that no source coordinate of the haloed window moves
    # by more than a quarter of its smallest distance to a cell edge: the FD then
    # never crosses a bilinear kink and must agree with the analytic derivative
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)[::7]
    J = im.jacobian(F, cfg.theta, cfg.pupil, 10, cfg.valid)
    A, b = geometry.inverse_from_misreg(cfg.theta, 96, 96, 80, 80)
    dmin = im.min_cell_edge_distance(A, b, 80, 80)
    Y, X = np.meshgrid(np.arange(-1, 81.0), np.arange(-1, 81.0), indexing="ij")
    for j, (dA, db) in enumerate(geometry.derivative_maps(cfg.theta, 96, 96, 80, 80)):
        disp = np.maximum(np.abs(dA[0, 0] * X + dA[0, 1] * Y + db[0]),
                          np.abs(dA[1, 0] * X + dA[1, 1] * Y + db[1])).max()
        h = 0.25 * dmin / disp
        fd = _fd(F, cfg.theta, j, h, cfg)
        assert np.max(np.abs(fd - J[j])) <= 1e-6 * np.abs(J[j]).max(), (j, h)


def test_min_cell_distance_of_small_geometry():
    cfg = wl.scao_small()
    A, b = geometry.inverse_from_misreg(cfg.theta, 96, 96, 80, 80)
    d = im.min_cell_edge_distance(A, b, 80, 80)
    assert 1e-6 < d < 1e-3      # generic position: every cell choice is unambiguous


def test_kink_protocol_at_adjoint_workload_steps():
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)
    theta = np.array(cfg.theta)
    steps = [1e-3, 1e-3, 1e-4, 1e-4]
    J = im.jacobian(F, theta, cfg.pupil, 10, cfg.valid)
    A, b = geometry.inverse_from_misreg(theta, 96, 96, 80, 80)
    xs, ys = warp.source_coords(A, b, 80, 80, 1)
    dmaps = geometry.derivative_maps(theta, 96, 96, 80, 80)
    Y, X = np.meshgrid(np.arange(-1, 81.0), np.arange(-1, 81.0), indexing="ij")
    nv = cfg.n_valid
    for j, h in enumerate(steps):
        fd = _fd(F, theta, j, h, cfg)
        dA, db = dmaps[j]
        mx = np.abs(dA[0, 0] * X + dA[0, 1] * Y + db[0]) * h
        my = np.abs(dA[1, 0] * X + dA[1, 1] * Y + db[1]) * h
        near = (np.abs(xs - np.round(xs)) <= 1.5 * mx) | (np.abs(ys - np.round(ys)) <= 1.5 * my)
        # a slope entry is unsafe if any pixel of its haloed stencil is near an edge
        bad = np.zeros(2 * nv, bool)
        for kk, k in enumerate(cfg.valid):
            v, u = divmod(int(k), 8)
            blk = near[v * 10:v * 10 + 12, u * 10:u * 10 + 12]
            bad[kk] = bad[nv + kk] = bool(blk.any())
        ok = ~bad
        assert ok.sum() > 0.4 * ok.size
        err = np.abs(fd[:, ok] - J[j][:, ok]).max() / np.abs(J[j]).max()
        assert err < 1e-6, (j, err)


def test_vjp_is_jacobian_contraction_and_matches_fd_of_inner_product():
    cfg = wl.scao_small()
    F = wl.if_stack(cfg.grid)[::5]
    rng = np.random.default_rng(3)
    theta = np.array(cfg.theta)
    G = rng.standard_normal((F.shape[0], 2 * cfg.n_valid))
    J = im.jacobian(F, theta, cfg.pupil, 10, cfg.valid)
    v = im.vjp(G, J)
    hs = [1e-6, 1e-6, 1e-7, 1e-6]      # below every kink (see the fine-FD test)
    for j, h in enumerate(hs):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fp = (G * im.im_build_misreg(F, tp, cfg.pupil, 10, cfg.valid)).sum()
        fm = (G * im.im_build_misreg(F, tm, cfg.pupil, 10, cfg.valid)).sum()
        assert abs((fp - fm) / (2 * h) - v[j]) < 1e-6 * max(1.0, abs(v[j]))
