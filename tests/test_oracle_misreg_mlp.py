"""Pins of the oracle's Gauss-Newton fit and FP64 MLP.

* Noise-free probe slopes at theta* are fitted back to theta* (GN is exact at
  a zero-residual solution).
* Probe slopes of the combined phase maps equal IM . C (linearity).
* MLP gradients against FP64 central differences on single weights; the first
  Adam step has the closed form p - lr * g / (|g| + eps).
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import im, misreg, mlp


@pytest.fixture(scope="module")
def probe():
    return wl.probe_config()


def test_probe_maps_are_linear_combinations(probe):
    cfg = probe.scao
    F = wl.if_stack(cfg.grid)
    theta = (1.3, -0.4, math.radians(0.3), 1.005)
    I = im.im_build_misreg(F, theta, cfg.pupil, 10, cfg.valid)
    S = misreg.probe_slopes(probe.probe_maps, theta, cfg.pupil, 10, cfg.valid)
    expect = probe.commands.T @ I
    # maps were rounded to float32 once: agreement to float32 resolution
    assert np.max(np.abs(S - expect)) < 1e-6 * np.abs(expect).max()


def test_probe_commands_fit_zernikes(probe):
    # tip (Noll 2) and defocus (Noll 4) fit by the 9x9 DM with small residual
    g = probe.scao.grid
    ifs = wl.if_stack(g).astype(np.float64)
    c = 63.5
    yy, xx = np.mgrid[0:128, 0:128].astype(np.float64)
    sel = np.hypot(xx - c, yy - c) <= 40.0
    for col, j in ((0, 2), (2, 4)):
        Z = wl.zernike_noll(j, 128, 80.0)[sel]
        fit = np.einsum("a,ap->p", probe.commands[:, col], ifs[:, sel])
        assert np.sqrt(np.mean((fit - Z) ** 2)) < 0.2


def test_zernike_orthonormal_on_fine_grid():
    n = 401
    Zs = [wl.zernike_noll(j, n, float(n - 1)) for j in range(1, 12)]
    c = (n - 1) / 2
    yy, xx = np.mgrid[0:n, 0:n]
    sel = np.hypot(xx - c, yy - c) <= (n - 1) / 2
    G = np.array([[np.mean(a[sel] * b[sel]) for b in Zs] for a in Zs])
    assert np.max(np.abs(G - np.eye(len(Zs)))) < 2e-2


@pytest.mark.parametrize("theta_star", [(2.0, -3.5, math.radians(0.6), 1.012),
                                        (-8.0, 6.0, math.radians(-0.9), 0.985)])
def test_gauss_newton_recovers_noise_free_theta(probe, theta_star):
    cfg = probe.scao
    maps = probe.probe_maps
    s = misreg.probe_slopes(maps, theta_star, cfg.pupil, 10, cfg.valid)
    scale = (wl.LABEL_HI - wl.LABEL_LO) / 2
    th, it, conv = misreg.gauss_newton(s, maps, cfg.pupil, 10, cfg.valid, scale)
    assert conv
    assert np.max(np.abs(th - np.array(theta_star)) / scale) < 1e-8


def _params(rng, sizes):
    return [(rng.standard_normal((o, i)) * math.sqrt(2.0 / i), rng.standard_normal(o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_mlp_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = [12, 9, 7, 4]
    P = _params(rng, sizes)
    x = rng.standard_normal((5, 12))
    t = rng.standard_normal((5, 4))
    y, acts = mlp.forward(x, P)
    grads = mlp.backward(acts, P, t)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0), (1, 2), (3, 1)]:
            W, b = P[l]
            if idx[0] >= W.shape[0] or idx[1] >= W.shape[1]:
                continue
            old = W[idx]
            W[idx] = old + h
            lp = mlp.mse(mlp.forward(x, P)[0], t)
            W[idx] = old - h
            lm = mlp.mse(mlp.forward(x, P)[0], t)
            W[idx] = old
            assert abs((lp - lm) / (2 * h) - grads[l][0][idx]) < 1e-7
        b = P[l][1]
        old = b[1]
        b[1] = old + h
        lp = mlp.mse(mlp.forward(x, P)[0], t)
        b[1] = old - h
        lm = mlp.mse(mlp.forward(x, P)[0], t)
        b[1] = old
        assert abs((lp - lm) / (2 * h) - grads[l][1][1]) < 1e-7


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 0.0])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    expect = p - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p1 - expect)) < 1e-15
