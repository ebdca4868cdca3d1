"""Interaction matrix, its misregistration Jacobian and the vector-Jacobian product.

IM column a = slopes(warp(F_a)) (paper Sec. 2.1 + Sec. 2.2).  Stored
actuator-major: ``im[a] = [s_x[0..N-1], s_y[0..N-1]]``, i.e. the transpose of the
paper's 2*N_valid x N_modes matrix.

Jacobian with respect to theta = (t_x, t_y, rho, m): the warp is
phi(p_o) = bilinear(F, p_s(p_o; theta)), so

    d phi / d theta_j = grad_s bilinear(F, p_s) . d p_s / d theta_j

with the floor-cell (right-continuous) bilinear gradient; the slope step is
linear, so d IM / d theta_j = slopes(d phi / d theta_j).
"""
from __future__ import annotations

import numpy as np

from . import geometry, slopes as _slopes, warp as _warp


def im_build(F, A, b, pupil, p: int, valid) -> np.ndarray:
    """[n_act][2*N_valid] float64."""
    H, W = pupil.shape
    phi = _warp.warp(F, A, b, H, W, halo=1)
    return _slopes.slopes(phi, pupil, p, valid)


def im_build_misreg(F, theta, pupil, p: int, valid, kappa: float = 1.0) -> np.ndarray:
    H, W = pupil.shape
    Hi, Wi = np.asarray(F).shape[-2:]
    A, b = geometry.inverse_from_misreg(theta, Hi, Wi, H, W, kappa)
    return im_build(F, A, b, pupil, p, valid)


def jacobian(F, theta, pupil, p: int, valid, kappa: float = 1.0) -> np.ndarray:
    """[4][n_act][2*N_valid] float64: d IM / d(t_x, t_y, rho, m)."""
    H, W = pupil.shape
    Hi, Wi = np.asarray(F).shape[-2:]
    A, b = geometry.inverse_from_misreg(theta, Hi, Wi, H, W, kappa)
    xs_s, ys_s = _warp.source_coords(A, b, H, W, 1)
    gx, gy = _warp.bilinear_gradient(F, xs_s, ys_s)
    Y, X = np.meshgrid(np.arange(-1, H + 1, dtype=np.float64),
                       np.arange(-1, W + 1, dtype=np.float64), indexing="ij")
    out = []
    for dA, db in geometry.derivative_maps(theta, Hi, Wi, H, W, kappa):
        dxs = dA[0, 0] * X + dA[0, 1] * Y + db[0]
        dys = dA[1, 0] * X + dA[1, 1] * Y + db[1]
        dphi = gx * dxs + gy * dys
        out.append(_slopes.slopes(dphi, pupil, p, valid))
    return np.stack(out)


def vjp(grad_im, J) -> np.ndarray:
    """grad_theta_j = <grad_im, dIM/dtheta_j> (Frobenius), float64[4]."""
    g = np.asarray(grad_im, dtype=np.float64)
    return np.array([(g * J[j]).sum() for j in range(J.shape[0])])


def min_cell_edge_distance(A, b, H: int, W: int) -> float:
    """Smallest distance of any haloed-window source coordinate to an integer.

    When this exceeds the coordinate error of a lower-precision evaluation, both
    evaluations pick the same bilinear cells everywhere (floor decisions agree).
    """
    xs_s, ys_s = _warp.source_coords(A, b, H, W, 1)
    dx = np.abs(xs_s - np.round(xs_s))
    dy = np.abs(ys_s - np.round(ys_s))
    return float(min(dx.min(), dy.min()))


def oob_count(A, b, pupil, p: int, valid, H_in: int, W_in: int) -> int:
    """Out-of-grid samples of one IF column (zero-filled by the warp, Sec. 2.1 with the
    zero-fill reading of the interpolation outside the IF grid).

    Counted per valid subaperture k: the haloed samples q whose central-difference
    coefficient in k is non-zero (c_x = [q-e_x in k, P=1] - [q+e_x in k, P=1], c_y
    likewise) and whose source point A q + b lies outside [0, W_in-1] x [0, H_in-1].
    A sample read by two subapertures counts twice.
    """
    H, W = pupil.shape
    n_sub_x = W // p
    xs_s, ys_s = _warp.source_coords(A, b, H, W, 1)
    out = (xs_s < 0) | (xs_s > W_in - 1) | (ys_s < 0) | (ys_s > H_in - 1)
    total = 0
    for k in np.asarray(valid).tolist():
        v, u = divmod(int(k), n_sub_x)
        m = np.zeros((H + 4, W + 4), np.int64)      # P=1 pixels of k, padded by 2
        m[v * p + 2:(v + 1) * p + 2, u * p + 2:(u + 1) * p + 2] = \
            pupil[v * p:(v + 1) * p, u * p:(u + 1) * p] > 0
        # haloed sample (y, x) in [-1, H] x [-1, W] sits at m[y + 2, x + 2]
        cx = m[1:-1, :-2] - m[1:-1, 2:]
        cy = m[:-2, 1:-1] - m[2:, 1:-1]
        total += int(np.count_nonzero(((cx != 0) | (cy != 0)) & out))
    return total
