"""G-tilt slopes by telescoping sums at the subaperture edges (the comparator
engine of paper Sec. 2.2), and the exact G-tilt of a continuous Gaussian IF
for the ablation against the numerical-derivative engine.

Test infrastructure: a plain FP64 statement of the definitions; the library
never imports it.

The G-tilt of a subaperture is its mean phase gradient over the illuminated
area.  Along one pixel row the integral of d(phi)/dx over a run of pupil pixels
telescopes to the phase difference between the run's two boundaries, so

    s_x[k] = (1 / n_k) * sum over rows y of k, over runs [xa, xb] of pupil pixels
             of k on that row:  phi(xb + 1/2, y) - phi(xa - 1/2, y)

and s_y likewise with the columns' runs and the points (x, ya - 1/2), (x, yb + 1/2).
n_k is the number of pupil pixels of k.  Every boundary value is read from the
IF by ONE bilinear interpolation through the composite map at the boundary
point itself (half-integer coordinate on the WFS grid), the engine's defining
difference from the central differences, which read pixel centres.  Units:
phase per WFS pixel; layout as ``oracle.im``.

Readings (the paper describes the engine only as evaluating the phase
difference strictly at the subaperture edges): the edges are those of the
pupil runs inside the subaperture (the pupil boundary where it cuts the
subaperture), one boundary point per pixel row or column at the pixel centre
line, and the same bilinear interpolation with zero fill as the warp.
"""
from __future__ import annotations

import math

import numpy as np

from . import warp as _warp


def edge_points(pupil, p: int, k: int, n_sub_x: int):
    """Boundary points of subaperture k: (xs, ys, coeff) for x and for y.

    x: points (x + 1/2, y) with coefficient [x in k] - [x + 1 in k] (pupil
    pixels of k), i.e. +1 at a run's right boundary, -1 at its left one;
    y: points (x, y + 1/2) with [y in k] - [y + 1 in k]."""
    v, u = divmod(int(k), n_sub_x)
    x0, y0 = u * p, v * p

    def inside(x, y):
        return x0 <= x < x0 + p and y0 <= y < y0 + p and pupil[y, x] > 0

    ptx, pty = [], []
    for y in range(y0, y0 + p):
        for x in range(x0 - 1, x0 + p):
            c = int(inside(x, y)) - int(inside(x + 1, y))
            if c:
                ptx.append((x + 0.5, float(y), c))
    for x in range(x0, x0 + p):
        for y in range(y0 - 1, y0 + p):
            c = int(inside(x, y)) - int(inside(x, y + 1))
            if c:
                pty.append((float(x), y + 0.5, c))
    return ptx, pty


def im_build_tsum(F, A, b, pupil, p: int, valid) -> np.ndarray:
    """[n_act][2N] telescoping-sum slopes of every IF of F through the map (A, b)."""
    F = np.asarray(F, dtype=np.float64)
    H, W = pupil.shape
    n_sub_x = W // p
    nv = len(valid)
    out = np.zeros((F.shape[0], 2 * nv))
    for kk, k in enumerate(np.asarray(valid).tolist()):
        v, u = divmod(int(k), n_sub_x)
        nk = int(np.count_nonzero(pupil[v * p:(v + 1) * p, u * p:(u + 1) * p]))
        if nk == 0:
            continue
        for comp, pts in enumerate(edge_points(pupil, p, k, n_sub_x)):
            if not pts:
                continue
            P = np.array(pts)
            xs = A[0, 0] * P[:, 0] + A[0, 1] * P[:, 1] + b[0]
            ys = A[1, 0] * P[:, 0] + A[1, 1] * P[:, 1] + b[1]
            phi = _warp.bilinear(F, xs, ys)            # [n][points]
            out[:, comp * nv + kk] = (phi * P[:, 2]).sum(axis=1) / nk
    return out


# ------------------------------------------------------ exact continuous G-tilt
_GL = np.polynomial.legendre.leggauss(24)


def _line_integral_gaussian(amp, cx, cy, sigma, A, b, pa, pb):
    """Integral over t in [0, 1] of G(A (pa + t (pb - pa)) + b) dt, G an
    isotropic Gaussian amp exp(-|q - c|^2 / (2 sigma^2)) on the IF grid, by
    24-point Gauss-Legendre quadrature (the integrand is smooth)."""
    t = 0.5 * (_GL[0] + 1.0)
    w = 0.5 * _GL[1]
    x = pa[0] + t * (pb[0] - pa[0])
    y = pa[1] + t * (pb[1] - pa[1])
    xs = A[0, 0] * x + A[0, 1] * y + b[0]
    ys = A[1, 0] * x + A[1, 1] * y + b[1]
    g = amp * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2.0 * sigma * sigma))
    return float((w * g).sum())


def gtilt_exact_gaussian(amp, cx, cy, sigma, A, b, pupil, p: int, valid) -> np.ndarray:
    """[2N] exact G-tilt of the continuous field phi(p_o) = G(A p_o + b) over the
    pupil pixels (unit squares) of every valid subaperture: by the divergence
    theorem along each pixel row, the mean of d(phi)/dx is the sum over rows of
    the integral over the row's height of phi(right boundary) - phi(left
    boundary), divided by the area n_k; likewise for y.  The boundaries are
    those of ``edge_points``; each boundary point becomes a unit segment
    across the row (column)."""
    H, W = pupil.shape
    n_sub_x = W // p
    nv = len(valid)
    out = np.zeros(2 * nv)
    for kk, k in enumerate(np.asarray(valid).tolist()):
        v, u = divmod(int(k), n_sub_x)
        nk = int(np.count_nonzero(pupil[v * p:(v + 1) * p, u * p:(u + 1) * p]))
        if nk == 0:
            continue
        ptx, pty = edge_points(pupil, p, k, n_sub_x)
        sx = sum(c * _line_integral_gaussian(amp, cx, cy, sigma, A, b, (x, y - 0.5), (x, y + 0.5))
                 for x, y, c in ptx)
        sy = sum(c * _line_integral_gaussian(amp, cx, cy, sigma, A, b, (x - 0.5, y), (x + 0.5, y))
                 for x, y, c in pty)
        out[kk] = sx / nk
        out[nv + kk] = sy / nk
    return out


def gaussian_if(amp, cx, cy, sigma, H: int, W: int) -> np.ndarray:
    """The Gaussian sampled at the IF grid's pixel centres [H][W] (float64)."""
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    return amp * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * sigma * sigma))


def rel_rms(est, ref) -> float:
    """RMS of est - ref over RMS of ref."""
    est, ref = np.asarray(est, np.float64), np.asarray(ref, np.float64)
    return math.sqrt(float(((est - ref) ** 2).mean()) / float((ref ** 2).mean()))
