"""Single bilinear resampling of IFs onto the WFS grid (paper Sec. 2.1, Sec. 2.2).

For every output pixel p_o in the haloed window {-h..W_out-1+h} x {-h..H_out-1+h}
the source point is p_s = A p_o + b.  With i = floor(x_s), j = floor(y_s),
a = x_s - i, c = y_s - j:

    phi = (1-a)(1-c) F[j,i] + a(1-c) F[j,i+1] + (1-a)c F[j+1,i] + a c F[j+1,i+1]

and F = 0 outside the IF grid.  The halo (1 px) provides the neighbours that the
central differences of the slope step need.
"""
from __future__ import annotations

import numpy as np


def source_coords(A, b, H_out: int, W_out: int, halo: int = 1):
    """x_s, y_s (float64) on the haloed output window, shape (H_out+2h, W_out+2h)."""
    ys = np.arange(-halo, H_out + halo, dtype=np.float64)
    xs = np.arange(-halo, W_out + halo, dtype=np.float64)
    X, Y = np.meshgrid(xs, ys)
    xs_s = A[0, 0] * X + A[0, 1] * Y + b[0]
    ys_s = A[1, 0] * X + A[1, 1] * Y + b[1]
    return xs_s, ys_s


def _tap(F, j, i):
    """F[..., j, i] with zero outside the grid (F has shape [n][H][W])."""
    H, W = F.shape[-2:]
    ok = (i >= 0) & (i < W) & (j >= 0) & (j < H)
    out = np.zeros(F.shape[:-2] + i.shape, dtype=np.float64)
    out[..., ok] = F[..., j[ok], i[ok]]
    return out


def bilinear(F, xs_s, ys_s):
    """Bilinear samples of every IF in F at the given source points."""
    F = np.asarray(F, dtype=np.float64)
    i = np.floor(xs_s).astype(np.int64)
    j = np.floor(ys_s).astype(np.int64)
    a = xs_s - i
    c = ys_s - j
    f00 = _tap(F, j, i)
    f01 = _tap(F, j, i + 1)
    f10 = _tap(F, j + 1, i)
    f11 = _tap(F, j + 1, i + 1)
    return (1 - a) * (1 - c) * f00 + a * (1 - c) * f01 + (1 - a) * c * f10 + a * c * f11


def bilinear_gradient(F, xs_s, ys_s):
    """Floor-cell (right-continuous) gradient of the bilinear interpolant.

    d phi/dx_s = (1-c)(F01-F00) + c(F11-F10),  d phi/dy_s = (1-a)(F10-F00) + a(F11-F01)
    where F_rc is the tap at (row j+r, column i+c).
    """
    F = np.asarray(F, dtype=np.float64)
    i = np.floor(xs_s).astype(np.int64)
    j = np.floor(ys_s).astype(np.int64)
    a = xs_s - i
    c = ys_s - j
    f00 = _tap(F, j, i)
    f01 = _tap(F, j, i + 1)
    f10 = _tap(F, j + 1, i)
    f11 = _tap(F, j + 1, i + 1)
    gx = (1 - c) * (f01 - f00) + c * (f11 - f10)
    gy = (1 - a) * (f10 - f00) + a * (f11 - f01)
    return gx, gy


def warp(F, A, b, H_out: int, W_out: int, halo: int = 1, count_oob: bool = False):
    """Warp an IF stack [n][H_in][W_in] to [n][H_out+2h][W_out+2h] (float64).

    With ``count_oob`` also return the number of output pixels of the haloed
    window whose source point lies outside the closed rectangle
    [0, W_in-1] x [0, H_in-1], i.e. that give a non-zero weight to a tap outside
    the IF grid (zero-filled).
    """
    xs_s, ys_s = source_coords(A, b, H_out, W_out, halo)
    out = bilinear(F, xs_s, ys_s)
    if not count_oob:
        return out
    H, W = np.asarray(F).shape[-2:]
    oob = (xs_s < 0) | (xs_s > W - 1) | (ys_s < 0) | (ys_s > H - 1)
    return out, int(oob.sum())


def warp_loops(F, A, b, H_out: int, W_out: int, halo: int = 1):
    """Per-pixel pure-Python loops: the same definition, for tiny grids only."""
    F = np.asarray(F, dtype=np.float64)
    n, H, W = F.shape
    out = np.zeros((n, H_out + 2 * halo, W_out + 2 * halo))
    import math
    for k in range(n):
        for yo in range(-halo, H_out + halo):
            for xo in range(-halo, W_out + halo):
                xs = A[0][0] * xo + A[0][1] * yo + b[0]
                ys = A[1][0] * xo + A[1][1] * yo + b[1]
                i = math.floor(xs)
                j = math.floor(ys)
                a = xs - i
                c = ys - j
                acc = 0.0
                for (dj, di, w) in ((0, 0, (1 - a) * (1 - c)), (0, 1, a * (1 - c)),
                                    (1, 0, (1 - a) * c), (1, 1, a * c)):
                    jj, ii = j + dj, i + di
                    if 0 <= jj < H and 0 <= ii < W:
                        acc += w * F[k, jj, ii]
                out[k, yo + halo, xo + halo] = acc
    return out
