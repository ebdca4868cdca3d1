"""Tomographic projection matrix P_opt (paper Sec. 2.5, after Fusco et al. 2001).

Test infrastructure: a plain FP64 statement of the definitions; the library
never imports it.

In MCAO the reconstructed atmosphere (virtual layers) is projected onto the
DMs for a set of optimisation directions.  With every DM influence function
and every layer mode sampled over the telescope pupil along each direction,

    P_opt = (P_DM^T P_DM + lambda I)^{-1} P_DM^T P_Layer,

where the rows of P_DM and P_Layer run over (direction, pupil sample) and
their columns over the DM actuators (all DMs) and the layer modes.

Sampling (the readings taken; the paper states the formula only):
* a component at conjugate altitude h (metres) holds its basis on its own grid
  of pixel size s (metres per pixel), centred on the optical axis at the grid
  centre; the pupil grid (pixel size s_p, centre c_p, mask M) is seen by
  direction theta = (theta_x, theta_y) (radians) through the footprint shift
  h theta, so pupil point r (metres from the axis) reads the component at
  grid coordinate c + (r + h theta) / s, by one bilinear interpolation (zero
  outside the grid) - the same single interpolation as the IM's composite map;
* with a binning factor b >= 1 (the 2x2 or larger binning the paper proposes)
  a row is one b x b block of the pupil grid: the mean of its b^2 samples,
  taken at the block's fine pixel centres; a block is kept if any of its fine
  pixels lies in the mask, and only those fine pixels are averaged;
* rows are ordered direction-major, blocks row-major within a direction.
"""
from __future__ import annotations

import numpy as np

from . import warp as _warp


def pupil_blocks(mask, b: int):
    """Kept blocks of a b x b binning of the pupil mask: list of (by, bx, [(y, x)...])
    in row-major block order, each with its fine pupil pixels."""
    H, W = mask.shape
    out = []
    for by in range(H // b):
        for bx in range(W // b):
            px = [(y, x) for y in range(by * b, by * b + b) for x in range(bx * b, bx * b + b)
                  if mask[y, x]]
            if px:
                out.append((by, bx, px))
    return out


def projection_matrix(stacks, directions, mask, pupil_pixel_m: float, b: int = 1) -> np.ndarray:
    """[n_dir * n_blocks][sum of basis sizes] float64.

    stacks: list of (F [n][H][W] basis on the component grid, altitude m, pixel m).
    directions: [n_dir][2] radians."""
    mask = np.asarray(mask) > 0
    H, W = mask.shape
    cpy, cpx = (H - 1) / 2.0, (W - 1) / 2.0
    blocks = pupil_blocks(mask, b)
    cols = []
    for F, h, s in stacks:
        F = np.asarray(F, dtype=np.float64)
        Hc, Wc = F.shape[-2:]
        cy, cx = (Hc - 1) / 2.0, (Wc - 1) / 2.0
        per_dir = []
        for tx, ty in directions:
            rows = []
            for _, _, px in blocks:
                ys = np.array([p[0] for p in px], np.float64)
                xs = np.array([p[1] for p in px], np.float64)
                gx = cx + ((xs - cpx) * pupil_pixel_m + h * tx) / s
                gy = cy + ((ys - cpy) * pupil_pixel_m + h * ty) / s
                rows.append(_warp.bilinear(F, gx, gy).mean(axis=-1))   # [n]
            per_dir.append(np.stack(rows))                              # [blocks][n]
        cols.append(np.concatenate(per_dir, axis=0))                    # [dir*blocks][n]
    return np.concatenate(cols, axis=1)


def p_opt(P_dm, P_layer, lam: float) -> np.ndarray:
    """(P_dm^T P_dm + lam I)^{-1} P_dm^T P_layer, by a plain linear solve."""
    P_dm = np.asarray(P_dm, np.float64)
    G = P_dm.T @ P_dm + lam * np.eye(P_dm.shape[1])
    return np.linalg.solve(G, P_dm.T @ np.asarray(P_layer, np.float64))
