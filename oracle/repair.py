"""Edge repair of an interpolated phase at a pre-masked IF's boundary (paper Sec. 2.3).

Test infrastructure: a plain FP64 statement of the method for checking the HIP
path; the library never imports it.

When the IF stack is pre-masked by the DM-side pupil mask M (binary, on the IF
grid), the single bilinear interpolation of Sec. 2.1 softens the mask edge: the
warped mask m = bilinear(M, A p_o + b) falls below 1 there and the warped phase
collapses towards zero.  The repair takes the paper's three steps, in its order:

1. strict binarisation and clearing: the core S = {m >= threshold} (threshold
   0.999999) keeps its phase, every pixel outside it is zeroed;
2. edge identification: the ring E = dilate(S) minus S, with the binary
   dilation by the 4-neighbour cross;
3. omnidirectional extrapolation: for every e in E and each cardinal direction
   d, with P1 = e + d and P2 = e + 2d: if P1 and P2 are in S the direction gives
   2 phi(P1) - phi(P2), if only P1 is in S it gives phi(P1), otherwise nothing;
   phi(e) becomes the mean of the estimates of the valid directions (every e has
   at least one, since some 4-neighbour of it lies in S).

Readings (the paper names the steps, not every detail): ">= threshold" for the
core; the cross as the dilation's structuring element (cardinal neighbours,
matching the four probe directions); P1 and P2 the first and second pixel from
e along d; pixels outside the evaluated window count as outside S.

On the WFS side the repaired phase feeds the unchanged slope step (Sec. 2.2).
"""
from __future__ import annotations

import numpy as np

from . import slopes as _slopes, warp as _warp

THRESHOLD = 0.999999
DIRS = ((1, 0), (-1, 0), (0, 1), (0, -1))     # (dx, dy): +x, -x, +y, -y


def strict_core(m, threshold: float = THRESHOLD) -> np.ndarray:
    """Step 1: the boolean core {m >= threshold}."""
    return np.asarray(m) >= threshold


def dilate_cross(S) -> np.ndarray:
    """Binary dilation by the 4-neighbour cross (outside the array: false)."""
    S = np.asarray(S, bool)
    D = S.copy()
    D[1:, :] |= S[:-1, :]
    D[:-1, :] |= S[1:, :]
    D[:, 1:] |= S[:, :-1]
    D[:, :-1] |= S[:, 1:]
    return D


def edge_ring(S) -> np.ndarray:
    """Step 2: E = dilate(S) \\ S."""
    S = np.asarray(S, bool)
    return dilate_cross(S) & ~S


def repair(phi, S) -> np.ndarray:
    """Steps 1 and 3 on one 2-D phase map (float64 copy): zero outside the core,
    then every edge pixel replaced by the mean of its directional extrapolations."""
    phi = np.asarray(phi, dtype=np.float64)
    S = np.asarray(S, bool)
    H, W = S.shape
    out = np.where(S, phi, 0.0)
    E = edge_ring(S)

    def inS(x, y):
        return 0 <= x < W and 0 <= y < H and S[y, x]

    for y, x in zip(*np.nonzero(E)):
        est = []
        for dx, dy in DIRS:
            x1, y1, x2, y2 = x + dx, y + dy, x + 2 * dx, y + 2 * dy
            if inS(x1, y1):
                est.append(2.0 * phi[y1, x1] - phi[y2, x2] if inS(x2, y2) else phi[y1, x1])
        out[y, x] = sum(est) / len(est)
    return out


def warp_repaired(F, M, A, b, H_out: int, W_out: int, halo: int = 1,
                  threshold: float = THRESHOLD) -> np.ndarray:
    """Warped and repaired phase of every IF of F (already masked by M) on the
    haloed WFS window [n][H_out+2h][W_out+2h]."""
    phi = _warp.warp(F, A, b, H_out, W_out, halo=halo)
    m = _warp.warp(np.asarray(M, dtype=np.float64)[None], A, b, H_out, W_out, halo=halo)[0]
    S = strict_core(m, threshold)
    return np.stack([repair(f, S) for f in phi])


def im_build_repaired(F, M, A, b, pupil, p: int, valid, threshold: float = THRESHOLD):
    """IM [n_act][2N] of a pre-masked IF stack with edge repair (Sec. 2.1-2.3)."""
    H, W = pupil.shape
    phi = warp_repaired(F, M, A, b, H, W, 1, threshold)
    return _slopes.slopes(phi, pupil, p, valid)
