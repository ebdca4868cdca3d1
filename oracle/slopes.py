"""Shack-Hartmann slopes by central differences and subaperture means (paper Sec. 2.2).

Input: a phase stack on the WFS grid with a 1-px halo, shape [n][H+2][W+2],
pixel (x, y) stored at [y+1][x+1].  At every pupil pixel (P = 1)

    g_x = (phi[y, x+1] - phi[y, x-1]) / 2,   g_y = (phi[y+1, x] - phi[y-1, x]) / 2

(neighbours taken from the resampled field whatever their mask value), and for
each valid subaperture k with n_k pupil pixels

    s_x[k] = sum_{pixels of k with P=1} g_x / n_k,   s_y[k] likewise.

The slope vector of one IF is [s_x[0..N-1], s_y[0..N-1]] (x block then y block),
in phase units per WFS pixel.
"""
from __future__ import annotations

import numpy as np


def subaperture_counts(pupil: np.ndarray, p: int) -> np.ndarray:
    """n_k for every subaperture (row-major), from the pupil mask."""
    h, w = pupil.shape
    return pupil.reshape(h // p, p, w // p, p).astype(np.int64).sum(axis=(1, 3)).ravel()


def slopes(phase, pupil: np.ndarray, p: int, valid: np.ndarray) -> np.ndarray:
    """[n][2*N_valid] float64 slopes of a haloed phase stack."""
    phase = np.asarray(phase, dtype=np.float64)
    P = pupil.astype(np.float64)
    H, W = P.shape
    gx = 0.5 * (phase[:, 1:H + 1, 2:W + 2] - phase[:, 1:H + 1, 0:W])
    gy = 0.5 * (phase[:, 2:H + 2, 1:W + 1] - phase[:, 0:H, 1:W + 1])
    n_sub_x = W // p
    nv = len(valid)
    out = np.zeros((phase.shape[0], 2 * nv))
    for kk, k in enumerate(np.asarray(valid)):
        v, u = divmod(int(k), n_sub_x)
        sl = (slice(None), slice(v * p, v * p + p), slice(u * p, u * p + p))
        msk = P[v * p:v * p + p, u * p:u * p + p]
        nk = msk.sum()
        out[:, kk] = (gx[sl] * msk).sum(axis=(1, 2)) / nk
        out[:, nv + kk] = (gy[sl] * msk).sum(axis=(1, 2)) / nk
    return out


def slopes_loops(phase, pupil, p: int, valid) -> np.ndarray:
    """The same definition as explicit per-pixel loops (tiny grids only)."""
    phase = np.asarray(phase, dtype=np.float64)
    H, W = pupil.shape
    n_sub_x = W // p
    nv = len(valid)
    out = np.zeros((phase.shape[0], 2 * nv))
    for a in range(phase.shape[0]):
        for kk, k in enumerate(valid):
            v, u = divmod(int(k), n_sub_x)
            sx = sy = 0.0
            nk = 0
            for y in range(v * p, v * p + p):
                for x in range(u * p, u * p + p):
                    if pupil[y, x]:
                        nk += 1
                        sx += 0.5 * (phase[a, y + 1, x + 2] - phase[a, y + 1, x])
                        sy += 0.5 * (phase[a, y + 2, x + 1] - phase[a, y, x + 1])
            out[a, kk] = sx / nk
            out[a, nv + kk] = sy / nk
    return out
