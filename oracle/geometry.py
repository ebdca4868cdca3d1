"""Composite affine geometry (paper Sec. 2.1).

The DM transform (shift, rotation, magnification), the LGS perspective at the
DM altitude (cone scaling and off-axis footprint shift) and the WFS transform
(rotation, anamorphic magnification, shift) are multiplied into one 3x3
homogeneous matrix, so the IF grid is resampled exactly once.

Coordinates: pixel centres at integers, x = column, y = row; a grid of n pixels
has its centre at (n-1)/2.  R(phi) = [[cos, -sin], [sin, cos]] acts on (x, y).

The warp needs the *inverse* map p_s = A p_o + b (WFS pixel -> IF pixel).  For
the four misregistration parameters theta = (t_x, t_y, rho, m) of a plain SCAO
system the forward map is p_o = c_o + t + (m/kappa) R(rho) (p_s - c_s), hence

    p_s = c_s + (kappa/m) R(-rho) (p_o - c_o - t).
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

HALF_PI = math.pi / 2.0


def rot(phi: float) -> np.ndarray:
    """R(phi); multiples of pi/2 (within 1e-12) give exact 0/+-1 entries."""
    q = phi / HALF_PI
    qr = round(q)
    if abs(q - qr) < 1e-12:
        c, s = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][int(qr) % 4]
    else:
        c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s], [s, c]], dtype=np.float64)


def centre(n: int) -> float:
    return (n - 1) / 2.0


def inverse_from_misreg(theta: Sequence[float], H_in: int, W_in: int, H_out: int, W_out: int,
                        kappa: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """(A, b) of p_s = A p_o + b for theta = (t_x, t_y, rho, m)."""
    tx, ty, rho, m = (float(v) for v in theta)
    A = (kappa / m) * rot(-rho)
    co = np.array([centre(W_out), centre(H_out)])
    cs = np.array([centre(W_in), centre(H_in)])
    b = cs - A @ (co + np.array([tx, ty]))
    return A, b


def derivative_maps(theta: Sequence[float], H_in: int, W_in: int, H_out: int, W_out: int,
                    kappa: float = 1.0):
    """[(dA_j, db_j)] with d p_s / d theta_j = dA_j p_o + db_j, j = t_x, t_y, rho, m.

    d/dt   = -(kappa/m) R(-rho) e
    d/drho = -(kappa/m) R(-rho) J (p_o - c_o - t),  J = [[0,-1],[1,0]]
    d/dm   = -(p_s - c_s) / m
    """
    tx, ty, rho, m = (float(v) for v in theta)
    A, _ = inverse_from_misreg(theta, H_in, W_in, H_out, W_out, kappa)
    co = np.array([centre(W_out), centre(H_out)])
    ct = co + np.array([tx, ty])
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    out = []
    out.append((np.zeros((2, 2)), -A[:, 0].copy()))
    out.append((np.zeros((2, 2)), -A[:, 1].copy()))
    AJ = A @ J
    out.append((-AJ, AJ @ ct))
    out.append((-A / m, (A @ ct) / m))
    return out


def forward_matrix(g) -> np.ndarray:
    """3x3 homogeneous forward map (DM px about the DM centre -> WFS px about the
    WFS centre) of a ``workloads.Geometry``-like object, composed in the order
    DM placement -> LGS footprint -> WFS."""
    def h(M, t):
        H = np.eye(3)
        H[:2, :2] = M
        H[:2, 2] = t
        return H
    dm = h(g.dm_mag * rot(g.dm_rot), [g.dm_shift_x, g.dm_shift_y])
    cone = h(np.eye(2) / (g.kappa * g.cone_scale),
             -np.array([g.footprint_x, g.footprint_y]) / (g.kappa * g.cone_scale))
    wfs = h(np.diag([g.wfs_mag_x, g.wfs_mag_y]) @ rot(g.wfs_rot), [g.wfs_shift_x, g.wfs_shift_y])
    return wfs @ cone @ dm


def inverse_from_geometry(g, H_in: int, W_in: int, H_out: int, W_out: int):
    """(A, b) of p_s = A p_o + b for a composite geometry (one matrix, one inverse)."""
    F = forward_matrix(g)
    Finv = np.linalg.inv(F)
    M = Finv[:2, :2]
    t = Finv[:2, 2]
    co = np.array([centre(W_out), centre(H_out)])
    cs = np.array([centre(W_in), centre(H_in)])
    # p_s - c_s = M (p_o - c_o) + t
    return M.copy(), cs + t - M @ co
