"""Probe slopes and the Gauss-Newton misregistration fit.

The online-tracking use of synthetic IMs (paper Sec. 5) regenerates IMs from
misregistration estimates.  Here the estimate theta = (t_x, t_y, rho, m) is fitted
to measured probe slopes:

* probe slopes S(theta) = IM(theta) . C for a command matrix C (one column per
  probe mode); by linearity this is the IM of the probe phase maps
  sum_a C[a, j] F_a, which is how it is evaluated here;
* J_S = dIM/dtheta . C, the Jacobian of the probe slopes;
* plain Gauss-Newton steps theta <- theta + (J^T J)^-1 J^T (s_meas - S(theta))
  from theta_0 = (0, 0, 0, 1), stopping when the step, divided per parameter by
  its label half-range, has norm < tol, or after max_iter steps.
"""
from __future__ import annotations

import numpy as np

from . import im as _im

THETA0 = np.array([0.0, 0.0, 0.0, 1.0])


def probe_slopes(maps, theta, pupil, p: int, valid) -> np.ndarray:
    """[n_probe][2*N_valid] float64."""
    return _im.im_build_misreg(maps, theta, pupil, p, valid)


def probe_jacobian(maps, theta, pupil, p: int, valid) -> np.ndarray:
    """[4][n_probe][2*N_valid] float64."""
    return _im.jacobian(maps, theta, pupil, p, valid)


def gauss_newton(s_meas, maps, pupil, p: int, valid, scale, theta0=THETA0,
                 max_iter: int = 20, tol: float = 1e-7):
    """Return (theta, iterations, converged)."""
    theta = np.array(theta0, dtype=np.float64)
    s_meas = np.asarray(s_meas, dtype=np.float64).ravel()
    scale = np.asarray(scale, dtype=np.float64)
    for it in range(1, max_iter + 1):
        S = probe_slopes(maps, theta, pupil, p, valid).ravel()
        J = probe_jacobian(maps, theta, pupil, p, valid).reshape(4, -1).T
        r = s_meas - S
        step = np.linalg.solve(J.T @ J, J.T @ r)
        theta = theta + step
        if np.linalg.norm(step / scale) < tol:
            return theta, it, True
    return theta, max_iter, False
