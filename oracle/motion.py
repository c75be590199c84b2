"""FP64 motion model, optimiser step and reprojection error — TEST INFRASTRUCTURE (oracle).

* The paper parameterises each of the six rigid parameters by a spline over
  the scan's views (Sec. II-B.1: N = 6 N_n free parameters mapped to
  12 N_p matrix entries). Here the spline is a uniform cubic B-spline with
  N_n coefficients and knots t_m = (m - 1) h, h = (N_p - 1)/(N_n - 3), so
  that exactly four basis functions cover every view 0..N_p-1.
  Coefficients are held in (mm, mm, mm, deg, deg, deg); theta in (mm, rad).
* Gradient descent with exponential step decay is Eq. 6; the solver used
  here is Adam (Kingma & Ba), which the paper's discussion suggests.
* Reprojection error (Sec. IV): mean detector distance (mm) between points
  projected with the estimated and the true geometry.
"""
from __future__ import annotations

import math

import numpy as np

UNIT = np.array([1.0, 1.0, 1.0, math.pi / 180.0, math.pi / 180.0, math.pi / 180.0])


def cubic_bspline(s):
    s = np.abs(np.asarray(s, dtype=np.float64))
    out = np.zeros_like(s)
    m1 = s < 1.0
    m2 = (s >= 1.0) & (s < 2.0)
    out[m1] = (4.0 - 6.0 * s[m1] ** 2 + 3.0 * s[m1] ** 3) / 6.0
    out[m2] = (2.0 - s[m2]) ** 3 / 6.0
    return out


def basis(n_views: int, n_nodes: int) -> np.ndarray:
    """B [n_views][n_nodes]"""
    if n_nodes < 4:
        raise ValueError("a cubic B-spline needs at least 4 coefficients")
    h = (n_views - 1) / (n_nodes - 3)
    B = np.zeros((n_views, n_nodes))
    for j in range(n_views):
        for m in range(n_nodes):
            B[j, m] = cubic_bspline((j - (m - 1) * h) / h)
    return B


def theta_from_coeffs(coeffs, n_views):
    """theta [n_views][6] (mm, rad) from coefficients [6][n_nodes] (mm, deg)."""
    c = np.asarray(coeffs, dtype=np.float64)
    B = basis(n_views, c.shape[1])
    return (B @ c.T) * UNIT[None, :]


def coeff_grad(grad_theta, n_nodes):
    """dL/dc [6][n_nodes] from dL/dtheta [n_views][6] (chain through theta = B c * unit)."""
    g = np.asarray(grad_theta, dtype=np.float64)
    B = basis(g.shape[0], n_nodes)
    return (B.T @ (g * UNIT[None, :])).T


def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based). Returns new (x, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return x - lr * mh / (np.sqrt(vh) + eps), m, v
