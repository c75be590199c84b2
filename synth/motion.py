"""Smooth random rigid motion for simulating motion-corrupted scans.

Motion is drawn as a uniform cubic B-spline per rigid parameter
(tx, ty, tz in mm; rx, ry, rz in rad), zero-centred over the scan and scaled
so that the largest translation and the largest rotation reach the requested
peaks. This only *creates* the ground-truth motion of a synthetic scan.
"""
from __future__ import annotations

import math

import numpy as np


def _b3(s: np.ndarray) -> np.ndarray:
    a = np.abs(s)
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def spline_matrix(n_views: int, n_nodes: int) -> np.ndarray:
    """[n_views][n_nodes] cubic B-spline basis with knots t_m = (m - 1) h, h = (n_views - 1)/(n_nodes - 3)."""
    h = (n_views - 1) / (n_nodes - 3)
    j = np.arange(n_views, dtype=np.float64)[:, None]
    t = (np.arange(n_nodes, dtype=np.float64) - 1.0) * h
    return _b3((j - t[None, :]) / h)


def random_motion(seed: int, n_views: int, n_nodes: int, peak_mm: float, peak_deg: float):
    """(theta [n_views][6], coeffs [6][n_nodes]) with theta = B @ coeffs.T, rotations in rad."""
    rng = np.random.default_rng(seed)
    B = spline_matrix(n_views, n_nodes)
    c = rng.standard_normal((6, n_nodes))
    th = B @ c.T
    shift = th.mean(axis=0)
    c = c - shift[:, None]          # partition of unity: a constant shift of all coefficients
    th = B @ c.T
    st = peak_mm / max(np.abs(th[:, :3]).max(), 1e-300)
    sr = math.radians(peak_deg) / max(np.abs(th[:, 3:]).max(), 1e-300)
    scale = np.array([st, st, st, sr, sr, sr])
    c = c * scale[:, None]
    return B @ c.T, c


def random_akima_motion(seed: int, n_views: int, n_nodes: int, peak_mm: float, peak_deg: float):
    """(theta [n_views][6], node values [6][n_nodes] in (mm, deg)) of a random Akima-spline motion:
    node values drawn per parameter, nodes evenly spaced from the first to the last view, each
    spline zero-centred over the scan, translations and rotations scaled to their peaks. The
    curves are evaluated with SciPy's Akima interpolator."""
    from scipy.interpolate import Akima1DInterpolator

    rng = np.random.default_rng(seed)
    xn = np.linspace(0.0, n_views - 1.0, n_nodes)
    xv = np.arange(n_views, dtype=np.float64)
    y = rng.standard_normal((6, n_nodes))
    th = np.stack([Akima1DInterpolator(xn, y[k])(xv) for k in range(6)], axis=1)
    y = y - th.mean(axis=0)[:, None]   # a constant shift of the nodes shifts the curve
    th = th - th.mean(axis=0)[None, :]
    st = peak_mm / max(np.abs(th[:, :3]).max(), 1e-300)
    sr = peak_deg / max(np.abs(th[:, 3:]).max(), 1e-300)
    scale = np.array([st, st, st, sr, sr, sr])
    y = y * scale[:, None]
    th = th * scale[None, :]
    th[:, 3:] = np.radians(th[:, 3:])
    return th, y
