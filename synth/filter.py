"""FDK pre-filtering of line integrals: cosine weight, Parker short-scan weight, ramp filter.

The paper filters its projections with a ramp kernel and weights them with a
cosine term (Sec. III), and uses Parker weights for the 200-degree clinical
short scans (Sec. V). It does not print the formulas, so the textbook forms
are used:

* Work on the virtual detector through the isocentre: spacing
  tau = pitch * D_so / D_sd, coordinates a = (c - c0) tau, b = (r - r0) tau.
* Cosine weight D_so / sqrt(D_so^2 + a^2 + b^2).
* Parker weight (Parker 1982, overscan form) over beta in [0, pi + 2 delta].
  With this module's geometry a ray with fan angle gamma (positive towards
  +u) at source angle beta has its conjugate at (beta + pi - 2 gamma,
  -gamma), which fixes the sign of gamma in the three branches.
* Ram-Lak kernel h[0] = 1/(4 tau^2), h[odd n] = -1/(pi^2 n^2 tau^2),
  h[even n != 0] = 0, applied along detector rows as a linear (zero-padded)
  convolution and scaled by tau.
* Angular weight: d_j = dbeta * q_j for a Parker-weighted short scan and
  (dbeta / 2) * q_j for a full circle. Backprojecting d_j with the FDK
  distance weight 1/w^2 then estimates the attenuation in 1/mm.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import ScanGeometry


def ramlak_kernel(n_half: int, tau: float) -> np.ndarray:
    """h[n] for n = -n_half..n_half."""
    n = np.arange(-n_half, n_half + 1)
    h = np.zeros(len(n))
    h[n == 0] = 1.0 / (4.0 * tau * tau)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (math.pi ** 2 * n[odd].astype(np.float64) ** 2 * tau * tau)
    return h


def cosine_weights(g: ScanGeometry) -> np.ndarray:
    """[det_h][det_w]"""
    tau = g.pitch_mm * g.dso_mm / g.dsd_mm
    a = (np.arange(g.det_w) - g.c0) * tau
    b = (np.arange(g.det_h) - g.r0) * tau
    return g.dso_mm / np.sqrt(g.dso_mm ** 2 + a[None, :] ** 2 + b[:, None] ** 2)


def fan_angles(g: ScanGeometry) -> np.ndarray:
    """Fan angle of each detector column [det_w]."""
    a = (np.arange(g.det_w) - g.c0) * g.pitch_mm
    return np.arctan(a / g.dsd_mm)


def parker_weight(beta, gamma, delta: float):
    """Parker weight for source angle beta and fan angle gamma, scan range [0, pi + 2 delta]."""
    beta = np.asarray(beta, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    beta, gamma = np.broadcast_arrays(beta, gamma)
    w = np.ones(beta.shape)
    lo = beta < 2.0 * (delta + gamma)
    hi = beta > math.pi + 2.0 * gamma
    with np.errstate(divide="ignore", invalid="ignore"):
        w_lo = np.sin(math.pi / 4.0 * beta / (delta + gamma)) ** 2
        w_hi = np.sin(math.pi / 4.0 * (math.pi + 2.0 * delta - beta) / (delta - gamma)) ** 2
    w = np.where(lo, w_lo, w)
    w = np.where(hi, w_hi, w)
    w = np.where((beta < 0) | (beta > math.pi + 2.0 * delta), 0.0, w)
    return w


def parker_weights(g: ScanGeometry) -> np.ndarray:
    """[n_views][det_w] Parker weights of the scan (ones for a full circle)."""
    if g.full_scan:
        return np.ones((g.n_views, g.det_w))
    delta = (math.radians(g.arc_deg) - math.pi) / 2.0
    if delta < g.max_fan_angle - 1e-12:
        raise ValueError("short scan shorter than pi + fan angle: Parker weights undefined")
    return parker_weight(g.betas[:, None], fan_angles(g)[None, :], delta)


def fdk_filter(g: ScanGeometry, p: np.ndarray) -> np.ndarray:
    """Filtered projections d [n_views][det_h][det_w] (float64) from line integrals p."""
    import torch

    tau = g.pitch_mm * g.dso_mm / g.dsd_mm
    W = g.det_w
    h = ramlak_kernel(W - 1, tau)           # covers every lag of a row
    nfft = 1 << int(math.ceil(math.log2(3 * W - 2)))
    Hf = torch.fft.rfft(torch.from_numpy(h), nfft)
    wscale = g.dbeta if not g.full_scan else g.dbeta / 2.0
    cw = torch.from_numpy(cosine_weights(g) * (wscale * tau))
    pw = torch.from_numpy(parker_weights(g))
    pt = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float64))
    out = np.empty(p.shape, dtype=np.float64)
    ot = torch.from_numpy(out)
    chunk = max(1, (1 << 25) // (g.det_h * nfft))
    for j0 in range(0, g.n_views, chunk):
        j1 = min(g.n_views, j0 + chunk)
        x = pt[j0:j1] * cw[None] * pw[j0:j1, None, :]
        y = torch.fft.irfft(torch.fft.rfft(x, nfft, dim=2) * Hf, nfft, dim=2)
        # linear convolution: output index n of x*h lives at n + (W-1)
        ot[j0:j1] = y[:, :, W - 1:2 * W - 1]
    return out
