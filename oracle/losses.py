"""FP64 volume losses and their seeds dL/dI — TEST INFRASTRUCTURE (oracle).

The paper's target is a learned quality map averaged to a scalar (Sec.
II-B.3), which needs trained weights that are not available. The hot path is
driven instead by two differentiable volume losses, defined here from first
principles in plain NumPy, float64:

* ``sumsq_grad``: sum over the three axes of squared forward differences
  between neighbouring voxels that both lie in the grid.
* ``entropy`` of a soft histogram: 64 bins of width D over [lo, hi], bin b
  centred at lo + (b + 1/2) D; every voxel value x adds B3((x - c_b)/D) to
  bin b, with B3 the uniform cubic B-spline (a Parzen window, support of four
  bins; mass that falls outside the bins is dropped). p_b = h_b / sum h,
  H = -sum_b p_b log p_b. The paper names low entropy as a property of a
  sharp image (Sec. I).
* ``tv``: isotropic total variation sum_p sqrt(|grad I(p)|^2 + eps^2) with
  forward differences, a difference that would leave the grid counting as 0
  (the paper's TV comparison metric, Sec. IV).
"""
from __future__ import annotations

import numpy as np


def sumsq_grad(I):
    I = np.asarray(I, dtype=np.float64)
    L = 0.0
    delta = np.zeros_like(I)
    for a in range(3):
        D = np.diff(I, axis=a)
        L += float(np.sum(D * D))
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[a] = slice(0, -1)
        hi[a] = slice(1, None)
        delta[tuple(hi)] += 2.0 * D
        delta[tuple(lo)] -= 2.0 * D
    return L, delta


def _b3(s):
    a = np.abs(s)
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3, np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def _db3(s):
    a = np.abs(s)
    d = np.where(a < 1.0, -2.0 * a + 1.5 * a * a, np.where(a < 2.0, -0.5 * (2.0 - a) ** 2, 0.0))
    return np.sign(s) * d


def soft_histogram(I, n_bins=64, lo=-0.01, hi=0.06):
    x = np.asarray(I, dtype=np.float64).ravel()
    D = (hi - lo) / n_bins
    s = (x - lo) / D - 0.5              # bin coordinate: bin b is centred at s = b
    base = np.floor(s).astype(np.int64)
    h = np.zeros(n_bins)
    for t in (-1, 0, 1, 2):
        b = base + t
        w = _b3(s - b)
        m = (b >= 0) & (b < n_bins) & (w > 0)
        h += np.bincount(b[m], weights=w[m], minlength=n_bins)
    return h


def entropy(I, n_bins=64, lo=-0.01, hi=0.06):
    """(H, dH/dI)"""
    I = np.asarray(I, dtype=np.float64)
    h = soft_histogram(I, n_bins, lo, hi)
    Z = h.sum()
    if Z <= 0:
        return 0.0, np.zeros_like(I)
    p = h / Z
    nz = p > 0
    H = float(-np.sum(p[nz] * np.log(p[nz])))
    # dH/dh_b = -(log p_b + H) / Z for occupied bins
    dh = np.zeros(n_bins)
    dh[nz] = -(np.log(p[nz]) + H) / Z
    D = (hi - lo) / n_bins
    x = I.ravel()
    s = (x - lo) / D - 0.5
    base = np.floor(s).astype(np.int64)
    g = np.zeros_like(x)
    for t in (-1, 0, 1, 2):
        b = base + t
        m = (b >= 0) & (b < n_bins)
        g[m] += dh[b[m]] * _db3(s[m] - b[m]) / D
    return H, g.reshape(I.shape)


def tv(I, eps=1e-5):
    """(TV, dTV/dI)"""
    I = np.asarray(I, dtype=np.float64)
    D = []
    for a in range(3):
        d = np.zeros_like(I)
        sl_lo = [slice(None)] * 3
        sl_lo[a] = slice(0, -1)
        d[tuple(sl_lo)] = np.diff(I, axis=a)
        D.append(d)
    N = np.sqrt(D[0] ** 2 + D[1] ** 2 + D[2] ** 2 + eps * eps)
    val = float(np.sum(N))
    g = np.zeros_like(I)
    for a in range(3):
        q = D[a] / N
        g -= q
        # the term at p - e_a depends on I(p) with +1
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[a] = slice(0, -1)
        sl_hi[a] = slice(1, None)
        g[tuple(sl_hi)] += q[tuple(sl_lo)]
    return val, g


def entropy_tv(I, lam, n_bins=64, lo=-0.01, hi=0.06, eps=1e-5):
    H, gH = entropy(I, n_bins, lo, hi)
    T, gT = tv(I, eps)
    return H + lam * T, gH + lam * gT, H, T
