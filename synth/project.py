"""Analytic cone-beam line integrals of ellipsoid phantoms under per-view rigid motion.

The paper simulates its scans with a third-party forward projector; here the
line integral of an ellipsoid along a ray is exact: mapping the ellipsoid to
the unit sphere turns the chord into the difference of the two roots of a
quadratic.

Motion convention: at view j the patient pose is T_j (rotation about the
isocentre, then translation), i.e. the density in world space is
mu(T_j^-1 x). The ray from source S_j through a pixel is therefore mapped by
T_j^-1 into the phantom frame, where the static phantom is integrated. A scan
simulated this way is reconstructed sharply by P_j T_j.
"""
from __future__ import annotations

import concurrent.futures as cf
import ctypes
import os
import subprocess

import numpy as np

from .geometry import ScanGeometry, detector_frames, rigid_transform, source_positions
from .phantom import Phantom


def _chord(src: np.ndarray, dirs: np.ndarray, centre, axes, rot) -> np.ndarray:
    """Chord length [n] of rays src + t*dirs (|dirs| = 1) through one ellipsoid."""
    s = ((src - centre) @ rot) / axes
    d = (dirs @ rot) / axes
    A = np.einsum("ij,ij->i", d, d)
    B = d @ s
    C = s @ s - 1.0
    disc = B * B - A * C
    out = np.zeros(len(A))
    m = disc > 0.0
    out[m] = 2.0 * np.sqrt(disc[m]) / A[m]
    return out


def _shadow_box(g: ScanGeometry, src: np.ndarray, e_u, e_v, e_w, centre, radius):
    """Conservative pixel box [c_lo, c_hi) x [r_lo, r_hi) hit by rays through a sphere.

    The sphere lies inside its axis-aligned bounding cube; when the whole cube is
    in front of the source, the cube's shadow is the convex hull of its 8
    projected corners, so their pixel bounding box (plus a margin) is safe.
    """
    corners = centre + radius * np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                                         dtype=np.float64)
    v = corners - src
    depth = v @ e_w
    if np.any(depth <= 1e-6):
        return 0, g.det_w, 0, g.det_h
    f = g.dsd_mm / g.pitch_mm
    u = f * (v @ e_u) / depth + g.c0
    w = f * (v @ e_v) / depth + g.r0
    c_lo = int(max(0, np.floor(u.min()) - 2))
    c_hi = int(min(g.det_w, np.ceil(u.max()) + 3))
    r_lo = int(max(0, np.floor(w.min()) - 2))
    r_hi = int(min(g.det_h, np.ceil(w.max()) + 3))
    return c_lo, c_hi, r_lo, r_hi


def _project_view(g: ScanGeometry, ph: Phantom, j: int, Tinv: np.ndarray, S, e_u, e_v, e_w,
                  cull: bool) -> np.ndarray:
    out = np.zeros((g.det_h, g.det_w))
    Rinv = Tinv[:3, :3]
    tinv = Tinv[:3, 3]
    src_ph = Rinv @ S[j] + tinv  # source in the phantom frame
    for e in range(ph.n):
        if cull:
            # the ellipsoid's bounding sphere, moved into the world frame of view j
            radius = ph.axes[e].max()
            centre_w = np.linalg.solve(Rinv, ph.centres[e] - tinv)
            c_lo, c_hi, r_lo, r_hi = _shadow_box(g, S[j], e_u[j], e_v[j], e_w[j], centre_w, radius)
        else:
            c_lo, c_hi, r_lo, r_hi = 0, g.det_w, 0, g.det_h
        if c_lo >= c_hi or r_lo >= r_hi:
            continue
        cc, rr = np.meshgrid(np.arange(c_lo, c_hi, dtype=np.float64),
                             np.arange(r_lo, r_hi, dtype=np.float64))
        a = (cc.ravel() - g.c0) * g.pitch_mm
        b = (rr.ravel() - g.r0) * g.pitch_mm
        dirs = g.dsd_mm * e_w[j][None, :] + a[:, None] * e_u[j][None, :] + b[:, None] * e_v[j][None, :]
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        dirs_ph = dirs @ Rinv.T
        ch = _chord(src_ph, dirs_ph, ph.centres[e], ph.axes[e], ph.rot[e])
        out[r_lo:r_hi, c_lo:c_hi] += ph.mu[e] * ch.reshape(r_hi - r_lo, c_hi - c_lo)
    return out


def line_integrals_numpy(g: ScanGeometry, ph: Phantom, theta=None, cull: bool = True,
                        workers: int = 1) -> np.ndarray:
    """NumPy version of ``line_integrals`` (slow; kept as the reference of the C version).

    Single-threaded by default: concurrent small matrix products from several Python
    threads were seen to corrupt results with the bundled BLAS.
    """
    if theta is None:
        theta = np.zeros((g.n_views, 6))
    T = rigid_transform(theta)
    Tinv = np.linalg.inv(T)
    S = source_positions(g)
    e_u, e_v, e_w = detector_frames(g)
    out = np.empty((g.n_views, g.det_h, g.det_w))

    def work(j):
        out[j] = _project_view(g, ph, j, Tinv[j], S, e_u, e_v, e_w, cull)

    if workers <= 1:
        for j in range(g.n_views):
            work(j)
    else:
        with cf.ThreadPoolExecutor(workers) as ex:
            list(ex.map(work, range(g.n_views)))
    return out


_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "_project.c")
_CLIB = os.path.join(_HERE, "libsynth.so")
_clib = None


def build_c(force: bool = False) -> str:
    if force or not os.path.exists(_CLIB) or os.path.getmtime(_CLIB) < os.path.getmtime(_CSRC):
        tmp = _CLIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _CSRC, "-o", tmp, "-lm"])
        os.replace(tmp, _CLIB)
    return _CLIB


def _c():
    global _clib
    if _clib is None:
        L = ctypes.CDLL(build_c())
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.synth_line_integrals.argtypes = [i32, i32, i32, f64, f64, f64, vp, vp, i32, vp, vp, vp, vp, vp]
        L.synth_line_integrals.restype = None
        _clib = L
    return _clib


def line_integrals(g: ScanGeometry, ph: Phantom, theta=None, cull: bool = True,
                   workers: int | None = None) -> np.ndarray:
    """Line integrals [n_views][det_h][det_w] (float64) of the phantom moved by T(theta_j)."""
    if not cull:
        return line_integrals_numpy(g, ph, theta, cull=False)
    if theta is None:
        theta = np.zeros((g.n_views, 6))
    Tinv = np.ascontiguousarray(np.linalg.inv(rigid_transform(theta)))
    betas = np.ascontiguousarray(g.betas)
    cen = np.ascontiguousarray(ph.centres, dtype=np.float64)
    ax = np.ascontiguousarray(ph.axes, dtype=np.float64)
    rot = np.ascontiguousarray(ph.rot, dtype=np.float64)
    mu = np.ascontiguousarray(ph.mu, dtype=np.float64)
    out = np.empty((g.n_views, g.det_h, g.det_w))
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _c().synth_line_integrals(g.n_views, g.det_w, g.det_h, g.pitch_mm, g.dso_mm, g.dsd_mm, p(betas), p(Tinv),
                              ph.n, p(cen), p(ax), p(rot), p(mu), p(out))
    return out
