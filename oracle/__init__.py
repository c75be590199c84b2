"""FP64 CPU oracle of the motion-compensation hot path — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU path (the two are
independent implementations of the paper's definitions); the only common
module is the seeded input generator ``synth``.

The numerical core is ``gmc_oracle.c`` (plain C, FP64, OpenMP over
independent voxels or views). This module compiles it on first use if the
shared library is missing and wraps it for NumPy arrays.

Functions (paper: Thies et al., arXiv 2401.09283):
  compose             Eq. 1 and the derivative matrices used by Eq. 2
  backproject         Eq. 3 over the whole grid
  backproject_voxels  Eq. 3 at chosen voxels
  backproject_points  Eq. 3 at arbitrary world points
  vjp / vjp_sparse    Eq. 4-5 contracted with a volume seed
  point_jacobian      Eq. 4-5 at single points (no contraction)
  chain               Eq. 2, G_j -> dL/dtheta_j
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WEIGHTING = {"paper": 0, "fdk": 1}
GRAD_MODE = {"paper": 0, "exact": 1}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("det_w", ctypes.c_int32), ("det_h", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("voxel", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("weighting", ctypes.c_int32), ("grad_mode", ctypes.c_int32)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        _lib.oracle_compose.argtypes = [i32, P, P, P, P]
        _lib.oracle_compose.restype = None
        _lib.oracle_rigid.argtypes = [P, P, P]
        _lib.oracle_rigid.restype = None
        for name in ("oracle_backproject",):
            getattr(_lib, name).argtypes = [P, P, P, P]
            getattr(_lib, name).restype = i64
        _lib.oracle_backproject_voxels.argtypes = [P, P, P, i64, P, P]
        _lib.oracle_backproject_voxels.restype = i64
        _lib.oracle_backproject_points.argtypes = [P, P, P, i64, P, i32, i32, P]
        _lib.oracle_backproject_points.restype = i64
        _lib.oracle_vjp.argtypes = [P, P, P, P, P]
        _lib.oracle_vjp.restype = i64
        _lib.oracle_vjp_sparse.argtypes = [P, P, P, i64, P, P, P]
        _lib.oracle_vjp_sparse.restype = i64
        _lib.oracle_point_jacobian.argtypes = [P, P, P, i64, P, i32, i32, P]
        _lib.oracle_point_jacobian.restype = i64
        _lib.oracle_chain.argtypes = [i32, P, P, P]
        _lib.oracle_chain.restype = None
        _lib.oracle_project_points.argtypes = [P, i64, P, P]
        _lib.oracle_project_points.restype = None
        _lib.oracle_forward_project.argtypes = [P, P, P, i32, P, ctypes.c_double, i32, i32, P]
        _lib.oracle_forward_project.restype = None
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def geom(n_views, det_w, det_h, shape, voxel, origin, weighting="fdk", grad_mode="paper") -> _Geom:
    g = _Geom()
    g.n_views, g.det_w, g.det_h = int(n_views), int(det_w), int(det_h)
    g.nx, g.ny, g.nz = (int(s) for s in shape)
    g.voxel = (ctypes.c_double * 3)(*[float(v) for v in voxel])
    g.origin = (ctypes.c_double * 3)(*[float(v) for v in origin])
    g.weighting = WEIGHTING[weighting] if isinstance(weighting, str) else int(weighting)
    g.grad_mode = GRAD_MODE[grad_mode] if isinstance(grad_mode, str) else int(grad_mode)
    return g


def geom_from(scan, grid, weighting="fdk", grad_mode="paper") -> _Geom:
    """Build the geometry record from ``synth`` scan and grid descriptions."""
    return geom(scan.n_views, scan.det_w, scan.det_h, grid.shape, grid.voxel_mm, grid.origin_mm,
                weighting, grad_mode)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def rigid(theta6):
    """T (4x4) and dT/dtheta (6x4x4) for one parameter vector."""
    th = _f64(theta6, (6,))
    T = np.empty((4, 4))
    dT = np.empty((6, 4, 4))
    _L().oracle_rigid(_ptr(th), _ptr(T), _ptr(dT))
    return T, dT


def compose(theta, P):
    """(Phat [n][3][4], dPhat [n][6][3][4]) from theta [n][6] and P [n][3][4]."""
    th = _f64(theta)
    n = th.shape[0]
    P = _f64(P, (n, 3, 4))
    Phat = np.empty((n, 3, 4))
    dPhat = np.empty((n, 6, 3, 4))
    _L().oracle_compose(n, _ptr(th), _ptr(P), _ptr(Phat), _ptr(dPhat))
    return Phat, dPhat


def backproject(g: _Geom, proj, Phat):
    """Whole volume [nx][ny][nz] (float64). Raises if any voxel has w <= 0."""
    proj = _f32(proj)
    Phat = _f64(Phat)
    vol = np.empty((g.nx, g.ny, g.nz))
    bad = _L().oracle_backproject(ctypes.byref(g), _ptr(proj), _ptr(Phat), _ptr(vol))
    if bad:
        raise ValueError("geometry has %d voxel-view pairs with w <= 0" % bad)
    return vol


def backproject_voxels(g: _Geom, proj, Phat, idx):
    proj = _f32(proj)
    Phat = _f64(Phat)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx))
    bad = _L().oracle_backproject_voxels(ctypes.byref(g), _ptr(proj), _ptr(Phat), len(idx), _ptr(idx), _ptr(out))
    if bad:
        raise ValueError("geometry has %d voxel-view pairs with w <= 0" % bad)
    return out


def backproject_points(g: _Geom, proj, Phat, pts, view_lo=0, view_hi=None):
    proj = _f32(proj)
    Phat = _f64(Phat)
    pts = _f64(pts).reshape(-1, 3)
    if view_hi is None:
        view_hi = g.n_views
    out = np.empty(len(pts))
    bad = _L().oracle_backproject_points(ctypes.byref(g), _ptr(proj), _ptr(Phat), len(pts), _ptr(pts),
                                         int(view_lo), int(view_hi), _ptr(out))
    if bad:
        raise ValueError("geometry has %d point-view pairs with w <= 0" % bad)
    return out


def vjp(g: _Geom, proj, Phat, delta):
    """G [n_views][3][4] = sum_p delta(p) dI(p)/dPhat_j."""
    proj = _f32(proj)
    Phat = _f64(Phat)
    delta = _f64(delta).reshape(g.nx, g.ny, g.nz)
    G = np.empty((g.n_views, 3, 4))
    bad = _L().oracle_vjp(ctypes.byref(g), _ptr(proj), _ptr(Phat), _ptr(delta), _ptr(G))
    if bad:
        raise ValueError("geometry has %d voxel-view pairs with w <= 0" % bad)
    return G


def vjp_sparse(g: _Geom, proj, Phat, idx, dval):
    proj = _f32(proj)
    Phat = _f64(Phat)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    dval = _f64(dval)
    G = np.empty((g.n_views, 3, 4))
    bad = _L().oracle_vjp_sparse(ctypes.byref(g), _ptr(proj), _ptr(Phat), len(idx), _ptr(idx), _ptr(dval), _ptr(G))
    if bad:
        raise ValueError("geometry has %d voxel-view pairs with w <= 0" % bad)
    return G


def point_jacobian(g: _Geom, proj, Phat, pts, view_lo=0, view_hi=None):
    """dI_j(p)/dPhat_j [n_pts][n_views_in_range][3][4]."""
    proj = _f32(proj)
    Phat = _f64(Phat)
    pts = _f64(pts).reshape(-1, 3)
    if view_hi is None:
        view_hi = g.n_views
    out = np.empty((len(pts), view_hi - view_lo, 3, 4))
    _L().oracle_point_jacobian(ctypes.byref(g), _ptr(proj), _ptr(Phat), len(pts), _ptr(pts),
                               int(view_lo), int(view_hi), _ptr(out))
    return out


def chain(G, dPhat):
    """dL/dtheta [n][6] from G [n][3][4] and dPhat [n][6][3][4]."""
    G = _f64(G)
    n = G.shape[0]
    dPhat = _f64(dPhat, (n, 6, 3, 4))
    out = np.empty((n, 6))
    _L().oracle_chain(n, _ptr(G), _ptr(dPhat), _ptr(out))
    return out


def project_points(Phat_j, pts):
    """(uh, vh, w) [n][3] of world points under one matrix, FP64."""
    Ph = _f64(Phat_j, (3, 4))
    pts = _f64(pts).reshape(-1, 3)
    out = np.empty((len(pts), 3))
    _L().oracle_project_points(_ptr(Ph), len(pts), _ptr(pts), _ptr(out))
    return out


def voxel_centres(g: _Geom, idx) -> np.ndarray:
    """World centres [n][3] of voxels given by linear index (i*ny + j)*nz + k."""
    idx = np.asarray(idx, dtype=np.int64)
    k = idx % g.nz
    j = (idx // g.nz) % g.ny
    i = idx // (g.nz * g.ny)
    return np.stack([g.origin[0] + i * g.voxel[0], g.origin[1] + j * g.voxel[1],
                     g.origin[2] + k * g.voxel[2]], axis=1)


def forward_project(g: _Geom, vol, Phat, step_vox=0.5, labels=None, part=0, view_lo=0, view_hi=None):
    """Ray-driven FP64 line integrals of the trilinear interpolant of vol (float32 [nx][ny][nz])
    under each Phat: [view_hi - view_lo][det_h][det_w] float64 (midpoint rule, steps of at most
    step_vox times the smallest voxel pitch). labels: optional uint8 volume; only voxels of
    `part` count."""
    v = _f32(vol)
    Ph = _f64(Phat).reshape(-1, 12)
    view_hi = g.n_views if view_hi is None else view_hi
    out = np.zeros((g.n_views, g.det_h, g.det_w))
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint8)
    _L().oracle_forward_project(ctypes.byref(g), _ptr(v), None if lab is None else _ptr(lab), int(part), _ptr(Ph),
                                float(step_vox), int(view_lo), int(view_hi), _ptr(out))
    return out[view_lo:view_hi]
