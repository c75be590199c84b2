"""Circular cone-beam scan geometry and calibrated projection matrices.

The paper describes a scan by one 3x4 projection matrix per view that maps
homogeneous world points to homogeneous detector points, unique up to scale
(Sec. II-A; Sec. II-B.1). It does not fix a coordinate convention, so this
module fixes one:

* World origin at the isocentre; the source rotates in the x-y plane (the
  source's plane of rotation is the reference plane of Fig. 4).
* View j has source angle beta_j = j * arc / n_views (counter-clockwise),
  source S = D_so (cos b, sin b, 0).
* Detector frame: e_u = (-sin b, cos b, 0), e_v = (0, 0, 1),
  e_w = -(cos b, sin b, 0) (from the source towards the detector).
* Pixel (c, r): c is the column (u, fastest in memory), r the row (v), both
  0-based with the pixel centre at integer coordinates. The principal point
  is the detector centre ((W-1)/2, (H-1)/2).
* P = K [R | -R S] / D_so with R = rows (e_u, e_v, e_w) and
  K = [[f, 0, c0], [0, f, r0], [0, 0, 1]], f = D_sd / pitch. Dividing by
  D_so fixes the free scale so that w = depth / D_so, i.e. w = 1 at the
  isocentre; FDK distance weighting 1/w^2 needs this fixed scale.

Voxel (i, j, k) of an (nx, ny, nz) grid has its centre at
origin + (i, j, k) * voxel, stored [i][j][k] with k fastest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class ScanGeometry:
    n_views: int
    det_w: int            # columns (u)
    det_h: int            # rows (v)
    pitch_mm: float       # detector pixel pitch
    dso_mm: float = 785.0   # source-isocentre distance (Sec. III)
    dsd_mm: float = 1200.0  # source-detector distance (Sec. III)
    arc_deg: float = 200.0  # angular range of the trajectory

    @property
    def betas(self) -> np.ndarray:
        return np.arange(self.n_views, dtype=np.float64) * math.radians(self.arc_deg) / self.n_views

    @property
    def dbeta(self) -> float:
        return math.radians(self.arc_deg) / self.n_views

    @property
    def c0(self) -> float:
        return (self.det_w - 1) / 2.0

    @property
    def r0(self) -> float:
        return (self.det_h - 1) / 2.0

    @property
    def focal_px(self) -> float:
        return self.dsd_mm / self.pitch_mm

    @property
    def full_scan(self) -> bool:
        return abs(self.arc_deg - 360.0) < 1e-9

    @property
    def max_fan_angle(self) -> float:
        return math.atan((self.det_w - 1) / 2.0 * self.pitch_mm / self.dsd_mm)


@dataclasses.dataclass(frozen=True)
class VolumeGrid:
    nx: int
    ny: int
    nz: int
    voxel_mm: tuple  # (dx, dy, dz)

    @property
    def origin_mm(self) -> tuple:
        """World coordinate of the centre of voxel (0, 0, 0); the grid is centred on the isocentre."""
        return tuple(-(n - 1) / 2.0 * d for n, d in zip((self.nx, self.ny, self.nz), self.voxel_mm))

    @property
    def shape(self) -> tuple:
        return (self.nx, self.ny, self.nz)

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    def coords(self, axis: int) -> np.ndarray:
        n = self.shape[axis]
        return self.origin_mm[axis] + np.arange(n, dtype=np.float64) * self.voxel_mm[axis]


def source_positions(g: ScanGeometry) -> np.ndarray:
    b = g.betas
    return g.dso_mm * np.stack([np.cos(b), np.sin(b), np.zeros_like(b)], axis=1)


def detector_frames(g: ScanGeometry):
    """(e_u, e_v, e_w), each [n_views][3]."""
    b = g.betas
    z = np.zeros_like(b)
    e_u = np.stack([-np.sin(b), np.cos(b), z], axis=1)
    e_v = np.stack([z, z, np.ones_like(b)], axis=1)
    e_w = -np.stack([np.cos(b), np.sin(b), z], axis=1)
    return e_u, e_v, e_w


def projection_matrices(g: ScanGeometry) -> np.ndarray:
    """Calibrated projection matrices [n_views][3][4] (float64) of the static scan."""
    e_u, e_v, e_w = detector_frames(g)
    S = source_positions(g)
    K = np.array([[g.focal_px, 0.0, g.c0], [0.0, g.focal_px, g.r0], [0.0, 0.0, 1.0]])
    P = np.empty((g.n_views, 3, 4))
    for j in range(g.n_views):
        R = np.stack([e_u[j], e_v[j], e_w[j]], axis=0)
        Rt = np.concatenate([R, (-R @ S[j])[:, None]], axis=1)
        P[j] = K @ Rt / g.dso_mm
    return P


def rigid_transform(theta: np.ndarray) -> np.ndarray:
    """Patient pose matrices [n][4][4] from (tx, ty, tz [mm], rx, ry, rz [rad]).

    Rotation order Rz @ Ry @ Rx about the isocentre, then translation. Used
    here only to *move the phantom* when simulating a motion-corrupted scan.
    """
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    n = theta.shape[0]
    T = np.zeros((n, 4, 4))
    for j in range(n):
        tx, ty, tz, rx, ry, rz = theta[j]
        cx, sx, cy, sy, cz, sz = math.cos(rx), math.sin(rx), math.cos(ry), math.sin(ry), math.cos(rz), math.sin(rz)
        Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
        Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
        Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
        T[j, :3, :3] = Rz @ Ry @ Rx
        T[j, :3, 3] = (tx, ty, tz)
        T[j, 3, 3] = 1.0
    return T


def detector_point(g: ScanGeometry, j: int, c: np.ndarray, r: np.ndarray) -> np.ndarray:
    """World position of detector pixel centres (c, r) of view j; shape [..., 3]."""
    e_u, e_v, e_w = detector_frames(g)
    S = source_positions(g)[j]
    a = (np.asarray(c, dtype=np.float64) - g.c0) * g.pitch_mm
    b = (np.asarray(r, dtype=np.float64) - g.r0) * g.pitch_mm
    return S + g.dsd_mm * e_w[j] + a[..., None] * e_u[j] + b[..., None] * e_v[j]
