"""The synthetic workloads: shapes, phantoms, motion and seeds of each case.

Stand-ins for the paper's head CT data (not available): the scanner distances
of Sec. III (785 / 1200 mm) with a 200-degree short-scan trajectory like the
clinical scans of Sec. V, and ellipsoid phantoms.

Cases
-----
tiny      64^3 @ 1 mm, 120 views, 128x128 @ 1.6 mm; 10 random ellipsoids
          (seed 0); motion seed 1: 10-node B-spline, +-2 mm / +-1 deg.
head256   256^3 @ 1 mm, 496 views, 620x480 @ 0.616 mm; head phantom seed 10;
          motion seed 11: 20-node B-spline, +-3 mm / +-2 deg.
head512   512^3 @ 0.5 mm, 496 views, 976x976 @ 0.308 mm; same seeds as head256.
serve128  128^3 @ 2 mm, 248 views, 310x240 @ 1.232 mm (serving mix).
serve384  384^3 @ 0.667 mm, 496 views, 620x480 @ 0.616 mm (serving mix).
paper128  the paper's own simulation shapes (Sec. III-IV): 360 views over a full circle,
          detector 500 rows x 700 columns @ 0.64 mm, estimation grid 128^3 @ 2 mm; head
          phantom seed 20; motion seed 21: 10-node Akima spline, +-5 mm / +-5 deg.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .filter import fdk_filter
from .geometry import ScanGeometry, VolumeGrid, projection_matrices
from .motion import random_akima_motion, random_motion
from .phantom import head_phantom, random_ellipsoids
from .project import line_integrals


@dataclasses.dataclass(frozen=True)
class CaseConfig:
    name: str
    n: int                 # cubic grid edge
    voxel_mm: float
    n_views: int
    det_w: int
    det_h: int
    pitch_mm: float
    phantom: str           # "random" | "head"
    phantom_seed: int
    motion_seed: int
    n_nodes: int
    peak_mm: float
    peak_deg: float
    arc_deg: float = 200.0
    motion_model: str = "bspline"   # "bspline" | "akima": spline of the simulated motion
    est_nodes: int = 0              # nodes of the estimated spline (0: n_nodes)

    @property
    def estimate_nodes(self) -> int:
        return self.est_nodes or self.n_nodes

    @property
    def scan(self) -> ScanGeometry:
        return ScanGeometry(self.n_views, self.det_w, self.det_h, self.pitch_mm, arc_deg=self.arc_deg)

    @property
    def grid(self) -> VolumeGrid:
        return VolumeGrid(self.n, self.n, self.n, (self.voxel_mm,) * 3)

    @property
    def updates(self) -> int:
        """voxel-view updates of one backprojection"""
        return self.n ** 3 * self.n_views


CONFIGS = {
    "tiny": CaseConfig("tiny", 64, 1.0, 120, 128, 128, 1.6, "random", 0, 1, 10, 2.0, 1.0),
    "head256": CaseConfig("head256", 256, 1.0, 496, 620, 480, 0.616, "head", 10, 11, 20, 3.0, 2.0),
    "head512": CaseConfig("head512", 512, 0.5, 496, 976, 976, 0.308, "head", 10, 11, 20, 3.0, 2.0),
    "serve128": CaseConfig("serve128", 128, 2.0, 248, 310, 240, 1.232, "head", 1000, 2000, 20, 3.0, 2.0),
    "serve256": CaseConfig("serve256", 256, 1.0, 496, 620, 480, 0.616, "head", 1000, 2000, 20, 3.0, 2.0),
    "serve384": CaseConfig("serve384", 384, 2.0 / 3.0, 496, 620, 480, 0.616, "head", 1000, 2000, 20, 3.0, 2.0),
    "paper128": CaseConfig("paper128", 128, 2.0, 360, 700, 500, 0.64, "head", 20, 21, 10, 5.0, 5.0,
                           arc_deg=360.0, motion_model="akima", est_nodes=30),
}


@dataclasses.dataclass
class Case:
    cfg: CaseConfig
    scan: ScanGeometry
    grid: VolumeGrid
    P: np.ndarray          # [n_views][3][4] float64 calibrated (static) matrices
    theta_true: np.ndarray  # [n_views][6] float64 motion of the simulated patient
    coeff_true: np.ndarray  # [6][n_nodes]
    proj: np.ndarray       # [n_views][det_h][det_w] float32 filtered projections
    phantom: object


def make_phantom(cfg: CaseConfig, seed: int | None = None):
    s = cfg.phantom_seed if seed is None else seed
    if cfg.phantom == "random":
        return random_ellipsoids(s)
    # the head phantom is sized for a 256 mm field of view; smaller grids shrink it
    fov = cfg.n * cfg.voxel_mm
    return head_phantom(s, scale=min(1.0, fov / 256.0))


def make_case(name_or_cfg, with_motion: bool = True, phantom_seed: int | None = None,
              motion_seed: int | None = None, workers: int | None = None) -> Case:
    cfg = CONFIGS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    scan = cfg.scan
    ph = make_phantom(cfg, phantom_seed)
    ms = cfg.motion_seed if motion_seed is None else motion_seed
    if with_motion and cfg.motion_model == "akima":
        theta, coeff = random_akima_motion(ms, cfg.n_views, cfg.n_nodes, cfg.peak_mm, cfg.peak_deg)
    elif with_motion:
        theta, coeff = random_motion(ms, cfg.n_views, cfg.n_nodes, cfg.peak_mm, cfg.peak_deg)
    else:
        theta, coeff = np.zeros((cfg.n_views, 6)), np.zeros((6, cfg.n_nodes))
    p = line_integrals(scan, ph, theta, workers=workers)
    d = fdk_filter(scan, p).astype(np.float32)
    return Case(cfg, scan, cfg.grid, projection_matrices(scan), theta, coeff, d, ph)
