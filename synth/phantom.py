"""Additive ellipsoid phantoms.

An ellipsoid is (centre [3] mm, semi-axes [3] mm, orientation [3][3] whose
columns are its axes in world coordinates, density mu [1/mm]). Densities add
where ellipsoids overlap. Phantoms stand in for the head CT volumes of the
paper's data set, which is not available here.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Phantom:
    centres: np.ndarray   # [n][3]
    axes: np.ndarray      # [n][3]
    rot: np.ndarray       # [n][3][3]
    mu: np.ndarray        # [n]

    @property
    def n(self) -> int:
        return len(self.mu)

    def density(self, pts: np.ndarray) -> np.ndarray:
        """Exact density at world points [..., 3] (static phantom)."""
        pts = np.asarray(pts, dtype=np.float64)
        out = np.zeros(pts.shape[:-1])
        for e in range(self.n):
            q = (pts - self.centres[e]) @ self.rot[e] / self.axes[e]
            out += np.where(np.sum(q * q, axis=-1) <= 1.0, self.mu[e], 0.0)
        return out

    def surface_distance_lower_bound(self, pts: np.ndarray) -> np.ndarray:
        """A lower bound of each point's distance to every ellipsoid surface (mm).

        A point at normalised radius rho lies on the surface of rho * E. For a
        convex E containing the ball of radius a_min, rho E = E + (rho - 1) E
        contains E + (rho - 1) a_min B (rho > 1), and likewise E contains
        rho E + (1 - rho) a_min B (rho < 1); so the distance to the surface of E
        is at least a_min |rho - 1|. Used to keep test regions away from edges.
        """
        pts = np.asarray(pts, dtype=np.float64)
        d = np.full(pts.shape[:-1], np.inf)
        for e in range(self.n):
            q = (pts - self.centres[e]) @ self.rot[e] / self.axes[e]
            rho = np.sqrt(np.sum(q * q, axis=-1))
            d = np.minimum(d, self.axes[e].min() * np.abs(rho - 1.0))
        return d


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (QR of a Gaussian matrix with sign fix)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_ellipsoids(seed: int, n: int = 10, axis_range=(4.0, 14.0), ball_radius=14.0,
                      mu_range=(0.0, 0.02)) -> Phantom:
    """n ellipsoids, semi-axes U[axis_range], centres uniform in a ball, random orientation."""
    rng = np.random.default_rng(seed)
    centres = np.empty((n, 3))
    for e in range(n):
        while True:
            p = rng.uniform(-ball_radius, ball_radius, 3)
            if p @ p <= ball_radius ** 2:
                centres[e] = p
                break
    axes = rng.uniform(axis_range[0], axis_range[1], (n, 3))
    rot = np.stack([random_rotation(rng) for _ in range(n)])
    mu = rng.uniform(mu_range[0], mu_range[1], n)
    return Phantom(centres, axes, rot, mu)


def head_phantom(seed: int, n_soft: int = 40, scale: float = 1.0) -> Phantom:
    """Head-like phantom: a 6 mm skull shell at 0.04/mm plus n_soft soft-tissue ellipsoids.

    Skull: outer ellipsoid (72, 92, 78) mm at +0.04 and inner (66, 86, 72) mm at
    -0.04. Soft tissue: semi-axes U[5, 15] mm, mu U[0.018, 0.022]/mm, rejection
    sampled so that they do not overlap each other (bounding spheres) and lie
    inside the inner skull. ``scale`` shrinks every length (same random draws).
    """
    rng = np.random.default_rng(seed)
    outer = np.array([72.0, 92.0, 78.0])
    inner = np.array([66.0, 86.0, 72.0])
    centres = [np.zeros(3), np.zeros(3)]
    axes = [outer, inner]
    rot = [np.eye(3), np.eye(3)]
    mu = [0.04, -0.04]
    placed = []  # (centre, bounding radius)
    tries = 0
    while len(placed) < n_soft:
        tries += 1
        if tries > 200000:
            raise RuntimeError("head phantom: could not place soft-tissue ellipsoids")
        a = rng.uniform(5.0, 15.0, 3)
        c = rng.uniform(-inner, inner)
        R = random_rotation(rng)
        m = rng.uniform(0.018, 0.022)
        rad = a.max()
        # inside the inner skull with a 2 mm gap: every point of the bounding sphere
        # must be inside the inner ellipsoid shrunk by 2 mm
        if np.any(np.abs(c) + rad + 2.0 > inner):
            continue
        q = (np.abs(c) + rad + 2.0) / inner
        if q @ q > 1.0:
            continue
        if any(np.linalg.norm(c - c2) < rad + r2 + 1.0 for c2, r2 in placed):
            continue
        placed.append((c, rad))
        centres.append(c)
        axes.append(a)
        rot.append(R)
        mu.append(m)
    return Phantom(np.array(centres) * scale, np.array(axes) * scale, np.array(rot), np.array(mu))


def single_ellipsoid(centre, axes, mu, rot=None) -> Phantom:
    return Phantom(np.array([centre], dtype=np.float64), np.array([axes], dtype=np.float64),
                   np.array([np.eye(3) if rot is None else rot], dtype=np.float64),
                   np.array([mu], dtype=np.float64))
