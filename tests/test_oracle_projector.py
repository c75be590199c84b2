"""Pins of the oracle's ray-driven forward projector (the adjoint partner of the
backprojection): a closed form, an independent trilinear sampler (SciPy), the quadrature's
convergence, and the equivalence of a rigid translation of the geometry with a shift of the
volume."""
import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import oracle
from synth.geometry import ScanGeometry, VolumeGrid, projection_matrices


def _setup(n=16, det=33, pitch=1.6, n_views=8):
    scan = ScanGeometry(n_views, det, det, pitch, arc_deg=360.0)
    grid = VolumeGrid(n, n, n, (1.0, 1.0, 1.0))
    g = oracle.geom_from(scan, grid)
    return scan, grid, g, projection_matrices(scan)


def _smooth_volume(n, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(n) - (n - 1) / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    v = np.zeros((n, n, n))
    for _ in range(4):
        c = rng.uniform(-n / 5, n / 5, 3)
        s = rng.uniform(n / 10, n / 5)
        v += rng.uniform(0.5, 1.0) * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s * s))
    return v.astype(np.float32)


def test_central_ray_through_a_constant_volume_is_n_voxels():
    scan, grid, g, P = _setup(n=16, det=33)
    vol = np.ones(grid.shape, dtype=np.float32)
    Phat, _ = oracle.compose(np.zeros((scan.n_views, 6)), P)
    out = oracle.forward_project(g, vol, Phat, step_vox=0.5)
    # view 0: the principal ray runs along -x through the isocentre, between voxel centres
    # in y and z; the interpolant is 1 between the outer centres and ramps to 0 over one voxel
    assert out[0, 16, 16] == pytest.approx(16.0, abs=1e-12)


def test_matches_an_independent_trilinear_sampler():
    scan, grid, g, P = _setup(n=16, det=33)
    vol = _smooth_volume(16, 1)
    rng = np.random.default_rng(2)
    theta = np.zeros((scan.n_views, 6))
    theta[:, :3] = rng.uniform(-2, 2, (scan.n_views, 3))
    theta[:, 3:] = np.radians(rng.uniform(-3, 3, (scan.n_views, 3)))
    Phat, _ = oracle.compose(theta, P)
    fine = oracle.forward_project(g, vol, Phat, step_vox=0.002)
    coarse = oracle.forward_project(g, vol, Phat, step_vox=0.5)
    org = np.asarray(grid.origin_mm)
    for (j, r, c) in [(0, 16, 16), (3, 10, 20), (5, 25, 7), (7, 16, 30)]:
        M = Phat[j][:, :3]
        S = -np.linalg.solve(M, Phat[j][:, 3])
        d = np.linalg.solve(M, np.array([c, r, 1.0]))
        # dense sampling of the ray over a range that covers the volume, SciPy's order-1 spline
        # (trilinear, zero outside) on voxel coordinates
        w = np.linspace(0.5, 1.5, 400001)
        pts = (S[None, :] + w[:, None] * d[None, :] - org[None, :]) / 1.0
        vals = map_coordinates(vol.astype(np.float64), pts.T, order=1, mode="grid-constant", cval=0.0)
        ref = np.trapezoid(vals, w) * np.linalg.norm(d)
        assert fine[j, r, c] == pytest.approx(ref, rel=2e-5, abs=1e-9)
        assert coarse[j, r, c] == pytest.approx(ref, rel=5e-3, abs=1e-6)


def test_translation_of_the_geometry_equals_a_shift_of_the_volume():
    scan, grid, g, P = _setup(n=16, det=33)
    vol = _smooth_volume(16, 3)
    vol[:, :, -1] = 0.0
    th = np.zeros((scan.n_views, 6))
    th[:, 2] = 1.0          # tz = one voxel: points are moved by +z before projection
    Ph1, _ = oracle.compose(th, P)
    Ph0, _ = oracle.compose(np.zeros_like(th), P)
    shifted = np.zeros_like(vol)
    shifted[:, :, 1:] = vol[:, :, :-1]
    a = oracle.forward_project(g, vol, Ph1, step_vox=0.05)
    b = oracle.forward_project(g, shifted, Ph0, step_vox=0.05)
    assert np.max(np.abs(a - b)) <= 1e-3 * np.max(np.abs(b))
