"""Pins of the oracle's geometry (Eq. 1) and of the synthetic scan it consumes.

Each check compares against something other than the oracle's own formula:
the textbook Feldkamp coordinates of a circular scan, a closed-form identity
between a rotated patient and a rotated gantry, finite differences, and an
independent rigid-transform implementation.
"""
import math

import numpy as np
import pytest

import oracle
from synth.geometry import ScanGeometry, VolumeGrid, projection_matrices, rigid_transform


SCAN = ScanGeometry(n_views=36, det_w=96, det_h=80, pitch_mm=1.2, arc_deg=200.0)


def feldkamp_coords(g: ScanGeometry, beta, p):
    """Textbook circular cone-beam coordinates: s along the source direction, t across it,
    U = (D_so - s)/D_so, detector position on the virtual detector with pitch tau."""
    x, y, z = p
    s = x * math.cos(beta) + y * math.sin(beta)
    t = -x * math.sin(beta) + y * math.cos(beta)
    U = (g.dso_mm - s) / g.dso_mm
    tau = g.pitch_mm * g.dso_mm / g.dsd_mm
    return t / (U * tau) + g.c0, z / (U * tau) + g.r0, U


def test_projection_matrix_matches_feldkamp_coordinates():
    P = projection_matrices(SCAN)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-60, 60, (50, 3))
    for j in range(0, SCAN.n_views, 5):
        got = oracle.project_points(P[j], pts)
        for q in range(len(pts)):
            uh, vh, U = feldkamp_coords(SCAN, SCAN.betas[j], pts[q])
            assert got[q, 0] == pytest.approx(uh, abs=1e-9)
            assert got[q, 1] == pytest.approx(vh, abs=1e-9)
            assert got[q, 2] == pytest.approx(U, abs=1e-12)


def test_isocentre_projects_to_principal_point_with_unit_w():
    P = projection_matrices(SCAN)
    for j in range(SCAN.n_views):
        uvw = P[j] @ np.array([0.0, 0.0, 0.0, 1.0])
        assert uvw[2] == pytest.approx(1.0, abs=1e-14)
        assert uvw[0] / uvw[2] == pytest.approx(SCAN.c0, abs=1e-9)
        assert uvw[1] / uvw[2] == pytest.approx(SCAN.r0, abs=1e-9)


def test_rigid_transform_is_a_rotation_and_matches_independent_build():
    rng = np.random.default_rng(5)
    for _ in range(20):
        th = np.concatenate([rng.uniform(-5, 5, 3), rng.uniform(-0.3, 0.3, 3)])
        T, _ = oracle.rigid(th)
        R = T[:3, :3]
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(T, rigid_transform(th)[0], atol=1e-14)


def test_rigid_derivatives_match_finite_differences():
    rng = np.random.default_rng(6)
    for _ in range(10):
        th = np.concatenate([rng.uniform(-5, 5, 3), rng.uniform(-0.5, 0.5, 3)])
        _, dT = oracle.rigid(th)
        for k in range(6):
            h = 1e-5
            e = np.zeros(6)
            e[k] = h
            Tp, _ = oracle.rigid(th + e)
            Tm, _ = oracle.rigid(th - e)
            fd = (Tp - Tm) / (2 * h)
            assert np.allclose(dT[k], fd, atol=1e-9), k


def test_compose_rotation_about_z_equals_rotated_gantry():
    """Rotating the patient by rz = alpha at source angle beta is the static scan at beta - alpha."""
    full = ScanGeometry(n_views=72, det_w=64, det_h=48, pitch_mm=1.0, arc_deg=360.0)
    P = projection_matrices(full)
    step = 2.0 * math.pi / full.n_views
    for j in range(3, full.n_views, 7):
        for m in (1, 2, 3):
            alpha = m * step
            th = np.array([[0, 0, 0, 0, 0, alpha]], dtype=np.float64)
            Phat, _ = oracle.compose(th, P[j:j + 1])
            assert np.allclose(Phat[0], P[j - m], atol=1e-11)


def test_compose_moves_points_like_the_patient_pose():
    P = projection_matrices(SCAN)
    rng = np.random.default_rng(8)
    th = np.concatenate([rng.uniform(-4, 4, (SCAN.n_views, 3)), rng.uniform(-0.2, 0.2, (SCAN.n_views, 3))], 1)
    Phat, dPhat = oracle.compose(th, P)
    T = rigid_transform(th)
    pts = np.concatenate([rng.uniform(-50, 50, (20, 3)), np.ones((20, 1))], 1)
    for j in range(SCAN.n_views):
        assert np.allclose(pts @ Phat[j].T, (pts @ T[j].T) @ P[j].T, rtol=1e-12, atol=1e-9)
    # derivative matrices by finite differences of the composition
    for k in range(6):
        h = 1e-6
        e = np.zeros(6)
        e[k] = h
        Pp, _ = oracle.compose(th + e, P)
        Pm, _ = oracle.compose(th - e, P)
        assert np.allclose(dPhat[:, k], (Pp - Pm) / (2 * h), rtol=1e-6, atol=1e-6)


def test_voxel_grid_is_centred_on_isocentre():
    grid = VolumeGrid(5, 4, 3, (1.0, 2.0, 0.5))
    assert grid.coords(0).tolist() == [-2, -1, 0, 1, 2]
    assert grid.coords(1).tolist() == [-3, -1, 1, 3]
    assert grid.coords(2).tolist() == [-0.5, 0, 0.5]
