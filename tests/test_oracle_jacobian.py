"""Pins of the oracle's Jacobian (Eq. 4-5) and of the chain to the rigid parameters (Eq. 2).

* Euler identity: a projection matrix is unique only up to scale (Sec.
  II-B.1), so the Eq. 3 value is invariant under Phat -> s Phat and its
  gradient is orthogonal to Phat; with the FDK weight the value scales as
  s^-2, so <G_j, Phat_j> = -2 sum_p delta(p) I_j(p).
* Affine detector images have exact central differences, so Eq. 4 is then
  the exact derivative and must match finite differences tightly.
* The "exact" gradient mode (derivative of the bilinear interpolant) must
  match finite differences on any data.
* A hand-worked single point (tests/golden/isocentre_point.json).
* Finite differences through the composition Phat = P T(theta).
"""
import json
import os

import numpy as np
import pytest

import oracle
from synth.geometry import ScanGeometry, VolumeGrid, projection_matrices

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_case(seed, n_views=8, det=(96, 80), grid_n=10, voxel=2.5, motion=True):
    scan = ScanGeometry(n_views=n_views, det_w=det[0], det_h=det[1], pitch_mm=1.0)
    grid = VolumeGrid(grid_n, grid_n, grid_n, (voxel,) * 3)
    rng = np.random.default_rng(seed)
    P = projection_matrices(scan)
    th = np.zeros((n_views, 6))
    if motion:
        th = np.concatenate([rng.uniform(-2, 2, (n_views, 3)), rng.uniform(-0.03, 0.03, (n_views, 3))], 1)
    Phat, dPhat = oracle.compose(th, P)
    return scan, grid, P, th, Phat, dPhat, rng


def affine_images(scan, rng):
    a = rng.integers(-3, 4, scan.n_views) / 8.0
    b = rng.integers(-3, 4, scan.n_views) / 16.0
    g = rng.integers(-20, 21, scan.n_views).astype(np.float64)
    c = np.arange(scan.det_w)[None, None, :]
    r = np.arange(scan.det_h)[None, :, None]
    return (a[:, None, None] * c + b[:, None, None] * r + g[:, None, None]).astype(np.float32)


@pytest.mark.parametrize("weighting", ["paper", "fdk"])
@pytest.mark.parametrize("grad_mode", ["paper", "exact"])
def test_euler_identity(weighting, grad_mode):
    scan, grid, P, th, Phat, dPhat, rng = small_case(1)
    d = rng.standard_normal((scan.n_views, scan.det_h, scan.det_w)).astype(np.float32)
    delta = rng.standard_normal(grid.shape)
    geo = oracle.geom_from(scan, grid, weighting, grad_mode)
    G = oracle.vjp(geo, d, Phat, delta)
    lhs = np.einsum("jrc,jrc->j", G, Phat)
    scale = np.einsum("jrc,jrc->j", np.abs(G), np.abs(Phat))
    if weighting == "paper":
        assert np.all(np.abs(lhs) <= 1e-12 * scale)
    else:
        X, Y, Z = np.meshgrid(grid.coords(0), grid.coords(1), grid.coords(2), indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
        for j in range(scan.n_views):
            Ij = oracle.backproject_points(geo, d, Phat, pts, j, j + 1)
            assert lhs[j] == pytest.approx(-2.0 * np.dot(delta.ravel(), Ij), abs=1e-12 * scale[j])


def _loss(geo, d, Phat, delta):
    return float(np.dot(oracle.backproject(geo, d, Phat).ravel(), delta.ravel()))


@pytest.mark.parametrize("weighting", ["paper", "fdk"])
def test_affine_images_gradient_matches_finite_differences(weighting):
    scan, grid, P, th, Phat, dPhat, rng = small_case(2, n_views=4, det=(200, 160), grid_n=6, voxel=4.0)
    d = affine_images(scan, rng)
    delta = rng.standard_normal(grid.shape)
    geo = oracle.geom_from(scan, grid, weighting, "paper")
    G = oracle.vjp(geo, d, Phat, delta)
    for j in range(scan.n_views):
        for e in range(12):
            r, c = divmod(e, 4)
            h = 1e-6 * max(1.0, abs(Phat[j, r, c]))
            Pp, Pm = Phat.copy(), Phat.copy()
            Pp[j, r, c] += h
            Pm[j, r, c] -= h
            fd = (_loss(geo, d, Pp, delta) - _loss(geo, d, Pm, delta)) / (2 * h)
            assert fd == pytest.approx(G[j, r, c], rel=1e-7, abs=1e-8 * np.abs(G[j]).max())


@pytest.mark.parametrize("weighting", ["paper", "fdk"])
def test_exact_mode_matches_finite_differences(weighting):
    scan, grid, P, th, Phat, dPhat, rng = small_case(3, n_views=8, det=(96, 80), grid_n=16, voxel=1.5)
    d = rng.standard_normal((scan.n_views, scan.det_h, scan.det_w)).astype(np.float32)
    delta = rng.standard_normal(grid.shape)
    geo = oracle.geom_from(scan, grid, weighting, "exact")
    G = oracle.vjp(geo, d, Phat, delta)
    for j in (0, 5):
        for e in range(12):
            r, c = divmod(e, 4)
            # a step that moves detector positions by ~1e-8 px keeps almost every sample inside
            # its bilinear cell, where the interpolant is smooth
            h = 1e-9 * max(1.0, abs(Phat[j, r, c]))
            Pp, Pm = Phat.copy(), Phat.copy()
            Pp[j, r, c] += h
            Pm[j, r, c] -= h
            fd = (_loss(geo, d, Pp, delta) - _loss(geo, d, Pm, delta)) / (2 * h)
            assert fd == pytest.approx(G[j, r, c], rel=1e-6, abs=1e-6 * np.abs(G[j]).max())


def test_paper_mode_differs_from_exact_but_agrees_in_direction():
    """The paper's interpolated central differences are not the derivative of the bilinear
    interpolant; on smooth images both gradients point the same way."""
    scan, grid, P, th, Phat, dPhat, rng = small_case(4, n_views=6, det=(96, 80), grid_n=12, voxel=2.0)
    c = np.arange(scan.det_w)[None, None, :]
    r = np.arange(scan.det_h)[None, :, None]
    ph = rng.uniform(0, 6.28, (scan.n_views, 1, 1))
    d = (np.sin(0.15 * c + ph) * np.cos(0.11 * r)).astype(np.float32)
    delta = rng.standard_normal(grid.shape)
    Gp = oracle.vjp(oracle.geom_from(scan, grid, "fdk", "paper"), d, Phat, delta).ravel()
    Ge = oracle.vjp(oracle.geom_from(scan, grid, "fdk", "exact"), d, Phat, delta).ravel()
    assert not np.allclose(Gp, Ge, rtol=1e-6)
    cos = np.dot(Gp, Ge) / np.linalg.norm(Gp) / np.linalg.norm(Ge)
    assert cos > 0.999


@pytest.mark.parametrize("weighting", ["paper", "fdk"])
def test_hand_worked_isocentre_point(weighting):
    gold = json.load(open(os.path.join(GOLDEN, "isocentre_point.json")))
    scan = ScanGeometry(n_views=1, det_w=gold["W"], det_h=gold["H"], pitch_mm=1.0)
    P = projection_matrices(scan)
    d = np.tile(np.arange(gold["W"], dtype=np.float32)[None, None, :], (1, gold["H"], 1))
    grid = VolumeGrid(1, 1, 1, (1.0, 1.0, 1.0))
    geo = oracle.geom_from(scan, grid, weighting, "paper")
    I = oracle.backproject_points(geo, d, P, np.array([gold["point"]]))
    J = oracle.point_jacobian(geo, d, P, np.array([gold["point"]]))[0, 0]
    assert I[0] == pytest.approx(gold[weighting]["I"], abs=1e-12)
    assert np.allclose(J, np.array(gold[weighting]["G"], dtype=np.float64), atol=1e-12)


def test_chain_matches_finite_differences_of_rigid_parameters():
    scan, grid, P, th, Phat, dPhat, rng = small_case(5, n_views=3, det=(200, 160), grid_n=6, voxel=4.0)
    d = affine_images(scan, rng)
    delta = rng.standard_normal(grid.shape)
    geo = oracle.geom_from(scan, grid, "fdk", "paper")
    G = oracle.vjp(geo, d, Phat, delta)
    g = oracle.chain(G, dPhat)

    def loss(t):
        Ph, _ = oracle.compose(t, P)
        return _loss(geo, d, Ph, delta)

    for j in range(scan.n_views):
        for k in range(6):
            h = 1e-5 if k < 3 else 1e-7
            tp, tm = th.copy(), th.copy()
            tp[j, k] += h
            tm[j, k] -= h
            fd = (loss(tp) - loss(tm)) / (2 * h)
            assert fd == pytest.approx(g[j, k], rel=1e-6, abs=1e-9 * np.abs(g[:, k]).max())


def test_sparse_seed_equals_dense_seed():
    scan, grid, P, th, Phat, dPhat, rng = small_case(6)
    d = rng.standard_normal((scan.n_views, scan.det_h, scan.det_w)).astype(np.float32)
    idx = rng.choice(grid.n_voxels, 50, replace=False)
    val = rng.standard_normal(50)
    delta = np.zeros(grid.n_voxels)
    delta[idx] = val
    geo = oracle.geom_from(scan, grid, "fdk", "paper")
    assert np.allclose(oracle.vjp(geo, d, Phat, delta), oracle.vjp_sparse(geo, d, Phat, idx, val), rtol=1e-13, atol=0)
    vol = oracle.backproject(geo, d, Phat).ravel()
    assert np.allclose(oracle.backproject_voxels(geo, d, Phat, idx), vol[idx], rtol=1e-14, atol=0)


def test_paper_jacobian_memory_figure():
    """The Discussion's 290 GB: one 3x4 block per voxel and view, 4-byte entries."""
    gold = json.load(open(os.path.join(GOLDEN, "jacobian_memory.json")))
    scan = ScanGeometry(n_views=1, det_w=9, det_h=7, pitch_mm=1.0)
    geo = oracle.geom_from(scan, VolumeGrid(1, 1, 1, (1.0,) * 3))
    P = projection_matrices(scan)
    d = np.ones((1, 7, 9), dtype=np.float32)
    block = oracle.point_jacobian(geo, d, P, np.zeros((1, 3)))
    assert block.shape[-2:] == (3, 4) and block[0, 0].size == gold["entries_per_view"]
    nbytes = gold["voxels"] * gold["views"] * block[0, 0].size * gold["bytes_per_entry"]
    assert abs(nbytes / 1e9 - gold["paper_gigabytes"]) <= gold["rounding_gigabytes"]
