"""Pins of the oracle's readings at the detector border and of its optimiser steps.

The paper leaves the border open: it names bilinear interpolation of the filtered projections
(Eq. 3) and central differences of them for g_u, g_v (Sec. II-B.2), but not what happens at
the first and last column and row or outside the detector. The oracle reads it as: taps
outside [0, W-1] x [0, H-1] are zero; the difference images are (d[c+1] - d[c-1]) / 2 inside
and one-sided d[1] - d[0], d[W-1] - d[W-2] on the first and last column (rows alike), i.e.
NumPy's ``gradient`` with ``edge_order=1``. These tests check those readings against
independent implementations: NumPy's ``gradient`` at every pixel centre, SciPy's zero-padded
bilinear sampler (``map_coordinates``, order 1, ``grid-constant``) at points straddling and
beyond the border, and an angle-based Feldkamp backprojection that zero-pads, on a grid that
projects partly off the detector.

The oracle is probed through its Jacobian: with Phat = [[1,0,0,u0],[0,1,0,v0],[0,0,0,1]] a
point (x, y, 0) projects to (x + u0, y + v0) at depth w = 1, so in the paper weighting
dI/dPhat has g_u in entry (0, 3), g_v in entry (1, 3), and I is the bilinear value itself.

Optimiser: Adam's bias-corrected steps against ``torch.optim.Adam`` (an independent
implementation), and the decaying gradient step of Eq. 6 against hand-worked step sizes,
the geometric-series total and the closed form of a quadratic.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import oracle
from oracle import motion
from synth.geometry import ScanGeometry, VolumeGrid, projection_matrices
from tests.test_oracle_backprojection import feldkamp_backprojection

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _probe(d, pts_uv):
    """(I, g_u, g_v) of the oracle at detector positions pts_uv [n][2] (paper weighting, w = 1)."""
    H, W = d.shape
    Phat = np.array([[[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0]]])
    geo = oracle.geom(1, W, H, (1, 1, 1), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), "paper", "paper")
    pts = np.column_stack([pts_uv[:, 0], pts_uv[:, 1], np.zeros(len(pts_uv))])
    img = d[None].astype(np.float32)
    I = oracle.backproject_points(geo, img, Phat, pts)
    J = oracle.point_jacobian(geo, img, Phat, pts)[:, 0]
    return I, J[:, 0, 3], J[:, 1, 3]


def _images(seed, H=13, W=17):
    rng = np.random.default_rng(seed)
    rand = rng.standard_normal((H, W)).astype(np.float32)
    c = np.arange(W)[None, :]
    r = np.arange(H)[:, None]
    quad = (0.25 * c * c - 0.5 * r * r + 0.125 * c * r + 3.0).astype(np.float32)   # curved: edges differ from centre
    return {"random": rand, "quadratic": quad}


@pytest.mark.parametrize("kind", ["random", "quadratic"])
def test_gradient_images_at_every_pixel_centre(kind):
    d = _images(40)[kind]
    H, W = d.shape
    rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    pts = np.column_stack([cc.ravel(), rr.ravel()]).astype(np.float64)
    I, gu, gv = _probe(d, pts)
    d64 = d.astype(np.float64)
    ref_u = np.gradient(d64, axis=1, edge_order=1)
    ref_v = np.gradient(d64, axis=0, edge_order=1)
    scale = np.abs(d64).max()
    assert np.max(np.abs(I - d64.ravel())) <= 1e-14 * scale
    assert np.max(np.abs(gu - ref_u.ravel())) <= 1e-13 * scale
    assert np.max(np.abs(gv - ref_v.ravel())) <= 1e-13 * scale
    # the border columns and rows are where the one-sided rule applies; check them by hand too
    gu2 = gu.reshape(H, W)
    gv2 = gv.reshape(H, W)
    assert np.allclose(gu2[:, 0], d64[:, 1] - d64[:, 0], rtol=0, atol=1e-13 * scale)
    assert np.allclose(gu2[:, -1], d64[:, -1] - d64[:, -2], rtol=0, atol=1e-13 * scale)
    assert np.allclose(gv2[0, :], d64[1, :] - d64[0, :], rtol=0, atol=1e-13 * scale)
    assert np.allclose(gv2[-1, :], d64[-1, :] - d64[-2, :], rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("kind", ["random", "quadratic"])
def test_off_detector_taps_are_zero_padded(kind):
    """Points in a band two pixels wide around the detector (half of them off it) and points
    wholly outside: value and difference images sampled as SciPy's zero-padded bilinear."""
    d = _images(41)[kind]
    H, W = d.shape
    rng = np.random.default_rng(42)
    n = 4000
    side = rng.integers(0, 4, n)
    t = rng.uniform(0.0, 1.0, n)
    off = rng.uniform(-1.6, 1.6, n)       # across the border line, up to 1.6 px either way
    u = np.where(side == 0, off, np.where(side == 1, W - 1 + off, t * (W - 1)))
    v = np.where(side == 2, off, np.where(side == 3, H - 1 + off, t * (H - 1)))
    far = np.array([[-3.0, 2.0], [W + 2.5, 4.0], [5.0, -2.2], [6.0, H + 1.5], [-1.0, -1.0], [W, H]])
    pts = np.vstack([np.column_stack([u, v]), far])
    I, gu, gv = _probe(d, pts)
    d64 = d.astype(np.float64)
    coords = [pts[:, 1], pts[:, 0]]

    def zero_padded(img):
        return map_coordinates(img, coords, order=1, mode="grid-constant", cval=0.0)

    scale = np.abs(d64).max()
    assert np.max(np.abs(I - zero_padded(d64))) <= 1e-12 * scale
    assert np.max(np.abs(gu - zero_padded(np.gradient(d64, axis=1, edge_order=1)))) <= 1e-12 * scale
    assert np.max(np.abs(gv - zero_padded(np.gradient(d64, axis=0, edge_order=1)))) <= 1e-12 * scale
    assert np.all(I[-6:-1] == 0.0) and np.all(gu[-6:-1] == 0.0) and np.all(gv[-6:-1] == 0.0)
    # a sample half a pixel outside the first column sees half of that column's value
    I1, gu1, _ = _probe(d, np.array([[-0.5, 4.0]]))
    assert I1[0] == pytest.approx(0.5 * d64[4, 0], abs=1e-14 * scale)
    assert gu1[0] == pytest.approx(0.5 * (d64[4, 1] - d64[4, 0]), abs=1e-14 * scale)


def test_grid_partly_off_the_detector_equals_zero_padded_fdk():
    """A grid wider and taller than the detector's field of view: the voxels near the grid's
    faces project partly or wholly off the detector in most views."""
    scan = ScanGeometry(n_views=36, det_w=30, det_h=22, pitch_mm=1.6)
    grid = VolumeGrid(16, 16, 14, (2.5, 2.5, 2.5))
    rng = np.random.default_rng(43)
    d = (1.0 + rng.standard_normal((scan.n_views, scan.det_h, scan.det_w))).astype(np.float32)
    P = projection_matrices(scan)
    Phat, _ = oracle.compose(np.zeros((scan.n_views, 6)), P)
    geo = oracle.geom_from(scan, grid, "fdk")
    vol = oracle.backproject(geo, d, Phat)
    X, Y, Z = np.meshgrid(grid.coords(0), grid.coords(1), grid.coords(2), indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    ref = feldkamp_backprojection(scan, d.astype(np.float64), pts).reshape(vol.shape)
    # the case must really leave the detector: count (voxel, view) pairs whose 4 taps are not all inside
    uvw = np.einsum("jrc,nc->jnr", Phat, np.column_stack([pts, np.ones(len(pts))]))
    uh, vh = uvw[..., 0] / uvw[..., 2], uvw[..., 1] / uvw[..., 2]
    partly = (uh < 0) | (uh > scan.det_w - 1) | (vh < 0) | (vh > scan.det_h - 1)
    straddle = partly & (uh > -1) & (uh < scan.det_w) & (vh > -1) & (vh < scan.det_h)
    assert partly.mean() > 0.2 and straddle.mean() > 0.02
    assert np.max(np.abs(vol - ref)) <= 1e-12 * np.max(np.abs(ref))


# ----------------------------------------------------------------------------- optimiser steps

def test_adam_steps_match_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(44)
    x0 = rng.standard_normal(120)
    grads = [rng.standard_normal(120) * (0.1 + k) for k in range(6)]
    for lr, b1, b2, eps in ((0.05, 0.9, 0.999, 1e-8), (0.3, 0.8, 0.99, 1e-3)):
        xt = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([xt], lr=lr, betas=(b1, b2), eps=eps)
        x, m, v = x0.copy(), np.zeros(120), np.zeros(120)
        for t, g in enumerate(grads, start=1):
            xt.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            x, m, v = motion.adam_step(x, g, m, v, t, lr, b1, b2, eps)
            ref = xt.detach().numpy()
            assert np.max(np.abs(x - ref)) <= 1e-13 * (1.0 + np.abs(ref).max()), (lr, t)


def test_eq6_step_sizes_hand_worked():
    gold = json.load(open(os.path.join(GOLDEN, "eq6_schedule.json")))
    for n, s in gold["hand_worked_steps"].items():
        assert motion.gd_step_size(int(n), gold["s0"], gold["decay"]) == pytest.approx(s, rel=1e-14)
    # total step over the paper's 100 iterations: geometric series s0 (1 - t^N) / (1 - t)
    s0, t, N = gold["s0"], gold["decay"], gold["iterations"]
    total = sum(motion.gd_step_size(n, s0, t) for n in range(N))
    assert total == pytest.approx(s0 * (1.0 - t ** N) / (1.0 - t), rel=1e-13)


def test_eq6_updates_against_the_negative_gradient():
    rng = np.random.default_rng(45)
    x = rng.standard_normal(180)
    g = rng.standard_normal(180)
    x1 = motion.gd_step(x, g, 0, 100.0, 0.97)
    assert np.allclose(x1, x - 100.0 * g, rtol=0, atol=1e-12)
    x5 = motion.gd_step(x, g, 5, 100.0, 0.97)
    assert np.allclose(x5, x - 100.0 * 0.97 ** 5 * g, rtol=0, atol=1e-12)
    assert np.dot(x5 - x, g) < 0.0


def test_eq6_on_a_quadratic_has_a_product_closed_form():
    """f(x) = a x^2 / 2 has gradient a x, so N steps of Eq. 6 from x0 give
    x0 * prod_n (1 - a s0 t^n)."""
    a, s0, t, x0, N = 0.004, 100.0, 0.97, np.array([2.0, -3.0, 0.5]), 100
    x = x0.copy()
    for n in range(N):
        x = motion.gd_step(x, a * x, n, s0, t)
    prod = math.prod(1.0 - a * s0 * t ** n for n in range(N))
    assert np.allclose(x, x0 * prod, rtol=1e-12, atol=0)
