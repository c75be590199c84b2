"""GPU ray-driven forward projector against the FP64 oracle: every ray of the tiny case under
per-view motion, several independently moving parts, and sampled views at the paper's own
simulation shape (360 views, 700 x 500 detector, 128^3 @ 2 mm)."""
import numpy as np
import pytest
import torch

import oracle
from parity import VOL_TOL, case

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd import gmc  # noqa: E402
from paper_2401_09283_amd.autograd import Backprojector  # noqa: E402

DEV = "cuda"


def _t(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def _blobs(shape, seed):
    rng = np.random.default_rng(seed)
    n = shape[0]
    x = np.arange(n) - (n - 1) / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    v = np.zeros(shape)
    for _ in range(6):
        c = rng.uniform(-n / 4, n / 4, 3)
        s = rng.uniform(n / 16, n / 6)
        v += rng.uniform(0.2, 1.0) * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s * s))
    return v.astype(np.float32)


def _err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def test_forward_projection_matches_oracle_tiny():
    c = case("tiny")
    bp = Backprojector.from_case(c)
    vol = _blobs(c.grid.shape, 1)
    out = torch.empty(bp.plan.proj_shape, dtype=torch.float32, device=DEV)
    gmc.gmc_forward_project(bp.plan, _t(vol, torch.float32), bp.P, _t(c.theta_true, torch.float64), out, bp.workspace)
    Phat, _ = oracle.compose(c.theta_true, c.P)
    ref = oracle.forward_project(oracle.geom_from(c.scan, c.grid), vol, Phat)
    e = _err(out.cpu().numpy(), ref)
    print("[projector tiny] err %.2e" % e, flush=True)
    assert e <= VOL_TOL


@pytest.mark.parametrize("nz", [1, 2, 3])
def test_forward_projection_of_thin_volumes(nz):
    """One, two and three slices: every z tap pair is clamped at the grid's top or bottom (nz = 1
    takes the single-load path, nz >= 2 the paired loads); ragged x and y."""
    c = case("tiny")
    shape = (21, 18, nz)
    origin = tuple(-(n - 1) / 2.0 for n in shape)
    bp = Backprojector(c.scan.n_views, c.scan.det_w, c.scan.det_h, shape, (1.0, 1.0, 1.0), origin, c.P)
    vol = np.random.default_rng(5 + nz).uniform(0.1, 1.0, shape).astype(np.float32)
    out = torch.empty(bp.plan.proj_shape, dtype=torch.float32, device=DEV)
    gmc.gmc_forward_project(bp.plan, _t(vol, torch.float32), bp.P, _t(c.theta_true, torch.float64), out, bp.workspace)
    Phat, _ = oracle.compose(c.theta_true, c.P)
    g = oracle.geom(c.scan.n_views, c.scan.det_w, c.scan.det_h, shape, (1.0, 1.0, 1.0), origin)
    ref = oracle.forward_project(g, vol, Phat)
    e = _err(out.cpu().numpy(), ref)
    print("[projector thin nz=%d] err %.2e" % (nz, e), flush=True)
    assert np.max(np.abs(ref)) > 0 and e <= VOL_TOL


def test_forward_projection_of_moving_parts():
    c = case("tiny")
    bp = Backprojector.from_case(c)
    vol = _blobs(c.grid.shape, 2)
    labels = np.zeros(c.grid.shape, dtype=np.uint8)
    labels[c.grid.shape[0] // 2:] = 1            # two halves move independently
    labels[:, :, :4] = 7                         # a slab that belongs to no part
    rng = np.random.default_rng(3)
    th = np.zeros((2, c.scan.n_views, 6))
    th[0] = c.theta_true
    th[1, :, :3] = rng.uniform(-2, 2, 3)
    th[1, :, 3:] = np.radians(rng.uniform(-2, 2, 3))
    out = torch.empty(bp.plan.proj_shape, dtype=torch.float32, device=DEV)
    gmc.gmc_forward_project_parts(bp.plan, _t(vol, torch.float32), _t(labels, torch.uint8), 2, bp.P,
                                  _t(th, torch.float64), out, bp.workspace)
    g = oracle.geom_from(c.scan, c.grid)
    ref = sum(oracle.forward_project(g, vol, oracle.compose(th[k], c.P)[0], labels=labels, part=k) for k in range(2))
    e = _err(out.cpu().numpy(), ref)
    print("[projector parts] err %.2e" % e, flush=True)
    assert e <= VOL_TOL


def test_forward_projection_paper_shape_sampled_views():
    from synth import CONFIGS, make_case

    cfg = CONFIGS["paper128"]
    cs = make_case("paper128", with_motion=True)
    bp = Backprojector.from_case(cs)
    vol = _blobs(cs.grid.shape, 4) * 0.02
    out = torch.empty(bp.plan.proj_shape, dtype=torch.float32, device=DEV)
    th = _t(cs.theta_true, torch.float64)
    gmc.gmc_forward_project(bp.plan, _t(vol, torch.float32), bp.P, th, out, bp.workspace)
    torch.cuda.synchronize()
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ev[0].record()
    for _ in range(3):
        gmc.gmc_forward_project(bp.plan, _t(vol, torch.float32), bp.P, th, out, bp.workspace)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / 3
    Phat, _ = oracle.compose(cs.theta_true, cs.P)
    g = oracle.geom_from(cs.scan, cs.grid)
    o = out.cpu().numpy()
    worst = 0.0
    for j in (0, 97, 181, 359):
        ref = oracle.forward_project(g, vol, Phat, view_lo=j, view_hi=j + 1)[0]
        worst = max(worst, _err(o[j], ref))
    rays = cfg.n_views * cfg.det_w * cfg.det_h
    print("[projector paper128] err %.2e, %.2f ms per 360-view projection (%.1f Grays/s)"
          % (worst, ms, rays / ms / 1e6), flush=True)
    assert worst <= VOL_TOL
