"""The allocation-free VJP entry point (static device scratch) against the workspace one.

Two calls in a row through the C ABI, the second on a smaller problem, each compared with
gmc_backproject_vjp on the same inputs (same kernels: bitwise equal) and with the FP64 oracle
(gradient bar 1e-3 per parameter type); then the first problem again, which must reproduce its
first result bitwise (nothing of the smaller call leaks through the shared buffer)."""
import numpy as np
import pytest
import torch

import oracle
from parity import GRAD_TOL, case, grad_err, mat_err
from synth.geometry import ScanGeometry, VolumeGrid, projection_matrices

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd import gmc  # noqa: E402

DEV = "cuda"


def _t(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


class Problem:
    def __init__(self, scan, grid, P, theta, proj, seed):
        self.scan, self.grid, self.P, self.theta, self.proj = scan, grid, P, theta, proj
        g = gmc.make_geometry(scan.n_views, scan.det_w, scan.det_h, grid.shape, grid.voxel_mm, grid.origin_mm)
        self.plan = gmc.Plan(g, P)
        rng = np.random.default_rng(seed)
        self.delta = rng.standard_normal(grid.shape).astype(np.float32)
        self.d = dict(proj=_t(proj, torch.float32), P=_t(P, torch.float64), theta=_t(theta, torch.float64),
                      delta=_t(self.delta, torch.float32))

    def with_workspace(self):
        n = self.scan.n_views
        gt = torch.empty((n, 6), dtype=torch.float64, device=DEV)
        gP = torch.empty((n, 3, 4), dtype=torch.float64, device=DEV)
        ws = self.plan.new_workspace(DEV)
        gmc.gmc_backproject_vjp(self.plan, self.d["proj"], self.d["P"], self.d["theta"], self.d["delta"], gt, gP, ws)
        return gt.cpu().numpy(), gP.cpu().numpy()

    def noalloc(self):
        n = self.scan.n_views
        gt = torch.full((n, 6), float("nan"), dtype=torch.float64, device=DEV)
        gP = torch.full((n, 3, 4), float("nan"), dtype=torch.float64, device=DEV)
        flag = torch.full((1,), 7, dtype=torch.int32, device=DEV)
        gmc.gmc_backproject_vjp_noalloc(self.plan, self.d["proj"], self.d["P"], self.d["theta"], self.d["delta"], gt,
                                        gP, flag)
        torch.cuda.synchronize()
        return gt.cpu().numpy(), gP.cpu().numpy(), int(flag.item())

    def oracle_grad(self):
        geo = oracle.geom_from(self.scan, self.grid, "fdk", "paper")
        Phat, dPhat = oracle.compose(self.theta, self.P)
        G = oracle.vjp(geo, self.proj, Phat, self.delta.astype(np.float64))
        return oracle.chain(G, dPhat), G


def _small_problem():
    scan = ScanGeometry(n_views=64, det_w=100, det_h=90, pitch_mm=1.6)
    grid = VolumeGrid(40, 36, 30, (1.5, 1.5, 1.5))
    rng = np.random.default_rng(71)
    P = projection_matrices(scan)
    theta = np.concatenate([rng.uniform(-2, 2, (scan.n_views, 3)), rng.uniform(-0.02, 0.02, (scan.n_views, 3))], 1)
    proj = rng.standard_normal((scan.n_views, scan.det_h, scan.det_w)).astype(np.float32)
    return Problem(scan, grid, P, theta, proj, 72)


def test_noalloc_vjp_matches_the_workspace_entry_point():
    c = case("tiny")
    big = Problem(c.scan, c.grid, c.P, c.theta_true, c.proj, 99)
    small = _small_problem()
    print("[noalloc] tiny 64^3 x 120 views, then 40x36x30 x 64 views, then tiny again", flush=True)
    first = big.noalloc()
    second = small.noalloc()
    third = big.noalloc()
    for name, prob, got in (("tiny", big, first), ("small", small, second)):
        gt, gP, flag = got
        ref_t, ref_P = prob.with_workspace()
        assert flag == 0
        assert np.array_equal(gt, ref_t) and np.array_equal(gP, ref_P), name
        o_t, o_G = prob.oracle_grad()
        e = grad_err(gt, o_t)
        eP = mat_err(gP, o_G)
        print("[noalloc %s] equal to gmc_backproject_vjp; oracle err per parameter %s, dL/dPhat %.2e"
              % (name, np.array2string(e, precision=2), eP), flush=True)
        assert np.all(e <= GRAD_TOL) and eP <= GRAD_TOL
    assert np.array_equal(third[0], first[0]) and np.array_equal(third[1], first[1])
