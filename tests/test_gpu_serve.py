"""Serving on the GPU: one batched launch over several geometries gives bitwise the same
results as the single calls, and a request's solve is the same alone and in the mix, with
requests on their own streams or in lockstep batched launches."""
import dataclasses

import numpy as np
import pytest
import torch

from synth import CONFIGS, make_case
from synth.geometry import ScanGeometry, VolumeGrid, projection_matrices

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd import gmc  # noqa: E402
from paper_2401_09283_amd.autograd import Backprojector  # noqa: E402
from paper_2401_09283_amd.serve import GpuExecutor, Request, Server, summarize  # noqa: E402

DEV = "cuda"


def _items():
    """Four different geometries: the tiny case, a ragged small scan, a coarse head, coarse
    voxels on a fine detector."""
    out = []
    c = make_case("tiny")
    out.append((c.scan, c.grid, c.P, c.theta_true, c.proj))
    scan = ScanGeometry(n_views=37, det_w=75, det_h=41, pitch_mm=1.3)
    grid = VolumeGrid(37, 29, 21, (1.7, 1.9, 1.6))
    rng = np.random.default_rng(17)
    th = np.concatenate([rng.uniform(-6, 6, (37, 3)), rng.uniform(-0.1, 0.1, (37, 3))], 1)
    out.append((scan, grid, projection_matrices(scan), th,
                rng.standard_normal((37, 41, 75)).astype(np.float32)))
    cfg = dataclasses.replace(CONFIGS["serve128"], n_views=60, n=64, voxel_mm=4.0)
    c = make_case(cfg)
    out.append((c.scan, c.grid, c.P, c.theta_true, c.proj))
    # coarse voxels on a fine detector: this plan takes 8-voxel bricks and the largest tile, so
    # the batched launch splits the items into one group per brick depth
    scan = ScanGeometry(n_views=23, det_w=700, det_h=500, pitch_mm=0.64, arc_deg=360.0)
    grid = VolumeGrid(40, 36, 50, (2.0, 2.0, 2.0))
    th = np.concatenate([rng.uniform(-5, 5, (23, 3)), rng.uniform(-0.08, 0.08, (23, 3))], 1)
    out.append((scan, grid, projection_matrices(scan), th, rng.standard_normal((23, 500, 700)).astype(np.float32)))
    return out


def test_batched_launch_is_bitwise_equal_to_single_calls():
    items = []
    for scan, grid, P, th, proj in _items():
        bp = Backprojector(scan.n_views, scan.det_w, scan.det_h, grid.shape, grid.voxel_mm, grid.origin_mm, P)
        d = dict(bp=bp, proj=torch.from_numpy(proj).to(DEV), theta=torch.from_numpy(th).to(DEV))
        d["seed"] = torch.randn(grid.shape, generator=torch.Generator(DEV).manual_seed(len(items)), device=DEV)
        items.append(d)
    # single calls
    ref_vol = [it["bp"].forward(it["proj"], it["theta"]).clone() for it in items]
    ref_g = [it["bp"].vjp(it["proj"], it["theta"], it["seed"]).clone() for it in items]
    # one batched call per phase
    vols = [torch.empty_like(v) for v in ref_vol]
    gts = [torch.empty_like(g) for g in ref_g]
    gmc.gmc_launch_batch([dict(plan=it["bp"].plan, proj=it["proj"], P=it["bp"].P, theta=it["theta"], vol=v,
                               workspace=it["bp"].workspace, phase=0) for it, v in zip(items, vols)])
    gmc.gmc_launch_batch([dict(plan=it["bp"].plan, proj=it["proj"], P=it["bp"].P, theta=it["theta"],
                               grad_vol=it["seed"], grad_theta=g, workspace=it["bp"].workspace, phase=1)
                          for it, g in zip(items, gts)])
    for a, b in zip(ref_vol, vols):
        assert torch.equal(a, b)
    for a, b in zip(ref_g, gts):
        assert torch.equal(a, b)


def test_shared_workspace_is_rejected():
    scan, grid, P, th, proj = _items()[0]
    bp = Backprojector(scan.n_views, scan.det_w, scan.det_h, grid.shape, grid.voxel_mm, grid.origin_mm, P)
    pr, tt = torch.from_numpy(proj).to(DEV), torch.from_numpy(th).to(DEV)
    v = torch.empty(grid.shape, device=DEV)
    with pytest.raises(gmc.GmcError):
        gmc.gmc_launch_batch([dict(plan=bp.plan, proj=pr, P=bp.P, theta=tt, vol=v, workspace=bp.workspace, phase=0)] * 2)


def _req_inputs(i):
    cfg = dataclasses.replace(CONFIGS["serve128"], n_views=60 + 10 * i, n=48 + 16 * (i % 2), voxel_mm=4.0,
                              n_nodes=8)
    c = make_case(cfg, phantom_seed=1000 + i, motion_seed=2000 + i)
    g = gmc.make_geometry(cfg.n_views, cfg.det_w, cfg.det_h, c.grid.shape, c.grid.voxel_mm, c.grid.origin_mm)
    return dict(geometry=g, proj=c.proj, P=c.P, n_nodes=cfg.n_nodes)


def _solo(inputs, n_iter):
    """A plain solve: the solver's own iterations on the current stream."""
    solo = Request(100, 0.0, n_iter, dict(inputs))
    ex = GpuExecutor(mode="batched")
    ex.admit(solo)
    s = solo.state
    for _ in range(n_iter):
        s.iteration()
    return ex.result(solo)


@pytest.mark.parametrize("mode,policy", [("streams", "srpt"), ("streams", "all"), ("batched", "srpt"),
                                         ("batched", "all")])
def test_served_results_equal_solo_solves(mode, policy):
    inputs = [_req_inputs(i) for i in range(4)]
    reqs = [Request(i, 0.0 if i < 2 else 0.002 * i, 6 + i, dict(inputs[i])) for i in range(4)]
    # srpt with a tick budget of about two of these requests: some ticks share the GPU, some not
    ex = GpuExecutor(mode=mode)
    srv = Server(ex, hbm_budget_bytes=int(50e9), max_active=3, policy=policy, tick_work=2.6e7)
    done = srv.run(reqs)
    s = summarize(done)
    print("[serve %s/%s] %s mean batch %.2f" % (mode, policy, s, np.mean(srv.batch_sizes)), flush=True)
    assert s["done"] == 4
    assert max(srv.batch_sizes) > 1          # requests did share ticks
    for r in done:
        res = _solo(inputs[r.rid], r.n_iter)
        assert np.array_equal(res["coeffs"], r.result["coeffs"]), r.rid
