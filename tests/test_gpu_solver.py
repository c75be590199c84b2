"""Motion estimation end to end on the GPU: the solver reduces its loss and the
reprojection error of a motion-corrupted synthetic scan; a step equals the oracle's Adam
step on the oracle's gradient."""
import numpy as np
import pytest
import torch

import oracle
from oracle import losses as olosses, motion as omotion
from parity import case

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd.autograd import Backprojector  # noqa: E402
from paper_2401_09283_amd.solver import MotionSolver, SolverConfig, reprojection_error  # noqa: E402


def test_one_iteration_matches_oracle_chain():
    c = case("tiny")
    bp = Backprojector.from_case(c)
    proj = torch.from_numpy(c.proj).to(bp.device)
    s = MotionSolver(bp, proj, SolverConfig(n_nodes=c.cfg.n_nodes, loss="sumsq", lr=0.05))
    s.calibrate()
    s.iteration()
    g_dev = s.gc.cpu().numpy()
    coeff_dev = s.coeffs.cpu().numpy()
    # oracle: theta = 0 -> volume -> loss seed -> G -> dL/dtheta -> dL/dc -> Adam
    th = omotion.theta_from_coeffs(np.zeros((6, c.cfg.n_nodes)), c.cfg.n_views)
    Phat, dPhat = oracle.compose(th, c.P)
    geo = oracle.geom_from(c.scan, c.grid, "fdk", "paper")
    vol = oracle.backproject(geo, c.proj, Phat)
    _, delta = olosses.sumsq_grad(vol)
    gth = oracle.chain(oracle.vjp(geo, c.proj, Phat, delta), dPhat)
    gc = omotion.coeff_grad(gth, c.cfg.n_nodes)
    err = np.max(np.abs(g_dev - gc)) / np.max(np.abs(gc))
    print("[solver step] coefficient-gradient err=%.2e" % err, flush=True)
    assert err <= 1e-3
    x1, _, _ = omotion.adam_step(np.zeros_like(gc), gc, np.zeros_like(gc), np.zeros_like(gc), 1, 0.05)
    # first Adam step is lr * sign(g): equal wherever the gradient is not tiny
    big = np.abs(gc) > 1e-3 * np.abs(gc).max()
    assert np.allclose(coeff_dev[big], x1[big], atol=1e-9)


def test_solver_reduces_loss_and_reprojection_error():
    c = case("tiny")
    bp = Backprojector.from_case(c)
    proj = torch.from_numpy(c.proj).to(bp.device)
    s = MotionSolver(bp, proj, SolverConfig(n_iter=60, n_nodes=c.cfg.n_nodes, loss="entropy_tv", lr=0.05))
    rpe0 = reprojection_error(c.P, np.zeros_like(c.theta_true), c.theta_true, c.cfg.pitch_mm)
    out = s.run(record_loss=True)
    rpe1 = reprojection_error(c.P, out["theta"], c.theta_true, c.cfg.pitch_mm)
    print("[solver tiny] rpe %.3f -> %.3f mm, loss %.5g -> %.5g, %.2f ms/iter"
          % (rpe0, rpe1, out["losses"][0], out["losses"][-1], out["ms_per_iter"]), flush=True)
    assert out["losses"][-1] < out["losses"][0]
    assert rpe1 < rpe0


@pytest.mark.parametrize("optimizer", ["adam", "gd"])
def test_checkpoint_and_resume_is_bitwise_identical(tmp_path, optimizer):
    """Six iterations straight equal three, a saved and reloaded state in a fresh solver, and
    three more: the kernels are deterministic and the state is complete."""
    c = case("tiny")
    proj_h = c.proj

    def solver():
        bp = Backprojector.from_case(c)
        return MotionSolver(bp, torch.from_numpy(proj_h).to(bp.device),
                            SolverConfig(n_nodes=c.cfg.n_nodes, loss="entropy_tv", optimizer=optimizer, lr=0.05))

    a = solver()
    a.calibrate()
    for _ in range(6):
        a.iteration()
    b = solver()
    b.calibrate()
    for _ in range(3):
        b.iteration()
    torch.save(b.state_dict(), tmp_path / "ck.pt")
    r = solver()
    r.load_state_dict(torch.load(tmp_path / "ck.pt", weights_only=True))
    for _ in range(3):
        r.iteration()
    assert r.it == 6
    assert torch.equal(a.coeffs, r.coeffs) and torch.equal(a.m, r.m) and torch.equal(a.v, r.v)
    # a checkpoint of another problem is refused
    other = MotionSolver(r.bp, r.proj, SolverConfig(n_nodes=c.cfg.n_nodes + 1))
    with pytest.raises(ValueError):
        other.load_state_dict(r.state_dict())
