"""The gradient-free baseline's GPU side: a population evaluated in one batched launch gives
exactly the losses of the candidates evaluated one at a time through the plain entry points."""
import numpy as np
import pytest
import torch

from parity import case

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd import gmc  # noqa: E402
from paper_2401_09283_amd.autograd import Backprojector  # noqa: E402
from paper_2401_09283_amd.cmaes import CMAES, PopulationEvaluator  # noqa: E402


def test_population_losses_equal_single_evaluations():
    c = case("tiny")
    bp = Backprojector.from_case(c)
    proj = torch.from_numpy(c.proj).cuda()
    nn = 10
    es = CMAES(np.zeros(6 * nn), 0.5, seed=2, popsize=5)
    X = es.ask()
    ev = PopulationEvaluator(bp, proj, nn, 5, motion="bspline", lam=1e-4)
    f = ev(X)
    ref = []
    for x in X:
        th = torch.empty((c.scan.n_views, 6), dtype=torch.float64, device="cuda")
        gmc.gmc_bspline_theta(c.scan.n_views, nn, torch.from_numpy(x.reshape(6, nn)).cuda(), th)
        vol = bp.forward(proj, th)
        g = torch.empty_like(vol)
        loss = torch.empty(5, dtype=torch.float64, device="cuda")
        cfg = ev.cfg
        gmc.gmc_loss_entropy_tv(bp.plan, vol, 1e-4, cfg.hist_lo, cfg.hist_hi, cfg.tv_eps, g, loss, bp.workspace)
        ref.append(float(loss[0]))
    assert np.array_equal(f, np.array(ref))
    es.tell(f)
    assert es.gen == 1
