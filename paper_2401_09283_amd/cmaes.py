"""The gradient-free baseline of Sec. IV: CMA-ES over the spline node values.

The paper compares its gradient descent with CMA-ES (covariance matrix adaptation evolution
strategy) on the same target and reports the gradient-based estimate to be about 19 times
faster. Here CMA-ES follows Hansen's published description of the (mu/mu_w, lambda)-CMA-ES
with its default strategy parameters (weighted recombination, cumulative step-size
adaptation, rank-one and rank-mu covariance updates); the strategy itself is a few small
matrix operations per generation on the host. Each generation's population is evaluated on
the GPU with the forward only (Eq. 3) and the volume loss: one batched backprojection launch
for the whole population (gmc_launch_batch), one loss per candidate, one transfer of the
population's losses to the host.

``python -m paper_2401_09283_amd.cmaes --config paper128 --evals 10000`` runs CMA-ES and the
gradient-based solver on the same case and prints both times, losses and reprojection errors.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np


class CMAES:
    """(mu/mu_w, lambda)-CMA-ES minimising f over R^n from mean x0 and step size sigma0."""

    def __init__(self, x0, sigma0, seed=0, popsize=None):
        x0 = np.asarray(x0, dtype=np.float64).ravel()
        n = x0.size
        self.n = n
        self.lam = int(popsize or 4 + int(3 * math.log(n)))
        self.mu = self.lam // 2
        w = math.log(self.mu + 0.5) - np.log(np.arange(1, self.mu + 1))
        self.w = w / w.sum()
        self.mueff = 1.0 / float(np.sum(self.w ** 2))
        self.cs = (self.mueff + 2.0) / (n + self.mueff + 5.0)
        self.ds = 1.0 + 2.0 * max(0.0, math.sqrt((self.mueff - 1.0) / (n + 1.0)) - 1.0) + self.cs
        self.cc = (4.0 + self.mueff / n) / (n + 4.0 + 2.0 * self.mueff / n)
        self.c1 = 2.0 / ((n + 1.3) ** 2 + self.mueff)
        self.cmu = min(1.0 - self.c1, 2.0 * (self.mueff - 2.0 + 1.0 / self.mueff) / ((n + 2.0) ** 2 + self.mueff))
        self.chin = math.sqrt(n) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n))
        self.m = x0.copy()
        self.sigma = float(sigma0)
        self.pc = np.zeros(n)
        self.ps = np.zeros(n)
        self.C = np.eye(n)
        self.B = np.eye(n)
        self.D = np.ones(n)
        self.rng = np.random.default_rng(seed)
        self.gen = 0
        self.evals = 0
        self._since_eig = 0
        self._y = None

    def ask(self):
        """lambda candidates [lambda][n]: m + sigma B D z, z ~ N(0, I)."""
        z = self.rng.standard_normal((self.lam, self.n))
        self._y = (z * self.D[None, :]) @ self.B.T
        return self.m[None, :] + self.sigma * self._y

    def tell(self, f):
        """Update the distribution from the candidates' values f [lambda] (the last ask)."""
        f = np.asarray(f, dtype=np.float64)
        order = np.argsort(f, kind="stable")
        ysel = self._y[order[:self.mu]]
        yw = self.w @ ysel
        self.m = self.m + self.sigma * yw
        # conjugate evolution path: C^(-1/2) yw = B D^-1 B^T yw
        self.ps = (1.0 - self.cs) * self.ps + math.sqrt(self.cs * (2.0 - self.cs) * self.mueff) * (
            self.B @ ((self.B.T @ yw) / self.D))
        norm_ps = float(np.linalg.norm(self.ps))
        hsig = norm_ps / math.sqrt(1.0 - (1.0 - self.cs) ** (2 * (self.gen + 1))) / self.chin < 1.4 + 2.0 / (self.n + 1)
        self.pc = (1.0 - self.cc) * self.pc + (math.sqrt(self.cc * (2.0 - self.cc) * self.mueff) * yw if hsig else 0.0)
        dh = 0.0 if hsig else self.cc * (2.0 - self.cc)
        rank_mu = (ysel * self.w[:, None]).T @ ysel
        self.C = ((1.0 - self.c1 - self.cmu) * self.C + self.c1 * (np.outer(self.pc, self.pc) + dh * self.C)
                  + self.cmu * rank_mu)
        self.sigma *= math.exp((self.cs / self.ds) * (norm_ps / self.chin - 1.0))
        self.gen += 1
        self.evals += self.lam
        self._since_eig += self.lam
        # eigendecomposition of C only every n / (10 (c1 + cmu)) evaluations (O(n^2) per sample)
        if self._since_eig > self.lam / (self.c1 + self.cmu) / self.n / 10.0:
            self._since_eig = 0
            self.C = np.triu(self.C) + np.triu(self.C, 1).T
            d2, self.B = np.linalg.eigh(self.C)
            self.D = np.sqrt(np.maximum(d2, 1e-300))
        return order[0]


class PopulationEvaluator:
    """Loss of a whole population of spline node sets on the GPU: Akima or B-spline theta per
    candidate, composition and set-up per candidate, ONE batched forward launch for the
    population, one loss per candidate, one device-to-host copy of the losses."""

    def __init__(self, bp, proj, n_nodes, popsize, motion="akima", lam=None, loss_cfg=None):
        import torch

        from . import gmc
        from .solver import SolverConfig

        self.torch, self.gmc = torch, gmc
        self.bp, self.proj = bp, proj
        self.n_nodes, self.motion = n_nodes, motion
        self.cfg = loss_cfg or SolverConfig()
        dev = bp.device
        n = bp.geometry.n_views
        self.n_views = n
        self.pop = popsize
        self.coeffs = torch.zeros((popsize, 6, n_nodes), dtype=torch.float64, device=dev)
        self.theta = torch.zeros((popsize, n, 6), dtype=torch.float64, device=dev)
        self.vol = torch.empty((popsize,) + tuple(bp.plan.vol_shape), dtype=torch.float32, device=dev)
        self.gvol = torch.empty((popsize,) + tuple(bp.plan.vol_shape), dtype=torch.float32, device=dev)
        self.ws = [bp.plan.new_workspace(dev) for _ in range(popsize)]
        self.loss = torch.zeros((popsize, 5), dtype=torch.float64, device=dev)
        self.lam = lam

    def __call__(self, X):
        torch, gmc = self.torch, self.gmc
        X = np.asarray(X, dtype=np.float64).reshape(-1, 6, self.n_nodes)
        k = X.shape[0]
        self.coeffs[:k].copy_(torch.from_numpy(X))
        items = []
        for i in range(k):
            if self.motion == "akima":
                gmc.gmc_akima_theta(self.n_views, self.n_nodes, self.coeffs[i], self.theta[i])
            else:
                gmc.gmc_bspline_theta(self.n_views, self.n_nodes, self.coeffs[i], self.theta[i])
            gmc.gmc_prepare(self.bp.plan, self.bp.P, self.theta[i], 0, self.ws[i])
            items.append(dict(plan=self.bp.plan, proj=self.proj, vol=self.vol[i], workspace=self.ws[i], phase=0,
                              flags=gmc.WORK_PREPARED))
        gmc.gmc_launch_batch(items)
        c = self.cfg
        for i in range(k):
            gmc.gmc_loss_entropy_tv(self.bp.plan, self.vol[i], self.lam, c.hist_lo, c.hist_hi, c.tv_eps, self.gvol[i],
                                    self.loss[i], self.ws[i])
        return self.loss[:k, 0].cpu().numpy()


def main(argv=None):
    import argparse

    import torch

    from synth import CONFIGS, make_case

    from .autograd import Backprojector
    from .solver import MotionSolver, SolverConfig, reprojection_error

    ap = argparse.ArgumentParser(description="CMA-ES against gradient descent on one synthetic case")
    ap.add_argument("--config", default="paper128")
    ap.add_argument("--evals", type=int, default=10000)
    ap.add_argument("--sigma0", type=float, default=0.5, help="initial step (mm and deg)")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--gd-iters", type=int, default=100)
    args = ap.parse_args(argv)

    cfg = CONFIGS[args.config]
    case = make_case(args.config)
    motion = cfg.motion_model
    nn = cfg.estimate_nodes
    bp = Backprojector.from_case(case)
    proj = torch.from_numpy(case.proj).to(bp.device)

    # the gradient-based reference: Eq. 6 steps as in the paper (s0 normalised by the first gradient)
    gd = MotionSolver(bp, proj, SolverConfig(n_iter=args.gd_iters, n_nodes=nn, motion=motion, optimizer="gd",
                                             gd_first_step=0.5))
    gd.calibrate()
    out_gd = gd.run(record_loss=True)
    gd_loss = out_gd["losses"][-1]
    gd_time = out_gd["ms_per_iter"] * args.gd_iters / 1e3
    rpe0 = reprojection_error(case.P, np.zeros_like(case.theta_true), case.theta_true, cfg.pitch_mm)
    gd_rpe = reprojection_error(case.P, out_gd["theta"], case.theta_true, cfg.pitch_mm)
    print("cmaes: gradient descent %d iterations in %.2f s, loss %.6f, RPE %.3f -> %.3f mm"
          % (args.gd_iters, gd_time, gd_loss, rpe0, gd_rpe), flush=True)

    es = CMAES(np.zeros(6 * nn), args.sigma0, seed=args.seed)
    ev = PopulationEvaluator(bp, proj, nn, es.lam, motion=motion, lam=gd.lam)
    ev(es.ask())   # warm-up of the batched path (not counted)
    es = CMAES(np.zeros(6 * nn), args.sigma0, seed=args.seed)
    best_f, best_x = math.inf, np.zeros(6 * nn)
    reach_t = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last_print = t0
    while es.evals + es.lam <= args.evals:
        X = es.ask()
        f = ev(X)
        i = es.tell(f)
        if f[i] < best_f:
            best_f, best_x = float(f[i]), X[i].copy()
        if reach_t is None and best_f <= gd_loss:
            reach_t = time.perf_counter() - t0
        if time.perf_counter() - last_print > 20.0:
            last_print = time.perf_counter()
            print("cmaes: %d evaluations, best loss %.6f, sigma %.4f" % (es.evals, best_f, es.sigma), flush=True)
    t_es = time.perf_counter() - t0
    # reprojection error of the best candidate
    th = torch.zeros((bp.geometry.n_views, 6), dtype=torch.float64, device=bp.device)
    c = torch.from_numpy(best_x.reshape(6, nn)).to(bp.device)
    from . import gmc
    if motion == "akima":
        gmc.gmc_akima_theta(bp.geometry.n_views, nn, c, th)
    else:
        gmc.gmc_bspline_theta(bp.geometry.n_views, nn, c, th)
    es_rpe = reprojection_error(case.P, th.cpu().numpy(), case.theta_true, cfg.pitch_mm)
    res = dict(config=args.config, motion=motion, nodes=nn, dims=6 * nn, popsize=es.lam, evaluations=es.evals,
               generations=es.gen, cmaes_s=t_es, cmaes_ms_per_eval=t_es * 1e3 / max(es.evals, 1),
               cmaes_best_loss=best_f, cmaes_rpe_mm=es_rpe, gd_iters=args.gd_iters, gd_s=gd_time, gd_loss=gd_loss,
               gd_rpe_mm=gd_rpe, rpe_initial_mm=rpe0, time_ratio=t_es / gd_time,
               cmaes_s_to_reach_gd_loss=reach_t)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
