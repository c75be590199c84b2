"""Gradient-based rigid motion estimation on one GPU (Sec. II-C, Fig. 2).

One iteration: spline coefficients -> per-view rigid parameters (Akima or B-spline, Sec. II-B.1) ->
composition and backprojection (Eq. 1, Eq. 3) -> volume loss and its seed -> VJP (Eq. 4-5)
-> dL/dtheta (Eq. 2) -> dL/dcoefficients (spline adjoint) -> Adam step, or the paper's
gradient descent with exponentially decaying steps (Eq. 6). Every step is a libgmc kernel
on the current stream; the host only launches (no synchronisation inside an iteration).

The quality metric of the paper is a trained network (Sec. II-B.3); the losses here are
differentiable volume-sharpness targets: soft-histogram entropy plus total variation, or the
sum of squared neighbour differences.

``python -m paper_2401_09283_amd.solver --config head256 --iters 100`` runs the synthetic
workload and prints the reprojection error before and after, and the time per iteration.
"""
from __future__ import annotations

import dataclasses
import json
import math
import time

import numpy as np
import torch

from . import gmc
from .autograd import Backprojector

DEG = math.pi / 180.0


@dataclasses.dataclass
class SolverConfig:
    n_iter: int = 100
    n_nodes: int = 20
    motion: str = "bspline"       # "bspline" | "akima" (the paper's motion model, Sec. II-B.1)
    loss: str = "entropy_tv"      # "entropy_tv" | "sumsq" | "unet" (learned metric, timing only)
    unet_channels: tuple = (8, 16, 32, 64)
    optimizer: str = "adam"       # "adam" | "gd"
    lr: float = 0.05              # Adam step (coefficient units: mm, deg)
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    gd_s0: float = 100.0          # Eq. 6 initial step
    gd_decay: float = 0.97        # Eq. 6 decay factor
    gd_first_step: float = 0.0    # > 0: s0 = gd_first_step / max|df/dx| at x = 0 (coefficient
                                  # units), for losses whose scale differs from the paper's metric
    hist_lo: float = -0.01
    hist_hi: float = 0.06
    tv_eps: float = 1e-5
    lam: float | None = None      # TV weight; None: equal seed norms at the start


class MotionSolver:
    """Owns the device state of one motion-estimation problem (projections stay resident)."""

    def __init__(self, bp: Backprojector, proj: torch.Tensor, cfg: SolverConfig | None = None):
        self.bp = bp
        self.cfg = cfg or SolverConfig()
        self.proj = proj
        dev = bp.device
        n = bp.geometry.n_views
        nn = self.cfg.n_nodes
        self.n_views = n
        self.coeffs = torch.zeros((6, nn), dtype=torch.float64, device=dev)
        self.m = torch.zeros_like(self.coeffs)
        self.v = torch.zeros_like(self.coeffs)
        self.gc = torch.zeros_like(self.coeffs)
        self.theta = torch.zeros((n, 6), dtype=torch.float64, device=dev)
        self.gtheta = torch.zeros((n, 6), dtype=torch.float64, device=dev)
        self.vol = torch.empty(bp.plan.vol_shape, dtype=torch.float32, device=dev)
        self.gvol = torch.empty_like(self.vol)
        self.loss = torch.zeros(5, dtype=torch.float64, device=dev)
        self.lam = self.cfg.lam
        self.it = 0
        self.gd_s0 = self.cfg.gd_s0
        self._unet = None
        if self.cfg.motion not in ("bspline", "akima"):
            raise ValueError("unknown motion model %r" % self.cfg.motion)

    def _theta(self):
        n, nn = self.n_views, self.cfg.n_nodes
        if self.cfg.motion == "akima":
            gmc.gmc_akima_theta(n, nn, self.coeffs, self.theta)
        else:
            gmc.gmc_bspline_theta(n, nn, self.coeffs, self.theta)

    def _coeff_grad(self):
        n, nn = self.n_views, self.cfg.n_nodes
        if self.cfg.motion == "akima":
            gmc.gmc_akima_grad(n, nn, self.coeffs, self.gtheta, self.gc)
        else:
            gmc.gmc_bspline_grad(n, nn, self.gtheta, self.gc)

    # ---------------------------------------------------------------- pieces of one iteration
    def _loss(self, lam):
        c, plan, ws = self.cfg, self.bp.plan, self.bp.workspace
        if c.loss == "entropy_tv":
            gmc.gmc_loss_entropy_tv(plan, self.vol, lam, c.hist_lo, c.hist_hi, c.tv_eps, self.gvol, self.loss, ws)
        elif c.loss == "sumsq":
            gmc.gmc_loss_sumsq_grad(plan, self.vol, self.gvol, self.loss[:1], ws)
        elif c.loss == "unet":
            if self._unet is None:
                from .unet import UNetMetric

                self._unet = UNetMetric(c.unet_channels, device=self.bp.device)
            self.loss[0] = self._unet(self.vol, self.gvol)
        else:
            raise ValueError("unknown loss %r" % c.loss)

    def calibrate(self):
        """TV weight that gives the entropy and TV seeds equal norms at the current estimate."""
        if self.cfg.loss != "entropy_tv" or self.lam is not None:
            if self.lam is None:
                self.lam = 0.0
            if self.cfg.loss != "entropy_tv" and self.cfg.optimizer == "gd" and self.cfg.gd_first_step > 0.0:
                self._normalise_gd()
            return self.lam
        plan, ws = self.bp.plan, self.bp.workspace
        self._theta()
        gmc.gmc_prepare(plan, self.bp.P, self.theta, 1, ws)
        gmc.gmc_bp_forward(plan, self.proj, self.vol, ws)
        self._loss(0.0)
        l0 = self.loss.cpu().numpy()
        self.lam = float(math.sqrt(l0[3] / max(l0[4], 1e-300)))
        if self.cfg.optimizer == "gd" and self.cfg.gd_first_step > 0.0:
            self._normalise_gd()
        return self.lam

    def _normalise_gd(self):
        """Eq. 6 with the initial step normalised by the gradient at the current estimate."""
        plan, ws = self.bp.plan, self.bp.workspace
        self._theta()
        gmc.gmc_prepare(plan, self.bp.P, self.theta, 1, ws)
        gmc.gmc_bp_forward(plan, self.proj, self.vol, ws)
        self._loss(self.lam if self.lam is not None else 0.0)
        gmc.gmc_bp_vjp(plan, self.proj, self.gvol, ws)
        gmc.gmc_bp_vjp_finish(plan, self.gtheta, None, ws)
        self._coeff_grad()
        gmax = float(self.gc.abs().max())
        self.gd_s0 = self.cfg.gd_first_step / max(gmax, 1e-300)

    def iteration(self, events=None):
        """Launch one iteration on the current stream. events: optional dict of
        torch.cuda.Event recorded around the forward ('f0','f1') and VJP ('v0','v1') kernels."""
        if self.lam is None:
            self.calibrate()
        c, plan, ws = self.cfg, self.bp.plan, self.bp.workspace
        self._theta()
        gmc.gmc_prepare(plan, self.bp.P, self.theta, 1, ws)
        if events:
            events["f0"].record()
        gmc.gmc_bp_forward(plan, self.proj, self.vol, ws)
        if events:
            events["f1"].record()
        self._loss(self.lam)
        if events:
            events["v0"].record()
        gmc.gmc_bp_vjp(plan, self.proj, self.gvol, ws)
        if events:
            events["v1"].record()
        gmc.gmc_bp_vjp_finish(plan, self.gtheta, None, ws)
        self._coeff_grad()
        self.it += 1
        if c.optimizer == "adam":
            gmc.gmc_adam_step(self.coeffs, self.gc, self.m, self.v, self.it, c.lr, c.beta1, c.beta2, c.adam_eps)
        elif c.optimizer == "gd":
            gmc.gmc_gd_step(self.coeffs, self.gc, self.it - 1, self.gd_s0, c.gd_decay)
        else:
            raise ValueError("unknown optimizer %r" % c.optimizer)

    # ---------------------------------------------------------------- checkpoint / resume
    def state_dict(self) -> dict:
        """Everything an interrupted solve needs to continue bitwise identically: the
        coefficients, Adam moments, iteration count, TV weight and Eq. 6 step (host copies;
        save with torch.save, load with torch.load(..., weights_only=True))."""
        return dict(coeffs=self.coeffs.cpu(), m=self.m.cpu(), v=self.v.cpu(), it=int(self.it),
                    lam=None if self.lam is None else float(self.lam),
                    gd_s0=None if self.gd_s0 is None else float(self.gd_s0),
                    n_nodes=int(self.cfg.n_nodes), motion=self.cfg.motion, n_views=int(self.n_views))

    def load_state_dict(self, st: dict) -> None:
        if (int(st["n_nodes"]) != self.cfg.n_nodes or st["motion"] != self.cfg.motion
                or int(st["n_views"]) != self.n_views):
            raise ValueError("checkpoint of another problem (nodes, motion model or views differ)")
        for name in ("coeffs", "m", "v"):
            src = st[name]
            if tuple(src.shape) != tuple(self.coeffs.shape):
                raise ValueError("checkpoint tensor %s has shape %s" % (name, tuple(src.shape)))
            getattr(self, name).copy_(src.to(device=self.coeffs.device, dtype=torch.float64))
        self.it = int(st["it"])
        self.lam = st["lam"]
        self.gd_s0 = st["gd_s0"]

    def run(self, n_iter=None, record_loss=False):
        """n_iter iterations; the loss of every iteration is kept on the device and read once."""
        n_iter = self.cfg.n_iter if n_iter is None else n_iter
        hist = torch.zeros(max(n_iter, 1), dtype=torch.float64, device=self.bp.device)
        self.calibrate()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_iter):
            self.iteration()
            if record_loss:
                hist[i].copy_(self.loss[0], non_blocking=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        self._theta()
        return dict(theta=self.theta.cpu().numpy(), coeffs=self.coeffs.cpu().numpy(),
                    losses=hist[:n_iter].cpu().tolist() if record_loss else [],
                    ms_per_iter=dt * 1e3 / max(n_iter, 1))


# ------------------------------------------------------------------------- evaluation (host)

def _rigid(theta6):
    tx, ty, tz, rx, ry, rz = theta6
    cx, sx, cy, sy, cz, sz = math.cos(rx), math.sin(rx), math.cos(ry), math.sin(ry), math.cos(rz), math.sin(rz)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    T = np.eye(4)
    T[:3, :3] = Rz @ Ry @ Rx
    T[:3, 3] = (tx, ty, tz)
    return T


def reprojection_error(P, theta_est, theta_true, pitch_mm, radii=(25.0, 50.0, 100.0), n_per_radius=100, seed=7):
    """Mean detector distance (mm) between points projected with the estimated and the true
    geometry (Sec. IV). Points are uniform on spheres of the given radii about the isocentre.
    Both parameter sets are zero-centred over the views first: a global rigid motion does not
    change the reconstruction's sharpness and cannot be recovered by an autofocus target."""
    rng = np.random.default_rng(seed)
    pts = []
    for r in radii:
        d = rng.standard_normal((n_per_radius, 3))
        pts.append(r * d / np.linalg.norm(d, axis=1, keepdims=True))
    pts = np.concatenate(pts)
    ph = np.concatenate([pts, np.ones((len(pts), 1))], 1)
    te = np.asarray(theta_est, dtype=np.float64)
    tt = np.asarray(theta_true, dtype=np.float64)
    te = te - te.mean(axis=0)
    tt = tt - tt.mean(axis=0)
    err = 0.0
    for j in range(len(P)):
        a = ph @ (P[j] @ _rigid(te[j])).T
        b = ph @ (P[j] @ _rigid(tt[j])).T
        da = a[:, :2] / a[:, 2:3] - b[:, :2] / b[:, 2:3]
        err += np.mean(np.sqrt(np.sum(da * da, axis=1)))
    return err / len(P) * pitch_mm


def main(argv=None):
    import argparse

    from synth import CONFIGS, make_case

    ap = argparse.ArgumentParser(description="motion estimation on a synthetic scan")
    ap.add_argument("--config", default="head256")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--loss", default="entropy_tv")
    ap.add_argument("--optimizer", default=None, help="adam | gd (default: gd for Akima cases, else adam)")
    ap.add_argument("--motion", default=None, help="bspline | akima (default: the case's motion model)")
    ap.add_argument("--nodes", type=int, default=0, help="nodes of the estimated spline (default: the case's)")
    ap.add_argument("--gd-s0", type=float, default=100.0)
    ap.add_argument("--gd-decay", type=float, default=0.97)
    ap.add_argument("--gd-first-step", type=float, default=None,
                    help="normalise s0 so that the first step moves the largest coefficient this far")
    ap.add_argument("--unet-channels", default="8,16,32,64", help="feature maps per level of the U-Net metric")
    args = ap.parse_args(argv)
    cfg = CONFIGS[args.config]
    motion = args.motion or cfg.motion_model
    optimizer = args.optimizer or ("gd" if motion == "akima" else "adam")
    first = args.gd_first_step if args.gd_first_step is not None else (0.5 if optimizer == "gd" else 0.0)
    case = make_case(args.config)
    bp = Backprojector.from_case(case)
    proj = torch.from_numpy(case.proj).to(bp.device)
    solver = MotionSolver(bp, proj, SolverConfig(n_iter=args.iters, n_nodes=args.nodes or cfg.estimate_nodes, lr=args.lr,
                                                 loss=args.loss, optimizer=optimizer, motion=motion, gd_s0=args.gd_s0,
                                                 gd_decay=args.gd_decay, gd_first_step=first,
                                                 unet_channels=tuple(int(x) for x in args.unet_channels.split(","))))
    rpe0 = reprojection_error(case.P, np.zeros_like(case.theta_true), case.theta_true, cfg.pitch_mm)
    out = solver.run(record_loss=True)
    rpe1 = reprojection_error(case.P, out["theta"], case.theta_true, cfg.pitch_mm)
    bp.check()
    print(json.dumps(dict(config=args.config, iters=args.iters, loss=args.loss, optimizer=optimizer, motion=motion,
                          nodes=solver.cfg.n_nodes, gd_s0=solver.gd_s0 if optimizer == "gd" else None,
                          lam=solver.lam, rpe_initial_mm=rpe0, rpe_final_mm=rpe1,
                          ms_per_iter=out["ms_per_iter"], loss_first=out["losses"][0], loss_last=out["losses"][-1])))


if __name__ == "__main__":
    main()
