"""Continuous-batching service for motion-estimation requests (one GPU).

Requests arrive over time (e.g. a Poisson stream). The server admits a waiting request as
soon as an active slot is free and its HBM footprint (projections, volumes, optimiser state,
workspace) fits the budget, keeps everything of an admitted request resident on the device,
and advances the active requests with scheduler ticks; a tick enqueues one solver iteration
(spline -> compose -> backprojection -> loss -> VJP -> chain -> Adam) for each request the
policy picks. A request that finishes its iterations retires and frees its memory; the next
tick admits new arrivals. Each request's arithmetic is the same as when it runs alone, so
its result is bitwise identical to a plain solve.

Two executors:
* streams (default): every admitted request has its own HIP stream and its iterations are
  enqueued there, at most ``depth`` iterations ahead of the device, with no device-wide
  synchronisation: the host only polls events. Requests on different streams overlap on
  the GPU, so the phases of one request that leave the GPU partly idle (loss, set-up,
  reduction, optimiser, launch gaps) run beside the backprojection of another.
* batched: every tick is one backprojection launch and one VJP launch over the voxel bricks of
  all ticked requests (gmc_launch_batch), in lockstep, with a device synchronisation per tick.

Which active requests a tick advances is the policy: ``"all"`` advances every active request
(processor sharing), ``"srpt"`` (the default) advances the requests with the least remaining
work first (remaining iterations times the voxel-view updates of one iteration), adding
requests to the tick until its work reaches ``tick_work`` updates (at least one request, and
at least ``min_batch`` while that many are active): small requests finish early, a large
request runs with at most a few others. With ``max_wait`` set, requests that arrived more
than ``max_wait`` seconds ago go first, oldest first, which bounds how long a large request
can be overtaken. Results do not depend on the policy or the executor.

The scheduler is independent of the GPU: ``Server`` drives an executor with four calls
(footprint, admit, step, release), an optional fifth (work: updates per iteration) and, for
asynchronous executors (``depth`` > 0), three more (in_flight, finished, wait), so its
admission, policy and retirement logic is tested on the CPU with fake executors and a fake
clock.

``python -m paper_2401_09283_amd.serve`` runs the synthetic serving workload (Poisson
arrivals drawn from 128^3 x 248, 256^3 x 496 and 384^3 x 496 views, 30 iterations each)
served and as sequential plain solves, and prints latency percentiles and throughput of both.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import math
import sys
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                    # seconds after the start of the run
    n_iter: int
    inputs: Callable[[], dict] | dict  # dict(geometry=..., proj=np f32, P=np f64, n_nodes=...) or a factory
    # filled by the server
    t_admit: float | None = None
    t_done: float | None = None
    status: str = "waiting"           # waiting | active | done | failed
    error: str | None = None
    result: dict | None = None
    iters_done: int = 0
    state: object = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class Server:
    """Continuous batching over an executor (see module docstring)."""

    def __init__(self, executor, hbm_budget_bytes: int, max_active: int = 16, clock=None, sleep=None,
                 policy: str = "srpt", tick_work: float = 8e9, max_wait: float | None = None, min_batch: int = 1):
        if policy not in ("all", "srpt"):
            raise ValueError("policy must be 'all' or 'srpt'")
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.max_active = int(max_active)
        self.policy = policy
        self.tick_work = float(tick_work)
        self.max_wait = None if max_wait is None else float(max_wait)
        self.min_batch = max(1, int(min_batch))
        # asynchronous executors enqueue work and report completion through in_flight/finished/wait
        self.depth = int(getattr(executor, "depth", 0) or 0)
        self._now = lambda: 0.0
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.used = 0
        self.ticks = 0
        self.batch_sizes = []
        self._cancelled = set()

    def cancel(self, rid: int) -> None:
        """Cancel request rid (callable from another thread or from the executor): it leaves the
        queue or its slot at the next tick, its memory is released, status 'cancelled'."""
        self._cancelled.add(rid)

    def _apply_cancellations(self, pending, waiting, active, t):
        if not self._cancelled:
            return pending, waiting, active
        hit = set(self._cancelled)

        def drop(lst, release):
            keep = []
            for r in lst:
                if r.rid in hit:
                    r.status, r.error, r.t_done = "cancelled", "cancelled", t
                    if release:
                        self._release(r)
                else:
                    keep.append(r)
            return keep

        return drop(pending, False), drop(waiting, False), drop(active, True)

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = list(reqs)
        waiting, active = [], []
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        self._now = now
        while pending or waiting or active:
            t = now()
            pending, waiting, active = self._apply_cancellations(pending, waiting, active, t)
            while pending and pending[0].arrival <= t:
                waiting.append(pending.pop(0))
            # FIFO admission by slots and HBM footprint
            while waiting and len(active) < self.max_active:
                r = waiting[0]
                need = self.ex.footprint(r)
                if need > self.budget:
                    waiting.pop(0)
                    r.status, r.error, r.t_done = "failed", "footprint %d exceeds the budget" % need, now()
                    continue
                if self.used + need > self.budget:
                    break
                waiting.pop(0)
                try:
                    self.ex.admit(r)
                except Exception as e:  # a request that cannot be set up fails alone
                    r.status, r.error, r.t_done = "failed", "admit: %s" % e, now()
                    continue
                self.used += need
                r.t_admit = now()
                r.status = "active"
                active.append(r)
            if self.depth:
                active = self._retire_finished(active, now)
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            # the policy chooses among the requests with iterations left; of those, a tick enqueues
            # the ones with fewer than `depth` iterations in flight (asynchronous executors), and
            # waits for the device when none can take more
            chosen = self._pick([r for r in active if r.iters_done < r.n_iter])
            batch = [r for r in chosen if not self.depth or self.ex.in_flight(r) < self.depth]
            if not batch:
                self.ex.wait([r for r in (chosen or active) if r.iters_done > 0])
                continue
            try:
                self.ex.step(batch)
            except Exception as e:
                # a failed tick fails its requests and frees their slots; others go on
                for r in batch:
                    r.status, r.error, r.t_done = "failed", "step: %s" % e, now()
                    self._release(r)
                active = [r for r in active if r.status == "active"]
                continue
            self.ticks += 1
            self.batch_sizes.append(len(batch))
            for r in batch:
                r.iters_done += 1
            if not self.depth:
                t = now()
                for r in batch:
                    if r.iters_done >= r.n_iter:
                        self._retire(r, t)
                active = [r for r in active if r.status == "active"]
        return reqs

    def _retire(self, r, t):
        r.result = self.ex.result(r)
        r.status, r.t_done = "done", t
        self._release(r)

    def _retire_finished(self, active, now):
        for r in active:
            if r.iters_done >= r.n_iter and self.ex.finished(r):
                self._retire(r, now())
        return [r for r in active if r.status == "active"]

    def _work(self, r):
        f = getattr(self.ex, "work", None)
        return float(f(r)) if f is not None else 1.0

    def _pick(self, active):
        """The requests this tick advances (in admission order)."""
        if self.policy == "all":
            return list(active)
        t = self._now()

        def key(r):
            if self.max_wait is not None and t - r.arrival > self.max_wait:
                return (0, r.arrival, r.rid)
            return (1, (r.n_iter - r.iters_done) * self._work(r), r.rid)

        order = sorted(active, key=key)
        chosen, total = [], 0.0
        for r in order:
            if len(chosen) >= self.min_batch and total + self._work(r) > self.tick_work:
                break
            chosen.append(r)
            total += self._work(r)
        keep = {id(r) for r in chosen}
        return [r for r in active if id(r) in keep]

    def _release(self, r):
        try:
            self.used -= self.ex.footprint(r)
            self.ex.release(r)
        except Exception:
            pass


def summarize(reqs, t_end=None):
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(0)
    span = (max(r.t_done for r in done) - min(r.arrival for r in reqs)) if done else float("nan")
    return dict(requests=len(reqs), done=len(done), failed=sum(r.status == "failed" for r in reqs),
                p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
                p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
                mean_s=float(lat.mean()) if len(lat) else None,
                throughput_req_per_s=len(done) / span if done else None, makespan_s=span)


# ---------------------------------------------------------------------------------- GPU side

class GpuExecutor:
    """Device state of each admitted request and the per-tick work.

    mode "streams" (asynchronous, ``depth`` > 0): every request owns a HIP stream (default
    priority); a tick enqueues one iteration per ticked request on its stream and records an
    event, and the server polls the events. mode "batched": a tick is one backprojection launch
    and one VJP launch over all ticked requests, then a device synchronisation."""

    def __init__(self, device="cuda", lr=0.05, loss="entropy_tv", mode="streams", depth=2, poll_s=50e-6):
        import torch

        if mode not in ("streams", "batched"):
            raise ValueError("mode must be 'streams' or 'batched'")
        self.torch = torch
        self.device = torch.device(device)
        self.lr = lr
        self.loss = loss
        self.mode = mode
        self.depth = int(depth) if mode == "streams" else 0
        self.poll_s = float(poll_s)

    def _inputs(self, r):
        if callable(r.inputs):
            r.inputs = r.inputs()
        return r.inputs

    def footprint(self, r):
        """Bytes of HBM an admitted request holds: projections, volume and seed, workspace,
        and 1 MiB for parameters and optimiser state."""
        inp = self._inputs(r)
        if "footprint" not in inp:
            from . import gmc

            g = inp["geometry"]
            plan = gmc.Plan(g)   # the workspace size does not depend on the matrices
            nvox = g.nx * g.ny * g.nz
            inp["footprint"] = int(inp["proj"].nbytes + 2 * 4 * nvox + plan.workspace_bytes + (1 << 20))
            plan.close()
        return inp["footprint"]

    def work(self, r):
        """Voxel-view updates of one iteration (the scheduler's unit of work)."""
        g = self._inputs(r)["geometry"]
        return float(g.nx) * g.ny * g.nz * g.n_views

    def admit(self, r):
        from .autograd import Backprojector
        from .solver import MotionSolver, SolverConfig

        inp = self._inputs(r)
        g = inp["geometry"]
        torch = self.torch
        bp = Backprojector(g.n_views, g.det_w, g.det_h, (g.nx, g.ny, g.nz), tuple(g.voxel_mm), tuple(g.origin_mm),
                           inp["P"], weighting=g.weighting, grad_mode=g.grad_mode, device=self.device)
        proj = torch.from_numpy(inp["proj"]).to(self.device)
        s = MotionSolver(bp, proj, SolverConfig(n_iter=r.n_iter, n_nodes=inp["n_nodes"], lr=self.lr, loss=self.loss))
        if self.depth:
            r.stream = torch.cuda.Stream(device=self.device)
            r.stream.wait_stream(torch.cuda.current_stream(self.device))   # inputs were copied there
            r.events = collections.deque()
            with torch.cuda.stream(r.stream):
                s.calibrate()
        else:
            s.calibrate()
        r.state = s

    def step(self, reqs):
        if self.depth:
            torch = self.torch
            for r in reqs:
                with torch.cuda.stream(r.stream):
                    r.state.iteration()
                    ev = torch.cuda.Event()
                    ev.record(r.stream)
                    r.events.append(ev)
            return
        from . import gmc

        fwd, vjp = [], []
        for r in reqs:
            s = r.state
            s._theta()
            gmc.gmc_prepare(s.bp.plan, s.bp.P, s.theta, 1, s.bp.workspace)
            fwd.append(dict(plan=s.bp.plan, proj=s.proj, vol=s.vol, workspace=s.bp.workspace, phase=0,
                            flags=gmc.WORK_PREPARED))
        gmc.gmc_launch_batch(fwd)
        for r in reqs:
            r.state._loss(r.state.lam)
        for r in reqs:
            s = r.state
            vjp.append(dict(plan=s.bp.plan, proj=s.proj, grad_vol=s.gvol, grad_theta=s.gtheta,
                            workspace=s.bp.workspace, phase=1, flags=gmc.WORK_PREPARED))
        gmc.gmc_launch_batch(vjp)
        for r in reqs:
            s = r.state
            s._coeff_grad()
            s.it += 1
            gmc.gmc_adam_step(s.coeffs, s.gc, s.m, s.v, s.it, s.cfg.lr, s.cfg.beta1, s.cfg.beta2, s.cfg.adam_eps)
        self.torch.cuda.synchronize()

    # asynchronous mode: completion of enqueued iterations
    def in_flight(self, r):
        ev = r.events
        while ev and ev[0].query():
            ev.popleft()
        return len(ev)

    def finished(self, r):
        return self.in_flight(r) == 0

    def wait(self, reqs):
        """Return once some enqueued iteration of reqs has completed (polling, host idle)."""
        import time as _time

        counts = [self.in_flight(r) for r in reqs]
        if not any(counts):
            return
        while True:
            for r, n in zip(reqs, counts):
                if self.in_flight(r) < n:
                    return
            _time.sleep(self.poll_s)

    def result(self, r):
        s = r.state
        if self.depth:
            r.stream.synchronize()
            with self.torch.cuda.stream(r.stream):
                s._theta()
                out = dict(coeffs=s.coeffs.cpu().numpy(), theta=s.theta.cpu().numpy())
            return out
        s._theta()
        return dict(coeffs=s.coeffs.cpu().numpy(), theta=s.theta.cpu().numpy())

    def release(self, r):
        # the request's stream must be idle before its memory can be reused on another stream
        if getattr(r, "stream", None) is not None:
            r.stream.synchronize()
        r.state = None
        r.stream = None
        r.events = None


def run_sequential(requests, device="cuda", lr=0.05, loss="entropy_tv", clock=None, sleep=None):
    """Plain solves one after another in arrival order (single-request launches)."""
    import torch

    ex = GpuExecutor(device, lr, loss, mode="batched")   # synchronous: admit and result on the current stream
    clock = clock or time.perf_counter
    sleep = sleep or time.sleep
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    t0 = clock()
    for r in reqs:
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        ex.admit(r)
        r.t_admit = clock() - t0
        s = r.state
        for _ in range(r.n_iter):
            s.iteration()
        torch.cuda.synchronize()
        r.result = ex.result(r)
        r.t_done = clock() - t0
        r.status = "done"
        ex.release(r)
    return reqs


# ---------------------------------------------------------------------------------- workload

SERVE_SIZES = ("serve128", "serve256", "serve384")


def poisson_requests(n, lam, seed, n_iter, sizes=SERVE_SIZES, size_seed=None):
    """Arrival times of a Poisson stream (rate lam per second) and uniformly drawn sizes."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / lam, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    pick = rng.integers(0, len(sizes), n)
    return [(int(i), float(arrivals[i]), sizes[int(pick[i])], n_iter) for i in range(n)]


def make_request_inputs(size, i):
    """Inputs of request i: its own phantom (seed 1000 + i) and motion (seed 2000 + i)."""
    from synth import CONFIGS, make_case

    from . import gmc

    cfg = CONFIGS[size]
    c = make_case(cfg, phantom_seed=1000 + i, motion_seed=2000 + i)
    g = gmc.make_geometry(cfg.n_views, cfg.det_w, cfg.det_h, c.grid.shape, c.grid.voxel_mm, c.grid.origin_mm)
    return dict(geometry=g, proj=c.proj, P=c.P, n_nodes=cfg.n_nodes, theta_true=c.theta_true, size=size)


def main(argv=None):
    import argparse
    import concurrent.futures as cf

    import torch

    from .solver import reprojection_error

    ap = argparse.ArgumentParser(description="continuous-batching motion-estimation service")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=2.0)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--seed", type=int, default=40)
    ap.add_argument("--max-active", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--skip-sequential", action="store_true")
    ap.add_argument("--mode", choices=("streams", "batched", "both"), default="streams",
                    help="executor: requests on their own streams, or lockstep batched launches")
    ap.add_argument("--policy", choices=("all", "srpt", "both"), default="srpt",
                    help="which active requests a tick advances (both: run the two policies)")
    ap.add_argument("--tick-work", type=float, default=8e9, help="srpt: voxel-view updates per tick")
    ap.add_argument("--min-batch", type=int, default=2, help="srpt: requests per tick while that many are active")
    ap.add_argument("--depth", type=int, default=2, help="streams: iterations a request may have in flight")
    ap.add_argument("--max-wait", type=float, default=10.0,
                    help="srpt: requests older than this many seconds go first (<= 0: never)")
    ap.add_argument("--out", default=None, help="also write the JSON summary to this file")
    args = ap.parse_args(argv)

    spec = poisson_requests(args.requests, args.rate, args.seed, args.iters)
    t = time.perf_counter()
    inputs = [None] * len(spec)
    with cf.ThreadPoolExecutor(4) as pool:
        futs = {pool.submit(make_request_inputs, s[2], s[0]): s[0] for s in spec}
        for n, f in enumerate(cf.as_completed(futs)):
            inputs[futs[f]] = f.result()
            if (n + 1) % 8 == 0:
                print("serve: generated %d/%d requests (%.0f s)" % (n + 1, len(spec), time.perf_counter() - t),
                      flush=True)

    def fresh():
        return [Request(rid, arr, it, dict(inputs[rid])) for rid, arr, size, it in spec]

    # warm the kernels once
    warm = GpuExecutor(mode="batched")
    w = Request(-1, 0.0, 1, dict(inputs[0]))
    warm.admit(w)
    warm.step([w])
    warm.release(w)
    torch.cuda.synchronize()

    out = dict(requests=args.requests, rate_per_s=args.rate, iters=args.iters, seed=args.seed,
               sizes={s: sum(1 for x in spec if x[2] == s) for s in SERVE_SIZES})
    policies = ("all", "srpt") if args.policy == "both" else (args.policy,)
    modes = ("streams", "batched") if args.mode == "both" else (args.mode,)
    runs = {}
    for mode in modes:
        for pol in policies:
            ex = GpuExecutor(mode=mode, depth=args.depth)
            srv = Server(ex, int(args.budget_gb * 1e9), args.max_active, policy=pol, tick_work=args.tick_work,
                         max_wait=args.max_wait if args.max_wait > 0 else None, min_batch=args.min_batch)
            reqs = srv.run(fresh())
            key = "served_%s_%s" % (mode, pol)
            out[key] = summarize(reqs)
            out[key].update(mode=mode, policy=pol, mean_batch=float(np.mean(srv.batch_sizes)) if srv.batch_sizes else 0.0)
            if pol == "srpt":
                out[key].update(max_wait_s=args.max_wait if args.max_wait > 0 else None, min_batch=args.min_batch,
                                tick_work=args.tick_work)
            if mode == "streams":
                out[key]["depth"] = args.depth
            out[key]["rpe_final_mm_mean"] = float(np.mean([
                reprojection_error(inputs[r.rid]["P"], r.result["theta"], inputs[r.rid]["theta_true"],
                                   _pitch(inputs[r.rid]["size"])) for r in reqs if r.status == "done"]))
            runs[key] = reqs
            print("serve: %s %s" % (key, json.dumps(out[key])), flush=True)
    if not args.skip_sequential:
        print("serve: sequential plain solves", flush=True)
        seq = run_sequential(fresh())
        out["sequential"] = summarize(seq)
        out["sequential"]["rpe_final_mm_mean"] = float(np.mean([
            reprojection_error(inputs[r.rid]["P"], r.result["theta"], inputs[r.rid]["theta_true"],
                               _pitch(inputs[r.rid]["size"])) for r in seq]))
        # offered load: arrival rate times the mean GPU time of one plain solve (> 1: the queue
        # grows for as long as requests keep arriving, and latency is mostly waiting)
        service = float(np.mean([r.t_done - r.t_admit for r in seq]))
        out["sequential"]["mean_service_s"] = service
        out["offered_load_rho"] = args.rate * service
        same = all(np.array_equal(a.result["coeffs"], b.result["coeffs"])
                   for reqs in runs.values()
                   for a, b in zip(sorted(reqs, key=lambda r: r.rid), sorted(seq, key=lambda r: r.rid))
                   if a.status == "done")
        out["identical_results"] = bool(same)
    out["rpe_initial_mm_mean"] = float(np.mean([
        reprojection_error(inputs[i]["P"], np.zeros_like(inputs[i]["theta_true"]), inputs[i]["theta_true"],
                           _pitch(inputs[i]["size"])) for i in range(len(spec))]))
    out["command"] = "python -m paper_2401_09283_amd.serve " + " ".join(argv if argv is not None else sys.argv[1:])
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)


def _pitch(size):
    from synth import CONFIGS

    return CONFIGS[size].pitch_mm


if __name__ == "__main__":
    main()
