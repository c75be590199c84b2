#!/usr/bin/env python3
"""Throughput of the motion-compensation hot path on one MI355X.

A step is one iteration of gradient-based motion estimation over a 256^3 volume
(1 mm voxels) reconstructed from 496 views (200-degree short scan, 620x480
detector at 0.616 mm, 785/1200 mm): cubic B-spline motion model -> Eq. 1
composition and brick set-up -> FDK backprojection (Eq. 3) -> entropy + TV
loss and its seed -> Jacobian-vector product (Eq. 4-5) -> reduction and chain
to the rigid parameters (Eq. 2) -> B-spline adjoint -> Adam step. Inputs are
seeded synthetic data (head-like ellipsoid phantom, analytic projections,
FDK pre-filter), resident in HBM before timing starts.

Prints one JSON line. ``value`` is voxel-view updates per second of the whole
step (GUPS = K * N_p / t_step / 1e9). The roofline object is for the dominant
kernel (the VJP), timed with HIP events on the stream it runs on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GUPS (voxel·view/s) fwd+Jacobian 256³×496 views; p50/p99 solve latency"
# algorithmic FP32 flops per voxel-view update (FMA = 2), FDK weighting, paper gradient
FLOPS_FWD = 23
FLOPS_VJP = 66
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (published)
# Measured plain (non-packed) FP32 VALU issue ceiling of this GPU: independent v_fma_f32 and
# v_mul_f32 chains at 32 waves per CU issue one wave64 instruction per 0.242 ns per CU, i.e.
# 64 lanes x 2 flops / 0.242 ns x 256 CUs = 135 TFLOP/s counting every instruction as an FMA
# (a throughput probe run on this machine; a single dependent FMA chain per register reaches half).
MEASURED_FP32_TFLOPS = 135.4
PEAK_HBM_GBS = 8000.0
LDS_BYTES_PER_UPDATE = 64     # 4 taps forward + 12-tap neighbourhood VJP, 4 B each
PEAK_LDS_TBPS = 128 * 256 * 2.4e9 / 1e12   # 128 B/clk/CU (CDNA3 figure) x 256 CUs x 2.4 GHz
# HBM bytes per launch of the dominant kernel, from the FETCH_SIZE / WRITE_SIZE counters of
# two rocprofv3 --pmc runs of this script, scaled by the same counters read for a plain
# elementwise kernel of known size (--copy-calib-mib). Valid only for the kernel source the
# counters were taken on: the file records its hash, and traffic is null when it differs.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bp_vjp_head256_traffic.md")
# the code that decides the recorded counters: the kernel, its descriptors (tiles, modes) and
# the plan (tile configuration, view chunks)
KERNEL_SOURCES = ("paper_2401_09283_amd/csrc/backproject.hip", "paper_2401_09283_amd/csrc/gmc_internal.hpp",
                  "paper_2401_09283_amd/csrc/compose.hip", "paper_2401_09283_amd/csrc/api.hip")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def kernel_source_hash():
    """Hash of the backprojection kernel's code: its sources with comments and whitespace
    removed, so that an edit of a comment does not invalidate recorded counters."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def recorded_traffic(config):
    """Counter-derived HBM bytes per VJP launch recorded for this configuration and the
    current kernel source, else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = [ln for ln in fh if ln.startswith("TRAFFIC ")]
    except OSError:
        return None
    for ln in lines:
        rec = json.loads(ln[len("TRAFFIC "):])
        if rec.get("config") == config and rec.get("kernel_sha") == kernel_source_hash():
            return rec
    return None


def copy_calibration(mib):
    """One plain elementwise kernel (negation) over mib MiB of FP32: reads and writes exactly
    mib MiB, the reference against which the HBM counters are scaled."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case, n_views_sample, n_views_single=4):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload: forward and
    VJP over the whole grid for the first n_views_sample views on every OpenMP thread, and the
    same for n_views_single views on one thread (scaling)."""
    import ctypes
    import dataclasses

    import numpy as np

    import oracle

    rng = np.random.default_rng(99)
    delta = rng.standard_normal(case.grid.shape)
    gomp = ctypes.CDLL("libgomp.so.1")

    def run(nv):
        scan = dataclasses.replace(case.scan, n_views=nv)
        geo = oracle.geom_from(scan, case.grid, "fdk", "paper")
        Phat, dPhat = oracle.compose(case.theta_true[:nv], case.P[:nv])
        proj = np.ascontiguousarray(case.proj[:nv])
        t0 = time.perf_counter()
        oracle.backproject(geo, proj, Phat)
        t1 = time.perf_counter()
        G = oracle.vjp(geo, proj, Phat, delta)
        oracle.chain(G, dPhat)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, case.grid.n_voxels * nv

    oracle.build()
    threads = int(gomp.omp_get_max_threads())
    tf, tv, upd = run(n_views_sample)
    out = {"value": upd / (tf + tv) / 1e9, "unit": "GUPS", "cores": threads, "kind": "oracle",
           "sample": "FP64 oracle forward (%.1f s) + VJP with chain (%.1f s) over the full %s grid for %d of %d views"
                     % (tf, tv, "x".join(map(str, case.grid.shape)), n_views_sample, case.scan.n_views),
           "gups_forward": upd / tf / 1e9, "gups_vjp": upd / tv / 1e9, "cpu_model": _cpu_model()}
    if n_views_single > 0:
        gomp.omp_set_num_threads(1)
        try:
            sf, sv, supd = run(n_views_single)
        finally:
            gomp.omp_set_num_threads(threads)
        out["single_thread"] = {"value": supd / (sf + sv) / 1e9, "unit": "GUPS", "cores": 1,
                                "sample": "forward + VJP with chain over the full grid for %d views (%.1f s)"
                                          % (n_views_single, sf + sv)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="head256")
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--cpu-views", type=int, default=160, help="views of the oracle's bounded CPU sample")
    ap.add_argument("--cpu-single-views", type=int, default=4,
                    help="views of the oracle's single-thread sample (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one elementwise kernel over this many MiB first (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2401_09283_amd.autograd import Backprojector
    from paper_2401_09283_amd.solver import MotionSolver, SolverConfig
    from synth import CONFIGS, make_case

    cfg = CONFIGS[args.config]
    t_gen = time.perf_counter()
    case = make_case(args.config)
    t_gen = time.perf_counter() - t_gen
    print("bench: generated %s inputs in %.1f s" % (args.config, t_gen), file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    if args.copy_calib_mib > 0:
        copy_calibration(args.copy_calib_mib)
    bp = Backprojector.from_case(case, device=dev)
    proj = torch.from_numpy(case.proj).to(dev)
    solver = MotionSolver(bp, proj, SolverConfig(n_nodes=cfg.n_nodes, lr=args.lr, loss="entropy_tv"))
    solver.calibrate()   # TV weight from the seed norms at theta = 0 (one sync, untimed)

    ev = {k: [] for k in ("f0", "f1", "v0", "v1", "s0", "s1")}

    def step(timed):
        e = {k: torch.cuda.Event(enable_timing=True) for k in ev} if timed else None
        if timed:
            e["s0"].record()
        solver.iteration(events=e)
        if timed:
            e["s1"].record()
            for k in ev:
                ev[k].append(e[k])

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bp.check()

    ms_step = (t1 - t0) * 1e3 / args.steps
    t_fwd = [a.elapsed_time(b) for a, b in zip(ev["f0"], ev["f1"])]
    t_vjp = [a.elapsed_time(b) for a, b in zip(ev["v0"], ev["v1"])]
    t_stp = [a.elapsed_time(b) for a, b in zip(ev["s0"], ev["s1"])]
    upd = cfg.updates
    fwd_ms, vjp_ms = float(np.mean(t_fwd)), float(np.mean(t_vjp))
    achieved = FLOPS_VJP * upd / (vjp_ms * 1e-3) / 1e12
    traffic = recorded_traffic(args.config)
    out = {
        "metric": METRIC,
        "value": upd / (ms_step * 1e-3) / 1e9,
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %d^3 @ %g mm, %d views over %g deg, %dx%d detector @ %g mm; one motion-estimation "
                        "iteration (B-spline, compose, FDK backprojection, entropy+TV loss, VJP, chain, Adam)"
                        % (cfg.name, cfg.n, cfg.voxel_mm, cfg.n_views, cfg.arc_deg, cfg.det_w, cfg.det_h,
                           cfg.pitch_mm),
            "voxel_view_updates": upd,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_bp VJP (Eq. 4-5)",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_unit": "bytes per launch (HBM read + write)",
            "flops_per_update": FLOPS_VJP,
            "avg_launch_ms": vjp_ms,
        },
        "kernels": {
            "bp_forward_ms": fwd_ms,
            "bp_vjp_ms": vjp_ms,
            "gups_forward": upd / (fwd_ms * 1e-3) / 1e9,
            "gups_vjp": upd / (vjp_ms * 1e-3) / 1e9,
            "gups_fwd_plus_jacobian": upd / ((fwd_ms + vjp_ms) * 1e-3) / 1e9,
            "forward_tflops": FLOPS_FWD * upd / (fwd_ms * 1e-3) / 1e12,
        },
        "context": {
            # both passes at the method's 89 flops per update, against the published FP32 vector
            # peak and the measured plain-FP32 issue ceiling; the VJP against the measured
            # ceiling; LDS at the algorithmic 64 B of tap reads per update against
            # 128 B/clk/CU x 256 CUs x 2.4 GHz
            "fwd_plus_vjp_tflops": (FLOPS_FWD + FLOPS_VJP) * upd / ((fwd_ms + vjp_ms) * 1e-3) / 1e12,
            "frac_fp32_peak": (FLOPS_FWD + FLOPS_VJP) * upd / ((fwd_ms + vjp_ms) * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "measured_fp32_ceiling_tflops": MEASURED_FP32_TFLOPS,
            "frac_measured_fp32_ceiling": (FLOPS_FWD + FLOPS_VJP) * upd / ((fwd_ms + vjp_ms) * 1e-3) / 1e12
                                          / MEASURED_FP32_TFLOPS,
            "vjp_frac_measured_fp32_ceiling": achieved / MEASURED_FP32_TFLOPS,
            "lds_tb_per_s": LDS_BYTES_PER_UPDATE * upd / ((fwd_ms + vjp_ms) * 1e-3) / 1e12,
            "frac_lds_peak": LDS_BYTES_PER_UPDATE * upd / ((fwd_ms + vjp_ms) * 1e-3) / 1e12 / PEAK_LDS_TBPS,
            "vjp_hbm_tb_per_s": (traffic["bytes"] / (vjp_ms * 1e-3) / 1e12) if traffic else None,
        },
        "latency_ms": {"step_p50": percentile(t_stp, 50), "step_p99": percentile(t_stp, 99)},
        "peak_hbm_gb": torch.cuda.max_memory_allocated() / 1e9,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on %d views" % args.cpu_views, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_views, args.cpu_single_views)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
