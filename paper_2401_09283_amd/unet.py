"""The paper's learned quality metric in the gradient chain (Sec. II-B.3), for timing only.

A 3D U-Net regresses a voxel-wise quality map from the reconstructed volume; its mean is the
target f, and backpropagation through the network gives the seed dL/dI for the Jacobian-vector
product of the backprojection. The trained weights and the training data (CQ500) are not
available, so the network here is randomly initialised (seeded): it measures what the metric
costs per iteration, not how well it guides the estimate.

Architecture (Sec. II-B.3): basic blocks of two 3x3x3 convolutions with ReLU per level, four
levels, max-pooling down and transposed convolutions up with skip connections, a final 1x1x1
convolution without activation. The feature maps per level are printed as "8^l, l = 1..4";
the default reads it as 8, 16, 32, 64 (doubling per level); ``channels=(8, 64, 512, 4096)``
gives the literal powers of 8. FP32 torch layers (MIOpen convolutions): this stage is a library
network, not part of the hand-written path.
"""
from __future__ import annotations

import torch
from torch import nn


class _Block(nn.Module):
    def __init__(self, cin, cout):
        super().__init__()
        self.c1 = nn.Conv3d(cin, cout, 3, padding=1)
        self.c2 = nn.Conv3d(cout, cout, 3, padding=1)

    def forward(self, x):
        return torch.relu(self.c2(torch.relu(self.c1(x))))


class UNet3D(nn.Module):
    def __init__(self, channels=(8, 16, 32, 64)):
        super().__init__()
        ch = list(channels)
        self.down = nn.ModuleList()
        cin = 1
        for c in ch:
            self.down.append(_Block(cin, c))
            cin = c
        self.up = nn.ModuleList()
        self.upconv = nn.ModuleList()
        for l in range(len(ch) - 1, 0, -1):
            self.upconv.append(nn.ConvTranspose3d(ch[l], ch[l - 1], 2, stride=2))
            self.up.append(_Block(2 * ch[l - 1], ch[l - 1]))
        self.head = nn.Conv3d(ch[0], 1, 1)

    def forward(self, x):
        skips = []
        for l, blk in enumerate(self.down):
            x = blk(x)
            if l < len(self.down) - 1:
                skips.append(x)
                x = torch.max_pool3d(x, 2)
        for uc, blk in zip(self.upconv, self.up):
            x = uc(x)
            x = blk(torch.cat([x, skips.pop()], dim=1))
        return self.head(x)


class UNetMetric:
    """f(I) = mean of the U-Net's quality map and its seed dL/dI, for one volume shape."""

    def __init__(self, channels=(8, 16, 32, 64), seed=0, device="cuda"):
        g = torch.Generator().manual_seed(seed)
        net = UNet3D(channels)
        with torch.no_grad():
            for p in net.parameters():
                p.copy_(torch.randn(p.shape, generator=g) * (2.0 / max(1, p[0].numel())) ** 0.5)
        self.net = net.to(device).float().eval()
        for p in self.net.parameters():
            p.requires_grad_(False)

    def __call__(self, vol, grad_out):
        """vol [nx][ny][nz] float32 (device); writes dL/dI into grad_out; returns f (device scalar)."""
        x = vol.detach().reshape((1, 1) + tuple(vol.shape)).requires_grad_(True)
        with torch.enable_grad():
            f = self.net(x).mean()
            (g,) = torch.autograd.grad(f, x)
        grad_out.copy_(g.reshape(vol.shape))
        return f.detach()


def main(argv=None):
    """Per-iteration cost of gradient-based motion estimation with the U-Net metric in the chain:
    ``python -m paper_2401_09283_amd.unet --config paper128 --iters 10``."""
    import argparse
    import json
    import time

    from synth import CONFIGS, make_case

    from .autograd import Backprojector
    from .solver import MotionSolver, SolverConfig

    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--config", default="paper128")
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--channels", default="8,16,32,64")
    ap.add_argument("--no-find", dest="find", action="store_false",
                    help="keep the convolution library's default algorithms (no MIOpen find step)")
    args = ap.parse_args(argv)
    # MIOpen times its convolution algorithms for each shape once (during the warm-up)
    torch.backends.cudnn.benchmark = args.find
    cfg = CONFIGS[args.config]
    case = make_case(args.config)
    bp = Backprojector.from_case(case)
    proj = torch.from_numpy(case.proj).to(bp.device)
    ch = tuple(int(x) for x in args.channels.split(","))
    s = MotionSolver(bp, proj, SolverConfig(n_nodes=cfg.estimate_nodes, motion=cfg.motion_model, loss="unet",
                                            optimizer="gd", gd_first_step=0.5, unet_channels=ch))
    s.calibrate()
    for _ in range(args.warmup):
        s.iteration()
    torch.cuda.synchronize()
    keys = ("f0", "f1", "v0", "v1")
    rec = []
    t0 = time.perf_counter()
    for _ in range(args.iters):
        e = {k: torch.cuda.Event(enable_timing=True) for k in keys}
        s.iteration(events=e)
        rec.append(e)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.iters
    fwd = sum(e["f0"].elapsed_time(e["f1"]) for e in rec) / args.iters
    mid = sum(e["f1"].elapsed_time(e["v0"]) for e in rec) / args.iters
    vjp = sum(e["v0"].elapsed_time(e["v1"]) for e in rec) / args.iters
    print(json.dumps(dict(config=args.config, channels=ch, find=args.find, ms_per_iter=ms, bp_forward_ms=fwd, unet_fwd_bwd_ms=mid,
                          bp_vjp_ms=vjp, s_per_100_iters=ms / 10.0)), flush=True)


if __name__ == "__main__":
    main()
