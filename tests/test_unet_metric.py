"""Shape and seed of the U-Net metric stage (CPU, small volume): the quality map has the
volume's shape, and the seed equals the gradient of the map's mean computed in FP64 with the
same weights, which in turn matches a central finite difference."""
import copy

import torch

from paper_2401_09283_amd.unet import UNet3D, UNetMetric


def test_unet_map_shape_and_seed():
    net = UNet3D((2, 4, 8, 16))
    x = torch.randn(1, 1, 16, 16, 16, generator=torch.Generator().manual_seed(1))
    assert net(x).shape == x.shape
    m = UNetMetric((2, 4, 8, 16), device="cpu")
    vol = torch.randn(16, 16, 16, generator=torch.Generator().manual_seed(2))
    g = torch.empty_like(vol)
    f = m(vol, g)
    net64 = copy.deepcopy(m.net).double()
    v64 = vol.double().reshape(1, 1, 16, 16, 16).requires_grad_(True)
    (g64,) = torch.autograd.grad(net64(v64).mean(), v64)
    g64 = g64.reshape(16, 16, 16)
    assert torch.max(torch.abs(g.double() - g64)) <= 1e-4 * torch.max(torch.abs(g64))
    e = torch.zeros(1, 1, 16, 16, 16, dtype=torch.float64)
    e[0, 0, 5, 6, 7] = 1e-4
    with torch.no_grad():
        fd = (net64(v64.detach() + e).mean() - net64(v64.detach() - e).mean()) / 2e-4
    assert abs(float(fd) - float(g64[5, 6, 7])) <= 1e-6 * max(1.0, float(torch.max(torch.abs(g64))))
    assert torch.isfinite(f)
