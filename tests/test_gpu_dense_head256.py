"""Dense parity at the benchmarked shape: 256^3 @ 1 mm, 496 views over 200 degrees, 620 x 480
detector @ 0.616 mm, head phantom under B-spline motion. Every voxel of the GPU volume against
the FP64 oracle's backprojection (Eq. 3), and the whole VJP (Eq. 4-5, chained by Eq. 2) over all
views with two dense seeds: N(0, 1) from rng(99), and the entropy + TV loss seed that the solver
uses (each side derives it from its own volume). Both weightings. Bars: volume 1e-4 normwise,
gradients 1e-3 per parameter type (tests/parity.py). The oracle takes about a minute of host
time per weighting on 16 threads.

The loss kernel is checked on its own input: the GPU seed against the oracle's seed of the GPU's
volume (1e-4). Seeds derived from the two volumes differ by more than that: the TV term's seed
(a sum of normalised differences D / sqrt(|D|^2 + eps^2)) changes by up to about 1/eps times a
change of the volume, so the volumes' 2e-6 difference shows up as about 3e-4 in the seed. The
end-to-end gradient, the quantity the solver uses, is held to the gradient bar."""
import functools
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import losses as olosses
from parity import GRAD_TOL, VOL_TOL, case, grad_err, mat_err, vol_err

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd import gmc  # noqa: E402
from paper_2401_09283_amd.autograd import Backprojector  # noqa: E402

HIST = (-0.01, 0.06)
TV_EPS = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _release_device_memory():
    yield
    _gpu.cache_clear()
    torch.cuda.empty_cache()


@functools.lru_cache(maxsize=1)
def _inputs():
    return case("head256")


@functools.lru_cache(maxsize=2)
def _oracle_volume(weighting):
    c = _inputs()
    Phat, dPhat = oracle.compose(c.theta_true, c.P)
    t0 = time.perf_counter()
    vol = oracle.backproject(oracle.geom_from(c.scan, c.grid, weighting, "paper"), c.proj, Phat)
    print("[dense head256] oracle %s volume in %.1f s" % (weighting, time.perf_counter() - t0), flush=True)
    return vol, Phat, dPhat


@functools.lru_cache(maxsize=2)
def _gpu(weighting):
    c = _inputs()
    bp = Backprojector.from_case(c, weighting=weighting)
    proj = torch.from_numpy(c.proj).cuda()
    theta = torch.from_numpy(c.theta_true).cuda()
    return bp, proj, theta


def _vjp_pair(weighting, delta_gpu, delta_oracle):
    c = _inputs()
    bp, proj, theta = _gpu(weighting)
    gP = torch.empty((c.scan.n_views, 3, 4), dtype=torch.float64, device="cuda")
    g = bp.vjp(proj, theta, delta_gpu, grad_P=gP).cpu().numpy()
    bp.check()
    _, Phat, dPhat = _oracle_volume(weighting)
    t0 = time.perf_counter()
    G = oracle.vjp(oracle.geom_from(c.scan, c.grid, weighting, "paper"), c.proj, Phat, delta_oracle)
    t1 = time.perf_counter() - t0
    return grad_err(g, oracle.chain(G, dPhat)), mat_err(gP.cpu().numpy(), G), t1


@pytest.mark.parametrize("weighting", ["fdk", "paper"])
def test_dense_volume(weighting):
    c = _inputs()
    bp, proj, theta = _gpu(weighting)
    vol = bp.forward(proj, theta).cpu().numpy()
    bp.check()
    ref, _, _ = _oracle_volume(weighting)
    e = vol_err(vol, ref)
    print("[dense head256 volume %s] err %.2e over %d voxels" % (weighting, e, vol.size), flush=True)
    assert e <= VOL_TOL


@pytest.mark.parametrize("weighting", ["fdk", "paper"])
def test_dense_vjp_random_seed(weighting):
    c = _inputs()
    delta = np.random.default_rng(99).standard_normal(c.grid.shape).astype(np.float32)
    e, eP, t = _vjp_pair(weighting, torch.from_numpy(delta).cuda(), delta.astype(np.float64))
    print("[dense head256 vjp N(0,1) %s] err per parameter %s, dL/dPhat %.2e (oracle %.1f s)"
          % (weighting, np.array2string(e, precision=2), eP, t), flush=True)
    assert np.all(e <= GRAD_TOL) and eP <= GRAD_TOL


@pytest.mark.parametrize("weighting", ["fdk", "paper"])
def test_dense_vjp_entropy_tv_seed(weighting):
    c = _inputs()
    bp, proj, theta = _gpu(weighting)
    ref, _, _ = _oracle_volume(weighting)
    # TV weight from the oracle's volume (equal seed norms), used by both sides
    _, gH = olosses.entropy(ref, 64, *HIST)
    _, gT = olosses.tv(ref, TV_EPS)
    lam = float(np.linalg.norm(gH) / np.linalg.norm(gT))
    L_r, delta_r, _, _ = olosses.entropy_tv(ref, lam, 64, HIST[0], HIST[1], TV_EPS)
    vol = bp.forward(proj, theta)
    seed = torch.empty_like(vol)
    loss = torch.empty(5, dtype=torch.float64, device="cuda")
    gmc.gmc_loss_entropy_tv(bp.plan, vol, lam, HIST[0], HIST[1], TV_EPS, seed, loss, bp.workspace)
    # the loss kernel on its own input: the oracle's loss and seed of the GPU volume
    L_own, delta_own, _, _ = olosses.entropy_tv(vol.cpu().numpy().astype(np.float64), lam, 64, HIST[0], HIST[1], TV_EPS)
    es_own = vol_err(seed.cpu().numpy(), delta_own)
    es = vol_err(seed.cpu().numpy(), delta_r)
    L = float(loss[0])
    e, eP, t = _vjp_pair(weighting, seed, delta_r)
    print("[dense head256 vjp entropy+TV %s] lambda %.3g loss rel err %.1e (own volume %.1e) seed err %.2e on the "
          "GPU volume, %.2e end to end; gradient err %s, dL/dPhat %.2e (oracle %.1f s)"
          % (weighting, lam, abs(L - L_r) / abs(L_r), abs(L - L_own) / abs(L_own), es_own, es,
             np.array2string(e, precision=2), eP, t), flush=True)
    assert L == pytest.approx(L_own, rel=1e-5) and L == pytest.approx(L_r, rel=1e-5)
    assert es_own <= VOL_TOL
    assert np.all(e <= GRAD_TOL) and eP <= GRAD_TOL
