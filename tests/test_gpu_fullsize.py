"""GPU parity at the full 256^3 x 496-view size, in the launch configuration bench.py times.

The oracle cannot evaluate the whole volume or a dense VJP in test time, so:
* forward: the full GPU volume against the oracle at 3000 sampled voxels (uniform, plus voxels
  near the field-of-view border and in the slabs that leave the detector);
* VJP: a seed that is nonzero only at 400 voxels, so the oracle's sum is exact;
* properties that hold at any size with a dense seed: with the Eq. 3 weighting the gradient
  of every view is orthogonal to its matrix (scale invariance); with the FDK weighting
  <G_j, Phat_j> = -2 sum_p seed(p) I_j(p), with I_j from a one-view backprojection;
* bitwise determinism of a full-size pass;
* finite differences of the loss through the spline coefficients (50 random coefficients).
"""
import numpy as np
import pytest
import torch

import oracle
from parity import GRAD_TOL, VOL_TOL, case, grad_err

pytestmark = pytest.mark.gpu

from paper_2401_09283_amd import gmc  # noqa: E402
from paper_2401_09283_amd.autograd import Backprojector  # noqa: E402

DEV = "cuda"


def _t(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


@pytest.fixture(scope="module")
def c1():
    return case("head256")


@pytest.fixture(scope="module")
def c1_dev(c1):
    return dict(proj=_t(c1.proj, torch.float32), theta=_t(c1.theta_true, torch.float64))


def _report(name, **kv):
    print("[%s] " % name + " ".join("%s=%s" % (k, v) for k, v in kv.items()), flush=True)


def sample_voxels(grid, seed=5):
    rng = np.random.default_rng(seed)
    n = grid.nx
    uni = rng.integers(0, grid.n_voxels, 2000)
    # near the in-plane border of the field of view and in the top/bottom slabs
    i = rng.integers(0, n, 500)
    j = rng.choice(np.r_[0:24, n - 24:n], 500)
    k = rng.integers(0, n, 500)
    border = (i * n + j) * n + k
    k2 = rng.choice(np.r_[0:56, n - 56:n], 500)
    slabs = (rng.integers(0, n, 500) * n + rng.integers(0, n, 500)) * n + k2
    return np.unique(np.concatenate([uni, border, slabs]))


@pytest.mark.parametrize("weighting", ["fdk", "paper"])
def test_forward_fullsize_sampled(c1, c1_dev, weighting):
    bp = Backprojector.from_case(c1, weighting=weighting)
    vol = bp.forward(c1_dev["proj"], c1_dev["theta"]).cpu().numpy().ravel()
    bp.check()
    idx = sample_voxels(c1.grid)
    Phat, _ = oracle.compose(c1.theta_true, c1.P)
    ref = oracle.backproject_voxels(oracle.geom_from(c1.scan, c1.grid, weighting), c1.proj, Phat, idx)
    e = float(np.max(np.abs(vol[idx] - ref)) / np.max(np.abs(ref)))
    _report("forward 256^3", weighting=weighting, voxels=len(idx), err=e)
    assert e <= VOL_TOL


@pytest.mark.parametrize("weighting", ["fdk", "paper"])
def test_vjp_fullsize_sparse_seed(c1, c1_dev, weighting):
    bp = Backprojector.from_case(c1, weighting=weighting)
    rng = np.random.default_rng(99)
    idx = np.unique(np.concatenate([rng.integers(0, c1.grid.n_voxels, 300), sample_voxels(c1.grid, 6)[:100]]))
    val = rng.standard_normal(len(idx))
    delta = np.zeros(c1.grid.n_voxels, dtype=np.float32)
    delta[idx] = val
    val = delta[idx].astype(np.float64)
    gP = torch.empty((c1.scan.n_views, 3, 4), dtype=torch.float64, device=DEV)
    g = bp.vjp(c1_dev["proj"], c1_dev["theta"], _t(delta.reshape(c1.grid.shape), torch.float32), grad_P=gP)
    Phat, dPhat = oracle.compose(c1.theta_true, c1.P)
    G = oracle.vjp_sparse(oracle.geom_from(c1.scan, c1.grid, weighting), c1.proj, Phat, idx, val)
    e = grad_err(g.cpu().numpy(), oracle.chain(G, dPhat))
    _report("vjp 256^3 sparse", weighting=weighting, voxels=len(idx), err=np.array2string(e, precision=2))
    assert np.all(e <= GRAD_TOL)


def test_vjp_fullsize_dense_scale_invariance(c1, c1_dev):
    """Eq. 3 weighting: sum_rc G_j[r,c] Phat_j[r,c] = 0 for every view, any seed."""
    bp = Backprojector.from_case(c1, weighting="paper")
    delta = torch.randn(c1.grid.shape, generator=torch.Generator(DEV).manual_seed(3), device=DEV)
    gP = torch.empty((c1.scan.n_views, 3, 4), dtype=torch.float64, device=DEV)
    bp.vjp(c1_dev["proj"], c1_dev["theta"], delta, grad_P=gP)
    G = gP.cpu().numpy()
    Phat, _ = oracle.compose(c1.theta_true, c1.P)
    lhs = np.einsum("jrc,jrc->j", G, Phat)
    scale = np.einsum("jrc,jrc->j", np.abs(G), np.abs(Phat))
    finite = np.isfinite(G).all(axis=(1, 2))
    # the short-scan (Parker) weight is zero on the first view: no data, gradient exactly 0
    no_data = np.abs(c1.proj).reshape(c1.scan.n_views, -1).max(axis=1) == 0
    _report("euler 256^3 paper", nonfinite_views=np.flatnonzero(~finite)[:10].tolist(),
            no_data_views=np.flatnonzero(no_data).tolist(), zero_views=np.flatnonzero(scale == 0).tolist(),
            worst=float(np.max(np.abs(lhs[scale > 0]) / scale[scale > 0])))
    assert finite.all()
    assert np.all(scale[no_data] == 0) and np.all(scale[~no_data] > 0)
    assert np.all(np.abs(lhs) <= 1e-4 * scale)


def test_vjp_fullsize_dense_fdk_euler(c1, c1_dev):
    """FDK weighting: <G_j, Phat_j> = -2 sum_p seed(p) I_j(p), I_j from one-view plans."""
    bp = Backprojector.from_case(c1, weighting="fdk")
    delta = torch.randn(c1.grid.shape, generator=torch.Generator(DEV).manual_seed(4), device=DEV)
    gP = torch.empty((c1.scan.n_views, 3, 4), dtype=torch.float64, device=DEV)
    bp.vjp(c1_dev["proj"], c1_dev["theta"], delta, grad_P=gP)
    G = gP.cpu().numpy()
    Phat, _ = oracle.compose(c1.theta_true, c1.P)
    s, gr = c1.scan, c1.grid
    for j in (0, 123, 247, 495):
        one = Backprojector(1, s.det_w, s.det_h, gr.shape, gr.voxel_mm, gr.origin_mm, c1.P[j:j + 1], "fdk")
        Ij = one.forward(c1_dev["proj"][j:j + 1].contiguous(), c1_dev["theta"][j:j + 1].contiguous())
        rhs = -2.0 * float(torch.sum(delta.double() * Ij.double()))
        lhs = float(np.sum(G[j] * Phat[j]))
        scale = float(np.sum(np.abs(G[j]) * np.abs(Phat[j])))
        _report("euler 256^3 fdk", view=j, lhs=lhs, rhs=rhs, scale=scale)
        assert abs(lhs - rhs) <= 1e-4 * scale


def test_fullsize_determinism(c1, c1_dev):
    bp = Backprojector.from_case(c1)
    a = bp.forward(c1_dev["proj"], c1_dev["theta"]).clone()
    b = bp.forward(c1_dev["proj"], c1_dev["theta"])
    assert torch.equal(a, b)
    g1 = bp.vjp(c1_dev["proj"], c1_dev["theta"], a).clone()
    g2 = bp.vjp(c1_dev["proj"], c1_dev["theta"], a)
    assert torch.equal(g1, g2)


def _sumsq64(vol):
    """The sum-of-squared-differences loss of a GPU volume, summed in FP64 (torch)."""
    v = vol.double()
    return float(((v[1:] - v[:-1]) ** 2).sum() + ((v[:, 1:] - v[:, :-1]) ** 2).sum()
                 + ((v[:, :, 1:] - v[:, :, :-1]) ** 2).sum())


def _loss_fn(bp, proj, n_nodes, n_views):
    """sum-of-squared-differences loss of the volume reconstructed with spline coefficients c.
    The library's loss scalar is an FP32 sum (one ulp is 3e-5 at a loss of 276), which would
    quantise central differences with steps of 1e-3 to multiples of 0.015; the finite differences therefore take the same loss of the same GPU volume summed in FP64,
    while the gradient's seed comes from the library's loss kernel."""
    theta = torch.empty((n_views, 6), dtype=torch.float64, device=DEV)
    vol = torch.empty(bp.plan.vol_shape, dtype=torch.float32, device=DEV)
    gvol = torch.empty_like(vol)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)

    def f(c, grad=False):
        gmc.gmc_bspline_theta(n_views, n_nodes, c, theta)
        bp.forward(proj, theta, out=vol)
        if not grad:
            return _sumsq64(vol)
        gmc.gmc_loss_sumsq_grad(bp.plan, vol, gvol, loss, bp.workspace)
        L64 = _sumsq64(vol)
        assert abs(float(loss.item()) - L64) <= 1e-5 * L64   # the FP32 scalar, to its precision
        gt = bp.vjp(proj, theta, gvol)
        gc = torch.empty_like(c)
        gmc.gmc_bspline_grad(n_views, n_nodes, gt, gc)
        return L64, gc.cpu().numpy()

    return f


@pytest.fixture(scope="module")
def c1_smooth_proj(c1):
    """The same projections blurred along both detector axes (Gaussian, sigma 4 px): the
    central differences of Sec. II-B.2 are then close to the true detector derivative."""
    from scipy.ndimage import gaussian_filter1d

    p = gaussian_filter1d(c1.proj, 4.0, axis=2, mode="constant")
    p = gaussian_filter1d(p, 4.0, axis=1, mode="constant")
    return _t(p.astype(np.float32), torch.float32)


# (gradient mode, data, step in mm or deg, bound on the normwise error, bound on the cosine).
# The exact mode is the derivative of the forward: the step trades the bilinear kinks it
# averages over (large steps) against FP32 noise of the volume (small steps); 0.001 is the best
# (about 1 %). The paper's interpolated central differences are not the derivative of the
# bilinear forward: on ramp-filtered data, rich in content near the pixel Nyquist rate, they
# deviate from finite differences by 37.7 % normwise (cosine 0.927); on smooth data they agree.
# The raw-data paper-mode case therefore cannot bound an error; its measured deviation is held
# as a regression value instead (PAPER_RAW_FD): a gradient a few percent off in scale or
# direction moves it out of the band. The dense oracle parity tests pin that gradient itself.
FD_CASES = [("exact", "raw", 1e-3, 3e-2, 0.9995), ("paper", "smooth", 3e-3, 5e-2, 0.999),
            ("exact", "smooth", 3e-3, 3e-2, 0.9995), ("paper", "raw", 3e-3, None, None)]
PAPER_RAW_FD = (0.3775, 0.9267)   # (normwise deviation, cosine) measured on MI355X


@pytest.mark.parametrize("grad_mode,data,eps,max_rel,min_cos", FD_CASES)
def test_finite_differences_through_spline_coefficients(c1, c1_dev, c1_smooth_proj, grad_mode, data, eps, max_rel,
                                                        min_cos):
    """50 random spline coefficients (seeded): central differences of the loss against the
    analytic gradient through compose, backprojection, loss, VJP, chain and spline adjoint."""
    cfg = c1.cfg
    bp = Backprojector.from_case(c1, grad_mode=grad_mode)
    proj = c1_dev["proj"] if data == "raw" else c1_smooth_proj
    f = _loss_fn(bp, proj, cfg.n_nodes, cfg.n_views)
    rng = np.random.default_rng(12)
    c0 = torch.zeros((6, cfg.n_nodes), dtype=torch.float64, device=DEV)
    L0, g = f(c0, grad=True)
    picks = [(int(rng.integers(0, 6)), int(rng.integers(0, cfg.n_nodes))) for _ in range(50)]
    fd, an = [], []
    for k, m in picks:
        cp, cm = c0.clone(), c0.clone()
        cp[k, m] += eps
        cm[k, m] -= eps
        fd.append((f(cp) - f(cm)) / (2 * eps))
        an.append(g[k, m])
    fd, an = np.array(fd), np.array(an)
    rel = np.linalg.norm(fd - an) / np.linalg.norm(fd)
    cos = float(np.dot(fd, an) / np.linalg.norm(fd) / np.linalg.norm(an))
    _report("fd 256^3", grad=grad_mode, data=data, eps=eps, normwise=rel, cosine=cos, loss=L0)
    if max_rel is None:
        assert abs(rel - PAPER_RAW_FD[0]) <= 0.01 and abs(cos - PAPER_RAW_FD[1]) <= 0.002
    else:
        assert rel <= max_rel and cos >= min_cos
