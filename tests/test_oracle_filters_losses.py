"""Pins of the FDK pre-filter (inputs), the motion model and the volume losses (oracle).

Filter and weights: the Ram-Lak kernel has zero DC gain, Parker weights of a
ray and its geometrically computed conjugate sum to one, the cosine weight is
one at the principal point. Motion model: cubic B-spline knot values,
partition of unity, reproduction of linear motion, adjointness. Optimiser:
Adam's first step is lr * sign(g). Losses: closed forms and finite
differences.
"""
import math

import numpy as np
import pytest

from oracle import losses, motion
from synth.filter import cosine_weights, parker_weight, ramlak_kernel
from synth.geometry import ScanGeometry


def test_ramlak_has_zero_dc_gain():
    tau = 0.4
    for n_half in (101, 1001, 10001):
        h = ramlak_kernel(n_half, tau)
        # the tail beyond n_half of sum 2/(pi^2 n^2 tau^2) over odd n is ~ 1/(pi^2 tau^2 n_half)
        assert abs(h.sum()) <= 1.1 / (math.pi ** 2 * tau * tau * n_half)
    assert ramlak_kernel(3, tau)[3] == pytest.approx(1 / (4 * tau * tau))


def test_parker_weights_of_conjugate_rays_sum_to_one():
    """Conjugate ray found geometrically: the other source position on the same line."""
    dso = 785.0
    delta = math.radians(10.0)
    rng = np.random.default_rng(4)
    for _ in range(300):
        beta = rng.uniform(0, math.pi + 2 * delta)
        gamma = rng.uniform(-math.radians(9.0), math.radians(9.0))
        S = dso * np.array([math.cos(beta), math.sin(beta)])
        # central ray points from the source to the isocentre; positive gamma turns towards e_u
        central = -S / dso
        e_u = np.array([-math.sin(beta), math.cos(beta)])
        d = math.cos(gamma) * central + math.sin(gamma) * e_u
        # second intersection of the line S + t d with the source circle
        t = -2.0 * np.dot(S, d)
        S2 = S + t * d
        beta2 = math.atan2(S2[1], S2[0]) % (2 * math.pi)
        d2 = -d
        central2 = -S2 / dso
        e_u2 = np.array([-math.sin(beta2), math.cos(beta2)])
        # fan angle of the reversed ray at the second source, positive towards that view's e_u
        gamma2 = math.atan2(np.dot(d2, e_u2), np.dot(d2, central2))
        w1 = parker_weight(beta, gamma, delta)
        if beta2 <= math.pi + 2 * delta:
            w2 = parker_weight(beta2, gamma2, delta)
            assert w1 + w2 == pytest.approx(1.0, abs=1e-12)
        else:
            assert w1 == pytest.approx(1.0, abs=1e-12)


def test_cosine_weight_is_one_at_principal_point():
    g = ScanGeometry(n_views=1, det_w=31, det_h=21, pitch_mm=0.5)
    cw = cosine_weights(g)
    assert cw[10, 15] == pytest.approx(1.0, abs=1e-15)
    assert np.all(cw <= 1.0)


def test_cubic_bspline_knot_values_and_partition_of_unity():
    assert motion.cubic_bspline(np.array([0.0]))[0] == pytest.approx(2 / 3)
    assert motion.cubic_bspline(np.array([1.0, -1.0])) == pytest.approx([1 / 6, 1 / 6])
    assert motion.cubic_bspline(np.array([2.0, -2.5]))[0] == 0.0
    for n_views, n_nodes in ((496, 20), (120, 10), (37, 4)):
        B = motion.basis(n_views, n_nodes)
        assert np.allclose(B.sum(1), 1.0, atol=1e-14)
        assert np.all((B > 0).sum(1) <= 4)
        # linear motion is reproduced exactly by coefficients at the knots t_m = (m - 1) h
        h = (n_views - 1) / (n_nodes - 3)
        t = (np.arange(n_nodes) - 1.0) * h
        assert np.allclose(B @ t, np.arange(n_views), atol=1e-10)


def test_coefficient_gradient_is_the_adjoint():
    rng = np.random.default_rng(9)
    c = rng.standard_normal((6, 20))
    g = rng.standard_normal((496, 6))
    th = motion.theta_from_coeffs(c, 496)
    assert np.sum(g * th) == pytest.approx(np.sum(motion.coeff_grad(g, 20) * c), rel=1e-12)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(10)
    x = rng.standard_normal(50)
    g = rng.standard_normal(50)
    x1, m, v = motion.adam_step(x, g, np.zeros(50), np.zeros(50), 1, lr=0.05)
    assert np.allclose(x1, x - 0.05 * np.sign(g), atol=1e-8)


def test_sumsq_grad_closed_form():
    n = (5, 6, 7)
    i, j, k = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in n], indexing="ij")
    I = 0.5 * i - 0.25 * j + 2.0 * k
    L, d = losses.sumsq_grad(I)
    pairs = [(n[0] - 1) * n[1] * n[2], n[0] * (n[1] - 1) * n[2], n[0] * n[1] * (n[2] - 1)]
    assert L == pytest.approx(0.25 * pairs[0] + 0.0625 * pairs[1] + 4.0 * pairs[2], rel=1e-14)
    # the seed is a discrete Laplacian: zero in the interior for a linear volume
    assert np.allclose(d[1:-1, 1:-1, 1:-1], 0.0, atol=1e-12)


def test_entropy_closed_form_single_bin():
    lo, hi, nb = -0.01, 0.06, 64
    D = (hi - lo) / nb
    I = np.full((4, 4, 4), lo + (20 + 0.5) * D)    # every voxel at the centre of bin 20
    H, g = losses.entropy(I, nb, lo, hi)
    p = np.array([1 / 6, 2 / 3, 1 / 6])
    assert H == pytest.approx(-np.sum(p * np.log(p)), rel=1e-12)
    # by symmetry of the window, moving any voxel changes H only at second order
    assert np.allclose(g, 0.0, atol=1e-9)


def test_tv_of_constant_and_of_a_step():
    I = np.full((6, 6, 6), 0.3)
    T, g = losses.tv(I, eps=1e-5)
    assert T == pytest.approx(216 * 1e-5, rel=1e-12)
    assert np.allclose(g, 0.0)
    J = np.zeros((6, 6, 6))
    J[3:] = 1.0
    T, _ = losses.tv(J, eps=1e-12)
    assert T == pytest.approx(36.0, rel=1e-9)


@pytest.mark.parametrize("which", ["sumsq", "entropy", "tv", "entropy_tv"])
def test_loss_seeds_match_finite_differences(which):
    rng = np.random.default_rng(12)
    I = 0.025 + 0.015 * rng.standard_normal((7, 6, 5))
    f = {"sumsq": losses.sumsq_grad, "entropy": losses.entropy, "tv": lambda v: losses.tv(v, 1e-3),
         "entropy_tv": lambda v: losses.entropy_tv(v, 0.3, eps=1e-3)}[which]
    L, g = f(I)[:2]
    for q in rng.choice(I.size, 25, replace=False):
        e = np.zeros(I.size)
        e[q] = 1e-7
        fd = (f(I + e.reshape(I.shape))[0] - f(I - e.reshape(I.shape))[0]) / 2e-7
        assert fd == pytest.approx(g.ravel()[q], rel=1e-5, abs=1e-6 * np.abs(g).max())
