"""Pins of the oracle's Akima motion model (Sec. II-B.1) against things it does not compute
itself: SciPy's Akima interpolator (an independent implementation of Akima 1970), exact
reproduction of straight lines, interpolation of the nodes, and central finite differences of
the node-value derivatives."""
import numpy as np
import pytest
from scipy.interpolate import Akima1DInterpolator

from oracle import motion


def _eval(y, xq, x_last):
    return np.array([motion._val(z) for z in motion.akima_eval(list(y), np.asarray(xq, dtype=np.float64), x_last)])


@pytest.mark.parametrize("n,n_views", [(3, 40), (10, 360), (30, 360), (20, 496)])
def test_akima_matches_scipy(n, n_views):
    rng = np.random.default_rng(n)
    y = rng.standard_normal(n) * 3.0
    xn = np.linspace(0.0, n_views - 1.0, n)
    ref = Akima1DInterpolator(xn, y)(np.arange(n_views))
    assert np.max(np.abs(_eval(y, np.arange(n_views), n_views - 1) - ref)) < 1e-12


def test_akima_reproduces_lines_and_nodes():
    n, nv = 12, 300
    xn = np.linspace(0.0, nv - 1.0, n)
    y = 0.7 - 0.013 * xn
    assert np.max(np.abs(_eval(y, np.arange(nv), nv - 1) - (0.7 - 0.013 * np.arange(nv)))) < 1e-12
    z = np.random.default_rng(3).standard_normal(n)
    assert np.max(np.abs(_eval(z, xn, nv - 1) - z)) < 1e-12


def test_akima_theta_units_and_shape():
    v = np.zeros((6, 10))
    v[2] = 1.5      # tz 1.5 mm everywhere
    v[4] = 2.0      # ry 2 deg everywhere
    th = motion.akima_theta(v, 100)
    assert th.shape == (100, 6)
    assert np.allclose(th[:, 2], 1.5) and np.allclose(th[:, 4], np.radians(2.0)) and np.allclose(th[:, [0, 1, 3, 5]], 0)


def test_akima_node_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    n, nv = 10, 120
    v = rng.standard_normal((6, n))
    g = rng.standard_normal((nv, 6))
    an = motion.akima_node_grad(v, g)
    eps = 1e-6
    fd = np.zeros_like(v)
    for k in range(6):
        for m in range(n):
            vp, vm = v.copy(), v.copy()
            vp[k, m] += eps
            vm[k, m] -= eps
            fd[k, m] = (np.sum(g * motion.akima_theta(vp, nv)) - np.sum(g * motion.akima_theta(vm, nv))) / (2 * eps)
    assert np.max(np.abs(an - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))
