"""CMA-ES (host side of the gradient-free baseline) on functions with known minima: it must
reach them from a distant start, and the same seed must give the same run."""
import numpy as np

from paper_2401_09283_amd.cmaes import CMAES


def _run(f, x0, sigma0, evals, seed=1):
    es = CMAES(x0, sigma0, seed=seed)
    best = np.inf
    while es.evals + es.lam <= evals:
        X = es.ask()
        v = np.array([f(x) for x in X])
        best = min(best, v.min())
        es.tell(v)
    return best, es


def test_sphere_converges():
    best, _ = _run(lambda x: float(np.sum(x * x)), np.full(10, 3.0), 1.0, 4000)
    assert best < 1e-10


def test_rotated_ill_conditioned_ellipsoid_converges():
    n = 8
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((n, n)))
    scale = 1e3 ** (np.arange(n) / (n - 1))      # condition number 1e6 in f
    f = lambda x: float(np.sum((scale * (Q @ (x - 1.0))) ** 2))   # noqa: E731
    best, es = _run(f, np.zeros(n), 0.5, 12000)
    assert best < 1e-8
    assert np.allclose(es.m, 1.0, atol=1e-3)


def test_seeded_runs_are_identical():
    f = lambda x: float(np.sum(np.abs(x)) + np.sum(x ** 2))   # noqa: E731
    b1, e1 = _run(f, np.ones(6), 0.3, 600, seed=4)
    b2, e2 = _run(f, np.ones(6), 0.3, 600, seed=4)
    assert b1 == b2 and np.array_equal(e1.m, e2.m)
