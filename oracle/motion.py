"""FP64 motion model, optimiser step and reprojection error — TEST INFRASTRUCTURE (oracle).

* The paper parameterises each of the six rigid parameters by a spline over
  the scan's views (Sec. II-B.1: N = 6 N_n free parameters mapped to
  12 N_p matrix entries). Here the spline is a uniform cubic B-spline with
  N_n coefficients and knots t_m = (m - 1) h, h = (N_p - 1)/(N_n - 3), so
  that exactly four basis functions cover every view 0..N_p-1.
  Coefficients are held in (mm, mm, mm, deg, deg, deg); theta in (mm, rad).
* Gradient descent with exponential step decay is Eq. 6 (Sec. II-C): the
  estimate moves against the gradient by s_n = s0 * t^n at iteration n,
  counted from 0; the workloads' solver is Adam (Kingma & Ba), which the
  paper's discussion suggests.
* Reprojection error (Sec. IV): mean detector distance (mm) between points
  projected with the estimated and the true geometry.
* The paper's own motion model (Sec. II-B.1) is an Akima spline per rigid parameter
  with N_n nodes evenly spaced over the scan, the first on the first view and the last
  on the last view. `akima_*` evaluate it from Akima's construction (secant slopes, two
  extrapolated secants at each end, node slopes weighted by the differences of the
  neighbouring secants, cubic Hermite pieces) and differentiate it in forward mode with
  dual numbers (no hand-derived adjoint).
"""
from __future__ import annotations

import math

import numpy as np

UNIT = np.array([1.0, 1.0, 1.0, math.pi / 180.0, math.pi / 180.0, math.pi / 180.0])


def cubic_bspline(s):
    s = np.abs(np.asarray(s, dtype=np.float64))
    out = np.zeros_like(s)
    m1 = s < 1.0
    m2 = (s >= 1.0) & (s < 2.0)
    out[m1] = (4.0 - 6.0 * s[m1] ** 2 + 3.0 * s[m1] ** 3) / 6.0
    out[m2] = (2.0 - s[m2]) ** 3 / 6.0
    return out


def basis(n_views: int, n_nodes: int) -> np.ndarray:
    """B [n_views][n_nodes]"""
    if n_nodes < 4:
        raise ValueError("a cubic B-spline needs at least 4 coefficients")
    h = (n_views - 1) / (n_nodes - 3)
    B = np.zeros((n_views, n_nodes))
    for j in range(n_views):
        for m in range(n_nodes):
            B[j, m] = cubic_bspline((j - (m - 1) * h) / h)
    return B


def theta_from_coeffs(coeffs, n_views):
    """theta [n_views][6] (mm, rad) from coefficients [6][n_nodes] (mm, deg)."""
    c = np.asarray(coeffs, dtype=np.float64)
    B = basis(n_views, c.shape[1])
    return (B @ c.T) * UNIT[None, :]


def coeff_grad(grad_theta, n_nodes):
    """dL/dc [6][n_nodes] from dL/dtheta [n_views][6] (chain through theta = B c * unit)."""
    g = np.asarray(grad_theta, dtype=np.float64)
    B = basis(g.shape[0], n_nodes)
    return (B.T @ (g * UNIT[None, :])).T


def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based). Returns new (x, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return x - lr * mh / (np.sqrt(vh) + eps), m, v


def gd_step_size(n, s0, decay):
    """Step size of Eq. 6 at iteration n (0-based): s0 * decay^n (Sec. II-C)."""
    return float(s0) * float(decay) ** int(n)


def gd_step(x, g, n, s0, decay):
    """One update of Eq. 6: x^(n+1) = x^(n) - s^(n) g, with s^(n) = s0 decay^n."""
    return np.asarray(x, dtype=np.float64) - gd_step_size(n, s0, decay) * np.asarray(g, dtype=np.float64)


# ------------------------------------------------------------------------------ Akima spline

class Dual:
    """Value and gradient with respect to the node values (forward-mode differentiation)."""

    def __init__(self, v, d):
        self.v = float(v)
        self.d = np.asarray(d, dtype=np.float64)

    def _wrap(self, o):
        return o if isinstance(o, Dual) else Dual(o, np.zeros_like(self.d))

    def __add__(self, o):
        o = self._wrap(o)
        return Dual(self.v + o.v, self.d + o.d)

    __radd__ = __add__

    def __sub__(self, o):
        o = self._wrap(o)
        return Dual(self.v - o.v, self.d - o.d)

    def __rsub__(self, o):
        return self._wrap(o) - self

    def __mul__(self, o):
        o = self._wrap(o)
        return Dual(self.v * o.v, self.v * o.d + o.v * self.d)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = self._wrap(o)
        return Dual(self.v / o.v, (self.d * o.v - self.v * o.d) / (o.v * o.v))


def _dabs(x):
    if not isinstance(x, Dual):
        return abs(x)
    s = 1.0 if x.v > 0 else (-1.0 if x.v < 0 else 0.0)
    return Dual(abs(x.v), s * x.d)


def _val(x):
    return x.v if isinstance(x, Dual) else float(x)


def akima_slopes(y, dx):
    """Node slopes of Akima's interpolant of values y (list of Dual or float, n >= 3) at
    uniformly spaced nodes (spacing dx)."""
    n = len(y)
    if n < 3:
        raise ValueError("an Akima spline needs at least 3 nodes")
    m = [(y[i + 1] - y[i]) / dx for i in range(n - 1)]
    ext = [3.0 * m[0] - 2.0 * m[1], 2.0 * m[0] - m[1]] + m + [2.0 * m[-1] - m[-2], 3.0 * m[-1] - 2.0 * m[-2]]
    t = []
    for i in range(n):
        a, b, c, d = ext[i], ext[i + 1], ext[i + 2], ext[i + 3]   # m_(i-2), m_(i-1), m_i, m_(i+1)
        w1, w2 = _dabs(d - c), _dabs(b - a)
        if _val(w1) + _val(w2) == 0.0:
            t.append((b + c) * 0.5)
        else:
            t.append((w1 * b + w2 * c) / (w1 + w2))
    return t


def akima_eval(y, x_q, x_last):
    """Akima interpolant of node values y on nodes evenly spaced over [0, x_last], at x_q."""
    n = len(y)
    dx = x_last / (n - 1)
    t = akima_slopes(y, dx)
    out = []
    for xq in x_q:
        i = min(int(math.floor(xq / dx)), n - 2)
        s = (xq - i * dx) / dx
        h00, h10 = 2 * s ** 3 - 3 * s ** 2 + 1, s ** 3 - 2 * s ** 2 + s
        h01, h11 = -2 * s ** 3 + 3 * s ** 2, s ** 3 - s ** 2
        out.append(y[i] * h00 + t[i] * (h10 * dx) + y[i + 1] * h01 + t[i + 1] * (h11 * dx))
    return out


def akima_theta(values, n_views):
    """theta [n_views][6] (mm, rad) from Akima node values [6][n_nodes] (mm, deg); node m sits
    at view m (n_views - 1)/(n_nodes - 1)."""
    v = np.asarray(values, dtype=np.float64)
    out = np.zeros((n_views, 6))
    for k in range(6):
        out[:, k] = [float(z) for z in akima_eval(list(v[k]), np.arange(n_views, dtype=np.float64), n_views - 1)]
    return out * UNIT[None, :]


def akima_jacobian(values_k, n_views):
    """d theta_j / d node_m [n_views][n_nodes] for one rigid parameter (in node units)."""
    y0 = np.asarray(values_k, dtype=np.float64)
    n = len(y0)
    y = [Dual(y0[i], np.eye(n)[i]) for i in range(n)]
    ev = akima_eval(y, np.arange(n_views, dtype=np.float64), n_views - 1)
    return np.array([e.d for e in ev])


def akima_node_grad(values, grad_theta):
    """dL/d nodes [6][n_nodes] from dL/dtheta [n_views][6] through theta = Akima(nodes) * unit."""
    v = np.asarray(values, dtype=np.float64)
    g = np.asarray(grad_theta, dtype=np.float64)
    out = np.zeros_like(v)
    for k in range(6):
        out[k] = akima_jacobian(v[k], g.shape[0]).T @ (g[:, k] * UNIT[k])
    return out
