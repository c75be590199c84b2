// Motion models and optimiser steps (Sec. II-B.1, Sec. II-C).
//
// The paper's motion model is an Akima spline per rigid parameter: N_n nodes evenly spaced over
// the views (node m at view m (N_p - 1)/(N_n - 1)), secant slopes between nodes, two secants
// extrapolated linearly at each end, node slopes t = (|m+1 - m| m-1 + |m-1 - m-2| m) / (sum of the
// two weights) (the mean of the two middle secants when both weights vanish), and a cubic
// Hermite piece per interval. Its adjoint differentiates through the slope weights
// (|x|' = sign(x), 0 at 0). The workloads' smooth stand-in is a uniform cubic B-spline:
//
// theta_jk = unit_k * sum_m c_km B3((j - t_m)/h), t_m = (m - 1) h, h = (n_views - 1)/(n_nodes - 3),
// with B3 the uniform cubic B-spline, coefficients in (mm, mm, mm, deg, deg, deg) and theta in
// (mm, rad). The adjoint gives dL/dc from dL/dtheta. Adam and the decaying gradient step of
// Eq. 6 update the coefficients. All FP64 (these are the motion parameters, not voxels).
#include "gmc_internal.hpp"

namespace gmc {

namespace {

__device__ __forceinline__ double bspline3(double s) {
    const double a = fabs(s);
    if (a >= 2.0) return 0.0;
    if (a >= 1.0) {
        const double t = 2.0 - a;
        return t * t * t / 6.0;
    }
    return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
}

__device__ __forceinline__ double unit_of(int k) { return k < 3 ? 1.0 : 0.017453292519943295769; }

}  // namespace

__global__ void k_bspline_theta(int n_views, int n_nodes, const double* __restrict__ c, double* __restrict__ theta) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_views * 6) return;
    const int j = q / 6, k = q % 6;
    const double h = (double)(n_views - 1) / (double)(n_nodes - 3);
    double s = 0.0;
    for (int m = 0; m < n_nodes; ++m) s += c[k * n_nodes + m] * bspline3(((double)j - (double)(m - 1) * h) / h);
    theta[q] = unit_of(k) * s;
}

// one block per coefficient (k, m): the threads split the views, then a fixed-order tree sum
__global__ void __launch_bounds__(256) k_bspline_grad(int n_views, int n_nodes, const double* __restrict__ g,
                                                      double* __restrict__ gc) {
    __shared__ double sh[256];
    const int q = blockIdx.x;
    const int k = q / n_nodes, m = q % n_nodes;
    const double h = (double)(n_views - 1) / (double)(n_nodes - 3);
    double s = 0.0;
    for (int j = threadIdx.x; j < n_views; j += 256) s += g[6 * j + k] * bspline3(((double)j - (double)(m - 1) * h) / h);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gc[q] = unit_of(k) * sh[0];
}

hipError_t launch_bspline_theta(int n_views, int n_nodes, const double* coeffs, double* theta, hipStream_t s) {
    k_bspline_theta<<<(n_views * 6 + 255) / 256, 256, 0, s>>>(n_views, n_nodes, coeffs, theta);
    return hipGetLastError();
}

hipError_t launch_bspline_grad(int n_views, int n_nodes, const double* grad_theta, double* grad_coeffs,
                               hipStream_t s) {
    k_bspline_grad<<<n_nodes * 6, 256, 0, s>>>(n_views, n_nodes, grad_theta, grad_coeffs);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ Akima spline

namespace {

// extended secant q (q = 0 .. n + 2 stands for m_(q-2)) of node values y[0..n-1], spacing dx
__device__ __forceinline__ double akima_secant(const double* y, int n, double dx, int q) {
    auto m = [&](int r) { return (y[r + 1] - y[r]) / dx; };
    if (q == 0) return 3.0 * m(0) - 2.0 * m(1);
    if (q == 1) return 2.0 * m(0) - m(1);
    if (q == n + 1) return 2.0 * m(n - 2) - m(n - 3);
    if (q == n + 2) return 3.0 * m(n - 2) - 2.0 * m(n - 3);
    return m(q - 2);
}

// slope at node i from its four secants a = m_(i-2), b = m_(i-1), c = m_i, d = m_(i+1), and the
// partial derivatives of the slope with respect to them
__device__ __forceinline__ double akima_slope(double a, double b, double c, double d, double* dt) {
    const double w1 = fabs(d - c), w2 = fabs(b - a), W = w1 + w2;
    if (W == 0.0) {
        if (dt) { dt[0] = 0.0; dt[1] = 0.5; dt[2] = 0.5; dt[3] = 0.0; }
        return 0.5 * (b + c);
    }
    const double t = (w1 * b + w2 * c) / W;
    if (dt) {
        const double sdc = (d > c) ? 1.0 : ((d < c) ? -1.0 : 0.0), sba = (b > a) ? 1.0 : ((b < a) ? -1.0 : 0.0);
        dt[0] = -(c - t) / W * sba;
        dt[1] = w1 / W + (c - t) / W * sba;
        dt[2] = w2 / W - (b - t) / W * sdc;
        dt[3] = (b - t) / W * sdc;
    }
    return t;
}

__device__ __forceinline__ double akima_node_slope(const double* y, int n, double dx, int i) {
    return akima_slope(akima_secant(y, n, dx, i), akima_secant(y, n, dx, i + 1), akima_secant(y, n, dx, i + 2),
                       akima_secant(y, n, dx, i + 3), nullptr);
}

__device__ __forceinline__ void hermite(double s, double& h00, double& h10, double& h01, double& h11) {
    const double s2 = s * s, s3 = s2 * s;
    h00 = 2.0 * s3 - 3.0 * s2 + 1.0;
    h10 = s3 - 2.0 * s2 + s;
    h01 = -2.0 * s3 + 3.0 * s2;
    h11 = s3 - s2;
}

__device__ __forceinline__ int akima_segment(int j, double dx, int n) {
    const int i = (int)floor((double)j / dx);
    return i < n - 2 ? i : n - 2;
}

}  // namespace

// theta[j][k] = unit_k * Akima(c[k][.])(j), one thread per (view, parameter)
__global__ void k_akima_theta(int n_views, int n_nodes, const double* __restrict__ c, double* __restrict__ theta) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_views * 6) return;
    const int j = q / 6, k = q % 6;
    const double* y = c + (long long)k * n_nodes;
    const double dx = (double)(n_views - 1) / (double)(n_nodes - 1);
    const int i = akima_segment(j, dx, n_nodes);
    const double s = ((double)j - (double)i * dx) / dx;
    double h00, h10, h01, h11;
    hermite(s, h00, h10, h01, h11);
    const double ti = akima_node_slope(y, n_nodes, dx, i), ti1 = akima_node_slope(y, n_nodes, dx, i + 1);
    theta[q] = unit_of(k) * (y[i] * h00 + ti * (h10 * dx) + y[i + 1] * h01 + ti1 * (h11 * dx));
}

// dL/dc[k][m] from dL/dtheta, one block per parameter k. Threads form the per-interval sums of
// the Hermite weights times dL/dtheta (views in increasing order); one thread then chains them
// through the node slopes, the extrapolated secants and the secants in a fixed order.
__global__ void __launch_bounds__(256) k_akima_grad(int n_views, int n_nodes, const double* __restrict__ c,
                                                    const double* __restrict__ g, double* __restrict__ gc) {
    __shared__ double A[256], B[256], C[256], D[256];
    __shared__ double dmext[259], dm[256];
    const int k = blockIdx.x;
    const double* y = c + (long long)k * n_nodes;
    const int n = n_nodes;
    const double dx = (double)(n_views - 1) / (double)(n - 1);
    for (int i = threadIdx.x; i < n - 1; i += 256) {
        double a = 0.0, b = 0.0, cc = 0.0, d = 0.0;
        const int j0 = (int)ceil((double)i * dx);
        for (int j = j0; j < n_views; ++j) {
            const int seg = akima_segment(j, dx, n);
            if (seg < i) continue;
            if (seg > i) break;
            const double s = ((double)j - (double)i * dx) / dx;
            double h00, h10, h01, h11;
            hermite(s, h00, h10, h01, h11);
            const double gj = g[6 * j + k];
            a += gj * h00;
            b += gj * h01;
            cc += gj * h10 * dx;
            d += gj * h11 * dx;
        }
        A[i] = a;
        B[i] = b;
        C[i] = cc;
        D[i] = d;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 0; q < n + 3; ++q) dmext[q] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double gt = (i < n - 1 ? C[i] : 0.0) + (i > 0 ? D[i - 1] : 0.0);   // dL/dt_i
        double dt[4];
        akima_slope(akima_secant(y, n, dx, i), akima_secant(y, n, dx, i + 1), akima_secant(y, n, dx, i + 2),
                    akima_secant(y, n, dx, i + 3), dt);
        for (int e = 0; e < 4; ++e) dmext[i + e] += gt * dt[e];
    }
    for (int r = 0; r < n - 1; ++r) dm[r] = dmext[r + 2];
    dm[0] += 3.0 * dmext[0] + 2.0 * dmext[1];
    dm[1] += -2.0 * dmext[0] - dmext[1];
    dm[n - 2] += 2.0 * dmext[n + 1] + 3.0 * dmext[n + 2];
    dm[n - 3] += -dmext[n + 1] - 2.0 * dmext[n + 2];
    for (int m = 0; m < n; ++m) {
        double v = (m < n - 1 ? A[m] : 0.0) + (m > 0 ? B[m - 1] : 0.0);
        if (m > 0) v += dm[m - 1] / dx;
        if (m < n - 1) v -= dm[m] / dx;
        gc[(long long)k * n + m] = unit_of(k) * v;
    }
}

hipError_t launch_akima_theta(int n_views, int n_nodes, const double* coeffs, double* theta, hipStream_t s) {
    k_akima_theta<<<(n_views * 6 + 255) / 256, 256, 0, s>>>(n_views, n_nodes, coeffs, theta);
    return hipGetLastError();
}

hipError_t launch_akima_grad(int n_views, int n_nodes, const double* coeffs, const double* grad_theta,
                             double* grad_coeffs, hipStream_t s) {
    k_akima_grad<<<6, 256, 0, s>>>(n_views, n_nodes, coeffs, grad_theta, grad_coeffs);
    return hipGetLastError();
}

__global__ void k_adam(long long n, double* __restrict__ x, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, double c1, double c2, double lr, double b1, double b2, double eps) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    x[i] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
}

hipError_t launch_adam(long long n, double* x, const double* g, double* m, double* v, int t, double lr,
                       double b1, double b2, double eps, hipStream_t s) {
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x, g, m, v, c1, c2, lr, b1, b2, eps);
    return hipGetLastError();
}

__global__ void k_gd(long long n, double* __restrict__ x, const double* __restrict__ g, double step) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] -= step * g[i];
}

hipError_t launch_gd(long long n, double* x, const double* g, double step, hipStream_t s) {
    k_gd<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x, g, step);
    return hipGetLastError();
}

}  // namespace gmc
