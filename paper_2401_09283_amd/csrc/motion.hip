// Motion model and optimiser steps (Sec. II-B.1, Sec. II-C).
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
