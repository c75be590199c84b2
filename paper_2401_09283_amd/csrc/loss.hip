// Volume losses that close the chain of Eq. 2: a scalar L(I) and its seed dL/dI for the VJP.
// The paper's own quality metric is a trained network averaged to a scalar (Sec. II-B.3);
// these kernels provide the differentiable stand-ins used by the solver:
//   * sum of squared forward differences between neighbouring voxels;
//   * soft-histogram entropy (64 bins, cubic B-spline Parzen window) plus lambda * total
//     variation (forward differences, a difference leaving the grid counts as 0).
// Voxel arithmetic is FP32; scalar sums and the 64-bin histogram are accumulated in FP64 in
// a fixed order (per-thread, per-block, then one final block), so results are reproducible.
#include "gmc_internal.hpp"

namespace gmc {

namespace {

__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// uniform cubic B-spline window and its derivative
__device__ __forceinline__ float b3(float s) {
    const float a = fabsf(s);
    if (a < 1.0f) return 2.0f / 3.0f - a * a + 0.5f * a * a * a;
    if (a < 2.0f) {
        const float t = 2.0f - a;
        return t * t * t * (1.0f / 6.0f);
    }
    return 0.0f;
}

__device__ __forceinline__ float db3(float s) {
    const float a = fabsf(s);
    float d = 0.0f;
    if (a < 1.0f)
        d = a * (1.5f * a - 2.0f);
    else if (a < 2.0f) {
        const float t = 2.0f - a;
        d = -0.5f * t * t;
    }
    return s < 0.0f ? -d : d;
}

}  // namespace

// ------------------------------------------------------------------ sum of squared differences
// Volume traversal without 64-bit division: blocks stride over (i, j) columns, threads
// over k (z fastest, coalesced).
#define FOR_EACH_VOXEL(nx, ny, nz)                                                             \
    for (int col = blockIdx.x; col < (nx) * (ny); col += gridDim.x)                            \
        for (int k = threadIdx.x; k < (nz); k += 256)

__global__ void __launch_bounds__(256) k_sumsq(const float* __restrict__ I, float* __restrict__ grad,
                                               double* __restrict__ part, int nx, int ny, int nz) {
    __shared__ double sh[256];
    const long long sx = (long long)ny * nz, sy = nz;
    double local = 0.0;
    FOR_EACH_VOXEL(nx, ny, nz) {
        const int i = col / ny, j = col % ny;
        const long long idx = (long long)col * nz + k;
        const float c = I[idx];
        float g = 0.0f;
        float s = 0.0f;
        if (i + 1 < nx) { const float d = I[idx + sx] - c; s = fmaf(d, d, s); g -= 2.0f * d; }
        if (i > 0) { g += 2.0f * (c - I[idx - sx]); }
        if (j + 1 < ny) { const float d = I[idx + sy] - c; s = fmaf(d, d, s); g -= 2.0f * d; }
        if (j > 0) { g += 2.0f * (c - I[idx - sy]); }
        if (k + 1 < nz) { const float d = I[idx + 1] - c; s = fmaf(d, d, s); g -= 2.0f * d; }
        if (k > 0) { g += 2.0f * (c - I[idx - 1]); }
        grad[idx] = g;
        local += (double)s;
    }
    const double b = block_sum(local, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// sums nparts partials of each of ncol columns (part[col * nparts + p]) in a fixed order
__global__ void __launch_bounds__(256) k_sum_cols(const double* __restrict__ part, int nparts, int ncol,
                                                  double* __restrict__ out) {
    __shared__ double sh[256];
    for (int col = 0; col < ncol; ++col) {
        double v = 0.0;
        for (int p = threadIdx.x; p < nparts; p += 256) v += part[(long long)col * nparts + p];
        const double s = block_sum(v, sh);
        if (threadIdx.x == 0) out[col] = s;
    }
}

hipError_t launch_loss_sumsq(const gmc_plan* p, const float* vol, float* grad, double* scratch, double* loss,
                             hipStream_t s) {
    k_sumsq<<<LOSS_BLOCKS, 256, 0, s>>>(vol, grad, scratch, p->g.nx, p->g.ny, p->g.nz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_cols<<<1, 256, 0, s>>>(scratch, LOSS_BLOCKS, 1, loss);
    return hipGetLastError();
}

// ------------------------------------------------------------------ entropy + TV
struct HistArgs {
    const float* I;
    long long N;
    float lo, inv_d;
};

// per-thread private histograms in LDS ([bin][thread], conflict free), summed per block in FP64
__global__ void __launch_bounds__(256) k_hist(HistArgs a, double* __restrict__ hist_part) {
    __shared__ float h[HIST_BINS * 256];
    const int t = threadIdx.x;
    for (int b = 0; b < HIST_BINS; ++b) h[b * 256 + t] = 0.0f;
    for (long long idx = (long long)blockIdx.x * 256 + t; idx < a.N; idx += (long long)gridDim.x * 256) {
        const float s = (a.I[idx] - a.lo) * a.inv_d - 0.5f;
        const float fb = floorf(s);
        if (!(fb > -3.0f && fb < (float)HIST_BINS + 1.0f)) continue;
        const int b0 = (int)fb;
#pragma unroll
        for (int o = -1; o <= 2; ++o) {
            const int b = b0 + o;
            if (b >= 0 && b < HIST_BINS) h[b * 256 + t] += b3(s - (float)b);
        }
    }
    __syncthreads();
    if (t < HIST_BINS) {
        double sum = 0.0;
        for (int q = 0; q < 256; ++q) sum += (double)h[t * 256 + q];
        hist_part[(long long)t * gridDim.x + blockIdx.x] = sum;
    }
}

// hist[b] = sum over blocks of the per-block partials (one block per bin, fixed-order tree)
__global__ void __launch_bounds__(256) k_hist_reduce(const double* __restrict__ hist_part, int nparts,
                                                     double* __restrict__ hist) {
    __shared__ double sh[256];
    const int b = blockIdx.x;
    double v = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 256) v += hist_part[(long long)b * nparts + p];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) hist[b] = s;
}

// coef[64..127] = dH/dh_b; hist[128] = H
__global__ void __launch_bounds__(64) k_hist_final(double* __restrict__ hist) {
    __shared__ double sh[64];
    const int b = threadIdx.x;
    const double h = hist[b];
    sh[b] = h;
    __syncthreads();
    double Z = 0.0;
    for (int q = 0; q < HIST_BINS; ++q) Z += sh[q];
    double H = 0.0;
    for (int q = 0; q < HIST_BINS; ++q)
        if (sh[q] > 0.0) {
            const double pq = sh[q] / Z;
            H -= pq * log(pq);
        }
    double coef = 0.0;
    if (h > 0.0 && Z > 0.0) coef = -(log(h / Z) + H) / Z;
    hist[HIST_BINS + b] = coef;
    if (b == 0) hist[2 * HIST_BINS] = H;
}

struct GradArgs {
    const float* I;
    float* grad;
    const double* hist;   // coef at [64..127]
    double* part;         // [3][nblocks]: TV, |gH|^2, |gTV|^2
    int nx, ny, nz;
    float lo, inv_d, eps2, lambda;
};

__device__ __forceinline__ float tv_norm(const float* __restrict__ I, long long idx, int i, int j, int k, int nx, int ny,
                                         int nz, long long sx, long long sy, float eps2, float& dxv, float& dyv,
                                         float& dzv) {
    const float c = I[idx];
    dxv = (i + 1 < nx) ? I[idx + sx] - c : 0.0f;
    dyv = (j + 1 < ny) ? I[idx + sy] - c : 0.0f;
    dzv = (k + 1 < nz) ? I[idx + 1] - c : 0.0f;
    return sqrtf(fmaf(dxv, dxv, fmaf(dyv, dyv, fmaf(dzv, dzv, eps2))));
}

__global__ void __launch_bounds__(256) k_entropy_tv_grad(GradArgs a) {
    __shared__ float coef[HIST_BINS];
    __shared__ double sh[256];
    if (threadIdx.x < HIST_BINS) coef[threadIdx.x] = (float)a.hist[HIST_BINS + threadIdx.x];
    __syncthreads();
    const long long sx = (long long)a.ny * a.nz, sy = a.nz;
    double tv = 0.0, gh2 = 0.0, gt2 = 0.0;
    FOR_EACH_VOXEL(a.nx, a.ny, a.nz) {
        const int i = col / a.ny, j = col % a.ny;
        const long long idx = (long long)col * a.nz + k;
        // entropy seed
        const float s = (a.I[idx] - a.lo) * a.inv_d - 0.5f;
        const float fb = floorf(s);
        float gh = 0.0f;
        if (fb > -3.0f && fb < (float)HIST_BINS + 1.0f) {
            const int b0 = (int)fb;
#pragma unroll
            for (int o = -1; o <= 2; ++o) {
                const int b = b0 + o;
                if (b >= 0 && b < HIST_BINS) gh = fmaf(coef[b], db3(s - (float)b), gh);
            }
        }
        gh *= a.inv_d;
        // TV seed: own term and the terms at the three backward neighbours
        float dx0, dy0, dz0;
        const float n0 = tv_norm(a.I, idx, i, j, k, a.nx, a.ny, a.nz, sx, sy, a.eps2, dx0, dy0, dz0);
        float gt = -(dx0 + dy0 + dz0) / n0;
        float p, q, r;
        if (i > 0) { const float nn = tv_norm(a.I, idx - sx, i - 1, j, k, a.nx, a.ny, a.nz, sx, sy, a.eps2, p, q, r); gt += p / nn; }
        if (j > 0) { const float nn = tv_norm(a.I, idx - sy, i, j - 1, k, a.nx, a.ny, a.nz, sx, sy, a.eps2, p, q, r); gt += q / nn; }
        if (k > 0) { const float nn = tv_norm(a.I, idx - 1, i, j, k - 1, a.nx, a.ny, a.nz, sx, sy, a.eps2, p, q, r); gt += r / nn; }
        a.grad[idx] = fmaf(a.lambda, gt, gh);
        tv += (double)n0;
        gh2 += (double)gh * (double)gh;
        gt2 += (double)gt * (double)gt;
    }
    const double b0 = block_sum(tv, sh);
    const double b1 = block_sum(gh2, sh);
    const double b2 = block_sum(gt2, sh);
    if (threadIdx.x == 0) {
        a.part[blockIdx.x] = b0;
        a.part[gridDim.x + blockIdx.x] = b1;
        a.part[2 * gridDim.x + blockIdx.x] = b2;
    }
}

__global__ void k_entropy_tv_final(const double* __restrict__ sums, const double* __restrict__ hist, double lambda,
                                   double* __restrict__ loss) {
    const double H = hist[2 * HIST_BINS];
    loss[0] = H + lambda * sums[0];
    loss[1] = H;
    loss[2] = sums[0];
    loss[3] = sums[1];
    loss[4] = sums[2];
}

hipError_t launch_loss_entropy_tv(const gmc_plan* p, const float* vol, double lambda, double lo, double hi,
                                  double eps, float* grad, double* scratch, double* hist, double* loss,
                                  hipStream_t s) {
    const long long N = (long long)p->g.nx * p->g.ny * p->g.nz;
    const float inv_d = (float)((double)HIST_BINS / (hi - lo));
    HistArgs ha{vol, N, (float)lo, inv_d};
    // hist scratch: [64][HIST_BLOCKS] partials, then 129 finals
    double* hist_part = hist;
    double* hist_final = hist + (long long)HIST_BINS * HIST_BLOCKS;
    k_hist<<<HIST_BLOCKS, 256, 0, s>>>(ha, hist_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_hist_reduce<<<HIST_BINS, 256, 0, s>>>(hist_part, HIST_BLOCKS, hist_final);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_hist_final<<<1, HIST_BINS, 0, s>>>(hist_final);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GradArgs ga;
    ga.I = vol;
    ga.grad = grad;
    ga.hist = hist_final;
    ga.part = scratch;
    ga.nx = p->g.nx;
    ga.ny = p->g.ny;
    ga.nz = p->g.nz;
    ga.lo = (float)lo;
    ga.inv_d = inv_d;
    ga.eps2 = (float)(eps * eps);
    ga.lambda = (float)lambda;
    k_entropy_tv_grad<<<LOSS_BLOCKS, 256, 0, s>>>(ga);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* sums = scratch + 3 * LOSS_BLOCKS;
    k_sum_cols<<<1, 256, 0, s>>>(scratch, LOSS_BLOCKS, 3, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_entropy_tv_final<<<1, 1, 0, s>>>(sums, hist_final, lambda, loss);
    return hipGetLastError();
}

}  // namespace gmc
