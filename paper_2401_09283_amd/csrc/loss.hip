// Volume losses that close the chain of Eq. 2: a scalar L(I) and its seed dL/dI for the VJP.
// The paper's own quality metric is a trained network averaged to a scalar (Sec. II-B.3);
// these kernels provide the differentiable stand-ins used by the solver:
//   * sum of squared forward differences between neighbouring voxels;
//   * soft-histogram entropy (64 bins, cubic B-spline Parzen window) plus lambda * total
//     variation (forward differences, a difference leaving the grid counts as 0).
// Arithmetic and accumulation are FP32: every scalar sum and the 64-bin histogram are
// accumulated per thread, then by fixed-order trees over the block and over the blocks, so the
// results are reproducible. Only the ABI's loss words are FP64 (converted at the end).
#include "gmc_internal.hpp"

namespace gmc {

namespace {

__device__ __forceinline__ float block_sum(float v, float* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const float r = sh[0];
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
                                               float* __restrict__ part, int nx, int ny, int nz) {
    __shared__ float sh[256];
    const long long sx = (long long)ny * nz, sy = nz;
    float local = 0.0f;
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
        local += s;
    }
    const float b = block_sum(local, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// sums nparts partials of each of ncol columns (part[col * nparts + p]) in a fixed order
__global__ void __launch_bounds__(256) k_sum_cols(const float* __restrict__ part, int nparts, int ncol,
                                                  float* __restrict__ out) {
    __shared__ float sh[256];
    for (int col = 0; col < ncol; ++col) {
        float v = 0.0f;
        for (int p = threadIdx.x; p < nparts; p += 256) v += part[(long long)col * nparts + p];
        const float s = block_sum(v, sh);
        if (threadIdx.x == 0) out[col] = s;
    }
}

__global__ void k_to_double(const float* __restrict__ src, double* __restrict__ dst, int n) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

hipError_t launch_loss_sumsq(const gmc_plan* p, const float* vol, float* grad, float* scratch, double* loss,
                             hipStream_t s) {
    k_sumsq<<<LOSS_BLOCKS, 256, 0, s>>>(vol, grad, scratch, p->g.nx, p->g.ny, p->g.nz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    float* total = scratch + LOSS_BLOCKS;
    k_sum_cols<<<1, 256, 0, s>>>(scratch, LOSS_BLOCKS, 1, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_to_double<<<1, 64, 0, s>>>(total, loss, 1);
    return hipGetLastError();
}

// ------------------------------------------------------------------ entropy + TV
struct HistArgs {
    const float* I;
    long long N;
    float lo, inv_d;
};

// Per-thread private histograms in LDS ([bin][thread], conflict free), summed per block by a
// fixed-order tree (thread t of the first 64 sums bin t). Voxels are read four at a time where
// the volume is 16-byte aligned.
__device__ __forceinline__ void hist_add(const HistArgs& a, float* h, int t, float x) {
    const float s = (x - a.lo) * a.inv_d - 0.5f;
    const float fb = floorf(s);
    if (!(fb > -3.0f && fb < (float)HIST_BINS + 1.0f)) return;
    const int b0 = (int)fb;
#pragma unroll
    for (int o = -1; o <= 2; ++o) {
        const int b = b0 + o;
        if (b >= 0 && b < HIST_BINS) h[b * 256 + t] += b3(s - (float)b);
    }
}

__global__ void __launch_bounds__(256) k_hist(HistArgs a, float* __restrict__ hist_part) {
    __shared__ float h[HIST_BINS * 256];
    const int t = threadIdx.x;
    for (int b = 0; b < HIST_BINS; ++b) h[b * 256 + t] = 0.0f;
    const long long stride = (long long)gridDim.x * 256, first = (long long)blockIdx.x * 256 + t;
    long long done = 0;
    if (((size_t)a.I & 15) == 0) {
        const float4* __restrict__ I4 = (const float4*)a.I;
        const long long n4 = a.N / 4;
        for (long long q = first; q < n4; q += stride) {
            const float4 v = I4[q];
            hist_add(a, h, t, v.x);
            hist_add(a, h, t, v.y);
            hist_add(a, h, t, v.z);
            hist_add(a, h, t, v.w);
        }
        done = 4 * n4;
    }
    for (long long idx = done + first; idx < a.N; idx += stride) hist_add(a, h, t, a.I[idx]);
    __syncthreads();
    // pairwise tree over the 256 threads' histograms, all 64 bins at once
    for (int w = 128; w > 0; w >>= 1) {
        for (int e = t; e < HIST_BINS * w; e += 256) {
            const int b = e / w, q = e % w;
            h[b * 256 + q] += h[b * 256 + q + w];
        }
        __syncthreads();
    }
    if (t < HIST_BINS) hist_part[(long long)t * gridDim.x + blockIdx.x] = h[t * 256];
}

// hist[b] = sum over blocks of the per-block partials (one block per bin, fixed-order tree)
__global__ void __launch_bounds__(256) k_hist_reduce(const float* __restrict__ hist_part, int nparts,
                                                     float* __restrict__ hist) {
    __shared__ float sh[256];
    const int b = blockIdx.x;
    float v = 0.0f;
    for (int p = threadIdx.x; p < nparts; p += 256) v += hist_part[(long long)b * nparts + p];
    const float s = block_sum(v, sh);
    if (threadIdx.x == 0) hist[b] = s;
}

// coef[64..127] = dH/dh_b; hist[128] = H (sums over the bins by fixed-order trees)
__global__ void __launch_bounds__(64) k_hist_final(float* __restrict__ hist) {
    __shared__ float sh[64], zs[64], hs[64];
    const int b = threadIdx.x;
    const float h = hist[b];
    sh[b] = h;
    zs[b] = h;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (b < w) zs[b] += zs[b + w];
        __syncthreads();
    }
    const float Z = zs[0];
    hs[b] = (h > 0.0f && Z > 0.0f) ? -(h / Z) * logf(h / Z) : 0.0f;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (b < w) hs[b] += hs[b + w];
        __syncthreads();
    }
    const float H = hs[0];
    float coef = 0.0f;
    if (h > 0.0f && Z > 0.0f) coef = -(logf(h / Z) + H) / Z;
    hist[HIST_BINS + b] = coef;
    if (b == 0) hist[2 * HIST_BINS] = H;
}

struct GradArgs {
    const float* I;
    float* grad;
    const float* hist;    // coef at [64..127]
    float* part;          // [3][nblocks]: TV, |gH|^2, |gTV|^2
    int nx, ny, nz;
    float lo, inv_d, eps2, lambda;
};

// One thread per run of four voxels along z (k = 4 kq .. 4 kq + 3 of column (i, j)); all the
// loads of a run are issued before the arithmetic. The TV seed of a voxel needs the norms at
// the voxel and at its three backward neighbours; along z the backward neighbour's norm is the
// previous voxel's own, so a run forms 13 norms for 4 voxels. Values outside the grid are never
// read (each load is guarded by the index test that makes its difference count).
template <typename IDX, bool VEC>
__global__ void __launch_bounds__(256) k_entropy_tv_grad(GradArgs a) {
    __shared__ float coef[HIST_BINS];
    __shared__ float sh[256];
    if (threadIdx.x < HIST_BINS) coef[threadIdx.x] = a.hist[HIST_BINS + threadIdx.x];
    __syncthreads();
    const float* __restrict__ I = a.I;
    float* __restrict__ G = a.grad;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long sx = (long long)ny * nz, sy = nz;
    const IDX nzq = (IDX)((nz + 3) / 4);
    const IDX nq = (IDX)nx * (IDX)ny * nzq;
    float tv = 0.0f, gh2 = 0.0f, gt2 = 0.0f;
    for (IDX q = (IDX)blockIdx.x * 256 + threadIdx.x; q < nq; q += (IDX)gridDim.x * 256) {
        const IDX col = q / nzq;
        const int k = 4 * (int)(q - col * nzq);
        const int i = (int)(col / (IDX)ny), j = (int)(col - (IDX)i * (IDX)ny);
        const long long base = (long long)col * nz + k;
        const bool xp = i + 1 < nx, yp = j + 1 < ny, xm = i > 0, ym = j > 0, zm = k > 0;
        // columns, index m = voxel k + m (m = -1 .. 4 where used)
        float C[6], XP[5], YP[5], XM[5], YM[5], XMYP[4], XPYM[4];
        if (VEC) {
            // nz % 4 == 0 and a 16-byte aligned volume: every run is four aligned floats
            const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            auto run = [&](long long off, bool ok) { return ok ? *(const float4*)(I + off) : z4; };
            const float4 c4 = run(base, true), xp4 = run(base + sx, xp), yp4 = run(base + sy, yp);
            const float4 xm4 = run(base - sx, xm), ym4 = run(base - sy, ym);
            const float4 xmyp4 = run(base - sx + sy, xm && yp), xpym4 = run(base + sx - sy, xp && ym);
            const bool z4p = k + 4 < nz;
            C[0] = zm ? I[base - 1] : 0.0f;
            C[1] = c4.x; C[2] = c4.y; C[3] = c4.z; C[4] = c4.w;
            C[5] = z4p ? I[base + 4] : 0.0f;
            XP[0] = (zm && xp) ? I[base + sx - 1] : 0.0f;
            XP[1] = xp4.x; XP[2] = xp4.y; XP[3] = xp4.z; XP[4] = xp4.w;
            YP[0] = (zm && yp) ? I[base + sy - 1] : 0.0f;
            YP[1] = yp4.x; YP[2] = yp4.y; YP[3] = yp4.z; YP[4] = yp4.w;
            XM[0] = xm4.x; XM[1] = xm4.y; XM[2] = xm4.z; XM[3] = xm4.w;
            XM[4] = (z4p && xm) ? I[base - sx + 4] : 0.0f;
            YM[0] = ym4.x; YM[1] = ym4.y; YM[2] = ym4.z; YM[3] = ym4.w;
            YM[4] = (z4p && ym) ? I[base - sy + 4] : 0.0f;
            XMYP[0] = xmyp4.x; XMYP[1] = xmyp4.y; XMYP[2] = xmyp4.z; XMYP[3] = xmyp4.w;
            XPYM[0] = xpym4.x; XPYM[1] = xpym4.y; XPYM[2] = xpym4.z; XPYM[3] = xpym4.w;
        } else {
#pragma unroll
        for (int m = -1; m <= 4; ++m) {
            const bool in = k + m < nz && (m >= 0 || zm);
            C[m + 1] = in ? I[base + m] : 0.0f;
            if (m <= 3) {
                XP[m + 1] = (in && xp) ? I[base + sx + m] : 0.0f;
                YP[m + 1] = (in && yp) ? I[base + sy + m] : 0.0f;
            }
            if (m >= 0) {
                XM[m] = (in && xm) ? I[base - sx + m] : 0.0f;
                YM[m] = (in && ym) ? I[base - sy + m] : 0.0f;
                if (m <= 3) {
                    XMYP[m] = (in && xm && yp) ? I[base - sx + sy + m] : 0.0f;
                    XPYM[m] = (in && xp && ym) ? I[base + sx - sy + m] : 0.0f;
                }
            }
        }
        }
        // own norm of voxel k - 1 (the z-neighbour of voxel k)
        float prev_n = 1.0f, prev_dz = 0.0f;
        if (zm) {
            const float c = C[0];
            const float dxv = xp ? XP[0] - c : 0.0f, dyv = yp ? YP[0] - c : 0.0f, dzv = C[1] - c;
            prev_n = sqrtf(fmaf(dxv, dxv, fmaf(dyv, dyv, fmaf(dzv, dzv, a.eps2))));
            prev_dz = dzv;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int kk = k + m;
            if (kk >= nz) break;
            const float c = C[m + 1];
            // entropy seed
            const float s = (c - a.lo) * a.inv_d - 0.5f;
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
            const bool zp = kk + 1 < nz;
            const float dx0 = xp ? XP[m + 1] - c : 0.0f, dy0 = yp ? YP[m + 1] - c : 0.0f;
            const float dz0 = zp ? C[m + 2] - c : 0.0f;
            const float n0 = sqrtf(fmaf(dx0, dx0, fmaf(dy0, dy0, fmaf(dz0, dz0, a.eps2))));
            float gt = -(dx0 + dy0 + dz0) / n0;
            if (xm) {   // norm at (i-1, j, kk)
                const float p = c - XM[m], qq = yp ? XMYP[m] - XM[m] : 0.0f, r = zp ? XM[m + 1] - XM[m] : 0.0f;
                gt += p / sqrtf(fmaf(p, p, fmaf(qq, qq, fmaf(r, r, a.eps2))));
            }
            if (ym) {   // norm at (i, j-1, kk)
                const float p = xp ? XPYM[m] - YM[m] : 0.0f, qq = c - YM[m], r = zp ? YM[m + 1] - YM[m] : 0.0f;
                gt += qq / sqrtf(fmaf(p, p, fmaf(qq, qq, fmaf(r, r, a.eps2))));
            }
            if (kk > 0) gt += prev_dz / prev_n;   // norm at (i, j, kk-1)
            G[base + m] = fmaf(a.lambda, gt, gh);
            tv += n0;
            gh2 = fmaf(gh, gh, gh2);
            gt2 = fmaf(gt, gt, gt2);
            prev_n = n0;
            prev_dz = dz0;
        }
    }
    const float b0 = block_sum(tv, sh);
    const float b1 = block_sum(gh2, sh);
    const float b2 = block_sum(gt2, sh);
    if (threadIdx.x == 0) {
        a.part[blockIdx.x] = b0;
        a.part[gridDim.x + blockIdx.x] = b1;
        a.part[2 * gridDim.x + blockIdx.x] = b2;
    }
}

__global__ void k_entropy_tv_final(const float* __restrict__ sums, const float* __restrict__ hist, float lambda,
                                   double* __restrict__ loss) {
    const float H = hist[2 * HIST_BINS];
    loss[0] = (double)fmaf(lambda, sums[0], H);
    loss[1] = (double)H;
    loss[2] = (double)sums[0];
    loss[3] = (double)sums[1];
    loss[4] = (double)sums[2];
}

hipError_t launch_loss_entropy_tv(const gmc_plan* p, const float* vol, double lambda, double lo, double hi,
                                  double eps, float* grad, float* scratch, float* hist, double* loss,
                                  hipStream_t s) {
    const long long N = (long long)p->g.nx * p->g.ny * p->g.nz;
    const float inv_d = (float)((double)HIST_BINS / (hi - lo));
    HistArgs ha{vol, N, (float)lo, inv_d};
    // hist scratch: [64][HIST_BLOCKS] partials, then 129 finals
    float* hist_part = hist;
    float* hist_final = hist + (long long)HIST_BINS * HIST_BLOCKS;
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
    const long long n_runs = (long long)p->g.nx * p->g.ny * ((p->g.nz + 3) / 4);
    const bool vec = p->g.nz % 4 == 0 && ((size_t)vol & 15) == 0;
    if (n_runs < (1LL << 31)) {
        if (vec)
            k_entropy_tv_grad<unsigned, true><<<LOSS_BLOCKS, 256, 0, s>>>(ga);
        else
            k_entropy_tv_grad<unsigned, false><<<LOSS_BLOCKS, 256, 0, s>>>(ga);
    } else {
        if (vec)
            k_entropy_tv_grad<unsigned long long, true><<<LOSS_BLOCKS, 256, 0, s>>>(ga);
        else
            k_entropy_tv_grad<unsigned long long, false><<<LOSS_BLOCKS, 256, 0, s>>>(ga);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float* sums = scratch + 3 * LOSS_BLOCKS;
    k_sum_cols<<<1, 256, 0, s>>>(scratch, LOSS_BLOCKS, 3, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_entropy_tv_final<<<1, 1, 0, s>>>(sums, hist_final, (float)lambda, loss);
    return hipGetLastError();
}

}  // namespace gmc
