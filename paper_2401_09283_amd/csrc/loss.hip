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

// Per-thread private histograms in LDS ([bin][thread], conflict free), 128 threads per block
// so that a block's 64 bins take 32 KB (five blocks per CU) and the bins b and b + 1 of a
// thread lie 128 words apart, one `ds_read2_b32` / `ds_write2_b32` pair each; summed per block
// by a fixed-order tree (thread t of the first 64 sums bin t). The window's weights at the four
// bins b0 - 1 .. b0 + 2 around a value are polynomials in its fraction f. Voxels are read four
// at a time where the volume is 16-byte aligned.
constexpr int HIST_THREADS = 128;

__device__ __forceinline__ void hist_add(const HistArgs& a, float* h, int t, float x) {
    const float s = (x - a.lo) * a.inv_d - 0.5f;
    const float fb = floorf(s);
    if (!(fb > -3.0f && fb < (float)HIST_BINS + 1.0f)) return;
    const int b0 = (int)fb;
    const float f = s - fb, g = 1.0f - f;
    const float w[4] = {g * g * g * (1.0f / 6.0f), fmaf(f * f, fmaf(0.5f, f, -1.0f), 2.0f / 3.0f),
                        fmaf(g * g, fmaf(0.5f, g, -1.0f), 2.0f / 3.0f), f * f * f * (1.0f / 6.0f)};
    if (b0 >= 1 && b0 <= HIST_BINS - 3) {
        float* p = h + (b0 - 1) * HIST_THREADS + t;
#pragma unroll
        for (int o = 0; o < 4; ++o) p[o * HIST_THREADS] += w[o];
    } else {
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int b = b0 - 1 + o;
            if (b >= 0 && b < HIST_BINS) h[b * HIST_THREADS + t] += w[o];
        }
    }
}

__global__ void __launch_bounds__(HIST_THREADS) k_hist(HistArgs a, float* __restrict__ hist_part) {
    __shared__ float h[HIST_BINS * HIST_THREADS];
    const int t = threadIdx.x;
    for (int b = 0; b < HIST_BINS; ++b) h[b * HIST_THREADS + t] = 0.0f;
    const long long stride = (long long)gridDim.x * HIST_THREADS, first = (long long)blockIdx.x * HIST_THREADS + t;
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
    // pairwise tree over the block's private histograms, all 64 bins at once
    for (int w = HIST_THREADS / 2; w > 0; w >>= 1) {
        for (int e = t; e < HIST_BINS * w; e += HIST_THREADS) {
            const int b = e / w, q = e % w;
            h[b * HIST_THREADS + q] += h[b * HIST_THREADS + q + w];
        }
        __syncthreads();
    }
    if (t < HIST_BINS) hist_part[(long long)t * gridDim.x + blockIdx.x] = h[t * HIST_THREADS];
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

// Tiles of 8 x 8 columns x 32 voxels along z. A block loads the tile and a one-voxel halo on
// every side (10 x 10 x 34 values, zero outside the grid) into LDS with loads coalesced along
// z, then computes the seeds of the tile's voxels from LDS: thread t takes z = t mod 32 and
// every eighth column of the tile, so that a wavefront's stores cover two columns of 32
// contiguous voxels. The TV seed of a voxel needs the norms at the voxel and at its three
// backward neighbours (13 values of the halo box); a difference that leaves the grid counts as
// 0, as in the definition. Norms come as reciprocal square roots (`v_rsq_f32`, about one ulp).
// Blocks stride over the tiles.
constexpr int TVX = 8, TVY = 8, TVZ = 32;
constexpr int TVBX = TVX + 2, TVBY = TVY + 2, TVBZ = TVZ + 2;

__global__ void __launch_bounds__(256) k_entropy_tv_grad(GradArgs a) {
    // coef[3 + b] = dH/dh_b for the 64 bins, 0 for the three bins on either side (the window of
    // a value in (-3, 65) bin widths reaches bins -3 .. 66; bins outside the range hold nothing)
    __shared__ float coef[HIST_BINS + 6];
    __shared__ float sh[256];
    __shared__ float box[TVBX * TVBY * TVBZ];
    const int t = threadIdx.x;
    if (t < HIST_BINS + 6) coef[t] = (t >= 3 && t < HIST_BINS + 3) ? a.hist[HIST_BINS + t - 3] : 0.0f;
    const float* __restrict__ I = a.I;
    float* __restrict__ G = a.grad;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long sx = (long long)ny * nz;
    const int ntx = (nx + TVX - 1) / TVX, nty = (ny + TVY - 1) / TVY, ntz = (nz + TVZ - 1) / TVZ;
    const long long n_tiles = (long long)ntx * nty * ntz;
    auto S = [&](int xl, int yl, int zl) { return box[(xl * TVBY + yl) * TVBZ + zl]; };
    float tv = 0.0f, gh2 = 0.0f, gt2 = 0.0f;
    for (long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int tz = (int)(tile % ntz);
        const long long txy = tile / ntz;
        const int ty = (int)(txy % nty), tx = (int)(txy / nty);
        const int i0 = tx * TVX, j0 = ty * TVY, k0 = tz * TVZ;
        __syncthreads();   // the previous tile's reads of box are done (and coef is in place)
        for (int e = t; e < TVBX * TVBY * TVBZ; e += 256) {
            const int zl = e % TVBZ, xy = e / TVBZ;
            const int yl = xy % TVBY, xl = xy / TVBY;
            const int i = i0 - 1 + xl, j = j0 - 1 + yl, k = k0 - 1 + zl;
            const bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny && (unsigned)k < (unsigned)nz;
            box[e] = in ? I[(long long)i * sx + (long long)j * nz + k] : 0.0f;
        }
        __syncthreads();
        const int zl = (t & 31) + 1, k = k0 + (t & 31);
        if (k >= nz) continue;
        const bool zp = k + 1 < nz, zm = k > 0;
#pragma unroll 2
        for (int cidx = t >> 5; cidx < TVX * TVY; cidx += 8) {
            const int xl = (cidx >> 3) + 1, yl = (cidx & 7) + 1;
            const int i = i0 + xl - 1, j = j0 + yl - 1;
            if (i >= nx || j >= ny) continue;
            const bool xp = i + 1 < nx, yp = j + 1 < ny, xm = i > 0, ym = j > 0;
            const float c = S(xl, yl, zl);
            // entropy seed: the window's derivative at the four bins b0 - 1 .. b0 + 2 around
            // the value, as polynomials in its fraction f (those of db3 at f + 1, f, f - 1, f - 2)
            const float sv = (c - a.lo) * a.inv_d - 0.5f;
            const float fb = floorf(sv);
            float gh = 0.0f;
            if (fb > -3.0f && fb < (float)HIST_BINS + 1.0f) {
                const int b0 = (int)fb + 3;
                const float f = sv - fb, g = 1.0f - f;
                gh = fmaf(coef[b0 - 1], -0.5f * g * g, fmaf(coef[b0], f * fmaf(1.5f, f, -2.0f),
                          fmaf(coef[b0 + 1], -g * fmaf(1.5f, g, -2.0f), coef[b0 + 2] * (0.5f * f * f))));
            }
            gh *= a.inv_d;
            // TV seed: own term and the terms at the three backward neighbours
            const float dx0 = xp ? S(xl + 1, yl, zl) - c : 0.0f, dy0 = yp ? S(xl, yl + 1, zl) - c : 0.0f;
            const float dz0 = zp ? S(xl, yl, zl + 1) - c : 0.0f;
            const float s0 = fmaf(dx0, dx0, fmaf(dy0, dy0, fmaf(dz0, dz0, a.eps2)));
            const float rn0 = __builtin_amdgcn_rsqf(s0), n0 = s0 * rn0;
            float gt = -(dx0 + dy0 + dz0) * rn0;
            if (xm) {   // norm at (i-1, j, k)
                const float m = S(xl - 1, yl, zl);
                const float p = c - m, q = yp ? S(xl - 1, yl + 1, zl) - m : 0.0f, r = zp ? S(xl - 1, yl, zl + 1) - m : 0.0f;
                gt = fmaf(p, __builtin_amdgcn_rsqf(fmaf(p, p, fmaf(q, q, fmaf(r, r, a.eps2)))), gt);
            }
            if (ym) {   // norm at (i, j-1, k)
                const float m = S(xl, yl - 1, zl);
                const float p = xp ? S(xl + 1, yl - 1, zl) - m : 0.0f, q = c - m, r = zp ? S(xl, yl - 1, zl + 1) - m : 0.0f;
                gt = fmaf(q, __builtin_amdgcn_rsqf(fmaf(p, p, fmaf(q, q, fmaf(r, r, a.eps2)))), gt);
            }
            if (zm) {   // norm at (i, j, k-1)
                const float m = S(xl, yl, zl - 1);
                const float p = xp ? S(xl + 1, yl, zl - 1) - m : 0.0f, q = yp ? S(xl, yl + 1, zl - 1) - m : 0.0f, r = c - m;
                gt = fmaf(r, __builtin_amdgcn_rsqf(fmaf(p, p, fmaf(q, q, fmaf(r, r, a.eps2)))), gt);
            }
            G[(long long)i * sx + (long long)j * nz + k] = fmaf(a.lambda, gt, gh);
            tv += n0;
            gh2 = fmaf(gh, gh, gh2);
            gt2 = fmaf(gt, gt, gt2);
        }
    }
    const float b0 = block_sum(tv, sh);
    const float b1 = block_sum(gh2, sh);
    const float b2 = block_sum(gt2, sh);
    if (t == 0) {
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
    k_hist<<<HIST_BLOCKS, HIST_THREADS, 0, s>>>(ha, hist_part);
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
    float* sums = scratch + 3 * LOSS_BLOCKS;
    k_sum_cols<<<1, 256, 0, s>>>(scratch, LOSS_BLOCKS, 3, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_entropy_tv_final<<<1, 1, 0, s>>>(sums, hist_final, (float)lambda, loss);
    return hipGetLastError();
}

}  // namespace gmc
