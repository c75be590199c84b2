// Voxel-driven backprojection (Eq. 3) and its Jacobian-vector product (Eq. 4-5) on gfx950.
//
// One workgroup of 256 threads owns a brick of 16 x 16 x BZ voxels; thread (li, lj) owns the
// column of BZ voxels at (li, lj). For every view the workgroup stages the brick's detector
// tile in LDS (the filtered projection with a one-pixel halo and, for the VJP, the two
// central-difference images of Sec. II-B.2 computed from it), then every thread walks its
// column: homogeneous position by FMA from the column base, one reciprocal, bilinear taps
// from LDS. The forward pass accumulates its BZ voxels in registers over all views and
// writes them once (z fastest). The VJP keeps the seed of its BZ voxels in registers, sums
// the per-sample row coefficients of Eq. 4 (6 running sums per thread, since x and y are
// constant along a column), reduces them over the workgroup with DPP at the end of each
// view and writes one 12-entry partial per (view, brick); k_reduce_chain finishes the sum.
//
// Workgroups are mapped to bricks so that each XCD (workgroup id mod 8) takes a contiguous
// range of z-slabs: its L2 then holds only the detector rows those slabs project to.
#include "gmc_internal.hpp"

namespace gmc {

namespace {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wavefront; the total ends in lane 63.
__device__ __forceinline__ float wave_sum_to_last(float v) {
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x124, 0xF>(v);  // row_ror:4
    v = dpp_add<0x128, 0xF>(v);  // row_ror:8
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

__device__ __forceinline__ float pix(const float* __restrict__ img, int W, int H, int r, int c) {
    return ((unsigned)r < (unsigned)H && (unsigned)c < (unsigned)W) ? img[(long long)r * W + c] : 0.0f;
}

// Twice the central-difference image along u at pixel (r, c): d[c+1] - d[c-1] inside,
// 2 (d[1] - d[0]) and 2 (d[W-1] - d[W-2]) on the border, 0 outside the detector.
__device__ __forceinline__ float grad_u2(float le, float ce, float ri, int c, int W) {
    if (W < 2) return 0.0f;
    if (c == 0) return 2.0f * (ri - ce);
    if (c == W - 1) return 2.0f * (ce - le);
    return ri - le;
}

struct Taps {
    float d00, d01, d10, d11;
    float u00, u01, u10, u11;   // 2 g_u
    float v00, v01, v10, v11;   // 2 g_v
};

// Global-memory sampler (tiles too large for LDS): same values as the LDS tile.
template <bool GRADS>
__device__ __forceinline__ void fetch_global(const float* __restrict__ img, int W, int H, int r, int c, Taps& t) {
    t.d00 = pix(img, W, H, r, c);
    t.d01 = pix(img, W, H, r, c + 1);
    t.d10 = pix(img, W, H, r + 1, c);
    t.d11 = pix(img, W, H, r + 1, c + 1);
    if (!GRADS) return;
    auto gu = [&](int rr, int cc) {
        if ((unsigned)rr >= (unsigned)H || (unsigned)cc >= (unsigned)W) return 0.0f;
        return grad_u2(pix(img, W, H, rr, cc - 1), pix(img, W, H, rr, cc), pix(img, W, H, rr, cc + 1), cc, W);
    };
    auto gv = [&](int rr, int cc) {
        if ((unsigned)rr >= (unsigned)H || (unsigned)cc >= (unsigned)W) return 0.0f;
        return grad_u2(pix(img, W, H, rr - 1, cc), pix(img, W, H, rr, cc), pix(img, W, H, rr + 1, cc), rr, H);
    };
    t.u00 = gu(r, c); t.u01 = gu(r, c + 1); t.u10 = gu(r + 1, c); t.u11 = gu(r + 1, c + 1);
    t.v00 = gv(r, c); t.v01 = gv(r, c + 1); t.v10 = gv(r + 1, c); t.v11 = gv(r + 1, c + 1);
}

}  // namespace

// WEIGHT: GMC_WEIGHT_*; GRAD: GMC_GRAD_*; VJP: false = Eq. 3, true = Eq. 4-5.
template <int TP, int TH, int BZ, int WEIGHT, int GRAD, bool VJP>
__global__ void __launch_bounds__(THREADS) k_bp(BpArgs a) {
    constexpr bool PLANES = VJP && GRAD == GMC_GRAD_PAPER;   // stage the gradient images
    constexpr int PLANE = TP * TH;
    __shared__ float sD[PLANE];
    __shared__ float sG[PLANES ? 2 * PLANE : 1];
    __shared__ float sRed[VJP ? 2 * 4 * 12 : 1];

    const int blk = blockIdx.x;
    const int brick = (blk & 7) * a.per_xcd + (blk >> 3);
    if (brick >= a.n_bricks) return;
    const int bj = brick % a.nby;
    const int bi = (brick / a.nby) % a.nbx;
    const int bk = brick / (a.nby * a.nbx);

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int li = t >> 4, lj = t & 15;
    const int i = bi * BXY + li, j = bj * BXY + lj, k0 = bk * BZ;
    const bool col_in = (i < a.nx) && (j < a.ny);
    const float qx = (float)li * a.dx, qy = (float)lj * a.dy, dz = a.dz;
    const long long col_off = ((long long)i * a.ny + j) * a.nz + k0;

    float acc[BZ];
    float seed[VJP ? BZ : 1];
    if (VJP) {
        // the paper gradient planes hold 2 g; fold the 1/2 into the seed
        const float sc = (GRAD == GMC_GRAD_PAPER) ? 0.5f : 1.0f;
#pragma unroll
        for (int k = 0; k < BZ; ++k) seed[k] = (col_in && k0 + k < a.nz) ? sc * a.gvol[col_off + k] : 0.0f;
    } else {
#pragma unroll
        for (int k = 0; k < BZ; ++k) acc[k] = 0.0f;
    }

    int prev_ou = 0, prev_ov = 0;
    for (int v = 0; v < a.n_views; ++v) {
        const BrickDesc* D = a.desc + (long long)v * a.n_bricks + brick;
        float m[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) m[e] = __builtin_nontemporal_load(&D->m[e]);
        const int ou = D->ou, ov = D->ov, tw = D->tw, th = D->th;

        __syncthreads();   // previous view's LDS reads are done
        if (VJP && v > 0 && t < 14) {
            float s;
            if (t < 12) {
                const float* rb = sRed + ((v - 1) & 1) * 48;
                s = ((rb[t] + rb[12 + t]) + rb[24 + t]) + rb[36 + t];
            } else {
                s = __int_as_float(t == 12 ? prev_ou : prev_ov);
            }
            a.part[((long long)(v - 1) * a.n_bricks + brick) * PART_STRIDE + t] = s;
        }
        prev_ou = ou;
        prev_ov = ov;

        float S0 = 0.f, S1 = 0.f, S2 = 0.f, T0 = 0.f, T1 = 0.f, T2 = 0.f;
        if (tw != 0) {
            const float* img = a.proj + (long long)v * a.plane;
            const bool lds = tw > 0;
            if (lds) {
                for (int r = wave; r < th; r += 4) {
                    const int gr = ov + r;
                    const bool rin = (unsigned)gr < (unsigned)a.H;
                    for (int c = lane; c < tw; c += 64) {
                        const int gc = ou + c;
                        float val = 0.0f;
                        if (rin && (unsigned)gc < (unsigned)a.W) val = img[(long long)gr * a.W + gc];
                        sD[r * TP + c] = val;
                    }
                }
                __syncthreads();
                if (PLANES) {
                    for (int r = 1 + wave; r < th - 1; r += 4) {
                        const int gr = ov + r;
                        const bool rin = (unsigned)gr < (unsigned)a.H;
                        for (int c = 1 + lane; c < tw - 1; c += 64) {
                            const int gc = ou + c;
                            float gu = 0.0f, gv = 0.0f;
                            if (rin && (unsigned)gc < (unsigned)a.W) {
                                const float ce = sD[r * TP + c];
                                gu = grad_u2(sD[r * TP + c - 1], ce, sD[r * TP + c + 1], gc, a.W);
                                gv = grad_u2(sD[(r - 1) * TP + c], ce, sD[(r + 1) * TP + c], gr, a.H);
                            }
                            sG[r * TP + c] = gu;
                            sG[PLANE + r * TP + c] = gv;
                        }
                    }
                    __syncthreads();
                }
            }
            const int twa = lds ? tw : -tw;
            const float ub = fmaf(m[0], qx, fmaf(m[1], qy, m[3]));
            const float vb = fmaf(m[4], qx, fmaf(m[5], qy, m[7]));
            const float wb = fmaf(m[8], qx, fmaf(m[9], qy, m[11]));
            const float du = m[2] * dz, dv = m[6] * dz, dw = m[10] * dz;
#pragma unroll
            for (int k = 0; k < BZ; ++k) {
                const float kf = (float)k;
                const float u = fmaf(kf, du, ub), vv = fmaf(kf, dv, vb), w = fmaf(kf, dw, wb);
                const float rw = __builtin_amdgcn_rcpf(w);
                const float uh = u * rw, vh = vv * rw;
                const float fu = floorf(uh), fv = floorf(vh);
                const float au = uh - fu, av = vh - fv;
                Taps tp;
                if (lds) {
                    const int ci = min(max((int)fu, 1), twa - 3);
                    const int ri = min(max((int)fv, 1), th - 3);
                    const int idx = ri * TP + ci;
                    tp.d00 = sD[idx]; tp.d01 = sD[idx + 1]; tp.d10 = sD[idx + TP]; tp.d11 = sD[idx + TP + 1];
                    if (PLANES) {
                        tp.u00 = sG[idx]; tp.u01 = sG[idx + 1]; tp.u10 = sG[idx + TP]; tp.u11 = sG[idx + TP + 1];
                        tp.v00 = sG[PLANE + idx]; tp.v01 = sG[PLANE + idx + 1];
                        tp.v10 = sG[PLANE + idx + TP]; tp.v11 = sG[PLANE + idx + TP + 1];
                    }
                } else {
                    fetch_global<PLANES>(img, a.W, a.H, (int)fv + ov, (int)fu + ou, tp);
                }
                const float e0 = tp.d01 - tp.d00, e1 = tp.d11 - tp.d10;
                const float top = fmaf(au, e0, tp.d00), bot = fmaf(au, e1, tp.d10);
                const float dtb = bot - top;
                const float val = fmaf(av, dtb, top);
                if (!VJP) {
                    acc[k] += (WEIGHT == GMC_WEIGHT_FDK) ? val * (rw * rw) : val;
                } else {
                    float gu, gv;
                    if (PLANES) {
                        const float ut = fmaf(au, tp.u01 - tp.u00, tp.u00), ubm = fmaf(au, tp.u11 - tp.u10, tp.u10);
                        gu = fmaf(av, ubm - ut, ut);
                        const float vt = fmaf(au, tp.v01 - tp.v00, tp.v00), vbm = fmaf(au, tp.v11 - tp.v10, tp.v10);
                        gv = fmaf(av, vbm - vt, vt);
                    } else {
                        // derivative of the bilinear interpolant
                        gu = fmaf(av, e1 - e0, e0);
                        gv = dtb;
                    }
                    // A = (g_u, g_v, -(g_u uh + g_v vh [+ 2 val])) scaled by seed / w (paper) or seed / w^3 (FDK);
                    // with the paper planes g is doubled and the seed halved, so the value term is 4 val
                    float e, tt;
                    if (WEIGHT == GMC_WEIGHT_FDK) {
                        e = seed[k] * (rw * rw * rw);
                        tt = fmaf(gu, uh, fmaf(gv, vh, (GRAD == GMC_GRAD_PAPER ? 4.0f : 2.0f) * val));
                    } else {
                        e = seed[k] * rw;
                        tt = fmaf(gu, uh, gv * vh);
                    }
                    const float ek = e * kf;
                    S0 = fmaf(e, gu, S0);
                    S1 = fmaf(e, gv, S1);
                    S2 = fmaf(e, tt, S2);
                    T0 = fmaf(ek, gu, T0);
                    T1 = fmaf(ek, gv, T1);
                    T2 = fmaf(ek, tt, T2);
                }
            }
        }
        if (VJP) {
            // G'' rows r: (qx S_r, qy S_r, dz T_r, S_r); row 2 carries the minus sign of Eq. 4
            float g[12] = {qx * S0, qy * S0, dz * T0, S0, qx * S1, qy * S1, dz * T1, S1,
                           -qx * S2, -qy * S2, -dz * T2, -S2};
#pragma unroll
            for (int e = 0; e < 12; ++e) g[e] = wave_sum_to_last(g[e]);
            if (lane == 63) {
                float* rb = sRed + (v & 1) * 48 + wave * 12;
#pragma unroll
                for (int e = 0; e < 12; ++e) rb[e] = g[e];
            }
        }
    }

    if (VJP) {
        __syncthreads();
        const int v = a.n_views;
        if (v > 0 && t < 14) {
            float s;
            if (t < 12) {
                const float* rb = sRed + ((v - 1) & 1) * 48;
                s = ((rb[t] + rb[12 + t]) + rb[24 + t]) + rb[36 + t];
            } else {
                s = __int_as_float(t == 12 ? prev_ou : prev_ov);
            }
            a.part[((long long)(v - 1) * a.n_bricks + brick) * PART_STRIDE + t] = s;
        }
    } else if (col_in) {
        float* out = a.vol + col_off;
#pragma unroll
        for (int k = 0; k < BZ; ++k)
            if (k0 + k < a.nz) out[k] = acc[k];
    }
}

namespace {

template <int TP, int TH, int BZ>
hipError_t launch_cfg(const gmc_plan* p, const BpArgs& a, bool vjp, hipStream_t s) {
    const unsigned grid = 8u * (unsigned)a.per_xcd;
    const int W = p->g.weighting, G = p->g.grad_mode;
    if (!vjp) {
        if (W == GMC_WEIGHT_FDK)
            k_bp<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_PAPER, false><<<grid, THREADS, 0, s>>>(a);
        else
            k_bp<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_PAPER, false><<<grid, THREADS, 0, s>>>(a);
    } else {
        if (W == GMC_WEIGHT_FDK && G == GMC_GRAD_PAPER)
            k_bp<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_PAPER, true><<<grid, THREADS, 0, s>>>(a);
        else if (W == GMC_WEIGHT_FDK)
            k_bp<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_EXACT, true><<<grid, THREADS, 0, s>>>(a);
        else if (G == GMC_GRAD_PAPER)
            k_bp<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_PAPER, true><<<grid, THREADS, 0, s>>>(a);
        else
            k_bp<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_EXACT, true><<<grid, THREADS, 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bp(const gmc_plan* p, const BpArgs& a, bool vjp, hipStream_t s) {
    if (p->bz != 16) return hipErrorInvalidValue;
    switch (p->tile_cfg) {
        case 0: return launch_cfg<TILE_CFGS[0].tp, TILE_CFGS[0].th, 16>(p, a, vjp, s);
        case 1: return launch_cfg<TILE_CFGS[1].tp, TILE_CFGS[1].th, 16>(p, a, vjp, s);
        case 2: return launch_cfg<TILE_CFGS[2].tp, TILE_CFGS[2].th, 16>(p, a, vjp, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- geometry-index check
__global__ void k_debug_project(const BrickDesc* __restrict__ desc, int n_bricks, int n_views, int nbx, int nby,
                                int nx, int ny, int nz, int bz, float dx, float dy, float dz, long long n,
                                const int64_t* __restrict__ voxel, const int32_t* __restrict__ view,
                                int32_t* __restrict__ cell, float* __restrict__ frac) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const long long L = voxel[q];
    const int vw = view[q];
    if (L < 0 || L >= (long long)nx * ny * nz || vw < 0 || vw >= n_views) {
        cell[2 * q] = cell[2 * q + 1] = INT32_MIN;
        frac[2 * q] = frac[2 * q + 1] = -1.0f;
        return;
    }
    const int k = (int)(L % nz), j = (int)((L / nz) % ny), i = (int)(L / ((long long)nz * ny));
    const int bi = i / BXY, bj = j / BXY, bk = k / bz;
    const int li = i % BXY, lj = j % BXY, kk = k % bz;
    const int brick = (bk * nbx + bi) * nby + bj;
    const BrickDesc& D = desc[(long long)vw * n_bricks + brick];
    // identical arithmetic to the sample loop of k_bp
    const float qx = (float)li * dx, qy = (float)lj * dy;
    const float ub = fmaf(D.m[0], qx, fmaf(D.m[1], qy, D.m[3]));
    const float vb = fmaf(D.m[4], qx, fmaf(D.m[5], qy, D.m[7]));
    const float wb = fmaf(D.m[8], qx, fmaf(D.m[9], qy, D.m[11]));
    const float du = D.m[2] * dz, dv = D.m[6] * dz, dw = D.m[10] * dz;
    const float kf = (float)kk;
    const float u = fmaf(kf, du, ub), vv = fmaf(kf, dv, vb), w = fmaf(kf, dw, wb);
    const float rw = __builtin_amdgcn_rcpf(w);
    const float uh = u * rw, vh = vv * rw;
    const float fu = floorf(uh), fv = floorf(vh);
    cell[2 * q] = (int)fu + D.ou;
    cell[2 * q + 1] = (int)fv + D.ov;
    frac[2 * q] = uh - fu;
    frac[2 * q + 1] = vh - fv;
}

hipError_t launch_debug_project(const gmc_plan* p, const BrickDesc* desc, long long n, const int64_t* voxel,
                                const int32_t* view, int32_t* cell, float* frac, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_debug_project<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        desc, p->n_bricks, p->g.n_views, p->nbx, p->nby, p->g.nx, p->g.ny, p->g.nz, p->bz, (float)p->g.voxel_mm[0],
        (float)p->g.voxel_mm[1], (float)p->g.voxel_mm[2], n, voxel, view, cell, frac);
    return hipGetLastError();
}

}  // namespace gmc
