// Voxel-driven backprojection (Eq. 3) and its Jacobian-vector product (Eq. 4-5) on gfx950.
//
// One workgroup of 256 threads owns a brick of 16 x 16 x BZ voxels; thread (li, lj) owns the
// column of BZ voxels at (li, lj). For every view the workgroup stages the brick's detector
// tile in LDS (the filtered projection; the VJP's tile has a one-pixel halo for the central
// differences of Sec. II-B.2, which are formed from the tile's taps on the fly), then every
// thread walks its column: homogeneous position by FMA from the column base, one reciprocal
// per column and a Newton step per sample, bilinear taps from LDS. A workgroup takes one
// item: a brick and a contiguous chunk of its views. The forward pass accumulates its BZ
// voxels in registers over the chunk's views and writes them once (z fastest; chunks after
// the first into partial volumes that are summed afterwards in chunk order). The VJP keeps
// the seed of its BZ voxels in registers, sums the per-sample row coefficients of Eq. 4 (6
// running sums per thread, since x and y are constant along a column), reduces them over the
// workgroup with cross-lane permutes at the end of each view and writes one 12-entry partial
// per (view, brick); k_reduce_chain finishes the sum.
//
// Items are numbered chunk-major and each XCD (workgroup id mod 8) takes a contiguous range
// of them: the workgroups resident on an XCD are neighbouring bricks over the same views,
// and every XCD gets a share of the whole volume (equal work).
#include "gmc_internal.hpp"

namespace gmc {

namespace {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Reduce-scatter of 12 per-lane values over the 64 lanes of a wavefront. Swapping 32-lane
// halves (v_permlane32_swap) pairs value i with i+6, swapping 16-lane rows (v_permlane16_swap)
// pairs i with i+3, and four DPP steps finish each 16-lane row. On return, every lane of row q
// (lanes 16q..16q+15) holds the wave totals of values 3q, 3q+1, 3q+2 in out[0..2].
__device__ __forceinline__ void wave_reduce12(const float g[12], float out[3]) {
    float h[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[i]), __float_as_uint(g[i + 6]), false, false);
        h[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(h[i]), __float_as_uint(h[i + 3]), false, false);
        float k = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        k = dpp_add<0xB1, 0xF>(k);   // quad_perm [1,0,3,2]
        k = dpp_add<0x4E, 0xF>(k);   // quad_perm [2,3,0,1]
        k = dpp_add<0x124, 0xF>(k);  // row_ror:4
        k = dpp_add<0x128, 0xF>(k);  // row_ror:8
        out[i] = k;
    }
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

// ---------------------------------------------------------------- per-sample arithmetic

// Positions along the thread's column. Sample k sits at (ub, vb, wb) + k (du, dv, dw) in the
// tile frame (homogeneous, one FMA per coordinate). The reciprocal depth of sample 0 comes from
// v_rcp_f32; every further sample refines its predecessor's with one Newton step,
// r_k = r_(k-1) (2 - w_k r_(k-1)), whose relative error is about (dw/w)^2 plus two roundings:
// dw/w, the relative change of depth per voxel along z, is below 1e-4 in the circular scans
// here and below 2e-3 for any cone-beam geometry with the source 500 voxels away. Samples are
// always visited in increasing k, so every path (and k_debug_project) sees the same positions.
struct Column {
    float ub, vb, wb, du, dv, dw;
    float rw;   // reciprocal depth of the last sample
};

struct Smp {
    float rw, uh, vh;
};

__device__ __forceinline__ Smp next_sample(Column& c, int k) {
    Smp s;
    if (k == 0) {
        c.rw = __builtin_amdgcn_rcpf(c.wb);
        s.rw = c.rw;
        s.uh = c.ub * s.rw;
        s.vh = c.vb * s.rw;
    } else {
        const float kf = (float)k;
        const float w = fmaf(kf, c.dw, c.wb);
        c.rw = c.rw * fmaf(-w, c.rw, 2.0f);
        s.rw = c.rw;
        s.uh = fmaf(kf, c.du, c.ub) * s.rw;
        s.vh = fmaf(kf, c.dv, c.vb) * s.rw;
    }
    return s;
}

// Cell (floor) and bilinear fraction of a tile coordinate x >= 1/2 without conversions:
// x + (2^23 - 1/2) rounds to 2^23 + floor(x) (to 2^23 + x - 1 when x is an integer; then the
// fraction is 1 and the bilinear value is the same). Every sample of a tile has tile
// coordinates >= 1 (the tile origin lies two pixels below the smallest projected corner).
constexpr int VJP_GROUP = 1;          // VJP samples whose LDS reads are issued together
constexpr int FWD_GROUP = 4;          // forward samples whose LDS reads are issued together
constexpr float RND23 = 8388607.5f;   // 2^23 - 1/2
constexpr float TWO23 = 8388608.0f;   // 2^23

struct Cell {
    float fu, fv;   // cell (integer-valued floats)
    float au, av;   // fractions in [0, 1]
    float fub;      // fu + 2^23 (its bit pattern is 0x4B000000 + fu)
};

__device__ __forceinline__ Cell cell_of(const Smp& s) {
    Cell c;
    c.fub = s.uh + RND23;
    c.fu = c.fub - TWO23;
    c.fv = (s.vh + RND23) - TWO23;
    c.au = s.uh - c.fu;
    c.av = s.vh - c.fv;
    return c;
}

// LDS byte addresses. An integer-valued float n in [0, 2^23) plus 2^23 has the bit pattern
// 0x4B000000 + n, so the address of element n of an LDS array of S-byte elements is
// (address of the array - S * 0x4B000000) + S * bits(n + 2^23), modulo 2^32: one shift-add per
// address, with the constant folded into the per-view base and the tap offsets into the
// instruction's offset fields.
typedef const __attribute__((address_space(3))) float LdsF;

__device__ __forceinline__ unsigned lds_addr(const void* p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) char*)p;
}
// per-view base for elements of `bytes` bytes
__device__ __forceinline__ unsigned lds_base(const void* p, unsigned bytes) { return lds_addr(p) - bytes * 0x4B000000u; }
__device__ __forceinline__ unsigned lds_index(unsigned base, unsigned bytes, float n) {
    return base + bytes * __float_as_uint(n + TWO23);
}
__device__ __forceinline__ LdsF* lds_f(unsigned addr) { return (LdsF*)(size_t)addr; }

// LDS address of the sample's cell (row-major, pitch TP). The linear cell is formed with the
// column's 2^23 bias already in place (fv TP + fu + 2^23, exact below 2^24), so its bits give
// the address without another add. No clamp: the tile spans the cells of the brick's projected
// corners plus one cell of margin on every side (and the halo beyond it), the projection of
// every voxel of the brick lies inside its corners' hull, and the FP32 positions differ from
// the set-up's FP64 corners by about 1e-3 pixel, so no cell leaves the margin.
template <int TP>
__device__ __forceinline__ unsigned tile_cell(const Cell& c, unsigned base) {
    return base + 4u * __float_as_uint(fmaf(c.fv, (float)TP, c.fub));
}

// Row coefficients of Eq. 4 for one sample, accumulated into the 6 running sums of the column:
// A = (g_u, g_v, g_u uh + g_v vh [+ 2 val]) * seed / w (Eq. 3 weighting) or * seed / w^3 (FDK).
// gu, gv are doubled central differences and the seed is halved (paper gradient), or exact
// bilinear derivatives with an unscaled seed (exact gradient). Samples arrive in increasing k;
// P_r += S_r after every sample but the last gives P_r = sum_k (BZ - 1 - k) A_r(k), so that the
// z-moment of the column is sum_k k A_r(k) = (BZ - 1) S_r - P_r.
template <int BZ, int WEIGHT, int GRAD>
__device__ __forceinline__ void accumulate(const Smp& p, float seed, float val, float gu, float gv, int k,
                                           float& S0, float& S1, float& S2, float& T0, float& T1, float& T2) {
    float e, tt;
    if (WEIGHT == GMC_WEIGHT_FDK) {
        e = seed * (p.rw * p.rw * p.rw);
        tt = fmaf(gu, p.uh, fmaf(gv, p.vh, (GRAD == GMC_GRAD_PAPER ? 4.0f : 2.0f) * val));
    } else {
        e = seed * p.rw;
        tt = fmaf(gu, p.uh, gv * p.vh);
    }
    S0 = fmaf(e, gu, S0);
    S1 = fmaf(e, gv, S1);
    S2 = fmaf(e, tt, S2);
    if (k == 0) {   // P starts at 0: a copy, not an add (which would also turn -0 into +0)
        T0 = S0;
        T1 = S1;
        T2 = S2;
    } else if (k < BZ - 1) {
        T0 += S0;
        T1 += S1;
        T2 += S2;
    }
}

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

// Taps of a sample whose taps, halo included, lie inside the detector (no border rule): the
// four bilinear taps and, for the paper gradient, the eight neighbours the central differences
// need. q addresses the tap at (row - 1, column - 1) of the sample's cell, so that every offset
// is positive.
struct Taps12 {
    float d00, d01, d10, d11;
    float bm, b2, cm, c2, a0, a1, f0, f1;
};

template <int TP, int GRAD, bool GRADS>
__device__ __forceinline__ void load_plain(LdsF* q, Taps12& t) {
    LdsF* b = q + TP + 1;
    t.d00 = b[0];
    t.d01 = b[1];
    t.d10 = b[TP];
    t.d11 = b[TP + 1];
    if (GRADS && GRAD == GMC_GRAD_PAPER) {
        t.bm = q[TP];
        t.b2 = q[TP + 3];
        t.cm = q[2 * TP];
        t.c2 = q[2 * TP + 3];
        t.a0 = q[1];
        t.a1 = q[2];
        t.f0 = q[3 * TP + 1];
        t.f1 = q[3 * TP + 2];
    }
}

// Bilinear value and, for the VJP, the interpolated doubled central differences (paper
// gradient) or the derivatives of the bilinear interpolant (exact gradient).
template <int GRAD, bool GRADS>
__device__ __forceinline__ void eval_plain(const Taps12& t, float au, float av, float& val, float& gu, float& gv) {
    const float e0 = t.d01 - t.d00, e1 = t.d11 - t.d10;
    const float top = fmaf(au, e0, t.d00), bot = fmaf(au, e1, t.d10);
    const float dtb = bot - top;
    val = fmaf(av, dtb, top);
    if (!GRADS) return;
    if (GRAD == GMC_GRAD_PAPER) {
        // doubled central differences at the four taps, interpolated bilinearly; along v the
        // rows are interpolated first: rows r0-1 and r0+2 give
        // (1-b)(row(r0+1) - row(r0-1)) + b (row(r0+2) - row(r0))
        gu = lerp(lerp(t.d01 - t.bm, t.b2 - t.d00, au), lerp(t.d11 - t.cm, t.c2 - t.d10, au), av);
        gv = lerp(bot - lerp(t.a0, t.a1, au), lerp(t.f0, t.f1, au) - top, av);
    } else {
        gu = fmaf(av, e1 - e0, e0);
        gv = dtb;
    }
}

template <int TP, int GRAD, bool GRADS>
__device__ __forceinline__ void taps_plain(LdsF* q, float au, float av, float& val, float& gu, float& gv) {
    Taps12 t;
    load_plain<TP, GRAD, GRADS>(q, t);
    eval_plain<GRAD, GRADS>(t, au, av, val, gu, gv);
}

// Taps of a sample near or across the detector border, masked with the border tables:
// (z, s) of the cell's two columns c0, c1 and two rows r0, r1 (z = 1 inside the detector,
// s = 2 on its first and last column/row for the one-sided differences). b addresses the cell.
template <int TP, int GRAD, bool GRADS>
__device__ __forceinline__ void taps_masked(LdsF* b, float au, float av, float2 c0, float2 c1, float2 r0, float2 r1,
                                            float& val, float& gu, float& gv) {
    const float d00 = b[0], d01 = b[1], d10 = b[TP], d11 = b[TP + 1];
    const float u0 = 1.0f - au, v0 = 1.0f - av;
    // bilinear weights with the outside taps masked (z)
    const float wc0 = u0 * c0.x, wc1 = au * c1.x, wr0 = v0 * r0.x, wr1 = av * r1.x;
    val = fmaf(wr0, fmaf(wc0, d00, wc1 * d01), wr1 * fmaf(wc0, d10, wc1 * d11));
    if (!GRADS) return;
    if (GRAD == GMC_GRAD_PAPER) {
        const float bm = b[-1], b2 = b[2], cm = b[TP - 1], c2 = b[TP + 2];
        const float a0 = b[-TP], a1 = b[-TP + 1], f0 = b[2 * TP], f1 = b[2 * TP + 1];
        // g_u: one-sided factor s per column, rows masked; g_v: s per row, columns masked
        const float sc0 = u0 * c0.y, sc1 = au * c1.y, sr0 = v0 * r0.y, sr1 = av * r1.y;
        gu = fmaf(wr0, fmaf(sc0, d01 - bm, sc1 * (b2 - d00)), wr1 * fmaf(sc0, d11 - cm, sc1 * (c2 - d10)));
        gv = fmaf(sr0, fmaf(wc0, d10 - a0, wc1 * (d11 - a1)), sr1 * fmaf(wc0, f0 - d00, wc1 * (f1 - d01)));
    } else {
        // derivative of the (masked) bilinear interpolant
        gu = fmaf(wr0, c1.x * d01 - c0.x * d00, wr1 * (c1.x * d11 - c0.x * d10));
        gv = fmaf(wc0, r1.x * d10 - r0.x * d00, wc1 * (r1.x * d11 - r0.x * d01));
    }
}

// ---------------------------------------------------------------- the kernel
//
// Per view v the workgroup (1) waits for its tile of view v and synchronises, (2) samples view
// v from LDS, (3) synchronises again and issues the asynchronous global->LDS loads of view
// v+1's tile into the same buffer, and the border tables of view v+1 if that tile crosses the
// detector border. The tile loads of one workgroup overlap the sampling of the others on the
// CU: with one buffer per workgroup, more workgroups fit (measured faster than two buffers per
// workgroup with the next tile's loads in flight during the sampling). Tiles are filled with clamped
// detector coordinates (the border pixel repeats outside the detector); the interior path
// never touches the repeats, the border path masks them with the tables:
//   column table (z, s): z = 1 inside the detector, 0 outside (bilinear taps of d, g_v);
//                        s = 2 on the first and last column, 1 elsewhere (g_u, one-sided)
//   row table likewise for rows (taps of d, g_u; s for g_v).
// With repeated border pixels the central difference is 0 outside the detector by itself.
__device__ __forceinline__ BrickDesc load_desc(const __attribute__((address_space(4))) BrickDesc* p) {
    BrickDesc d;
#pragma unroll
    for (int e = 0; e < 12; ++e) d.m[e] = p->m[e];
    d.ou = p->ou;
    d.ov = p->ov;
    d.kin = p->kin;
    d.kout = p->kout;
    d.tw = p->tw;
    d.th = p->th;
    d.mode = p->mode;
    d.pad = 0;
    return d;
}

// The work of one item (a brick and a contiguous chunk of its views); shared by the
// single-plan kernel and the batched one. Item q is brick q % n_bricks and chunk q / n_bricks;
// chunk c covers views [c n / vsplit, (c + 1) n / vsplit). The forward of chunk 0 writes the
// volume, chunk c > 0 its own partial volume (summed afterwards in a fixed order); the VJP
// partials are per view and brick, so every chunk writes its own views' rows.
template <int TP, int TH, int BZ, int WEIGHT, int GRAD, bool VJP>
__device__ __forceinline__ void bp_brick(const BpArgs& a, const BrickDesc* __restrict__ desc,
                                         const float* __restrict__ proj, float* __restrict__ vol,
                                         const float* __restrict__ gvol, float* __restrict__ part, const int item,
                                         float* __restrict__ sT, float* __restrict__ sCol, float* __restrict__ sRow,
                                         float* __restrict__ sRed) {
    constexpr int NSEG = (TP + 63) / 64;
    // The VJP stores the whole tile; the forward needs no halo and stores rows and columns
    // 1 .. extent - 2, its row r at buffer row r - 1 (so its buffer has TH - 2 rows). Border
    // tables hold (z, s) pairs for the VJP and z alone for the forward.
    constexpr int H0 = VJP ? 0 : 1;
    constexpr unsigned TBL = VJP ? 8u : 4u;
    static_assert(BZ % FWD_GROUP == 0, "the forward samples a column in whole groups");
    static_assert(BZ % 4 == 0, "seeds and voxels move in groups of 4 along z");
    static_assert(TP <= 128 && 128 + TH <= THREADS, "border tables: columns by threads 0 .. TP-1, rows by 128 ..");
    const int brick = item % a.n_bricks, chunk = item / a.n_bricks;
    const int v_lo = chunk * a.n_views / a.vsplit, v_hi = (chunk + 1) * a.n_views / a.vsplit;
    const int bj = brick % a.nby;
    const int bi = (brick / a.nby) % a.nbx;
    const int bk = brick / (a.nby * a.nbx);

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    typedef const __attribute__((address_space(4))) BrickDesc ConstDesc;
    // Each wave covers an 8 x 8 patch of columns and each half-wave (the lanes one LDS pass
    // serves) 4 (x) by 8 (y) of them, so that a half-wave's samples fall on few detector columns
    // and rows of a tile (fewer bank conflicts). The VJP transposes the half-wave patches to 8 by
    // 4 when, at the middle view of its chunk, the detector column moves faster along y than
    // along x (chunks span a few degrees of the arc; the forward's longer chunks keep 4 by 8).
    int li = 8 * (wave & 1) + (lane >> 3), lj = 8 * (wave >> 1) + (lane & 7);
    if (VJP && v_lo < v_hi) {
        const ConstDesc* dm = (ConstDesc*)(desc + brick) + (long long)((v_lo + v_hi) >> 1) * a.n_bricks;
        // d(u''/w)/dx and d(u''/w)/dy at the tile's middle column, both times w
        const float c = 0.5f * (float)dm->tw;
        const float ax = fabsf(fmaf(-c, dm->m[8], dm->m[0])), ay = fabsf(fmaf(-c, dm->m[9], dm->m[1]));
        if (dm->mode != TILE_SKIP && ay > ax) {
            const int tmp = li;
            li = lj;
            lj = tmp;
        }
    }
    const int i = bi * BXY + li, j = bj * BXY + lj, k0 = bk * BZ;
    const bool col_in = (i < a.nx) && (j < a.ny);
    const float qx = (float)li * a.dx, qy = (float)lj * a.dy, dz = a.dz;
    const long long col_off = ((long long)i * a.ny + j) * a.nz + k0;

    float acc[BZ];
    float seed[VJP ? BZ : 1];
    if (VJP) {
        const float sc = (GRAD == GMC_GRAD_PAPER) ? 0.5f : 1.0f;
#pragma unroll
        for (int k = 0; k < BZ; ++k) seed[k] = 0.0f;
        if (col_in && k0 + BZ <= a.nz && ((size_t)(gvol + col_off) & 15) == 0) {
            // whole column inside the volume, 16-byte aligned: one vector load per 4 voxels
            const float4* g4 = (const float4*)(gvol + col_off);
#pragma unroll
            for (int k4 = 0; k4 < BZ / 4; ++k4) {
                const float4 x = g4[k4];
                seed[4 * k4 + 0] = sc * x.x;
                seed[4 * k4 + 1] = sc * x.y;
                seed[4 * k4 + 2] = sc * x.z;
                seed[4 * k4 + 3] = sc * x.w;
            }
        } else if (col_in) {
#pragma unroll
            for (int k = 0; k < BZ; ++k)
                if (k0 + k < a.nz) seed[k] = sc * gvol[col_off + k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < BZ; ++k) acc[k] = 0.0f;
    }

    // the descriptors are read-only for the whole launch: read them through the constant
    // address space so that they arrive with scalar loads whatever the caller's pointer provenance
    ConstDesc* descs = (ConstDesc*)(desc + brick);
    const long long dstride = a.n_bricks;

    // Issue view vv's tile loads (asynchronous, no registers). Rows are
    // distributed over the four waves and walked with scalar registers; each lane carries one
    // clamped detector column per 64-column segment, lanes outside the tile's columns are masked
    // once per segment. Interior tiles need no row clamp and step their row address by four rows.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    auto stage = [&](const BrickDesc& D, int vv) {
        if (D.mode != TILE_INTERIOR && D.mode != TILE_EDGE) return;
        const float* __restrict__ img = proj + (long long)vv * a.plane;
        const int c_end = D.tw - H0, r_end = D.th - H0;
        // the lane index (and from it the thread index) is recomputed per view with mbcnt rather
        // than kept live across the sampling
        const int ln = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        const int tt = wv * 64 + ln;
#pragma unroll
        for (int q = 0; q < NSEG; ++q) {
            if (q * 64 >= c_end) break;
            const int c = q * 64 + ln;
            const unsigned cb = 4u * (unsigned)min(max(D.ou + c, 0), a.W - 1);
            if (c >= H0 && c < c_end) {   // lanes outside the tile's columns stay idle
                if (D.mode == TILE_INTERIOR) {
                    const char* row = (const char*)(img + (long long)(D.ov + H0 + wv) * a.W);
                    const long long step = 16LL * a.W;
                    for (int r = H0 + wv; r < r_end; r += 4, row += step)
                        __builtin_amdgcn_global_load_lds((const float*)(row + cb), sT + (r - H0) * TP + q * 64, 4, 0, 0);
                } else {
                    for (int r = H0 + wv; r < r_end; r += 4) {
                        const int gr = min(max(D.ov + r, 0), a.H - 1);
                        const char* row = (const char*)(img + (long long)gr * a.W);
                        __builtin_amdgcn_global_load_lds((const float*)(row + cb), sT + (r - H0) * TP + q * 64, 4, 0, 0);
                    }
                }
            }
        }
        if (D.mode == TILE_EDGE) {
            if (tt < TP) {
                const int gc = D.ou + tt;
                const float z = ((unsigned)gc < (unsigned)a.W) ? 1.0f : 0.0f;
                if (VJP) {
                    sCol[2 * tt] = z;
                    sCol[2 * tt + 1] = (gc == 0 || gc == a.W - 1) ? 2.0f : 1.0f;
                } else {
                    sCol[tt] = z;
                }
            } else if (tt >= 128 && tt < 128 + TH) {
                const int gr = D.ov + (tt - 128);
                const float z = ((unsigned)gr < (unsigned)a.H) ? 1.0f : 0.0f;
                if (VJP) {
                    sRow[2 * (tt - 128)] = z;
                    sRow[2 * (tt - 128) + 1] = (gr == 0 || gr == a.H - 1) ? 2.0f : 1.0f;
                } else {
                    sRow[tt - 128] = z;
                }
            }
        }
    };

    BrickDesc cur;
    if (v_lo < v_hi) {
        cur = load_desc(descs + (long long)v_lo * dstride);
        stage(cur, v_lo);
    }
    int prev_ou = 0, prev_ov = 0;
    for (int v = v_lo; v < v_hi; ++v) {
        __builtin_amdgcn_s_waitcnt(0);   // this wave's tile loads of view v have landed in LDS
        __syncthreads();                 // ... and everybody's
        if (VJP && v > v_lo && t < 14) {
            float s;
            if (t < 12) {
                const float* rb = sRed + ((v - 1) & 1) * 48;
                s = ((rb[t] + rb[12 + t]) + rb[24 + t]) + rb[36 + t];
            } else {
                s = __int_as_float(t == 12 ? prev_ou : prev_ov);
            }
            part[((long long)(v - 1) * a.n_bricks + brick) * PART_STRIDE + t] = s;
        }
        prev_ou = cur.ou;
        prev_ov = cur.ov;

        float S0 = 0.f, S1 = 0.f, S2 = 0.f, T0 = 0.f, T1 = 0.f, T2 = 0.f;
        const float* m = cur.m;
        Column col;
        col.ub = fmaf(m[0], qx, fmaf(m[1], qy, m[3]));
        col.vb = fmaf(m[4], qx, fmaf(m[5], qy, m[7]));
        col.wb = fmaf(m[8], qx, fmaf(m[9], qy, m[11]));
        col.du = m[2] * dz;
        col.dv = m[6] * dz;
        col.dw = m[10] * dz;
        // LDS byte address of tile row 0 (for the forward one row before its buffer; no
        // access lands there)
        const unsigned tile = lds_addr(sT) - 4u * (unsigned)(H0 * TP);
        const float cmax = (float)(cur.tw - 3), rmax = (float)(cur.th - 3);

        if (cur.mode == TILE_INTERIOR) {
            // cell (r, c) with 1 <= r <= rmax, 1 <= c <= cmax: every tap, halo included, in the tile
            const unsigned base = tile - 4u * 0x4B000000u;
            if (!VJP) {
                // per group of FWD_GROUP samples: positions first, then all LDS reads, then the
                // arithmetic, so that the reads of a group are in flight together
#pragma unroll
                for (int g = 0; g < BZ; g += FWD_GROUP) {
                    unsigned off[FWD_GROUP];
                    float au[FWD_GROUP], av[FWD_GROUP], ww[FWD_GROUP];
#pragma unroll
                    for (int k = 0; k < FWD_GROUP; ++k) {
                        const Smp p = next_sample(col, g + k);
                        const Cell c = cell_of(p);
                        off[k] = tile_cell<TP>(c, base);
                        au[k] = c.au;
                        av[k] = c.av;
                        ww[k] = (WEIGHT == GMC_WEIGHT_FDK) ? p.rw * p.rw : 1.0f;
                    }
                    float d00[FWD_GROUP], d01[FWD_GROUP], d10[FWD_GROUP], d11[FWD_GROUP];
#pragma unroll
                    for (int k = 0; k < FWD_GROUP; ++k) {
                        LdsF* b = lds_f(off[k]);
                        d00[k] = b[0];
                        d01[k] = b[1];
                        d10[k] = b[TP];
                        d11[k] = b[TP + 1];
                    }
#pragma unroll
                    for (int k = 0; k < FWD_GROUP; ++k) {
                        const float top = lerp(d00[k], d01[k], au[k]);
                        const float bot = lerp(d10[k], d11[k], au[k]);
                        const float val = lerp(top, bot, av[k]);
                        acc[g + k] = (WEIGHT == GMC_WEIGHT_FDK) ? fmaf(val, ww[k], acc[g + k]) : acc[g + k] + val;
                    }
                }
            } else {
                // taps addressed from (row - 1, column - 1), so that every LDS offset is positive
                const unsigned base_m = base - 4u * (TP + 1);
                // per group of VJP_GROUP samples: positions, then the LDS reads, then the arithmetic
#pragma unroll
                for (int g = 0; g < BZ; g += VJP_GROUP) {
                    Smp p[VJP_GROUP];
                    Cell c[VJP_GROUP];
                    Taps12 tp[VJP_GROUP];
#pragma unroll
                    for (int i = 0; i < VJP_GROUP; ++i) {
                        p[i] = next_sample(col, g + i);
                        c[i] = cell_of(p[i]);
                    }
#pragma unroll
                    for (int i = 0; i < VJP_GROUP; ++i)
                        load_plain<TP, GRAD, true>(lds_f(tile_cell<TP>(c[i], base_m)), tp[i]);
#pragma unroll
                    for (int i = 0; i < VJP_GROUP; ++i) {
                        float val, gu, gv;
                        eval_plain<GRAD, true>(tp[i], c[i].au, c[i].av, val, gu, gv);
                        accumulate<BZ, WEIGHT, GRAD>(p[i], seed[g + i], val, gu, gv, g + i, S0, S1, S2, T0, T1, T2);
                    }
                }
            }
        } else if (cur.mode == TILE_EDGE) {
            // per slice k (uniform branches): skip slices that miss the detector, plain taps for
            // slices inside it, masked taps for the slices across its border
            const unsigned tb = tile - 4u * 0x4B000000u, cb = lds_base(sCol, TBL), rb = lds_base(sRow, TBL);
            const unsigned kin = cur.kin, kout = cur.kout;
#pragma unroll
            for (int k = 0; k < BZ; ++k) {
                const Smp p = next_sample(col, k);
                if ((kout >> k) & 1u) {
                    if (VJP && k < BZ - 1) {   // the prefix sums still advance
                        T0 += S0;
                        T1 += S1;
                        T2 += S2;
                    }
                    continue;
                }
                const Cell cl = cell_of(p);
                float val, gu = 0.0f, gv = 0.0f;
                if ((kin >> k) & 1u) {
                    taps_plain<TP, GRAD, VJP>(lds_f(tile_cell<TP>(cl, tb - 4u * (TP + 1))), cl.au, cl.av, val,
                                              gu, gv);
                } else {
                    const float cf = __builtin_amdgcn_fmed3f(cl.fu, 1.0f, cmax);
                    const float rf = __builtin_amdgcn_fmed3f(cl.fv, 1.0f, rmax);
                    // border tables: (z, s) of columns cf, cf + 1 and rows rf, rf + 1 (the
                    // forward's tables hold z only; s is not used without gradients)
                    LdsF* ct = lds_f(lds_index(cb, TBL, cf));
                    LdsF* rt = lds_f(lds_index(rb, TBL, rf));
                    float2 c0, c1, r0, r1;
                    if (VJP) {
                        c0 = make_float2(ct[0], ct[1]);
                        c1 = make_float2(ct[2], ct[3]);
                        r0 = make_float2(rt[0], rt[1]);
                        r1 = make_float2(rt[2], rt[3]);
                    } else {
                        c0 = make_float2(ct[0], 1.0f);
                        c1 = make_float2(ct[1], 1.0f);
                        r0 = make_float2(rt[0], 1.0f);
                        r1 = make_float2(rt[1], 1.0f);
                    }
                    taps_masked<TP, GRAD, VJP>(lds_f(lds_index(tb, 4u, fmaf(rf, (float)TP, cf))), cl.au, cl.av, c0, c1,
                                               r0, r1, val, gu, gv);
                }
                if (!VJP)
                    acc[k] += (WEIGHT == GMC_WEIGHT_FDK) ? val * (p.rw * p.rw) : val;
                else
                    accumulate<BZ, WEIGHT, GRAD>(p, seed[k], val, gu, gv, k, S0, S1, S2, T0, T1, T2);
            }
        } else if (cur.mode == TILE_GLOBAL) {
            const float* __restrict__ img = proj + (long long)v * a.plane;
#pragma unroll 1
            for (int k = 0; k < BZ; ++k) {
                const Smp p = next_sample(col, k);
                const Cell cl = cell_of(p);
                const float au = cl.au, av = cl.av;
                Taps tp;
                // cells outside [-2^22, 2^22) cannot meet the detector: clamp before the conversion
                const int cu = (int)fminf(fmaxf(cl.fu, -4194304.0f), 4194304.0f);
                const int cv = (int)fminf(fmaxf(cl.fv, -4194304.0f), 4194304.0f);
                fetch_global<VJP && GRAD == GMC_GRAD_PAPER>(img, a.W, a.H, cv + cur.ov, cu + cur.ou, tp);
                const float e0 = tp.d01 - tp.d00, e1 = tp.d11 - tp.d10;
                const float top = fmaf(au, e0, tp.d00), bot = fmaf(au, e1, tp.d10);
                const float dtb = bot - top;
                const float val = fmaf(av, dtb, top);
                // acc / seed are indexed dynamically here (this path is rare): select by k
#pragma unroll
                for (int k2 = 0; k2 < BZ; ++k2) {
                    if (k2 != k) continue;
                    if (!VJP) {
                        acc[k2] += (WEIGHT == GMC_WEIGHT_FDK) ? val * (p.rw * p.rw) : val;
                    } else {
                        float gu, gv;
                        if (GRAD == GMC_GRAD_PAPER) {
                            gu = lerp(lerp(tp.u00, tp.u01, au), lerp(tp.u10, tp.u11, au), av);
                            gv = lerp(lerp(tp.v00, tp.v01, au), lerp(tp.v10, tp.v11, au), av);
                        } else {
                            gu = fmaf(av, e1 - e0, e0);
                            gv = dtb;
                        }
                        accumulate<BZ, WEIGHT, GRAD>(p, seed[k2], val, gu, gv, k2, S0, S1, S2, T0, T1, T2);
                    }
                }
            }
        }
        if (VJP) {
            // z-moments from the prefix sums; G'' rows r: (qx S_r, qy S_r, dz T_r, S_r); row 2
            // carries the minus sign of Eq. 4
            T0 = fmaf((float)(BZ - 1), S0, -T0);
            T1 = fmaf((float)(BZ - 1), S1, -T1);
            T2 = fmaf((float)(BZ - 1), S2, -T2);
            float g[12] = {qx * S0, qy * S0, dz * T0, S0, qx * S1, qy * S1, dz * T1, S1,
                           -qx * S2, -qy * S2, -dz * T2, -S2};
            float red[3] = {0.0f, 0.0f, 0.0f};
            if (cur.mode != TILE_SKIP) wave_reduce12(g, red);
            if ((lane & 15) == 0) {
                float* rb = sRed + (v & 1) * 48 + wave * 12 + 3 * (lane >> 4);
                rb[0] = red[0];
                rb[1] = red[1];
                rb[2] = red[2];
            }
        }
        if (v + 1 < v_hi) {
            cur = load_desc(descs + (long long)(v + 1) * dstride);
            __syncthreads();   // everybody has finished sampling view v: the tile can be refilled
            stage(cur, v + 1);
        }
    }

    if (VJP) {
        __syncthreads();
        const int v = v_hi;
        if (v > v_lo && t < 14) {
            float s;
            if (t < 12) {
                const float* rb = sRed + ((v - 1) & 1) * 48;
                s = ((rb[t] + rb[12 + t]) + rb[24 + t]) + rb[36 + t];
            } else {
                s = __int_as_float(t == 12 ? prev_ou : prev_ov);
            }
            part[((long long)(v - 1) * a.n_bricks + brick) * PART_STRIDE + t] = s;
        }
    } else if (col_in) {
        float* out = (chunk == 0 ? vol : a.vpart + (long long)(chunk - 1) * a.nx * a.ny * a.nz) + col_off;
        if (k0 + BZ <= a.nz && ((size_t)out & 15) == 0) {
            // whole column inside the volume, 16-byte aligned: one vector store per 4 voxels
#pragma unroll
            for (int k4 = 0; k4 < BZ / 4; ++k4)
                ((float4*)out)[k4] = make_float4(acc[4 * k4], acc[4 * k4 + 1], acc[4 * k4 + 2], acc[4 * k4 + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < BZ; ++k)
                if (k0 + k < a.nz) out[k] = acc[k];
        }
    }
}

template <int TP, int TH, bool VJP>
struct BpShared;
template <int TP, int TH>
struct BpShared<TP, TH, true> {
    float sT[TP * TH];
    float sCol[2 * TP];   // (z, s) per tile column
    float sRow[2 * TH];   // (z, s) per tile row
    float sRed[2 * 4 * 12];
    __device__ float* red() { return sRed; }
};
template <int TP, int TH>
struct BpShared<TP, TH, false> {
    float sT[TP * (TH - 2)];   // tile rows 1 .. TH - 2
    float sCol[TP];            // z per tile column
    float sRow[TH];            // z per tile row
    __device__ float* red() { return nullptr; }
};

#ifndef GMC_FWD_DEEP_OCC
#define GMC_FWD_DEEP_OCC 8
#endif
// Workgroups per CU the register budget is sized for. With deep bricks: 4 for the VJP (about
// 110 VGPRs with 16 seeds; at 5 it spills, and spilling costs more than the fifth workgroup
// gains); 8 for the forward, whose halo-free 80 x 62 buffer and z-only border tables take
// 20,416 bytes, so that eight fit in the 160 KB of LDS (64 VGPRs: 16 accumulators and samples
// read in groups of 4). With shallow bricks 6 and 8 (80 and 60 VGPRs). The largest tiles fit
// three (128 x 96) and four (VJP, 128 x 64) or five (forward) times.
constexpr int bp_occupancy(int plane, int bz, bool vjp) {
    return bz == BZ_DEEP ? (plane <= 80 * 64 ? (vjp ? 4 : GMC_FWD_DEEP_OCC) : 3)
                         : (plane <= 80 * 40 ? (vjp ? 6 : 8) : (vjp ? 4 : 5));
}

template <int TP, int TH, int BZ, int WEIGHT, int GRAD, bool VJP>
__global__ void __launch_bounds__(THREADS, bp_occupancy(TP * TH, BZ, VJP))
    k_bp(BpArgs a, const BrickDesc* __restrict__ desc, const float* __restrict__ proj, float* __restrict__ vol,
         const float* __restrict__ gvol, float* __restrict__ part) {
    __shared__ BpShared<TP, TH, VJP> sh;
    const int blk = blockIdx.x;
    const int item = (blk & 7) * a.per_xcd + (blk >> 3);
    if (item >= a.n_bricks * a.vsplit) return;
    bp_brick<TP, TH, BZ, WEIGHT, GRAD, VJP>(a, desc, proj, vol, gvol, part, item, sh.sT, sh.sCol, sh.sRow, sh.red());
}

// Several plans in one launch: the work items of all plans form one index space (plan q owns
// [begin_q, begin_q + n_bricks_q vsplit_q)), mapped to XCDs like a single plan's items.
template <int TP, int TH, int BZ, int WEIGHT, int GRAD, bool VJP>
__global__ void __launch_bounds__(THREADS, bp_occupancy(TP * TH, BZ, VJP)) k_bp_batch(BatchTable tab) {
    __shared__ BpShared<TP, TH, VJP> sh;
    const int blk = blockIdx.x;
    const int g = (blk & 7) * tab.per_xcd + (blk >> 3);
    if (g >= tab.total) return;
    int q = 0;
    for (int e = 1; e < tab.n; ++e)
        if (g >= tab.begin[e]) q = e;
    const BpArgs& a = tab.item[q];
    bp_brick<TP, TH, BZ, WEIGHT, GRAD, VJP>(a, a.desc, a.proj, a.vol, a.gvol, a.part, g - tab.begin[q], sh.sT, sh.sCol,
                                           sh.sRow, sh.red());
}

namespace {

template <int TP, int TH, int BZ>
hipError_t launch_cfg(const gmc_plan* p, const BpArgs& a, bool vjp, hipStream_t s) {
    const unsigned grid = 8u * (unsigned)a.per_xcd;
    const int W = p->g.weighting, G = p->g.grad_mode;
    if (!vjp) {
        if (W == GMC_WEIGHT_FDK)
            k_bp<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_PAPER, false><<<grid, THREADS, 0, s>>>(a, a.desc, a.proj, a.vol, a.gvol, a.part);
        else
            k_bp<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_PAPER, false><<<grid, THREADS, 0, s>>>(a, a.desc, a.proj, a.vol, a.gvol, a.part);
    } else {
        if (W == GMC_WEIGHT_FDK && G == GMC_GRAD_PAPER)
            k_bp<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_PAPER, true><<<grid, THREADS, 0, s>>>(a, a.desc, a.proj, a.vol, a.gvol, a.part);
        else if (W == GMC_WEIGHT_FDK)
            k_bp<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_EXACT, true><<<grid, THREADS, 0, s>>>(a, a.desc, a.proj, a.vol, a.gvol, a.part);
        else if (G == GMC_GRAD_PAPER)
            k_bp<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_PAPER, true><<<grid, THREADS, 0, s>>>(a, a.desc, a.proj, a.vol, a.gvol, a.part);
        else
            k_bp<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_EXACT, true><<<grid, THREADS, 0, s>>>(a, a.desc, a.proj, a.vol, a.gvol, a.part);
    }
    return hipGetLastError();
}

}  // namespace

template <int TP, int TH, int BZ>
hipError_t launch_batch_cfg(int W, int G, const BatchTable& tab, bool vjp, hipStream_t s) {
    const unsigned grid = 8u * (unsigned)tab.per_xcd;
    if (!vjp) {
        if (W == GMC_WEIGHT_FDK)
            k_bp_batch<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_PAPER, false><<<grid, THREADS, 0, s>>>(tab);
        else
            k_bp_batch<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_PAPER, false><<<grid, THREADS, 0, s>>>(tab);
    } else {
        if (W == GMC_WEIGHT_FDK && G == GMC_GRAD_PAPER)
            k_bp_batch<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_PAPER, true><<<grid, THREADS, 0, s>>>(tab);
        else if (W == GMC_WEIGHT_FDK)
            k_bp_batch<TP, TH, BZ, GMC_WEIGHT_FDK, GMC_GRAD_EXACT, true><<<grid, THREADS, 0, s>>>(tab);
        else if (G == GMC_GRAD_PAPER)
            k_bp_batch<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_PAPER, true><<<grid, THREADS, 0, s>>>(tab);
        else
            k_bp_batch<TP, TH, BZ, GMC_WEIGHT_PAPER, GMC_GRAD_EXACT, true><<<grid, THREADS, 0, s>>>(tab);
    }
    return hipGetLastError();
}

#define GMC_TILE(D, C) TILE_CFGS[D][C].tp, TILE_CFGS[D][C].th, (D == 0 ? BZ_DEEP : BZ_SHALLOW)

hipError_t launch_bp_batch(int bz, int tile_cfg, int weighting, int grad_mode, const BatchTable& tab, bool vjp,
                           hipStream_t s) {
    if (tab.n < 1 || tab.n > MAX_BATCH || tab.total < 1) return hipErrorInvalidValue;
    if (bz != BZ_DEEP && bz != BZ_SHALLOW) return hipErrorInvalidValue;
    switch (3 * depth_index(bz) + tile_cfg) {
        case 0: return launch_batch_cfg<GMC_TILE(0, 0)>(weighting, grad_mode, tab, vjp, s);
        case 1: return launch_batch_cfg<GMC_TILE(0, 1)>(weighting, grad_mode, tab, vjp, s);
        case 2: return launch_batch_cfg<GMC_TILE(0, 2)>(weighting, grad_mode, tab, vjp, s);
        case 3: return launch_batch_cfg<GMC_TILE(1, 0)>(weighting, grad_mode, tab, vjp, s);
        case 4: return launch_batch_cfg<GMC_TILE(1, 1)>(weighting, grad_mode, tab, vjp, s);
        case 5: return launch_batch_cfg<GMC_TILE(1, 2)>(weighting, grad_mode, tab, vjp, s);
        default: return hipErrorInvalidValue;
    }
}

// vol += partial volumes of chunks 1 .. vsplit-1, added in chunk order (deterministic)
__global__ void k_sum_chunks(float* __restrict__ vol, const float* __restrict__ vpart, long long n, int n_parts) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        float x = vol[e];
        for (int c = 0; c < n_parts; ++c) x += vpart[c * n + e];
        vol[e] = x;
    }
}

hipError_t launch_sum_chunks(const BpArgs& a, hipStream_t s) {
    if (a.vsplit <= 1) return hipSuccess;
    const long long n = (long long)a.nx * a.ny * a.nz;
    const unsigned grid = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid), dim3(256), 0, s, a.vol, (const float*)a.vpart, n, a.vsplit - 1);
    return hipGetLastError();
}

hipError_t launch_bp(const gmc_plan* p, const BpArgs& a, bool vjp, hipStream_t s) {
    if (p->bz != BZ_DEEP && p->bz != BZ_SHALLOW) return hipErrorInvalidValue;
    switch (3 * depth_index(p->bz) + p->tile_cfg) {
        case 0: return launch_cfg<GMC_TILE(0, 0)>(p, a, vjp, s);
        case 1: return launch_cfg<GMC_TILE(0, 1)>(p, a, vjp, s);
        case 2: return launch_cfg<GMC_TILE(0, 2)>(p, a, vjp, s);
        case 3: return launch_cfg<GMC_TILE(1, 0)>(p, a, vjp, s);
        case 4: return launch_cfg<GMC_TILE(1, 1)>(p, a, vjp, s);
        case 5: return launch_cfg<GMC_TILE(1, 2)>(p, a, vjp, s);
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
    Column col;
    col.ub = fmaf(D.m[0], qx, fmaf(D.m[1], qy, D.m[3]));
    col.vb = fmaf(D.m[4], qx, fmaf(D.m[5], qy, D.m[7]));
    col.wb = fmaf(D.m[8], qx, fmaf(D.m[9], qy, D.m[11]));
    col.du = D.m[2] * dz;
    col.dv = D.m[6] * dz;
    col.dw = D.m[10] * dz;
    Smp p = next_sample(col, 0);
    for (int s = 1; s <= kk; ++s) p = next_sample(col, s);
    const Cell c = cell_of(p);
    cell[2 * q] = (int)c.fu + D.ou;
    cell[2 * q + 1] = (int)c.fv + D.ov;
    frac[2 * q] = c.au;
    frac[2 * q + 1] = c.av;
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
