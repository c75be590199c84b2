// Ray-driven forward projection under the composed matrices Phat_j (the adjoint partner of the
// backprojection of Eq. 3; used to simulate scans under motion and to re-project volumes).
//
// Line integral, along the ray from the source through pixel (c, r), of the trilinear
// interpolant of the volume (values at voxel centres, zero outside the grid). With
// Phat = [M | p4] the source is C = -M^-1 p4 and the points projecting to (c, r) are
// C + w M^-1 (c, r, 1)^T. The ray's w-interval inside the interpolant's support (voxel
// coordinates [-1, n] per axis) is split into N = ceil(length / h) equal steps, h half the
// smallest voxel pitch, and the integral is the midpoint sum (mm x volume units).
//
// One thread per detector pixel, a workgroup per 4 columns x 64 rows of one view: a wave
// takes 64 rows of one column, whose rays cross the same (x, y) columns of the volume at
// nearby z, so each tap load of the wave touches one or two cache lines of the z-fastest
// volume. The ray set-up (inverse, clipping, entry point) is
// FP64; the march is FP32 from the entry point, so sample positions carry no cancellation
// against the distant source. Per sample the two taps along each axis are clamped into the
// grid and a tap outside it gets weight 0 (the zero extension), so the loads need no branches:
// the two z taps of each (x, y) column are adjacent in memory and read as one 8-byte load
// (four loads per sample instead of eight); indices are 32-bit when the volume has fewer than
// 2^31 voxels.
#include "gmc_internal.hpp"

namespace gmc {

namespace {

struct FpArgs {
    const float* vol;
    const uint8_t* labels;   // optional: only voxels with labels == part count
    const double* Phat;      // [n_views][12]
    float* out;              // [n_views][H][W]
    int nx, ny, nz, W, H, part, accumulate;
    unsigned max_off;        // interior path: byte offset of the last (x, y, z) pair base
    double vx, vy, vz, ox, oy, oz;
    double step_mm;
};

// The two taps of one axis: clamped indices and weights, 0 for a tap outside [0, n).
struct AxisTaps {
    int i0, i1;
    float w0, w1;
};

__device__ __forceinline__ AxisTaps axis_taps(int i, float frac, int n) {
    AxisTaps t;
    t.i0 = min(max(i, 0), n - 1);
    t.i1 = min(max(i + 1, 0), n - 1);
    t.w0 = ((unsigned)i < (unsigned)n) ? 1.0f - frac : 0.0f;
    t.w1 = ((unsigned)(i + 1) < (unsigned)n) ? frac : 0.0f;
    return t;
}

template <typename Idx, bool LABELS>
__device__ __forceinline__ float tap(const FpArgs& a, Idx idx) {
    const float x = a.vol[idx];
    return LABELS ? (a.labels[idx] == a.part ? x : 0.0f) : x;
}

// One sample of the trilinear interpolant at voxel coordinates (px, py, pz), anywhere in the
// support: taps clamped into the grid, zero weights outside it.
template <typename Idx, bool LABELS, bool PAIRZ>
__device__ __forceinline__ float clamped_sample(const FpArgs& a, float px, float py, float pz, Idx sx_i, Idx sy_i) {
    const float fx = floorf(px), fy = floorf(py), fz = floorf(pz);
    const AxisTaps tx = axis_taps((int)fx, px - fx, a.nx);
    const AxisTaps ty = axis_taps((int)fy, py - fy, a.ny);
    const AxisTaps tz = axis_taps((int)fz, pz - fz, a.nz);
    if constexpr (PAIRZ) {
        // both z taps of an (x, y) column in one 8-byte load: the pair starts at b, inside
        // [0, nz - 2], and each tap's weight moves to the element holding its clamped index
        // (same products and sums as the two single loads)
        const int b = min(max((int)fz, 0), a.nz - 2);
        const float e0 = (tz.i0 == b ? tz.w0 : 0.0f) + (tz.i1 == b ? tz.w1 : 0.0f);
        const float e1 = (tz.i0 == b + 1 ? tz.w0 : 0.0f) + (tz.i1 == b + 1 ? tz.w1 : 0.0f);
        const Idx q00 = (Idx)tx.i0 * sx_i + (Idx)ty.i0 * sy_i + b, q01 = (Idx)tx.i0 * sx_i + (Idx)ty.i1 * sy_i + b;
        const Idx q10 = (Idx)tx.i1 * sx_i + (Idx)ty.i0 * sy_i + b, q11 = (Idx)tx.i1 * sx_i + (Idx)ty.i1 * sy_i + b;
        float2 p00, p01, p10, p11;
        __builtin_memcpy(&p00, a.vol + q00, 8);
        __builtin_memcpy(&p01, a.vol + q01, 8);
        __builtin_memcpy(&p10, a.vol + q10, 8);
        __builtin_memcpy(&p11, a.vol + q11, 8);
        const float z00 = fmaf(e0, p00.x, e1 * p00.y), z01 = fmaf(e0, p01.x, e1 * p01.y);
        const float z10 = fmaf(e0, p10.x, e1 * p10.y), z11 = fmaf(e0, p11.x, e1 * p11.y);
        const float y0 = fmaf(ty.w0, z00, ty.w1 * z01), y1 = fmaf(ty.w0, z10, ty.w1 * z11);
        return fmaf(tx.w0, y0, tx.w1 * y1);
    } else {
        const Idx r00 = (Idx)tx.i0 * sx_i + (Idx)ty.i0 * sy_i, r01 = (Idx)tx.i0 * sx_i + (Idx)ty.i1 * sy_i;
        const Idx r10 = (Idx)tx.i1 * sx_i + (Idx)ty.i0 * sy_i, r11 = (Idx)tx.i1 * sx_i + (Idx)ty.i1 * sy_i;
        const float z00 = fmaf(tz.w0, tap<Idx, LABELS>(a, r00 + tz.i0), tz.w1 * tap<Idx, LABELS>(a, r00 + tz.i1));
        const float z01 = fmaf(tz.w0, tap<Idx, LABELS>(a, r01 + tz.i0), tz.w1 * tap<Idx, LABELS>(a, r01 + tz.i1));
        const float z10 = fmaf(tz.w0, tap<Idx, LABELS>(a, r10 + tz.i0), tz.w1 * tap<Idx, LABELS>(a, r10 + tz.i1));
        const float z11 = fmaf(tz.w0, tap<Idx, LABELS>(a, r11 + tz.i0), tz.w1 * tap<Idx, LABELS>(a, r11 + tz.i1));
        const float y0 = fmaf(ty.w0, z00, ty.w1 * z01), y1 = fmaf(ty.w0, z10, ty.w1 * z11);
        return fmaf(tx.w0, y0, tx.w1 * y1);
    }
}

// Floor, fraction and 1 - fraction of x in [0, 2^22) without conversions: (x - 1/2) + 1.5 2^23
// lies where FP32 numbers are spaced by 1, so it rounds to 1.5 2^23 + floor(x) (at an integer
// x the tie may give x - 1 with fraction 1, which interpolates to the same value); the integer
// is read from the bits. (Below 2^23 the spacing is 1/2: x + (2^23 - 1/2) would not round for
// x < 1/4.)
struct FastAxis {
    int i;
    float w0, w1;
};

__device__ __forceinline__ FastAxis fast_axis(float x) {
    const float b = (x - 0.5f) + 12582912.0f;
    const float f = x - (b - 12582912.0f);
    FastAxis t;
    t.i = __float_as_int(b) - 0x4B400000;
    t.w0 = 1.0f - f;
    t.w1 = f;
    return t;
}

// Samples whose eight taps are all inside the grid (every coordinate in [1e-3, n - 1 - 1e-3],
// far beyond the FP32 position error) form one interval [sa, sb) of the ray's samples; they
// take the unclamped path (four 8-byte loads from uniform bases at one 32-bit byte offset),
// the samples before and after it the clamped one. The products and sums are those of the
// clamped path, and the samples are added in the same order.
__device__ __forceinline__ void interior_range(float q, float st, int n, double& lo, double& hi) {
    const double A = 1e-3, B = (double)n - 1.0 - 1e-3;
    if (!(A <= B)) {   // fewer than two slices: no interior
        lo = 1.0;
        hi = 0.0;
        return;
    }
    if (st == 0.0f) {
        if (!((double)q >= A && (double)q <= B)) { lo = 1.0; hi = 0.0; }
        return;
    }
    double u = (A - (double)q) / (double)st, w = (B - (double)q) / (double)st;
    if (u > w) { const double x = u; u = w; w = x; }
    lo = fmax(lo, ceil(u));
    hi = fmin(hi, floor(w));
}

template <typename Idx, bool LABELS, bool PAIRZ, bool FAST>
__global__ void __launch_bounds__(256) k_forward_project(FpArgs a) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int r = blockIdx.y * 64 + (threadIdx.x & 63);
    const int v = blockIdx.z;
    if (c >= a.W || r >= a.H) return;
    const double* P = a.Phat + 12 * (long long)v;
    // M^-1 by cofactors
    const double m00 = P[0], m01 = P[1], m02 = P[2], m10 = P[4], m11 = P[5], m12 = P[6], m20 = P[8], m21 = P[9],
                 m22 = P[10];
    const double c00 = m11 * m22 - m12 * m21, c01 = m02 * m21 - m01 * m22, c02 = m01 * m12 - m02 * m11;
    const double c10 = m12 * m20 - m10 * m22, c11 = m00 * m22 - m02 * m20, c12 = m02 * m10 - m00 * m12;
    const double c20 = m10 * m21 - m11 * m20, c21 = m01 * m20 - m00 * m21, c22 = m00 * m11 - m01 * m10;
    const double idet = 1.0 / (m00 * c00 + m01 * c10 + m02 * c20);
    const double S[3] = {-(c00 * P[3] + c01 * P[7] + c02 * P[11]) * idet, -(c10 * P[3] + c11 * P[7] + c12 * P[11]) * idet,
                         -(c20 * P[3] + c21 * P[7] + c22 * P[11]) * idet};
    const double D[3] = {(c00 * c + c01 * r + c02) * idet, (c10 * c + c11 * r + c12) * idet, (c20 * c + c21 * r + c22) * idet};
    const double vox[3] = {a.vx, a.vy, a.vz}, org[3] = {a.ox, a.oy, a.oz};
    const int n[3] = {a.nx, a.ny, a.nz};
    double q0[3], dq[3], t0 = -1e300, t1 = 1e300;
    bool empty = false;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        q0[e] = (S[e] - org[e]) / vox[e];
        dq[e] = D[e] / vox[e];
        if (dq[e] == 0.0) {
            if (q0[e] <= -1.0 || q0[e] >= (double)n[e]) empty = true;
        } else {
            double ta = (-1.0 - q0[e]) / dq[e], tb = ((double)n[e] - q0[e]) / dq[e];
            if (ta > tb) { const double x = ta; ta = tb; tb = x; }
            t0 = fmax(t0, ta);
            t1 = fmin(t1, tb);
        }
    }
    float sum = 0.0f;
    double len = 0.0;
    long long N = 0;
    if (!empty && t1 > t0) {
        len = (t1 - t0) * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        N = (long long)ceil(len / a.step_mm - 1e-9);   // an exact multiple of the step is not split further
        const double dt = (t1 - t0) / (double)N;
        // FP32 march from the first sample
        const float qx = (float)(q0[0] + (t0 + 0.5 * dt) * dq[0]), qy = (float)(q0[1] + (t0 + 0.5 * dt) * dq[1]),
                    qz = (float)(q0[2] + (t0 + 0.5 * dt) * dq[2]);
        const float sx = (float)(dt * dq[0]), sy = (float)(dt * dq[1]), sz = (float)(dt * dq[2]);
        const Idx sx_i = (Idx)a.ny * a.nz, sy_i = a.nz;
        // sample counters are 32-bit (a ray has far fewer than 2^24 samples: (float)s is exact)
        const int n_s = (int)N;
        int sa = n_s, sb = n_s;   // the interior interval (empty: every sample clamped)
        if (FAST) {
            double lo = 0.0, hi = (double)(N - 1);
            interior_range(qx, sx, a.nx, lo, hi);
            interior_range(qy, sy, a.ny, lo, hi);
            interior_range(qz, sz, a.nz, lo, hi);
            if (lo <= hi) {
                sa = (int)lo;
                sb = (int)hi + 1;
            }
        }
        for (int s = 0; s < sa; ++s) {
            const float fs = (float)s;
            sum += clamped_sample<Idx, LABELS, PAIRZ>(a, fmaf(fs, sx, qx), fmaf(fs, sy, qy), fmaf(fs, sz, qz), sx_i, sy_i);
        }
        if (FAST) {
            // unclamped interior: byte offsets from four uniform bases (the volume has fewer
            // than 2^30 voxels, so every offset fits in 32 bits)
            const unsigned bx = 4u * (unsigned)a.ny * (unsigned)a.nz, by = 4u * (unsigned)a.nz;
            const char* b00 = (const char*)a.vol;
            const char* b01 = b00 + by;
            const char* b10 = b00 + bx;
            const char* b11 = b10 + by;
            // consecutive samples half a voxel apart often share their cell: the four pairs
            // are reloaded only when it changes
            float fs = (float)sa;
            unsigned prev = 0xFFFFFFFFu;
            float2 p00 = make_float2(0.f, 0.f), p01 = p00, p10 = p00, p11 = p00;
            for (int s = sa; s < sb; ++s, fs += 1.0f) {
                const FastAxis tx = fast_axis(fmaf(fs, sx, qx));
                const FastAxis ty = fast_axis(fmaf(fs, sy, qy));
                const FastAxis tz = fast_axis(fmaf(fs, sz, qz));
                // the interior interval keeps every index in [0, n - 2]; the clamp only guards
                // the loads
                const unsigned off = min(__umul24((unsigned)tx.i, bx) + __umul24((unsigned)ty.i, by) + 4u * (unsigned)tz.i,
                                         a.max_off);
                if (off != prev) {
                    __builtin_memcpy(&p00, b00 + off, 8);
                    __builtin_memcpy(&p01, b01 + off, 8);
                    __builtin_memcpy(&p10, b10 + off, 8);
                    __builtin_memcpy(&p11, b11 + off, 8);
                    prev = off;
                }
                const float z00 = fmaf(tz.w0, p00.x, tz.w1 * p00.y), z01 = fmaf(tz.w0, p01.x, tz.w1 * p01.y);
                const float z10 = fmaf(tz.w0, p10.x, tz.w1 * p10.y), z11 = fmaf(tz.w0, p11.x, tz.w1 * p11.y);
                const float y0 = fmaf(ty.w0, z00, ty.w1 * z01), y1 = fmaf(ty.w0, z10, ty.w1 * z11);
                sum += fmaf(tx.w0, y0, tx.w1 * y1);
            }
            for (int s = sb; s < n_s; ++s) {
                const float fs = (float)s;
                sum += clamped_sample<Idx, LABELS, PAIRZ>(a, fmaf(fs, sx, qx), fmaf(fs, sy, qy), fmaf(fs, sz, qz), sx_i, sy_i);
            }
        }
        sum *= (float)(len / (double)N);
    }
    float* o = a.out + ((long long)v * a.H + r) * a.W + c;
    *o = a.accumulate ? *o + sum : sum;
}

}  // namespace

hipError_t launch_forward_project(const gmc_plan* p, const float* vol, const uint8_t* labels, int part,
                                  const double* Phat, float* out, int accumulate, hipStream_t s) {
    FpArgs a;
    a.vol = vol;
    a.labels = labels;
    a.Phat = Phat;
    a.out = out;
    a.nx = p->g.nx;
    a.ny = p->g.ny;
    a.nz = p->g.nz;
    a.W = p->g.det_w;
    a.H = p->g.det_h;
    a.part = part;
    a.accumulate = accumulate;
    a.vx = p->g.voxel_mm[0];
    a.vy = p->g.voxel_mm[1];
    a.vz = p->g.voxel_mm[2];
    a.ox = p->g.origin_mm[0];
    a.oy = p->g.origin_mm[1];
    a.oz = p->g.origin_mm[2];
    a.step_mm = 0.5 * fmin(a.vx, fmin(a.vy, a.vz));
    const dim3 grid((unsigned)((a.W + 3) / 4), (unsigned)((a.H + 63) / 64), (unsigned)p->g.n_views);
    const bool small = (long long)a.nx * a.ny * a.nz < (1LL << 31);
    const bool pair = a.nz >= 2;
    a.max_off = 0;
    // the interior path needs two taps per axis, 32-bit byte offsets and 24-bit multiplier
    // operands (4 ny nz < 2^24)
    const bool fast = pair && a.nx >= 2 && a.ny >= 2 && (long long)a.nx * a.ny * a.nz < (1LL << 30) &&
                      (long long)a.ny * a.nz < (1LL << 22);
    if (fast)
        a.max_off = 4u * (unsigned)(((long long)a.nx - 2) * a.ny * a.nz + ((long long)a.ny - 2) * a.nz + (a.nz - 2));
    if (small && labels)
        k_forward_project<int, true, false, false><<<grid, 256, 0, s>>>(a);
    else if (fast)
        k_forward_project<int, false, true, true><<<grid, 256, 0, s>>>(a);
    else if (small && pair)
        k_forward_project<int, false, true, false><<<grid, 256, 0, s>>>(a);
    else if (small)
        k_forward_project<int, false, false, false><<<grid, 256, 0, s>>>(a);
    else if (labels)
        k_forward_project<long long, true, false, false><<<grid, 256, 0, s>>>(a);
    else if (pair)
        k_forward_project<long long, false, true, false><<<grid, 256, 0, s>>>(a);
    else
        k_forward_project<long long, false, false, false><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace gmc
