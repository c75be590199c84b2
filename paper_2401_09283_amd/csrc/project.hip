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
// One thread per detector pixel, a workgroup per 16 x 16 pixel patch and view (neighbouring
// rays share cache lines of the volume). The ray set-up (inverse, clipping, entry point) is
// FP64; the march is FP32 from the entry point, so sample positions carry no cancellation
// against the distant source.
#include "gmc_internal.hpp"

namespace gmc {

namespace {

struct FpArgs {
    const float* vol;
    const uint8_t* labels;   // optional: only voxels with labels == part count
    const double* Phat;      // [n_views][12]
    float* out;              // [n_views][H][W]
    int nx, ny, nz, W, H, part, accumulate;
    double vx, vy, vz, ox, oy, oz;
    double step_mm;
};

__device__ __forceinline__ float voxel_at(const FpArgs& a, int i, int j, int k) {
    if ((unsigned)i >= (unsigned)a.nx || (unsigned)j >= (unsigned)a.ny || (unsigned)k >= (unsigned)a.nz) return 0.0f;
    const long long idx = ((long long)i * a.ny + j) * a.nz + k;
    if (a.labels && a.labels[idx] != a.part) return 0.0f;
    return a.vol[idx];
}

__global__ void __launch_bounds__(256) k_forward_project(FpArgs a) {
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    const int r = blockIdx.y * 16 + (threadIdx.x >> 4);
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
        for (long long s = 0; s < N; ++s) {
            const float fs = (float)s;
            const float px = fmaf(fs, sx, qx), py = fmaf(fs, sy, qy), pz = fmaf(fs, sz, qz);
            const float fx = floorf(px), fy = floorf(py), fz = floorf(pz);
            const float ax = px - fx, ay = py - fy, az = pz - fz;
            const int i = (int)fx, j = (int)fy, k = (int)fz;
            const float v000 = voxel_at(a, i, j, k), v001 = voxel_at(a, i, j, k + 1);
            const float v010 = voxel_at(a, i, j + 1, k), v011 = voxel_at(a, i, j + 1, k + 1);
            const float v100 = voxel_at(a, i + 1, j, k), v101 = voxel_at(a, i + 1, j, k + 1);
            const float v110 = voxel_at(a, i + 1, j + 1, k), v111 = voxel_at(a, i + 1, j + 1, k + 1);
            const float z00 = fmaf(az, v001 - v000, v000), z01 = fmaf(az, v011 - v010, v010);
            const float z10 = fmaf(az, v101 - v100, v100), z11 = fmaf(az, v111 - v110, v110);
            const float y0 = fmaf(ay, z01 - z00, z00), y1 = fmaf(ay, z11 - z10, z10);
            sum += fmaf(ax, y1 - y0, y0);
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
    const dim3 grid((unsigned)((a.W + 15) / 16), (unsigned)((a.H + 15) / 16), (unsigned)p->g.n_views);
    k_forward_project<<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace gmc
