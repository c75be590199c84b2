// Geometry composition on the GPU, FP64.
//
// k_compose: Eq. 1, Phat_j = P_j T_j(theta_j) with T = [Rz(rz) Ry(ry) Rx(rx) | t], and the six
//   derivative matrices P_j dT_j/dtheta_jk that Eq. 2 contracts with dL/dPhat_j.
// k_setup:   composes each Phat_j further with the local frame of every voxel brick and the
//   origin of that brick's detector tile, and sizes the tile from the projections of the
//   brick's eight corners (w > 0 makes the projected box the hull of its corners).
#include "gmc_internal.hpp"

namespace gmc {

__global__ void k_compose(const double* __restrict__ theta, const double* __restrict__ P, double* __restrict__ Phat,
                          double* __restrict__ dPhat, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double* th = theta + 6 * j;
    double cx, sx, cy, sy, cz, sz;
    sincos(th[3], &sx, &cx);
    sincos(th[4], &sy, &cy);
    sincos(th[5], &sz, &cz);
    // R = Rz Ry Rx and its partial derivatives, written out
    const double R[3][3] = {{cz * cy, cz * sy * sx - sz * cx, cz * sy * cx + sz * sx},
                            {sz * cy, sz * sy * sx + cz * cx, sz * sy * cx - cz * sx},
                            {-sy, cy * sx, cy * cx}};
    const double Rrx[3][3] = {{0.0, cz * sy * cx + sz * sx, -cz * sy * sx + sz * cx},
                              {0.0, sz * sy * cx - cz * sx, -sz * sy * sx - cz * cx},
                              {0.0, cy * cx, -cy * sx}};
    const double Rry[3][3] = {{-cz * sy, cz * cy * sx, cz * cy * cx},
                              {-sz * sy, sz * cy * sx, sz * cy * cx},
                              {-cy, -sy * sx, -sy * cx}};
    const double Rrz[3][3] = {{-sz * cy, -sz * sy * sx - cz * cx, -sz * sy * cx + cz * sx},
                              {cz * cy, cz * sy * sx - sz * cx, cz * sy * cx + sz * sx},
                              {0.0, 0.0, 0.0}};
    const double* Pj = P + 12 * j;
    double* Ph = Phat + 12 * j;
    for (int r = 0; r < 3; ++r) {
        const double p0 = Pj[4 * r], p1 = Pj[4 * r + 1], p2 = Pj[4 * r + 2], p3 = Pj[4 * r + 3];
        for (int c = 0; c < 3; ++c) Ph[4 * r + c] = p0 * R[0][c] + p1 * R[1][c] + p2 * R[2][c];
        Ph[4 * r + 3] = p0 * th[0] + p1 * th[1] + p2 * th[2] + p3;
        if (!dPhat) continue;
        double* D = dPhat + 72 * j;
        // translations: dT/dt_k has a single 1 in column 3, row k
        D[0 * 12 + 4 * r + 0] = 0.0; D[0 * 12 + 4 * r + 1] = 0.0; D[0 * 12 + 4 * r + 2] = 0.0; D[0 * 12 + 4 * r + 3] = p0;
        D[1 * 12 + 4 * r + 0] = 0.0; D[1 * 12 + 4 * r + 1] = 0.0; D[1 * 12 + 4 * r + 2] = 0.0; D[1 * 12 + 4 * r + 3] = p1;
        D[2 * 12 + 4 * r + 0] = 0.0; D[2 * 12 + 4 * r + 1] = 0.0; D[2 * 12 + 4 * r + 2] = 0.0; D[2 * 12 + 4 * r + 3] = p2;
        for (int c = 0; c < 3; ++c) {
            D[3 * 12 + 4 * r + c] = p0 * Rrx[0][c] + p1 * Rrx[1][c] + p2 * Rrx[2][c];
            D[4 * 12 + 4 * r + c] = p0 * Rry[0][c] + p1 * Rry[1][c] + p2 * Rry[2][c];
            D[5 * 12 + 4 * r + c] = p0 * Rrz[0][c] + p1 * Rrz[1][c] + p2 * Rrz[2][c];
        }
        D[3 * 12 + 4 * r + 3] = 0.0;
        D[4 * 12 + 4 * r + 3] = 0.0;
        D[5 * 12 + 4 * r + 3] = 0.0;
    }
}

hipError_t launch_compose(const double* theta, const double* P, double* Phat, double* dPhat, int n_views,
                          hipStream_t s) {
    k_compose<<<(n_views + 127) / 128, 128, 0, s>>>(theta, P, Phat, dPhat, n_views);
    return hipGetLastError();
}

struct SetupArgs {
    const double* Phat;
    BrickDesc* desc;
    int* status;
    int n_views, n_bricks, nbx, nby, bz, W, H, tp, th_max, flags;
    double ox, oy, oz, dx, dy, dz;
};

// 1/w for w > 0: the hardware reciprocal and two Newton steps (relative error near 1e-16;
// tile bounds carry 2 pixels of margin and the slice classes 1e-3 pixel)
__device__ __forceinline__ double rcp64(double w) {
    double r = __builtin_amdgcn_rcp(w);
    r = fma(r, fma(-w, r, 1.0), r);
    return fma(r, fma(-w, r, 1.0), r);
}

__device__ void setup_one(const SetupArgs& a, const int v, const int b) {
    const long long idx = (long long)v * a.n_bricks + b;
    // bricks are numbered z-slab major: b = (bk * nbx + bi) * nby + bj
    const int bj = b % a.nby;
    const int bi = (b / a.nby) % a.nbx;
    const int bk = b / (a.nby * a.nbx);
    const double o[3] = {a.ox + (double)(bi * BXY) * a.dx, a.oy + (double)(bj * BXY) * a.dy,
                         a.oz + (double)(bk * a.bz) * a.dz};
    const double ext[3] = {(BXY - 1) * a.dx, (BXY - 1) * a.dy, (a.bz - 1) * a.dz};
    const double* Ph = a.Phat + 12 * v;
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    bool bad = false;
    for (int c = 0; c < 8; ++c) {
        const double x = o[0] + ((c & 1) ? ext[0] : 0.0);
        const double y = o[1] + ((c & 2) ? ext[1] : 0.0);
        const double z = o[2] + ((c & 4) ? ext[2] : 0.0);
        const double u = Ph[0] * x + Ph[1] * y + Ph[2] * z + Ph[3];
        const double vv = Ph[4] * x + Ph[5] * y + Ph[6] * z + Ph[7];
        const double w = Ph[8] * x + Ph[9] * y + Ph[10] * z + Ph[11];
        if (!(w > 0.0)) { bad = true; break; }
        const double rw = rcp64(w);   // tile bounds: one reciprocal per corner suffices
        const double uh = u * rw, vh = vv * rw;
        umin = fmin(umin, uh); umax = fmax(umax, uh);
        vmin = fmin(vmin, vh); vmax = fmax(vmax, vh);
    }
    BrickDesc d;
    if (bad || !(umax - umin < 1e6) || !(vmax - vmin < 1e6)) {
        for (int e = 0; e < 12; ++e) d.m[e] = 0.0f;
        d.ou = d.ov = 0;
        d.kin = d.kout = 0;
        d.tw = d.th = 0;
        d.mode = TILE_SKIP;
        d.pad = 0;
        atomicOr(a.status, 1);
        a.desc[idx] = d;
        return;
    }
    // taps of the samples lie in [floor(umin), floor(umax) + 1]; one column of rounding
    // margin and one of halo for the central differences on each side
    const double clo = floor(umin), chi = floor(umax) + 1.0;
    const double rlo = floor(vmin), rhi = floor(vmax) + 1.0;
    const int ou = (int)clo - 2, ov = (int)rlo - 2;
    const int tw = (int)(chi - clo) + 5, th = (int)(rhi - rlo) + 5;
    // M = S * Phat * T_brick
    double rows[3][4];
    for (int c = 0; c < 4; ++c) {
        rows[0][c] = Ph[c] - (double)ou * Ph[8 + c];
        rows[1][c] = Ph[4 + c] - (double)ov * Ph[8 + c];
        rows[2][c] = Ph[8 + c];
    }
    for (int r = 0; r < 3; ++r) {
        d.m[4 * r + 0] = (float)rows[r][0];
        d.m[4 * r + 1] = (float)rows[r][1];
        d.m[4 * r + 2] = (float)rows[r][2];
        d.m[4 * r + 3] = (float)(rows[r][0] * o[0] + rows[r][1] * o[1] + rows[r][2] * o[2] + rows[r][3]);
    }
    d.ou = ou;
    d.ov = ov;
    const bool outside = (ou + tw <= 0) || (ou >= a.W) || (ov + th <= 0) || (ov >= a.H);
    const bool inside = ou >= 0 && ov >= 0 && ou + tw <= a.W && ov + th <= a.H;
    if (outside) {
        d.mode = TILE_SKIP;
    } else if ((a.flags & GMC_FLAG_FORCE_GLOBAL) || tw > a.tp || th > a.th_max) {
        d.mode = TILE_GLOBAL;
    } else if (inside && !(a.flags & GMC_FLAG_FORCE_EDGE)) {
        d.mode = TILE_INTERIOR;
    } else {
        d.mode = TILE_EDGE;
    }
    d.tw = (uint8_t)(tw < 255 ? tw : 255);
    d.th = (uint8_t)(th < 255 ? th : 255);
    d.pad = 0;
    d.kin = d.kout = 0;
    if (d.mode == TILE_EDGE) {
        // Classify the brick's z-slices. At fixed z, u/w and v/w are linear-fractional in
        // (x, y), so the four corners of a slice bound its projection. A slice whose tap cells
        // (c, c+1) x (r, r+1) all satisfy 1 <= c, c+1 <= W-2, 1 <= r, r+1 <= H-2 needs no border
        // rule (central differences stay inside); a slice whose tap cells all lie outside the
        // detector contributes nothing (values and differences are 0 there). The corners are
        // evaluated in FP32 with the local matrix the sampling kernels use (tile-relative
        // positions below 2^8 pixels: about 1e-5 pixel of rounding, and the reciprocal within one
        // ulp); 1e-3 pixel of margin covers the difference to the kernels' positions, which
        // follow a Newton chain along the column.
        const float eps = 1e-3f;
        const float exf = (float)ext[0], eyf = (float)ext[1], dzf = (float)a.dz;
        const float ouf = (float)ou, ovf = (float)ov;
        for (int k = 0; k < a.bz && k < 16; ++k) {
            const float qz = (float)k * dzf;
            float ulo = 3.0e38f, uhi = -3.0e38f, vlo = 3.0e38f, vhi = -3.0e38f;
            bool ok = true;
            for (int c = 0; c < 4; ++c) {
                const float qx = (c & 1) ? exf : 0.0f, qy = (c & 2) ? eyf : 0.0f;
                const float w = fmaf(d.m[8], qx, fmaf(d.m[9], qy, fmaf(d.m[10], qz, d.m[11])));
                if (!(w > 0.0f)) { ok = false; break; }
                const float rw = __builtin_amdgcn_rcpf(w);
                const float uh = fmaf(d.m[0], qx, fmaf(d.m[1], qy, fmaf(d.m[2], qz, d.m[3]))) * rw;
                const float vh = fmaf(d.m[4], qx, fmaf(d.m[5], qy, fmaf(d.m[6], qz, d.m[7]))) * rw;
                ulo = fminf(ulo, uh); uhi = fmaxf(uhi, uh);
                vlo = fminf(vlo, vh); vhi = fmaxf(vhi, vh);
            }
            if (!ok) continue;
            // detector cells: tile-relative cell + tile origin (integer-valued floats, exact)
            const float c0 = floorf(ulo - eps) + ouf, c1 = floorf(uhi + eps) + 1.0f + ouf;
            const float r0 = floorf(vlo - eps) + ovf, r1 = floorf(vhi + eps) + 1.0f + ovf;
            if (c0 >= 1.0f && c1 <= (float)(a.W - 2) && r0 >= 1.0f && r1 <= (float)(a.H - 2)) d.kin |= (uint16_t)(1u << k);
            if (c1 < 0.0f || c0 > (float)(a.W - 1) || r1 < 0.0f || r0 > (float)(a.H - 1)) d.kout |= (uint16_t)(1u << k);
        }
    }
    a.desc[idx] = d;
}

// one thread per brick (x) and view (y, strided when there are more views than grid rows)
__global__ void k_setup(SetupArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.n_bricks) return;
    for (int v = blockIdx.y; v < a.n_views; v += gridDim.y)
        setup_one(a, v, b);
}

hipError_t launch_setup(const gmc_plan* p, const double* Phat, BrickDesc* desc, int* status, hipStream_t s) {
    SetupArgs a;
    a.Phat = Phat;
    a.desc = desc;
    a.status = status;
    a.n_views = p->g.n_views;
    a.n_bricks = p->n_bricks;
    a.nbx = p->nbx;
    a.nby = p->nby;
    a.bz = p->bz;
    a.W = p->g.det_w;
    a.H = p->g.det_h;
    a.tp = plan_tile(p).tp;
    a.th_max = plan_tile(p).th;
    a.flags = p->g.flags;
    a.ox = p->g.origin_mm[0];
    a.oy = p->g.origin_mm[1];
    a.oz = p->g.origin_mm[2];
    a.dx = p->g.voxel_mm[0];
    a.dy = p->g.voxel_mm[1];
    a.dz = p->g.voxel_mm[2];
    const dim3 grid((unsigned)((a.n_bricks + 255) / 256), (unsigned)std::min(a.n_views, 65535));
    k_setup<<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace gmc
