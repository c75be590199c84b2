// Finishing the Jacobian-vector product: the per-(view, brick) partials of G_j, taken in each
// brick's local frame, are moved back to the frame of Phat_j and summed over bricks in a
// fixed order (per-thread strided sums, then a pairwise tree over the block), giving
// G_j = dL/dPhat_j; Eq. 2 then contracts G_j with the derivative matrices P_j dT_j/dtheta_jk.
// The frame change and the sum are FP32 like the rest of the voxel arithmetic; the
// contraction with the FP64 derivative matrices, and the outputs, are FP64.
//
// Frame change: the kernels differentiate with respect to M = S Phat T_b, where T_b moves
// brick-local points to the world (origin o_b) and S = [[1,0,-ou],[0,1,-ov],[0,0,1]] shifts
// the detector to the tile origin. Hence dL/dPhat = S^T (dL/dM) T_b^T: row 2 loses
// ou * row 0 + ov * row 1, then columns 0..2 gain o_b * column 3.
#include "gmc_internal.hpp"

namespace gmc {

struct ReduceArgs {
    const float* part;
    const double* dPhat;
    double* G;
    double* grad_theta;
    double* grad_P;
    int n_bricks, nbx, nby, bz;
    double ox, oy, oz, dx, dy, dz;
};

__global__ void __launch_bounds__(256) k_reduce_chain(ReduceArgs a) {
    __shared__ float sh[256 * 12];
    __shared__ double shd[12];
    const int v = blockIdx.x;
    const int t = threadIdx.x;
    float acc[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[e] = 0.0f;
    for (int b = t; b < a.n_bricks; b += 256) {
        const float* p = a.part + ((long long)v * a.n_bricks + b) * PART_STRIDE;
        float q[14];
#pragma unroll
        for (int e = 0; e < 14; ++e) q[e] = p[e];
        const float ou = (float)__float_as_int(q[12]);
        const float ov = (float)__float_as_int(q[13]);
        const int bj = b % a.nby;
        const int bi = (b / a.nby) % a.nbx;
        const int bk = b / (a.nby * a.nbx);
        const float o[3] = {(float)(a.ox + (double)(bi * BXY) * a.dx), (float)(a.oy + (double)(bj * BXY) * a.dy),
                            (float)(a.oz + (double)(bk * a.bz) * a.dz)};
        float g[12];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            g[c] = q[c];
            g[4 + c] = q[4 + c];
            g[8 + c] = q[8 + c] - ou * q[c] - ov * q[4 + c];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[4 * r + c] += g[4 * r + c] + o[c] * g[4 * r + 3];
            acc[4 * r + 3] += g[4 * r + 3];
        }
    }
#pragma unroll
    for (int e = 0; e < 12; ++e) sh[e * 256 + t] = acc[e];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int e = 0; e < 12; ++e) sh[e * 256 + t] += sh[e * 256 + t + s];
        }
        __syncthreads();
    }
    if (t < 12) {
        const double gv = (double)sh[t * 256];
        shd[t] = gv;
        a.G[12 * v + t] = gv;
        if (a.grad_P) a.grad_P[12 * v + t] = gv;
    }
    __syncthreads();
    if (t < 6) {
        const double* D = a.dPhat + 72 * v + 12 * t;
        double s = 0.0;
        for (int e = 0; e < 12; ++e) s += shd[e] * D[e];
        a.grad_theta[6 * v + t] = s;
    }
}

hipError_t launch_reduce_chain(const gmc_plan* p, const float* part, const double* dPhat, double* G,
                               double* grad_theta, double* grad_P, hipStream_t s) {
    ReduceArgs a;
    a.part = part;
    a.dPhat = dPhat;
    a.G = G;
    a.grad_theta = grad_theta;
    a.grad_P = grad_P;
    a.n_bricks = p->n_bricks;
    a.nbx = p->nbx;
    a.nby = p->nby;
    a.bz = p->bz;
    a.ox = p->g.origin_mm[0];
    a.oy = p->g.origin_mm[1];
    a.oz = p->g.origin_mm[2];
    a.dx = p->g.voxel_mm[0];
    a.dy = p->g.voxel_mm[1];
    a.dz = p->g.voxel_mm[2];
    k_reduce_chain<<<p->g.n_views, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace gmc
