// Internal declarations shared by the HIP translation units of libgmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gmc.h"

namespace gmc {

// Voxel bricks are BXY x BXY columns of bz voxels; one workgroup of BXY*BXY threads owns a
// brick and each thread owns one column (a run of bz voxels along z). The tile the brick
// projects to is staged in LDS once per view. A plan takes deep bricks (16 voxels) where their
// tiles fit the small or middle tile configuration: each tile and the per-view work of a
// column (set-up, reciprocal, VJP wave reduction) then serve twice the samples of 8, at the
// price of registers (16 accumulators or seeds per thread). Coarse voxels on a fine detector
// project 16 voxels to taller tiles than the largest configuration holds at full occupancy;
// such plans take shallow bricks (8 voxels).
constexpr int BXY = 16;
constexpr int BZ_DEEP = 16, BZ_SHALLOW = 8;
constexpr int THREADS = BXY * BXY;

// One per (view, brick), 64 bytes, read with scalar loads by the backprojection kernels.
// The local matrix m maps brick-local coordinates q (mm, relative to the centre of the
// brick's first voxel) to (u'', v'', w) with u'' = u - ou*w and v'' = v - ov*w, so
// u''/w is the detector column relative to the tile origin ou.
enum TileMode : int32_t {
    TILE_SKIP = 0,      // nothing to sample: the tile misses the detector, or w <= 0 (flagged)
    TILE_INTERIOR = 1,  // tile inside the detector: plain bilinear taps from LDS
    TILE_EDGE = 2,      // tile crosses the detector border: taps weighted by border tables
    TILE_GLOBAL = 3     // tile larger than the LDS tile: taps gathered from global memory
};
struct BrickDesc {
    float m[12];
    int32_t ou, ov;       // detector column / row of tile index 0
    uint16_t kin, kout;   // border tiles: bit k is set when every tap of the brick's slice k lies
                          // inside the detector away from its border (plain formulas apply) /
                          // outside the detector (the slice contributes nothing)
    uint8_t tw, th;       // tile extent (columns, rows); 255 for tiles sampled from global memory
    uint8_t mode;         // TileMode
    uint8_t pad;
};
static_assert(sizeof(BrickDesc) == 64, "descriptor must be 64 bytes");

// Per-(view, brick) partial of the VJP: 12 entries of G in the brick-local frame, then
// the tile origin (ou, ov) as int bits, then 2 unused slots.
constexpr int PART_STRIDE = 16;

// Tile configurations (pitch TP floats, TH rows) compiled into the kernels, per brick depth;
// one tile per workgroup. 80 x 64 floats plus the border tables take 21 KB (the registers, not
// the 160 KB of LDS, then bound the workgroups per CU); a brick of 16 x 16 x 16 voxels at 1 mm
// in the 200-degree scan geometry projects to at most about 73 x 61 pixels, and a tile that
// exceeds the plan's configuration is sampled from global memory instead. 128 x 96 (49 KB,
// three workgroups per CU) and, for shallow bricks, 128 x 64 (34 KB, four per CU) serve coarse
// voxels on a fine detector. Within a depth the configurations grow in both extents, so a
// batched launch can run every plan with the largest configuration among them. A row pitch of
// 80 floats (16 banks apart modulo 32) spreads the neighbouring rows a wavefront reads over
// different LDS banks.
struct TileCfg {
    int tp, th;
};
constexpr int N_TILE_CFGS = 3;
constexpr TileCfg TILE_CFGS[2][N_TILE_CFGS] = {{{40, 64}, {80, 64}, {128, 96}},    // deep bricks
                                               {{40, 40}, {80, 40}, {128, 64}}};   // shallow bricks
__host__ __device__ constexpr int depth_index(int bz) { return bz == BZ_DEEP ? 0 : 1; }
static_assert(TILE_CFGS[0][0].tp <= TILE_CFGS[0][1].tp && TILE_CFGS[0][1].tp <= TILE_CFGS[0][2].tp &&
                  TILE_CFGS[0][0].th <= TILE_CFGS[0][1].th && TILE_CFGS[0][1].th <= TILE_CFGS[0][2].th &&
                  TILE_CFGS[1][0].tp <= TILE_CFGS[1][1].tp && TILE_CFGS[1][1].tp <= TILE_CFGS[1][2].tp &&
                  TILE_CFGS[1][0].th <= TILE_CFGS[1][1].th && TILE_CFGS[1][1].th <= TILE_CFGS[1][2].th,
              "tile configurations grow in both extents");

constexpr int LOSS_BLOCKS = 4096;   // blocks of the reduction kernels of the losses
constexpr int HIST_BLOCKS = 1024;   // blocks of the histogram kernel (32 KB of LDS each)
constexpr int HIST_BINS = 64;

}  // namespace gmc

struct gmc_plan {
    gmc_geometry g;
    int bz;                      // brick depth (voxels along z): BZ_DEEP or BZ_SHALLOW
    int nbx, nby, nbz, n_bricks;
    int tile_cfg;                // index into TILE_CFGS[depth_index(bz)]
    int vsplit_fwd, vsplit_vjp;  // view chunks per brick (items = bricks x chunks) of each pass
    // workspace layout (byte offsets)
    size_t off_phat, off_dphat, off_desc, off_part, off_G, off_status, off_loss, off_hist, off_vpart, ws_bytes;
};

namespace gmc {

inline TileCfg plan_tile(const gmc_plan* p) { return TILE_CFGS[depth_index(p->bz)][p->tile_cfg]; }

struct BpArgs {
    const float* proj;
    const BrickDesc* desc;
    float* vol;          // forward output
    const float* gvol;   // VJP seed
    float* part;         // VJP partials [view][brick][PART_STRIDE]
    int nx, ny, nz, W, H, n_views, nbx, nby, nbz, n_bricks, per_xcd;
    float dx, dy, dz;
    long long plane;     // W*H
    int vsplit;          // view chunks per brick: work item q is brick q % n_bricks, chunk q / n_bricks
    float* vpart;        // forward partial volumes of chunks 1 .. vsplit-1 ([vsplit-1][nx*ny*nz])
};

// Several plans in one launch (serving): work items of plan q are [begin[q], begin[q] + n_bricks * vsplit).
constexpr int MAX_BATCH = 16;
struct BatchTable {
    BpArgs item[MAX_BATCH];
    int begin[MAX_BATCH];
    int n, total, per_xcd;
};

// launchers (return hipError_t of the launch)
hipError_t launch_compose(const double* theta, const double* P, double* Phat, double* dPhat, int n_views,
                          hipStream_t s);
hipError_t launch_setup(const gmc_plan* p, const double* Phat, BrickDesc* desc, int* status, hipStream_t s);
hipError_t launch_bp(const gmc_plan* p, const BpArgs& a, bool vjp, hipStream_t s);
// one launch over all items of tab; every plan must share weighting, gradient mode and brick
// depth bz, and tile_cfg must be at least each plan's own tile configuration
hipError_t launch_bp_batch(int bz, int tile_cfg, int weighting, int grad_mode, const BatchTable& tab, bool vjp,
                           hipStream_t s);
// vol += sum of the chunk partial volumes (fixed order), for a forward run with a.vsplit > 1
hipError_t launch_sum_chunks(const BpArgs& a, hipStream_t s);
hipError_t launch_reduce_chain(const gmc_plan* p, const float* part, const double* dPhat, double* G,
                               double* grad_theta, double* grad_P, hipStream_t s);
hipError_t launch_debug_project(const gmc_plan* p, const BrickDesc* desc, long long n, const int64_t* voxel,
                                const int32_t* view, int32_t* cell, float* frac, hipStream_t s);
hipError_t launch_loss_sumsq(const gmc_plan* p, const float* vol, float* grad, float* scratch, double* loss,
                             hipStream_t s);
hipError_t launch_loss_entropy_tv(const gmc_plan* p, const float* vol, double lambda, double lo, double hi,
                                  double eps, float* grad, float* scratch, float* hist, double* loss,
                                  hipStream_t s);
hipError_t launch_bspline_theta(int n_views, int n_nodes, const double* coeffs, double* theta, hipStream_t s);
hipError_t launch_bspline_grad(int n_views, int n_nodes, const double* grad_theta, double* grad_coeffs,
                               hipStream_t s);
hipError_t launch_forward_project(const gmc_plan* p, const float* vol, const uint8_t* labels, int part,
                                  const double* Phat, float* out, int accumulate, hipStream_t s);
hipError_t launch_akima_theta(int n_views, int n_nodes, const double* coeffs, double* theta, hipStream_t s);
hipError_t launch_akima_grad(int n_views, int n_nodes, const double* coeffs, const double* grad_theta,
                             double* grad_coeffs, hipStream_t s);
hipError_t launch_adam(long long n, double* x, const double* g, double* m, double* v, int t, double lr,
                       double b1, double b2, double eps, hipStream_t s);
hipError_t launch_gd(long long n, double* x, const double* g, double step, hipStream_t s);

}  // namespace gmc
