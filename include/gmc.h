/*
 * gmc.h — C ABI of the MI355X (gfx950) hot path of gradient-based rigid head-motion
 * compensation in cone-beam CT (Thies et al., arXiv 2401.09283).
 *
 * The library evaluates the paper's differentiable backprojection r and its
 * Jacobian-vector product (Sec. II-B, Fig. 2):
 *   - per-view rigid parameters theta_j = (tx, ty, tz [mm], rx, ry, rz [rad]) and the
 *     calibrated projection matrices P_j give Phat_j = P_j T_j(theta_j)            (Eq. 1)
 *   - filtered projections d_j and Phat_j give the volume
 *         I(p) = sum_j omega_j(p) * bilinear(d_j, u/w, v/w),  (u, v, w) = Phat_j (p, 1)  (Eq. 3)
 *   - a volume seed delta = dL/dI gives G_j = sum_p delta(p) dI(p)/dPhat_j            (Eq. 4-5)
 *     and dL/dtheta_jk = <G_j, P_j dT_j/dtheta_jk>                                     (Eq. 2)
 * The full Jacobian is never formed (Sec. II-B.2, Sec. V).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer unless stated otherwise. The caller
 *     allocates and owns all buffers, including the workspace sized by
 *     gmc_workspace_bytes(); the library never frees caller memory and allocates no
 *     device memory per call.
 *   - Projections: [n_views][det_h][det_w] float32, column (u) fastest; pixel centres at
 *     integer detector coordinates; a bilinear tap outside the detector counts as 0.
 *   - Volumes: [nx][ny][nz] float32, z fastest; voxel (i,j,k) is centred at
 *     origin_mm + (i,j,k) * voxel_mm (world coordinates, mm).
 *   - Matrices: row-major 3x4 float64, scaled so that w > 0 for every voxel (the FDK
 *     weighting additionally assumes w = 1 at the isocentre).
 *   - Calls are asynchronous on the given HIP stream (hipStream_t passed as void*;
 *     NULL = default stream). Argument errors are returned synchronously and nothing is
 *     launched; launch failures are returned as GMC_E_HIP. A (voxel brick, view) pair
 *     with w <= 0 is skipped and raises a device flag read by gmc_check().
 *   - Calls that share a workspace must be ordered (same stream, or synchronised);
 *     calls with different workspaces may run concurrently. A plan is immutable.
 *   - Results are bitwise reproducible for identical inputs on the same device.
 *   - No C++ exception, abort() or exit() crosses this ABI. gmc_last_error() returns a
 *     thread-local description of the last failure.
 */
#ifndef GMC_H
#define GMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GMC_OK = 0,
    GMC_E_INVALID = -1,     /* bad argument: null pointer, size, shape, enum value      */
    GMC_E_WORKSPACE = -2,   /* workspace missing or too small                           */
    GMC_E_HIP = -3,         /* HIP runtime error (launch, copy)                         */
    GMC_E_GEOMETRY = -4,    /* gmc_check: some voxel had w <= 0 (behind the source)     */
    GMC_E_UNSUPPORTED = -5  /* configuration outside what the kernels implement         */
} gmc_status;

/* Voxel weighting omega of Eq. 3. PAPER: omega = 1 (Eq. 3 as printed).
 * FDK: omega = 1/w^2 (Feldkamp distance weight; needs w = 1 at the isocentre). */
enum { GMC_WEIGHT_PAPER = 0, GMC_WEIGHT_FDK = 1 };
/* Detector-gradient images g_u, g_v of Eq. 4. PAPER: bilinear samples of the
 * central-difference images (Sec. II-B.2; one-sided differences on the detector
 * border, per pixel). EXACT: the derivative of the bilinear interpolant. */
enum { GMC_GRAD_PAPER = 0, GMC_GRAD_EXACT = 1 };
/* geometry.flags bits */
enum {
    GMC_FLAG_FORCE_GLOBAL = 1,  /* testing: gather every tap from global memory              */
    GMC_FLAG_FORCE_EDGE = 2     /* testing: use the detector-border tap weights on every tile */
};

typedef struct {
    int32_t n_views, det_w, det_h;   /* projection stack [n_views][det_h][det_w]            */
    int32_t nx, ny, nz;              /* volume [nx][ny][nz], z fastest                      */
    double voxel_mm[3];              /* voxel pitch                                         */
    double origin_mm[3];             /* world position of the centre of voxel (0,0,0)       */
    int32_t weighting;               /* GMC_WEIGHT_*                                         */
    int32_t grad_mode;               /* GMC_GRAD_*                                           */
    int32_t flags;                   /* GMC_FLAG_* bits, 0 for normal use                    */
} gmc_geometry;

typedef struct gmc_plan gmc_plan;

/* Create a plan for one geometry. P_nominal (HOST pointer, [n_views][3][4] float64, or
 * NULL) is the static scan; it sizes the on-chip detector tiles and chooses the brick depth
 * (16 voxels, or 8 where 16 would need the largest tile; 16 without P_nominal). A pair whose
 * tile exceeds the chosen tile at run time is sampled from global memory instead, with
 * identical results. Host-only; allocates host memory only. GMC_E_UNSUPPORTED beyond 2^26
 * bricks of 16 x 16 x 16 voxels (about 2.7e11 voxels) or 2^33 (brick, view) pairs. */
gmc_status gmc_plan_create(const gmc_geometry* g, const double* P_nominal, gmc_plan** out);
gmc_status gmc_plan_destroy(gmc_plan* plan);
/* Bytes of device workspace every call on this plan needs (256-byte aligned pointer). */
size_t gmc_workspace_bytes(const gmc_plan* plan);
/* Launch configuration chosen by the plan: out[0] brick x, out[1] brick y, out[2] brick z,
 * out[3] tile pitch (floats), out[4] tile rows, out[5] number of bricks, out[6] and out[7]
 * view chunks per brick of the forward and of the VJP (each brick's views are split over
 * that many workgroups; the forward then adds the chunks' partial volumes in chunk order,
 * so results do not depend on scheduling). HOST pointer. */
gmc_status gmc_plan_info(const gmc_plan* plan, int64_t out[8]);

/* Eq. 1 and the derivative matrices of Eq. 2, FP64.
 * theta [n_views][6] (tx,ty,tz mm; rx,ry,rz rad), P [n_views][3][4] ->
 * Phat [n_views][3][4] = P_j T_j with T = [Rz(rz) Ry(ry) Rx(rx) | t],
 * dPhat [n_views][6][3][4] = P_j dT_j/dtheta_jk (may be NULL). */
gmc_status gmc_compose(const gmc_plan* plan, const double* theta, const double* P, double* Phat,
                       double* dPhat, void* hip_stream);

/* Eq. 3: vol = r(p(theta)). proj, P, theta as above; vol [nx][ny][nz] float32 (written,
 * not accumulated). */
gmc_status gmc_backproject(const gmc_plan* plan, const float* proj, const double* P, const double* theta,
                           float* vol, void* workspace, void* hip_stream);

/* Eq. 4-5 contracted with grad_vol = dL/dI ([nx][ny][nz] float32), then Eq. 2:
 * grad_theta [n_views][6] float64 (written). grad_P [n_views][3][4] float64 receives
 * G_j = dL/dPhat_j when not NULL. Sample positions are recomputed, never stored. */
gmc_status gmc_backproject_vjp(const gmc_plan* plan, const float* proj, const double* P, const double* theta,
                               const float* grad_vol, double* grad_theta, double* grad_P, void* workspace,
                               void* hip_stream);

/* Allocation-free form of gmc_backproject_vjp, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation). Same
 * arguments, kernels and results (bitwise) as gmc_backproject_vjp, but no workspace argument:
 * the matrices, brick descriptors, per-(view, brick) partials and status word live in a static
 * device buffer of GMC_NOALLOC_SCRATCH_BYTES (64 MiB) that every GPU the library runs on holds
 * until the process ends (set up on the first call on each device, with that device current;
 * a stream of another device returns GMC_E_INVALID). A plan whose VJP needs more returns
 * GMC_E_UNSUPPORTED before anything is launched: about 128 bytes per (brick, view) pair, i.e.
 * up to roughly 5e5 pairs (a 128^3 grid has 512 bricks of 16 x 16 x 16 voxels, so up to about
 * 1000 views; half as many with 8-voxel bricks). The call allocates nothing (no hipMalloc, no
 * hipFree). geometry_flag (device int32, or NULL) receives 1 if some (brick, view) pair hit
 * w <= 0 in this call, else 0: this variant's replacement for gmc_check. Every call on one
 * GPU shares that GPU's buffer and leaves its contents there; each call overwrites everything
 * it reads, so no clearing is needed between calls, but calls that overlap in time on one GPU
 * (different streams or host threads) race on the buffer and must be serialised by the
 * caller. */
#define GMC_NOALLOC_SCRATCH_BYTES (64u << 20)
gmc_status gmc_backproject_vjp_noalloc(const gmc_plan* plan, const float* proj, const double* P,
                                       const double* theta, const float* grad_vol, double* grad_theta,
                                       double* grad_P, int32_t* geometry_flag, void* hip_stream);

/* The two calls above in steps, for callers that reuse one geometry or time the kernels:
 *  gmc_prepare: Eq. 1 (and with with_deriv != 0 the derivative matrices of Eq. 2) into the
 *    workspace, then the per-(view, brick) local matrices and detector tiles;
 *  gmc_bp_forward: the Eq. 3 kernel alone (one launch) on the prepared workspace;
 *  gmc_bp_vjp: the Eq. 4-5 kernel alone (one launch), writing per-(view, brick) partials;
 *  gmc_bp_vjp_finish: sums the partials into G_j = dL/dPhat_j and applies Eq. 2 (needs a
 *    gmc_prepare with with_deriv != 0).
 * gmc_backproject = prepare + bp_forward; gmc_backproject_vjp = prepare(1) + bp_vjp + finish. */
gmc_status gmc_prepare(const gmc_plan* plan, const double* P, const double* theta, int32_t with_deriv,
                       void* workspace, void* hip_stream);
gmc_status gmc_bp_forward(const gmc_plan* plan, const float* proj, float* vol, void* workspace, void* hip_stream);
gmc_status gmc_bp_vjp(const gmc_plan* plan, const float* proj, const float* grad_vol, void* workspace,
                      void* hip_stream);
gmc_status gmc_bp_vjp_finish(const gmc_plan* plan, double* grad_theta, double* grad_P, void* workspace,
                             void* hip_stream);

/* Scalar volume losses and their seeds dL/dI (float32 volume, FP64 scalars).
 * Sum of squared forward differences over the three axes (pairs inside the grid):
 * loss[0] = L; grad_vol = dL/dI. loss: device float64[1]. */
gmc_status gmc_loss_sumsq_grad(const gmc_plan* plan, const float* vol, float* grad_vol, double* loss,
                               void* workspace, void* hip_stream);
/* Soft-histogram entropy plus lambda * total variation:
 *   H = -sum_b p_b log p_b, p_b = h_b / sum h, h_b = sum_p B3((I(p) - c_b)/D), 64 bins of width
 *   D = (hi - lo)/64 centred at c_b = lo + (b + 1/2) D, B3 the cubic B-spline window;
 *   TV = sum_p sqrt(|forward-difference gradient|^2 + eps^2), a difference leaving the grid = 0.
 * loss (device float64[5]) = {H + lambda TV, H, TV, |dH/dI|^2, |dTV/dI|^2};
 * grad_vol = dH/dI + lambda dTV/dI. */
gmc_status gmc_loss_entropy_tv(const gmc_plan* plan, const float* vol, double lambda, double lo, double hi,
                               double eps, float* grad_vol, double* loss, void* workspace, void* hip_stream);

/* Ray-driven forward projection under Phat_j = P_j T(theta_j) (Eq. 1): the adjoint partner of
 * the backprojection, for simulating scans under motion and re-projecting volumes (Sec. III
 * simulates its data by forward projection). proj_out[j][r][c] (float32 [n_views][det_h][det_w],
 * overwritten) is the line integral, along the ray from the source -M^-1 p4 (Phat = [M | p4])
 * through pixel (c, r), of the trilinear interpolant of vol (float32 [nx][ny][nz], values at the
 * voxel centres, zero outside the grid), by the midpoint rule over equal steps of at most half
 * the smallest voxel pitch (units: mm x volume units). Device pointers; the workspace's matrix
 * area is overwritten. GMC_E_UNSUPPORTED for an axis longer than 2^22 voxels or rays of more than
 * 2^24 steps. */
gmc_status gmc_forward_project(const gmc_plan* plan, const float* vol, const double* P, const double* theta,
                               float* proj_out, void* workspace, void* hip_stream);
/* Several independently moving rigid parts: voxel p belongs to part labels[p] (uint8 [nx][ny][nz],
 * values >= n_parts belong to no part); part k moves with theta[k] ([n_parts][n_views][6] float64)
 * and proj_out is the sum of the parts' projections. 1 <= n_parts <= 255; labels may be NULL
 * only for n_parts = 1. */
gmc_status gmc_forward_project_parts(const gmc_plan* plan, const float* vol, const uint8_t* labels, int32_t n_parts,
                                     const double* P, const double* theta, float* proj_out, void* workspace,
                                     void* hip_stream);

/* Motion model: uniform cubic B-spline per rigid parameter with n_nodes coefficients,
 * knots t_m = (m - 1) h, h = (n_views - 1)/(n_nodes - 3) (Sec. II-B.1 uses splines over
 * the views). coeffs [6][n_nodes] float64 in (mm, mm, mm, deg, deg, deg);
 * theta [n_views][6] float64 in (mm, rad). */
gmc_status gmc_bspline_theta(int32_t n_views, int32_t n_nodes, const double* coeffs, double* theta,
                             void* hip_stream);
/* Adjoint: grad_coeffs [6][n_nodes] = d/dcoeffs of <grad_theta, theta(coeffs)>. */
gmc_status gmc_bspline_grad(int32_t n_views, int32_t n_nodes, const double* grad_theta, double* grad_coeffs,
                            void* hip_stream);
/* The paper's motion model (Sec. II-B.1): an Akima spline per rigid parameter through
 * n_nodes node values evenly spaced over the views (node m at view m (n_views - 1)/(n_nodes - 1),
 * the first and the last node on the first and the last view). coeffs [6][n_nodes] float64
 * node values in (mm, mm, mm, deg, deg, deg); theta [n_views][6] float64 in (mm, rad).
 * 3 <= n_nodes <= 256, n_nodes <= n_views. */
gmc_status gmc_akima_theta(int32_t n_views, int32_t n_nodes, const double* coeffs, double* theta,
                           void* hip_stream);
/* Adjoint at coeffs: grad_coeffs [6][n_nodes] = (d theta / d coeffs)^T grad_theta. The spline is
 * not linear in its nodes (the node slopes weight neighbouring secants by their differences);
 * |x|' is taken as sign(x), 0 at 0. */
gmc_status gmc_akima_grad(int32_t n_views, int32_t n_nodes, const double* coeffs, const double* grad_theta,
                          double* grad_coeffs, void* hip_stream);
/* One Adam step (Kingma & Ba) on n float64 parameters x with gradient g and moments m, v;
 * step t >= 1. The paper's optimiser is gradient descent with decaying steps (Eq. 6). */
gmc_status gmc_adam_step(int64_t n, double* x, const double* g, double* m, double* v, int32_t t, double lr,
                         double beta1, double beta2, double eps, void* hip_stream);
/* Eq. 6: x <- x - s0 * decay^n * g. */
gmc_status gmc_gd_step(int64_t n, double* x, const double* g, int32_t n_iter, double s0, double decay,
                       void* hip_stream);

/* Geometry-index check: for n pairs (voxel linear index (i*ny + j)*nz + k, view), the
 * detector position exactly as the backprojection kernels compute it (after
 * gmc_backproject or gmc_backproject_vjp has run with this workspace): cell [n][2]
 * int32 = (floor(u/w), floor(v/w)) and frac [n][2] float32, detector pixel units. */
gmc_status gmc_debug_project(const gmc_plan* plan, int64_t n, const int64_t* voxel, const int32_t* view,
                             int32_t* cell, float* frac, const void* workspace, void* hip_stream);

/* Serving: several (plan, phase) work items in one backprojection launch.
 * phase 0 = backprojection (writes vol), 1 = VJP (writes grad_theta, and grad_P if set).
 * For each item the call first runs gmc_prepare (skipped when flags has GMC_WORK_PREPARED:
 * the caller already ran gmc_prepare on that workspace, with with_deriv = 1 for phase 1),
 * then ONE kernel launch processes the voxel bricks of all items of a phase together
 * (items are grouped by phase, weighting and gradient mode, at most 16 per launch), then
 * the VJP items are reduced and chained. Every item needs its own workspace. Items may
 * have different geometries; each result is bitwise identical to the corresponding single
 * call. */
enum { GMC_WORK_PREPARED = 1 };
typedef struct {
    const gmc_plan* plan;
    const float* proj;
    const double* P;
    const double* theta;
    float* vol;              /* phase 0 output                       */
    const float* grad_vol;   /* phase 1 input                        */
    double* grad_theta;      /* phase 1 output                       */
    double* grad_P;          /* phase 1 optional output (or NULL)    */
    void* workspace;
    int32_t phase;
    int32_t flags;           /* GMC_WORK_* bits                      */
} gmc_work;
gmc_status gmc_launch_batch(const gmc_work* items, int32_t n_items, void* hip_stream);

/* Synchronises the stream of the last call on this workspace (the default stream if
 * NULL) and returns GMC_E_GEOMETRY if any (brick, view) pair hit w <= 0 since the last
 * gmc_check on it, else GMC_OK. Clears the flag. */
gmc_status gmc_check(const gmc_plan* plan, void* workspace, void* hip_stream);

const char* gmc_status_string(gmc_status s);
const char* gmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMC_H */
