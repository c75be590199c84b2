/*
 * FP64 CPU oracle of the motion-compensation hot path (test infrastructure).
 *
 * This file is the reference that the GPU path is checked against. It is
 * deliberately plain: one voxel and one view at a time, straight from the
 * definitions, in double precision. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product never does.
 *
 * What it computes (Thies et al., "A gradient-based approach to fast and
 * accurate head motion compensation in cone-beam CT"):
 *   - Eq. 1: updated projection matrices  Phat_j = P_j * T_j(theta_j), with
 *     T = [Rz(rz) Ry(ry) Rx(rx) | (tx, ty, tz)] (six rigid parameters per view,
 *     Sec. II-A / II-B.1), and the six derivative matrices P_j * dT_j/dtheta_jk.
 *   - Eq. 3: voxel-driven backprojection I(p) = sum_j omega_j(p) d_j(g(Phat_j p~)),
 *     with bilinear interpolation of the filtered projection d_j at the
 *     dehomogenised detector position. omega = 1 is Eq. 3 as printed
 *     ("paper" weighting); omega = 1/w^2 is the FDK distance weight used when
 *     the matrices are scaled so that w = 1 at the isocentre ("fdk" weighting).
 *   - Eq. 4-5: the derivative of I(p) with respect to the 12 entries of Phat_j,
 *     contracted with a volume seed delta = dL/dI into G_j = sum_p delta(p) dI(p)/dPhat_j.
 *     g_u, g_v are bilinear samples of the central-difference images of d_j
 *     (Sec. II-B.2: central differences in the interior, one-sided at the
 *     detector edge, per pixel). An optional "exact" mode uses the derivative
 *     of the bilinear interpolant instead.
 *   - Eq. 2: the chain to the rigid parameters, dL/dtheta_jk = <G_j, dPhat_j/dtheta_jk>.
 *
 * Readings where the paper is silent (each is also taken by the GPU path):
 *   - pixel centres sit at integer detector coordinates; a bilinear tap outside
 *     [0, W-1] x [0, H-1] contributes zero (to d and to the gradient images);
 *   - projection data are stored [view][row][column], column (u) fastest;
 *   - the volume is stored [i][j][k], k (z) fastest, voxel (i,j,k) centred at
 *     origin + (i,j,k) * voxel;
 *   - a voxel with w <= 0 (at or behind the source plane) contributes nothing
 *     and is counted, so the caller can reject such a geometry.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    int32_t n_views, det_w, det_h;
    int32_t nx, ny, nz;
    double voxel[3];
    double origin[3];
    int32_t weighting; /* 0: Eq. 3 as printed (omega = 1); 1: FDK, omega = 1/w^2 */
    int32_t grad_mode; /* 0: interpolated central differences (Sec. II-B.2); 1: exact bilinear derivative */
} og_geom;

/* ---------------------------------------------------------------- Eq. 1 */

/* T(theta) = [Rz(rz) Ry(ry) Rx(rx) | t; 0 0 0 1]  and its six partial derivatives. */
static void mat3_mul(const double A[3][3], const double B[3][3], double C[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
            C[i][j] = s;
        }
}

static void rot_parts(double rx, double ry, double rz, double Rx[3][3], double Ry[3][3], double Rz[3][3],
                      double dRx[3][3], double dRy[3][3], double dRz[3][3]) {
    double cx = cos(rx), sx = sin(rx), cy = cos(ry), sy = sin(ry), cz = cos(rz), sz = sin(rz);
    double rx_[3][3] = {{1, 0, 0}, {0, cx, -sx}, {0, sx, cx}};
    double ry_[3][3] = {{cy, 0, sy}, {0, 1, 0}, {-sy, 0, cy}};
    double rz_[3][3] = {{cz, -sz, 0}, {sz, cz, 0}, {0, 0, 1}};
    double drx[3][3] = {{0, 0, 0}, {0, -sx, -cx}, {0, cx, -sx}};
    double dry[3][3] = {{-sy, 0, cy}, {0, 0, 0}, {-cy, 0, -sy}};
    double drz[3][3] = {{-sz, -cz, 0}, {cz, -sz, 0}, {0, 0, 0}};
    memcpy(Rx, rx_, sizeof rx_); memcpy(Ry, ry_, sizeof ry_); memcpy(Rz, rz_, sizeof rz_);
    memcpy(dRx, drx, sizeof drx); memcpy(dRy, dry, sizeof dry); memcpy(dRz, drz, sizeof drz);
}

void oracle_rigid(const double th[6], double T[16], double dT[6 * 16]) {
    double Rx[3][3], Ry[3][3], Rz[3][3], dRx[3][3], dRy[3][3], dRz[3][3], A[3][3], R[3][3];
    rot_parts(th[3], th[4], th[5], Rx, Ry, Rz, dRx, dRy, dRz);
    mat3_mul(Ry, Rx, A);
    mat3_mul(Rz, A, R);
    memset(T, 0, 16 * sizeof(double));
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T[i * 4 + j] = R[i][j];
        T[i * 4 + 3] = th[i];
    }
    T[15] = 1.0;
    if (!dT) return;
    memset(dT, 0, 6 * 16 * sizeof(double));
    for (int k = 0; k < 3; ++k) dT[k * 16 + k * 4 + 3] = 1.0; /* d/dt_k: unit entry in column 3 */
    double B[3][3], D[3][3];
    /* d/drx = Rz Ry dRx */
    mat3_mul(Ry, dRx, B); mat3_mul(Rz, B, D);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) dT[3 * 16 + i * 4 + j] = D[i][j];
    /* d/dry = Rz dRy Rx */
    mat3_mul(dRy, Rx, B); mat3_mul(Rz, B, D);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) dT[4 * 16 + i * 4 + j] = D[i][j];
    /* d/drz = dRz Ry Rx */
    mat3_mul(Ry, Rx, B); mat3_mul(dRz, B, D);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) dT[5 * 16 + i * 4 + j] = D[i][j];
}

/* Phat_j = P_j T_j (Eq. 1) and dPhat_j/dtheta_jk = P_j dT_j/dtheta_jk.
 * theta [n][6], P [n][3][4], Phat [n][3][4], dPhat [n][6][3][4] (may be NULL). */
void oracle_compose(int32_t n, const double* theta, const double* P, double* Phat, double* dPhat) {
    for (int32_t j = 0; j < n; ++j) {
        double T[16], dT[96];
        oracle_rigid(theta + 6 * j, T, dPhat ? dT : NULL);
        const double* Pj = P + 12 * j;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += Pj[r * 4 + k] * T[k * 4 + c];
                Phat[12 * j + r * 4 + c] = s;
            }
        if (!dPhat) continue;
        for (int q = 0; q < 6; ++q)
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 4; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < 4; ++k) s += Pj[r * 4 + k] * dT[q * 16 + k * 4 + c];
                    dPhat[72 * j + 12 * q + r * 4 + c] = s;
                }
    }
}

/* ------------------------------------------------------- detector sampling */

/* d_j[r][c], zero outside the detector */
static double pix(const og_geom* g, const float* img, long r, long c) {
    if (c < 0 || c >= g->det_w || r < 0 || r >= g->det_h) return 0.0;
    return (double)img[r * (long)g->det_w + c];
}

/* Central-difference images of Sec. II-B.2 (per pixel): (d[c+1] - d[c-1]) / 2 inside,
 * one-sided d[1]-d[0] and d[W-1]-d[W-2] at the edges; zero outside the detector. */
static double grad_u_pix(const og_geom* g, const float* img, long r, long c) {
    long W = g->det_w;
    if (c < 0 || c >= W || r < 0 || r >= g->det_h || W < 2) return 0.0;
    if (c == 0) return pix(g, img, r, 1) - pix(g, img, r, 0);
    if (c == W - 1) return pix(g, img, r, W - 1) - pix(g, img, r, W - 2);
    return 0.5 * (pix(g, img, r, c + 1) - pix(g, img, r, c - 1));
}

static double grad_v_pix(const og_geom* g, const float* img, long r, long c) {
    long H = g->det_h;
    if (c < 0 || c >= g->det_w || r < 0 || r >= H || H < 2) return 0.0;
    if (r == 0) return pix(g, img, 1, c) - pix(g, img, 0, c);
    if (r == H - 1) return pix(g, img, H - 1, c) - pix(g, img, H - 2, c);
    return 0.5 * (pix(g, img, r + 1, c) - pix(g, img, r - 1, c));
}

typedef double (*pixfn)(const og_geom*, const float*, long, long);

/* bilinear interpolation of a per-pixel function at detector position (uh, vh) */
static double bilinear(const og_geom* g, const float* img, pixfn f, double uh, double vh) {
    double cf = floor(uh), rf = floor(vh);
    long c0 = (long)cf, r0 = (long)rf;
    double a = uh - cf, b = vh - rf;
    return (1 - a) * (1 - b) * f(g, img, r0, c0) + a * (1 - b) * f(g, img, r0, c0 + 1) +
           (1 - a) * b * f(g, img, r0 + 1, c0) + a * b * f(g, img, r0 + 1, c0 + 1);
}

/* homogeneous projection (u, v, w) = Phat * (x, y, z, 1) */
static void project(const double* Ph, const double p[3], double uvw[3]) {
    for (int r = 0; r < 3; ++r)
        uvw[r] = Ph[r * 4 + 0] * p[0] + Ph[r * 4 + 1] * p[1] + Ph[r * 4 + 2] * p[2] + Ph[r * 4 + 3];
}

static void voxel_centre(const og_geom* g, long i, long j, long k, double p[3]) {
    p[0] = g->origin[0] + (double)i * g->voxel[0];
    p[1] = g->origin[1] + (double)j * g->voxel[1];
    p[2] = g->origin[2] + (double)k * g->voxel[2];
}

/* one view's contribution omega * d_j(uh, vh) at world point p; returns 0 and sets *bad if w <= 0 */
static double view_value(const og_geom* g, const float* img, const double* Ph, const double p[3], int* bad) {
    double uvw[3];
    project(Ph, p, uvw);
    if (!(uvw[2] > 0.0)) { *bad = 1; return 0.0; }
    double uh = uvw[0] / uvw[2], vh = uvw[1] / uvw[2];
    double val = bilinear(g, img, pix, uh, vh);
    if (g->weighting == 1) val /= uvw[2] * uvw[2];
    return val;
}

/* ---------------------------------------------------------------- Eq. 3 */

/* I(p) at arbitrary world points pts [n_pts][3]; views [view_lo, view_hi). Returns the number of
 * (point, view) pairs with w <= 0. */
int64_t oracle_backproject_points(const og_geom* g, const float* proj, const double* Phat, int64_t n_pts,
                                  const double* pts, int32_t view_lo, int32_t view_hi, double* out) {
    int64_t nbad = 0;
    const long plane = (long)g->det_w * g->det_h;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nbad)
    for (int64_t q = 0; q < n_pts; ++q) {
        double s = 0.0;
        for (int32_t j = view_lo; j < view_hi; ++j) {
            int bad = 0;
            s += view_value(g, proj + (long)j * plane, Phat + 12 * j, pts + 3 * q, &bad);
            nbad += bad;
        }
        out[q] = s;
    }
    return nbad;
}

/* Full volume, [nx][ny][nz] z fastest. */
int64_t oracle_backproject(const og_geom* g, const float* proj, const double* Phat, double* vol) {
    int64_t nbad = 0;
    const long plane = (long)g->det_w * g->det_h;
    const long nyz = (long)g->ny * g->nz;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nbad)
    for (long ij = 0; ij < (long)g->nx * g->ny; ++ij) {
        long i = ij / g->ny, jj = ij % g->ny;
        for (long k = 0; k < g->nz; ++k) {
            double p[3];
            voxel_centre(g, i, jj, k, p);
            double s = 0.0;
            for (int32_t v = 0; v < g->n_views; ++v) {
                int bad = 0;
                s += view_value(g, proj + (long)v * plane, Phat + 12 * v, p, &bad);
                nbad += bad;
            }
            vol[i * nyz + jj * g->nz + k] = s;
        }
    }
    return nbad;
}

/* Voxels given by linear index (i*ny + j)*nz + k. */
int64_t oracle_backproject_voxels(const og_geom* g, const float* proj, const double* Phat, int64_t n_idx,
                                  const int64_t* idx, double* out) {
    int64_t nbad = 0;
    const long plane = (long)g->det_w * g->det_h;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nbad)
    for (int64_t q = 0; q < n_idx; ++q) {
        long L = (long)idx[q];
        long k = L % g->nz, jj = (L / g->nz) % g->ny, i = L / ((long)g->nz * g->ny);
        double p[3];
        voxel_centre(g, i, jj, k, p);
        double s = 0.0;
        for (int32_t v = 0; v < g->n_views; ++v) {
            int bad = 0;
            s += view_value(g, proj + (long)v * plane, Phat + 12 * v, p, &bad);
            nbad += bad;
        }
        out[q] = s;
    }
    return nbad;
}

/* ------------------------------------------------------------- Eq. 4-5 */

/* dI_j(p)/dPhat_j (3x4, row-major) at world point p, added with factor delta into G. */
static int add_view_jacobian(const og_geom* g, const float* img, const double* Ph, const double p[3],
                             double delta, double G[12]) {
    double uvw[3];
    project(Ph, p, uvw);
    double w = uvw[2];
    if (!(w > 0.0)) return 1;
    double uh = uvw[0] / w, vh = uvw[1] / w;
    double gu, gv;
    if (g->grad_mode == 0) {
        gu = bilinear(g, img, grad_u_pix, uh, vh);
        gv = bilinear(g, img, grad_v_pix, uh, vh);
    } else {
        /* derivative of the bilinear interpolant itself */
        double cf = floor(uh), rf = floor(vh);
        long c0 = (long)cf, r0 = (long)rf;
        double a = uh - cf, b = vh - rf;
        double d00 = pix(g, img, r0, c0), d01 = pix(g, img, r0, c0 + 1);
        double d10 = pix(g, img, r0 + 1, c0), d11 = pix(g, img, r0 + 1, c0 + 1);
        gu = (1 - b) * (d01 - d00) + b * (d11 - d10);
        gv = (1 - a) * (d10 - d00) + a * (d11 - d01);
    }
    double pt[4] = {p[0], p[1], p[2], 1.0};
    double row[3];
    if (g->weighting == 0) {
        /* Eq. 4 with h(i) = g_u i u + g_v i v (Eq. 5): rows g_u p~/w, g_v p~/w, -(g_u u + g_v v) p~/w^2 */
        row[0] = gu / w;
        row[1] = gv / w;
        row[2] = -(gu * uvw[0] + gv * uvw[1]) / (w * w);
    } else {
        /* I_j = d(u/w, v/w) / w^2: rows g_u p~/w^3, g_v p~/w^3, -(g_u uh + g_v vh + 2 d) p~/w^3 */
        double val = bilinear(g, img, pix, uh, vh);
        double w3 = w * w * w;
        row[0] = gu / w3;
        row[1] = gv / w3;
        row[2] = -(gu * uh + gv * vh + 2.0 * val) / w3;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) G[r * 4 + c] += delta * row[r] * pt[c];
    return 0;
}

/* G_j = sum_p delta(p) dI(p)/dPhat_j for every view (G [n_views][3][4]); delta is the full
 * volume seed, [nx][ny][nz] z fastest. Views are independent; each sums voxels in index order. */
int64_t oracle_vjp(const og_geom* g, const float* proj, const double* Phat, const double* delta, double* G) {
    int64_t nbad = 0;
    const long plane = (long)g->det_w * g->det_h;
    const long nyz = (long)g->ny * g->nz;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nbad)
    for (int32_t v = 0; v < g->n_views; ++v) {
        double acc[12] = {0};
        for (long i = 0; i < g->nx; ++i)
            for (long jj = 0; jj < g->ny; ++jj)
                for (long k = 0; k < g->nz; ++k) {
                    double dv = delta[i * nyz + jj * g->nz + k];
                    if (dv == 0.0) continue;
                    double p[3];
                    voxel_centre(g, i, jj, k, p);
                    nbad += add_view_jacobian(g, proj + (long)v * plane, Phat + 12 * v, p, dv, acc);
                }
        memcpy(G + 12 * v, acc, sizeof acc);
    }
    return nbad;
}

/* Same with a sparse seed: delta is nonzero only at voxels idx[q] (linear index) with value dval[q]. */
int64_t oracle_vjp_sparse(const og_geom* g, const float* proj, const double* Phat, int64_t n_idx,
                          const int64_t* idx, const double* dval, double* G) {
    int64_t nbad = 0;
    const long plane = (long)g->det_w * g->det_h;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nbad)
    for (int32_t v = 0; v < g->n_views; ++v) {
        double acc[12] = {0};
        for (int64_t q = 0; q < n_idx; ++q) {
            long L = (long)idx[q];
            long k = L % g->nz, jj = (L / g->nz) % g->ny, i = L / ((long)g->nz * g->ny);
            double p[3];
            voxel_centre(g, i, jj, k, p);
            nbad += add_view_jacobian(g, proj + (long)v * plane, Phat + 12 * v, p, dval[q], acc);
        }
        memcpy(G + 12 * v, acc, sizeof acc);
    }
    return nbad;
}

/* dI(p)/dPhat_j at arbitrary points, one 3x4 block per (point, view) pair:
 * out [n_pts][view_hi-view_lo][12]. */
int64_t oracle_point_jacobian(const og_geom* g, const float* proj, const double* Phat, int64_t n_pts,
                              const double* pts, int32_t view_lo, int32_t view_hi, double* out) {
    int64_t nbad = 0;
    const long plane = (long)g->det_w * g->det_h;
    const int32_t nv = view_hi - view_lo;
    for (int64_t q = 0; q < n_pts; ++q)
        for (int32_t v = view_lo; v < view_hi; ++v) {
            double* o = out + (q * nv + (v - view_lo)) * 12;
            memset(o, 0, 12 * sizeof(double));
            nbad += add_view_jacobian(g, proj + (long)v * plane, Phat + 12 * v, pts + 3 * q, 1.0, o);
        }
    return nbad;
}

/* ---------------------------------------------------------------- Eq. 2 */

/* dL/dtheta_jk = sum_{r,c} G_j[r][c] dPhat_jk[r][c]; G [n][12], dPhat [n][6][12], out [n][6]. */
void oracle_chain(int32_t n, const double* G, const double* dPhat, double* grad_theta) {
    for (int32_t j = 0; j < n; ++j)
        for (int q = 0; q < 6; ++q) {
            double s = 0.0;
            for (int e = 0; e < 12; ++e) s += G[12 * j + e] * dPhat[72 * j + 12 * q + e];
            grad_theta[6 * j + q] = s;
        }
}

/* (uh, vh, w) of points under each view, FP64: out [n_pts][3] for one view. */
void oracle_project_points(const double* Ph, int64_t n_pts, const double* pts, double* out) {
    for (int64_t q = 0; q < n_pts; ++q) {
        double uvw[3];
        project(Ph, pts + 3 * q, uvw);
        out[3 * q + 0] = uvw[0] / uvw[2];
        out[3 * q + 1] = uvw[1] / uvw[2];
        out[3 * q + 2] = uvw[2];
    }
}

/* ---------------------------------------------------------------- ray-driven forward projection
 *
 * The adjoint partner of the backprojection (used to simulate scans under Phat_j): the line
 * integral, along the ray from the source through pixel (c, r), of the trilinear interpolant
 * of the volume (voxel values at the voxel centres, zero outside the grid).
 *
 * Ray: with Phat = [M | p4], the source is C = -M^-1 p4 and the points projecting to (c, r)
 * are C + w M^-1 (c, r, 1)^T, w the depth. The interpolant is supported in the box of voxel
 * coordinates [-1, n] per axis; the ray's w-interval inside that box is split into
 * N = ceil(length / h) equal steps (h = step_vox times the smallest voxel pitch) and the
 * integral is the midpoint sum over them (mm x volume units). Volume [i][j][k], k fastest;
 * out [n_views][det_h][det_w]; labels (optional, 255 = none) select the voxels of part `part`. */
static void mat3_inv(const double A[3][3], double B[3][3]) {
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

static double voxel_value(const og_geom* g, const float* vol, const uint8_t* labels, int part, long i, long j,
                          long k) {
    if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return 0.0;
    const long idx = (i * g->ny + j) * g->nz + k;
    if (labels && labels[idx] != part) return 0.0;
    return (double)vol[idx];
}

static double trilinear(const og_geom* g, const float* vol, const uint8_t* labels, int part, const double q[3]) {
    const double fi = floor(q[0]), fj = floor(q[1]), fk = floor(q[2]);
    const double a = q[0] - fi, b = q[1] - fj, c = q[2] - fk;
    const long i = (long)fi, j = (long)fj, k = (long)fk;
    double s = 0.0;
    for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj)
            for (int dk = 0; dk < 2; ++dk) {
                const double w = (di ? a : 1.0 - a) * (dj ? b : 1.0 - b) * (dk ? c : 1.0 - c);
                s += w * voxel_value(g, vol, labels, part, i + di, j + dj, k + dk);
            }
    return s;
}

void oracle_forward_project(const og_geom* g, const float* vol, const uint8_t* labels, int32_t part,
                            const double* Phat, double step_vox, int32_t view_lo, int32_t view_hi, double* out) {
    const double vmin = fmin(g->voxel[0], fmin(g->voxel[1], g->voxel[2]));
    const double h = step_vox * vmin;
    const int n[3] = {g->nx, g->ny, g->nz};
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int32_t jv = view_lo; jv < view_hi; ++jv)
        for (int32_t r = 0; r < g->det_h; ++r) {
            const double* Ph = Phat + 12 * jv;
            const double M[3][3] = {{Ph[0], Ph[1], Ph[2]}, {Ph[4], Ph[5], Ph[6]}, {Ph[8], Ph[9], Ph[10]}};
            double Mi[3][3];
            mat3_inv(M, Mi);
            double C[3];
            for (int a = 0; a < 3; ++a) C[a] = -(Mi[a][0] * Ph[3] + Mi[a][1] * Ph[7] + Mi[a][2] * Ph[11]);
            for (int32_t c = 0; c < g->det_w; ++c) {
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = Mi[a][0] * c + Mi[a][1] * r + Mi[a][2];
                /* voxel coordinates: q(w) = (C + w d - origin) / voxel */
                double q0[3], dq[3], t0 = -INFINITY, t1 = INFINITY;
                int empty = 0;
                for (int a = 0; a < 3; ++a) {
                    q0[a] = (C[a] - g->origin[a]) / g->voxel[a];
                    dq[a] = d[a] / g->voxel[a];
                    const double lo = -1.0, hi = (double)n[a];
                    if (dq[a] == 0.0) {
                        if (q0[a] <= lo || q0[a] >= hi) empty = 1;
                    } else {
                        double ta = (lo - q0[a]) / dq[a], tb = (hi - q0[a]) / dq[a];
                        if (ta > tb) { const double x = ta; ta = tb; tb = x; }
                        t0 = fmax(t0, ta);
                        t1 = fmin(t1, tb);
                    }
                }
                double sum = 0.0;
                if (!empty && t1 > t0) {
                    const double len = (t1 - t0) * sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    const long N = (long)ceil(len / h - 1e-9);   /* an exact multiple of h is not split further */
                    const double dt = (t1 - t0) / (double)N;
                    for (long s = 0; s < N; ++s) {
                        const double t = t0 + ((double)s + 0.5) * dt;
                        const double q[3] = {q0[0] + t * dq[0], q0[1] + t * dq[1], q0[2] + t * dq[2]};
                        sum += trilinear(g, vol, labels, part, q);
                    }
                    sum *= len / (double)N;
                }
                out[((long)jv * g->det_h + r) * g->det_w + c] = sum;
            }
        }
}
