/*
 * Analytic line integrals of additive ellipsoid phantoms under per-view rigid motion
 * (input generator; the same computation as synth/project.py, in C with OpenMP over views).
 *
 * For view j the ray from source S_j through pixel (c, r) is mapped by T_j^-1 into the
 * phantom frame; the chord through an ellipsoid (centre ce, semi-axes ax, axes as the
 * columns of R) follows from the roots of |A^-1 R^T (s + t d - ce)|^2 = 1.
 * Only pixels inside the projected bounding box of each ellipsoid's bounding cube are
 * evaluated (all eight corners in front of the source, else the whole detector).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

void synth_line_integrals(int32_t n_views, int32_t W, int32_t H, double pitch, double dso, double dsd,
                          const double* betas, const double* Tinv, int32_t n_ell, const double* centres,
                          const double* axes, const double* rot, const double* mu, double* out) {
    const double c0 = (W - 1) / 2.0, r0 = (H - 1) / 2.0, f = dsd / pitch;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < n_views; ++j) {
        const double cb = cos(betas[j]), sb = sin(betas[j]);
        const double S[3] = {dso * cb, dso * sb, 0.0};
        const double eu[3] = {-sb, cb, 0.0}, ev[3] = {0.0, 0.0, 1.0}, ew[3] = {-cb, -sb, 0.0};
        const double* Ti = Tinv + 16 * j;
        double* img = out + (int64_t)j * W * H;
        memset(img, 0, sizeof(double) * (size_t)W * H);
        /* source in the phantom frame */
        double sp[3];
        for (int a = 0; a < 3; ++a) sp[a] = Ti[4 * a] * S[0] + Ti[4 * a + 1] * S[1] + Ti[4 * a + 2] * S[2] + Ti[4 * a + 3];
        for (int32_t e = 0; e < n_ell; ++e) {
            const double* ce = centres + 3 * e;
            const double* ax = axes + 3 * e;
            const double* R = rot + 9 * e;
            /* bounding sphere of the ellipsoid, moved to the world frame: x = T (ce) */
            double rad = ax[0] > ax[1] ? ax[0] : ax[1];
            if (ax[2] > rad) rad = ax[2];
            /* world centre: solve Ti x = ce for the rigid Ti: x = Ri^T (ce - ti) */
            double cw[3];
            for (int a = 0; a < 3; ++a)
                cw[a] = Ti[a] * (ce[0] - Ti[3]) + Ti[4 + a] * (ce[1] - Ti[7]) + Ti[8 + a] * (ce[2] - Ti[11]);
            int clo = 0, chi = W, rlo = 0, rhi = H;
            {
                double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
                int behind = 0;
                for (int q = 0; q < 8; ++q) {
                    double p[3] = {cw[0] + ((q & 1) ? rad : -rad), cw[1] + ((q & 2) ? rad : -rad),
                                   cw[2] + ((q & 4) ? rad : -rad)};
                    double v[3] = {p[0] - S[0], p[1] - S[1], p[2] - S[2]};
                    double depth = v[0] * ew[0] + v[1] * ew[1] + v[2] * ew[2];
                    if (depth <= 1e-6) { behind = 1; break; }
                    double u = f * (v[0] * eu[0] + v[1] * eu[1] + v[2] * eu[2]) / depth + c0;
                    double w = f * (v[0] * ev[0] + v[1] * ev[1] + v[2] * ev[2]) / depth + r0;
                    if (u < umin) umin = u;
                    if (u > umax) umax = u;
                    if (w < vmin) vmin = w;
                    if (w > vmax) vmax = w;
                }
                if (!behind) {
                    clo = (int)fmax(0.0, floor(umin) - 2);
                    chi = (int)fmin((double)W, ceil(umax) + 3);
                    rlo = (int)fmax(0.0, floor(vmin) - 2);
                    rhi = (int)fmin((double)H, ceil(vmax) + 3);
                }
            }
            /* ellipsoid frame: s' = A^-1 R^T (sp - ce) */
            double s1[3];
            for (int a = 0; a < 3; ++a)
                s1[a] = (R[a] * (sp[0] - ce[0]) + R[3 + a] * (sp[1] - ce[1]) + R[6 + a] * (sp[2] - ce[2])) / ax[a];
            const double C = s1[0] * s1[0] + s1[1] * s1[1] + s1[2] * s1[2] - 1.0;
            for (int r = rlo; r < rhi; ++r) {
                const double b = (r - r0) * pitch;
                for (int c = clo; c < chi; ++c) {
                    const double a_ = (c - c0) * pitch;
                    double d[3];
                    for (int k = 0; k < 3; ++k) d[k] = dsd * ew[k] + a_ * eu[k] + b * ev[k];
                    const double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    /* direction in the phantom frame (rotation part of Ti), unit length */
                    double dp[3];
                    for (int k = 0; k < 3; ++k) dp[k] = (Ti[4 * k] * d[0] + Ti[4 * k + 1] * d[1] + Ti[4 * k + 2] * d[2]) / n;
                    double d1[3];
                    for (int k = 0; k < 3; ++k) d1[k] = (R[k] * dp[0] + R[3 + k] * dp[1] + R[6 + k] * dp[2]) / ax[k];
                    const double A = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
                    const double B = d1[0] * s1[0] + d1[1] * s1[1] + d1[2] * s1[2];
                    const double disc = B * B - A * C;
                    if (disc > 0.0) img[(int64_t)r * W + c] += mu[e] * 2.0 * sqrt(disc) / A;
                }
            }
        }
    }
}
