// C ABI of libgmc: plans, argument validation, workspace layout and the call sequences of
// the hot path (compose -> brick descriptors -> backprojection / VJP -> reduce and chain).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <new>
#include <string>
#include <vector>

#include "gmc_internal.hpp"

using namespace gmc;

namespace {

thread_local std::string g_last_error;

gmc_status fail(gmc_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

gmc_status hip_fail(hipError_t e, const char* where) {
    return fail(GMC_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool finite3(const double* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

gmc_status validate_geometry(const gmc_geometry* g) {
    if (!g) return fail(GMC_E_INVALID, "geometry is NULL");
    if (g->n_views < 1 || g->det_w < 1 || g->det_h < 1 || g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(GMC_E_INVALID, "sizes must be >= 1 (n_views=%d det=%dx%d vol=%dx%dx%d)", g->n_views, g->det_w,
                    g->det_h, g->nx, g->ny, g->nz);
    if (!finite3(g->voxel_mm) || g->voxel_mm[0] <= 0 || g->voxel_mm[1] <= 0 || g->voxel_mm[2] <= 0)
        return fail(GMC_E_INVALID, "voxel size must be finite and > 0");
    if (!finite3(g->origin_mm)) return fail(GMC_E_INVALID, "origin must be finite");
    if (g->weighting != GMC_WEIGHT_PAPER && g->weighting != GMC_WEIGHT_FDK)
        return fail(GMC_E_INVALID, "weighting must be GMC_WEIGHT_PAPER or GMC_WEIGHT_FDK");
    if (g->grad_mode != GMC_GRAD_PAPER && g->grad_mode != GMC_GRAD_EXACT)
        return fail(GMC_E_INVALID, "grad_mode must be GMC_GRAD_PAPER or GMC_GRAD_EXACT");
    if (g->flags & ~(GMC_FLAG_FORCE_GLOBAL | GMC_FLAG_FORCE_EDGE)) return fail(GMC_E_INVALID, "unknown flag bits 0x%x", g->flags);
    const long long nvox = (long long)g->nx * g->ny * g->nz;
    if (nvox > (1LL << 40) || (long long)g->det_w * g->det_h > (1LL << 31))
        return fail(GMC_E_UNSUPPORTED, "volume or detector too large");
    return GMC_OK;
}

// Same tile rule as k_setup, on the host and for the nominal matrices: the largest tile.
// Tile extents (columns, rows) of the nominal (motion-free) geometry for every brick whose tile
// meets the detector: every view for short scans, a subsample of long ones (a sizing
// heuristic: a tile that exceeds the chosen LDS tile at run time is sampled from global memory
// instead).
void nominal_tile_extents(const gmc_plan* p, const double* P, std::vector<std::pair<int, int>>& out) {
    const gmc_geometry& g = p->g;
    const double ext[3] = {(BXY - 1) * g.voxel_mm[0], (BXY - 1) * g.voxel_mm[1], (p->bz - 1) * g.voxel_mm[2]};
    const int vstride = std::max(1, g.n_views / 128);
    for (int v = 0; v < g.n_views; v += vstride) {
        const double* Ph = P + 12 * v;
        for (int b = 0; b < p->n_bricks; ++b) {
            const int bj = b % p->nby, bi = (b / p->nby) % p->nbx, bk = b / (p->nby * p->nbx);
            const double o[3] = {g.origin_mm[0] + (double)(bi * BXY) * g.voxel_mm[0],
                                 g.origin_mm[1] + (double)(bj * BXY) * g.voxel_mm[1],
                                 g.origin_mm[2] + (double)(bk * p->bz) * g.voxel_mm[2]};
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            bool bad = false;
            for (int c = 0; c < 8; ++c) {
                const double x = o[0] + ((c & 1) ? ext[0] : 0.0), y = o[1] + ((c & 2) ? ext[1] : 0.0),
                             z = o[2] + ((c & 4) ? ext[2] : 0.0);
                const double w = Ph[8] * x + Ph[9] * y + Ph[10] * z + Ph[11];
                if (!(w > 0.0)) { bad = true; break; }
                const double uh = (Ph[0] * x + Ph[1] * y + Ph[2] * z + Ph[3]) / w;
                const double vh = (Ph[4] * x + Ph[5] * y + Ph[6] * z + Ph[7]) / w;
                umin = std::min(umin, uh); umax = std::max(umax, uh);
                vmin = std::min(vmin, vh); vmax = std::max(vmax, vh);
            }
            if (bad || !(umax - umin < 1e6) || !(vmax - vmin < 1e6)) continue;
            const int tw = (int)(floor(umax) + 1.0 - floor(umin)) + 5;
            const int th = (int)(floor(vmax) + 1.0 - floor(vmin)) + 5;
            const int ou = (int)floor(umin) - 2, ov = (int)floor(vmin) - 2;
            if (ou + tw <= 0 || ou >= g.det_w || ov + th <= 0 || ov >= g.det_h) continue;
            out.emplace_back(tw, th);
        }
    }
}

// The smallest tile configuration of the plan's brick depth that holds at least 99 % of the
// nominal tiles with two columns and rows to spare for motion (a smaller LDS tile fits more
// workgroups per CU; the rest are sampled from global memory); N_TILE_CFGS when none does.
int choose_tile_cfg(const gmc_plan* p, const double* P) {
    std::vector<std::pair<int, int>> ext;
    nominal_tile_extents(p, P, ext);
    if (ext.empty()) return 0;
    const TileCfg* cfgs = TILE_CFGS[depth_index(p->bz)];
    for (int c = 0; c < N_TILE_CFGS; ++c) {
        size_t fit = 0;
        for (const auto& e : ext)
            if (e.first + 2 <= cfgs[c].tp && e.second + 2 <= cfgs[c].th) ++fit;
        if (fit >= (size_t)(0.99 * (double)ext.size())) return c;
    }
    return N_TILE_CFGS;
}

void set_depth(gmc_plan* p, int bz) {
    p->bz = bz;
    p->nbx = (p->g.nx + BXY - 1) / BXY;
    p->nby = (p->g.ny + BXY - 1) / BXY;
    p->nbz = (p->g.nz + bz - 1) / bz;
    p->n_bricks = (int)std::min<long long>((long long)p->nbx * p->nby * p->nbz, 1LL << 30);
}

struct WS {
    double* Phat;
    double* dPhat;
    BrickDesc* desc;
    float* part;
    double* G;
    int* status;
    float* loss;
    float* hist;
    float* vpart;
};

WS carve(const gmc_plan* p, void* ws) {
    char* b = (char*)ws;
    WS w;
    w.Phat = (double*)(b + p->off_phat);
    w.dPhat = (double*)(b + p->off_dphat);
    w.desc = (BrickDesc*)(b + p->off_desc);
    w.part = (float*)(b + p->off_part);
    w.G = (double*)(b + p->off_G);
    w.status = (int*)(b + p->off_status);
    w.loss = (float*)(b + p->off_loss);
    w.hist = (float*)(b + p->off_hist);
    w.vpart = (float*)(b + p->off_vpart);
    return w;
}

gmc_status check_plan_ws(const gmc_plan* p, const void* ws) {
    if (!p) return fail(GMC_E_INVALID, "plan is NULL");
    if (!ws) return fail(GMC_E_WORKSPACE, "workspace is NULL (need %zu bytes)", p->ws_bytes);
    if (((uintptr_t)ws) & 255) return fail(GMC_E_WORKSPACE, "workspace must be 256-byte aligned");
    return GMC_OK;
}

BpArgs bp_args(const gmc_plan* p, const float* proj, const WS& w, bool vjp) {
    BpArgs a;
    a.proj = proj;
    a.desc = w.desc;
    a.vol = nullptr;
    a.gvol = nullptr;
    a.part = w.part;
    a.nx = p->g.nx;
    a.ny = p->g.ny;
    a.nz = p->g.nz;
    a.W = p->g.det_w;
    a.H = p->g.det_h;
    a.n_views = p->g.n_views;
    a.nbx = p->nbx;
    a.nby = p->nby;
    a.nbz = p->nbz;
    a.n_bricks = p->n_bricks;
    a.vsplit = vjp ? p->vsplit_vjp : p->vsplit_fwd;
    a.vpart = w.vpart;
    a.per_xcd = (int)(((long long)p->n_bricks * a.vsplit + 7) / 8);
    a.dx = (float)p->g.voxel_mm[0];
    a.dy = (float)p->g.voxel_mm[1];
    a.dz = (float)p->g.voxel_mm[2];
    a.plane = (long long)p->g.det_w * p->g.det_h;
    return a;
}

__global__ void k_clear_int(int* p) { *p = 0; }

gmc_status prepare(const gmc_plan* p, const double* P, const double* theta, const WS& w, bool with_deriv,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, s, w.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "clear status");
    e = launch_compose(theta, P, w.Phat, with_deriv ? w.dPhat : nullptr, p->g.n_views, s);
    if (e != hipSuccess) return hip_fail(e, "compose");
    e = launch_setup(p, w.Phat, w.desc, w.status, s);
    if (e != hipSuccess) return hip_fail(e, "brick setup");
    return GMC_OK;
}

// ---------------------------------------------------------------- allocation-free VJP
//
// gmc_backproject_vjp_noalloc carves its workspace from this file-scope device array instead of
// a caller-owned buffer. In host code the name `scratch` is a host-side stand-in, not a device
// address: the address comes from hipGetSymbolAddress, once per device with that device current,
// and only that pointer reaches kernels. Every GPU the library runs on holds its own copy of the
// array until the process ends.
static __device__ __align__(256) unsigned char scratch[GMC_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

gmc_status scratch_of_current_device(hipStream_t stream, void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    // the buffer is the current device's: a stream of another device would run the kernels there
    if (stream) {
        hipDevice_t sdev = -1;
        e = hipStreamGetDevice(stream, &sdev);
        if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
        if (sdev != dev)
            return fail(GMC_E_INVALID, "the stream belongs to device %d but device %d is current", (int)sdev, dev);
    }
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(GMC_E_UNSUPPORTED, "device %d: the allocation-free entry point serves devices 0..%d", dev,
                    NOALLOC_MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(GMC_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GMC_OK;
}

__global__ void k_copy_int(const int* src, int32_t* dst) { *dst = *src; }

}  // namespace

extern "C" {

gmc_status gmc_plan_create(const gmc_geometry* g, const double* P_nominal, gmc_plan** out) {
    if (!out) return fail(GMC_E_INVALID, "out is NULL");
    *out = nullptr;
    gmc_status st = validate_geometry(g);
    if (st != GMC_OK) return st;
    gmc_plan* p = new (std::nothrow) gmc_plan();
    if (!p) return fail(GMC_E_INVALID, "out of host memory");
    p->g = *g;
    // work items (brick, view chunk) are numbered in 32 bits: at most 2^26 bricks (and 2^30 items)
    {
        const long long nb = (long long)((g->nx + BXY - 1) / BXY) * ((g->ny + BXY - 1) / BXY) *
                             ((g->nz + BZ_DEEP - 1) / BZ_DEEP);
        if (nb > (1LL << 26) || nb * g->n_views > (1LL << 33)) {
            delete p;
            return fail(GMC_E_UNSUPPORTED, "too many (brick, view) pairs");
        }
    }
    // Deep bricks with the middle tile when no nominal geometry is given. With one: deep bricks
    // if their tiles fit the small or middle configuration, else shallow bricks with the
    // smallest configuration that holds theirs (the largest when none does).
    set_depth(p, BZ_DEEP);
    p->tile_cfg = 1;
    if (P_nominal) {
        for (long long e = 0; e < 12LL * g->n_views; ++e)
            if (!isfinite(P_nominal[e])) {
                delete p;
                return fail(GMC_E_INVALID, "P_nominal has a non-finite entry");
            }
        p->tile_cfg = choose_tile_cfg(p, P_nominal);
        const long long nb_shallow = (long long)p->nbx * p->nby * ((g->nz + BZ_SHALLOW - 1) / BZ_SHALLOW);
        if (p->tile_cfg >= N_TILE_CFGS - 1 && nb_shallow <= (1LL << 26) && nb_shallow * g->n_views <= (1LL << 33)) {
            set_depth(p, BZ_SHALLOW);
            p->tile_cfg = choose_tile_cfg(p, P_nominal);
        }
        p->tile_cfg = std::min(p->tile_cfg, N_TILE_CFGS - 1);
    }
    const long long nb = p->n_bricks;
    // Each brick's views are split into chunks, one workgroup per (brick, chunk). The items of
    // a launch are numbered chunk-major and handed to the eight XCDs in contiguous ranges, so
    // with 4 chunks every pair of XCDs gets one chunk of the whole volume, split at its middle
    // z-slab (bricks near the ends of the cone are cheaper: symmetric halves keep the XCDs
    // equally loaded), and shorter items leave a shorter tail at the end of the launch. The
    // VJP's partials are per view already: it takes 32 chunks (4 per XCD; at most 2^30 items),
    // whose workgroups resident on an XCD read the tiles of fewer views at a time (half the L2
    // misses of 4 chunks), and whose half-wave orientation (chosen per chunk) then suits every
    // view of its 6-degree chunk. The forward pays one partial volume per extra chunk (capped
    // at 4 GiB) and a summation: 4 chunks, 8 below 3072 bricks (two rounds of the GPU's
    // workgroup slots).
    {
        const long long nv = g->n_views;
        const long long vol_bytes = (long long)g->nx * g->ny * g->nz * (long long)sizeof(float);
        const long long fwd = std::min<long long>({nb < 3072 ? 8LL : 4LL, nv, 1 + (4LL << 30) / vol_bytes});
        p->vsplit_fwd = (int)std::max<long long>(1, fwd);
        p->vsplit_vjp = (int)std::min<long long>({32LL, nv, std::max<long long>(1, (1LL << 30) / nb)});
    }
    const size_t n = (size_t)g->n_views;
    size_t off = 0;
    p->off_phat = off; off = align256(off + n * 12 * sizeof(double));
    p->off_dphat = off; off = align256(off + n * 72 * sizeof(double));
    p->off_desc = off; off = align256(off + n * (size_t)nb * sizeof(BrickDesc));
    p->off_part = off; off = align256(off + n * (size_t)nb * PART_STRIDE * sizeof(float));
    p->off_G = off; off = align256(off + n * 12 * sizeof(double));
    p->off_status = off; off = align256(off + sizeof(int));
    p->off_loss = off; off = align256(off + (4 * (size_t)LOSS_BLOCKS + 8) * sizeof(float));
    p->off_hist = off; off = align256(off + ((size_t)HIST_BINS * HIST_BLOCKS + 2 * HIST_BINS + 8) * sizeof(float));
    p->off_vpart = off;
    off = align256(off + (size_t)(p->vsplit_fwd - 1) * (size_t)g->nx * g->ny * g->nz * sizeof(float));
    p->ws_bytes = off;
    *out = p;
    return GMC_OK;
}

gmc_status gmc_plan_destroy(gmc_plan* plan) {
    delete plan;
    return GMC_OK;
}

size_t gmc_workspace_bytes(const gmc_plan* plan) { return plan ? plan->ws_bytes : 0; }

gmc_status gmc_plan_info(const gmc_plan* plan, int64_t out[8]) {
    if (!plan || !out) return fail(GMC_E_INVALID, "NULL argument");
    out[0] = BXY;
    out[1] = BXY;
    out[2] = plan->bz;
    out[3] = plan_tile(plan).tp;
    out[4] = plan_tile(plan).th;
    out[5] = plan->n_bricks;
    out[6] = plan->vsplit_fwd;
    out[7] = plan->vsplit_vjp;
    return GMC_OK;
}

gmc_status gmc_compose(const gmc_plan* plan, const double* theta, const double* P, double* Phat, double* dPhat,
                       void* hip_stream) {
    if (!plan || !theta || !P || !Phat) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_compose(theta, P, Phat, dPhat, plan->g.n_views, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "compose");
}

gmc_status gmc_prepare(const gmc_plan* plan, const double* P, const double* theta, int32_t with_deriv,
                       void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!P || !theta) return fail(GMC_E_INVALID, "NULL array argument");
    return prepare(plan, P, theta, carve(plan, workspace), with_deriv != 0, (hipStream_t)hip_stream);
}

gmc_status gmc_bp_forward(const gmc_plan* plan, const float* proj, float* vol, void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!proj || !vol) return fail(GMC_E_INVALID, "NULL array argument");
    BpArgs a = bp_args(plan, proj, carve(plan, workspace), false);
    a.vol = vol;
    hipError_t e = launch_bp(plan, a, false, (hipStream_t)hip_stream);
    if (e == hipSuccess && a.vsplit > 1) e = launch_sum_chunks(a, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "backprojection");
}

gmc_status gmc_bp_vjp(const gmc_plan* plan, const float* proj, const float* grad_vol, void* workspace,
                      void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!proj || !grad_vol) return fail(GMC_E_INVALID, "NULL array argument");
    BpArgs a = bp_args(plan, proj, carve(plan, workspace), true);
    a.gvol = grad_vol;
    hipError_t e = launch_bp(plan, a, true, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "vjp");
}

gmc_status gmc_bp_vjp_finish(const gmc_plan* plan, double* grad_theta, double* grad_P, void* workspace,
                             void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!grad_theta) return fail(GMC_E_INVALID, "NULL array argument");
    const WS w = carve(plan, workspace);
    hipError_t e = launch_reduce_chain(plan, w.part, w.dPhat, w.G, grad_theta, grad_P, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "reduce/chain");
}

gmc_status gmc_backproject(const gmc_plan* plan, const float* proj, const double* P, const double* theta, float* vol,
                           void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!proj || !P || !theta || !vol) return fail(GMC_E_INVALID, "NULL array argument");
    if ((st = gmc_prepare(plan, P, theta, 0, workspace, hip_stream)) != GMC_OK) return st;
    return gmc_bp_forward(plan, proj, vol, workspace, hip_stream);
}

gmc_status gmc_backproject_vjp(const gmc_plan* plan, const float* proj, const double* P, const double* theta,
                               const float* grad_vol, double* grad_theta, double* grad_P, void* workspace,
                               void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!proj || !P || !theta || !grad_vol || !grad_theta) return fail(GMC_E_INVALID, "NULL array argument");
    if ((st = gmc_prepare(plan, P, theta, 1, workspace, hip_stream)) != GMC_OK) return st;
    if ((st = gmc_bp_vjp(plan, proj, grad_vol, workspace, hip_stream)) != GMC_OK) return st;
    return gmc_bp_vjp_finish(plan, grad_theta, grad_P, workspace, hip_stream);
}

gmc_status gmc_backproject_vjp_noalloc(const gmc_plan* plan, const float* proj, const double* P,
                                       const double* theta, const float* grad_vol, double* grad_theta,
                                       double* grad_P, int32_t* geometry_flag, void* hip_stream) {
    if (!plan) return fail(GMC_E_INVALID, "plan is NULL");
    if (!proj || !P || !theta || !grad_vol || !grad_theta) return fail(GMC_E_INVALID, "NULL array argument");
    // the VJP touches the workspace up to the status word (matrices, descriptors, partials, G)
    const size_t need = plan->off_loss;
    if (need > (size_t)GMC_NOALLOC_SCRATCH_BYTES)
        return fail(GMC_E_UNSUPPORTED,
                    "allocation-free VJP: this plan needs %zu bytes of scratch (%d bricks x %d views), the static "
                    "buffer holds %zu; use gmc_backproject_vjp with a caller workspace",
                    need, plan->n_bricks, plan->g.n_views, (size_t)GMC_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    gmc_status st = scratch_of_current_device((hipStream_t)hip_stream, &ws);
    if (st != GMC_OK) return st;
    const hipStream_t s = (hipStream_t)hip_stream;
    const WS w = carve(plan, ws);
    if ((st = prepare(plan, P, theta, w, true, s)) != GMC_OK) return st;
    BpArgs a = bp_args(plan, proj, w, true);
    a.gvol = grad_vol;
    hipError_t e = launch_bp(plan, a, true, s);
    if (e != hipSuccess) return hip_fail(e, "vjp");
    e = launch_reduce_chain(plan, w.part, w.dPhat, w.G, grad_theta, grad_P, s);
    if (e != hipSuccess) return hip_fail(e, "reduce/chain");
    if (geometry_flag) {
        hipLaunchKernelGGL(k_copy_int, dim3(1), dim3(1), 0, s, (const int*)w.status, geometry_flag);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "geometry flag");
    }
    return GMC_OK;
}

gmc_status gmc_forward_project(const gmc_plan* plan, const float* vol, const double* P, const double* theta,
                               float* proj_out, void* workspace, void* hip_stream) {
    return gmc_forward_project_parts(plan, vol, nullptr, 1, P, theta, proj_out, workspace, hip_stream);
}

gmc_status gmc_forward_project_parts(const gmc_plan* plan, const float* vol, const uint8_t* labels, int32_t n_parts,
                                     const double* P, const double* theta, float* proj_out, void* workspace,
                                     void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!vol || !P || !theta || !proj_out) return fail(GMC_E_INVALID, "NULL array argument");
    if (n_parts < 1 || n_parts > 255 || (n_parts > 1 && !labels))
        return fail(GMC_E_INVALID, "need 1 <= n_parts <= 255 and labels when n_parts > 1");
    // the march counts samples and voxel coordinates in FP32 / 32-bit integers: every ray has
    // fewer than 2^24 samples (the support's diagonal over half the smallest voxel pitch)
    {
        const gmc_geometry& g = plan->g;
        const double ex = (g.nx + 1) * g.voxel_mm[0], ey = (g.ny + 1) * g.voxel_mm[1], ez = (g.nz + 1) * g.voxel_mm[2];
        const double h = 0.5 * std::min({g.voxel_mm[0], g.voxel_mm[1], g.voxel_mm[2]});
        if (std::max({g.nx, g.ny, g.nz}) > (1 << 22) || sqrt(ex * ex + ey * ey + ez * ez) / h + 2.0 > 16777216.0)
            return fail(GMC_E_UNSUPPORTED, "forward projection: more than 2^24 samples per ray or an axis longer than 2^22 voxels");
    }
    const WS w = carve(plan, workspace);
    const hipStream_t s = (hipStream_t)hip_stream;
    const long long nv = plan->g.n_views;
    for (int k = 0; k < n_parts; ++k) {
        hipError_t e = launch_compose(theta + 6 * nv * k, P, w.Phat, nullptr, plan->g.n_views, s);
        if (e != hipSuccess) return hip_fail(e, "compose");
        e = launch_forward_project(plan, vol, labels, k, w.Phat, proj_out, k > 0, s);
        if (e != hipSuccess) return hip_fail(e, "forward projection");
    }
    return GMC_OK;
}

gmc_status gmc_loss_sumsq_grad(const gmc_plan* plan, const float* vol, float* grad_vol, double* loss,
                               void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!vol || !grad_vol || !loss) return fail(GMC_E_INVALID, "NULL array argument");
    const WS w = carve(plan, workspace);
    hipError_t e = launch_loss_sumsq(plan, vol, grad_vol, w.loss, loss, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "loss");
}

gmc_status gmc_loss_entropy_tv(const gmc_plan* plan, const float* vol, double lambda, double lo, double hi, double eps,
                               float* grad_vol, double* loss, void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (!vol || !grad_vol || !loss) return fail(GMC_E_INVALID, "NULL array argument");
    if (!(hi > lo) || !isfinite(lo) || !isfinite(hi) || !(eps > 0) || !isfinite(lambda))
        return fail(GMC_E_INVALID, "need lo < hi, eps > 0 and a finite lambda");
    const WS w = carve(plan, workspace);
    hipError_t e = launch_loss_entropy_tv(plan, vol, lambda, lo, hi, eps, grad_vol, w.loss, w.hist, loss,
                                          (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "loss");
}

gmc_status gmc_bspline_theta(int32_t n_views, int32_t n_nodes, const double* coeffs, double* theta,
                             void* hip_stream) {
    if (n_views < 2 || n_nodes < 4 || n_nodes > 4096) return fail(GMC_E_INVALID, "need n_views >= 2, 4 <= n_nodes <= 4096");
    if (!coeffs || !theta) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_bspline_theta(n_views, n_nodes, coeffs, theta, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "bspline");
}

gmc_status gmc_bspline_grad(int32_t n_views, int32_t n_nodes, const double* grad_theta, double* grad_coeffs,
                            void* hip_stream) {
    if (n_views < 2 || n_nodes < 4 || n_nodes > 4096) return fail(GMC_E_INVALID, "need n_views >= 2, 4 <= n_nodes <= 4096");
    if (!grad_theta || !grad_coeffs) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_bspline_grad(n_views, n_nodes, grad_theta, grad_coeffs, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "bspline adjoint");
}

gmc_status gmc_akima_theta(int32_t n_views, int32_t n_nodes, const double* coeffs, double* theta,
                           void* hip_stream) {
    if (n_views < 2 || n_nodes < 3 || n_nodes > 256 || n_nodes > n_views)
        return fail(GMC_E_INVALID, "need n_views >= 2 and 3 <= n_nodes <= min(256, n_views)");
    if (!coeffs || !theta) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_akima_theta(n_views, n_nodes, coeffs, theta, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "akima");
}

gmc_status gmc_akima_grad(int32_t n_views, int32_t n_nodes, const double* coeffs, const double* grad_theta,
                          double* grad_coeffs, void* hip_stream) {
    if (n_views < 2 || n_nodes < 3 || n_nodes > 256 || n_nodes > n_views)
        return fail(GMC_E_INVALID, "need n_views >= 2 and 3 <= n_nodes <= min(256, n_views)");
    if (!coeffs || !grad_theta || !grad_coeffs) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_akima_grad(n_views, n_nodes, coeffs, grad_theta, grad_coeffs, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "akima adjoint");
}

gmc_status gmc_adam_step(int64_t n, double* x, const double* g, double* m, double* v, int32_t t, double lr,
                         double beta1, double beta2, double eps, void* hip_stream) {
    if (n < 0 || t < 1) return fail(GMC_E_INVALID, "need n >= 0 and t >= 1");
    if (n == 0) return GMC_OK;
    if (!x || !g || !m || !v) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_adam(n, x, g, m, v, t, lr, beta1, beta2, eps, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "adam");
}

gmc_status gmc_gd_step(int64_t n, double* x, const double* g, int32_t n_iter, double s0, double decay,
                       void* hip_stream) {
    if (n < 0 || n_iter < 0) return fail(GMC_E_INVALID, "need n >= 0 and n_iter >= 0");
    if (n == 0) return GMC_OK;
    if (!x || !g) return fail(GMC_E_INVALID, "NULL argument");
    hipError_t e = launch_gd(n, x, g, s0 * pow(decay, (double)n_iter), (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "gd");
}

gmc_status gmc_debug_project(const gmc_plan* plan, int64_t n, const int64_t* voxel, const int32_t* view, int32_t* cell,
                             float* frac, const void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    if (n < 0) return fail(GMC_E_INVALID, "n < 0");
    if (n == 0) return GMC_OK;
    if (!voxel || !view || !cell || !frac) return fail(GMC_E_INVALID, "NULL argument");
    const WS w = carve(plan, const_cast<void*>(workspace));
    hipError_t e = launch_debug_project(plan, w.desc, n, voxel, view, cell, frac, (hipStream_t)hip_stream);
    return e == hipSuccess ? GMC_OK : hip_fail(e, "debug project");
}

gmc_status gmc_launch_batch(const gmc_work* items, int32_t n_items, void* hip_stream) {
    if (n_items < 0 || (n_items > 0 && !items)) return fail(GMC_E_INVALID, "bad item list");
    hipStream_t s = (hipStream_t)hip_stream;
    // validate everything before launching anything
    for (int32_t q = 0; q < n_items; ++q) {
        const gmc_work& it = items[q];
        gmc_status st = check_plan_ws(it.plan, it.workspace);
        if (st != GMC_OK) return fail(st, "item %d: %s", q, g_last_error.c_str());
        if (it.phase != 0 && it.phase != 1) return fail(GMC_E_INVALID, "item %d: phase must be 0 or 1", q);
        if (it.flags & ~GMC_WORK_PREPARED) return fail(GMC_E_INVALID, "item %d: unknown flag bits", q);
        if (!it.proj || !(it.flags & GMC_WORK_PREPARED ? true : (it.P && it.theta)))
            return fail(GMC_E_INVALID, "item %d: NULL input", q);
        if (it.phase == 0 && !it.vol) return fail(GMC_E_INVALID, "item %d: NULL vol", q);
        if (it.phase == 1 && (!it.grad_vol || !it.grad_theta)) return fail(GMC_E_INVALID, "item %d: NULL gradient", q);
        for (int32_t r = 0; r < q; ++r)
            if (items[r].workspace == it.workspace)
                return fail(GMC_E_WORKSPACE, "items %d and %d share a workspace", r, q);
    }
    for (int32_t q = 0; q < n_items; ++q) {
        const gmc_work& it = items[q];
        if (it.flags & GMC_WORK_PREPARED) continue;
        gmc_status st = gmc_prepare(it.plan, it.P, it.theta, it.phase == 1 ? 1 : 0, it.workspace, hip_stream);
        if (st != GMC_OK) return st;
    }
    // one launch per (phase, weighting, gradient mode, brick depth) group and at most MAX_BATCH items
    std::vector<bool> done(n_items, false);
    for (int32_t q0 = 0; q0 < n_items; ++q0) {
        if (done[q0]) continue;
        const gmc_work& lead = items[q0];
        BatchTable tab;
        tab.n = 0;
        tab.total = 0;
        int cfg = 0;
        for (int32_t q = q0; q < n_items && tab.n < MAX_BATCH; ++q) {
            const gmc_work& it = items[q];
            if (done[q] || it.phase != lead.phase || it.plan->g.weighting != lead.plan->g.weighting ||
                it.plan->g.grad_mode != lead.plan->g.grad_mode || it.plan->bz != lead.plan->bz)
                continue;
            BpArgs ba = bp_args(it.plan, it.proj, carve(it.plan, it.workspace), it.phase == 1);
            // the items of one launch are numbered in 32 bits: a plan that would overflow them
            // waits for the next launch
            if (tab.n > 0 && (long long)tab.total + (long long)it.plan->n_bricks * ba.vsplit > (1LL << 30)) continue;
            ba.vol = it.vol;
            ba.gvol = it.grad_vol;
            tab.item[tab.n] = ba;
            tab.begin[tab.n] = tab.total;
            tab.total += it.plan->n_bricks * ba.vsplit;
            tab.n++;
            cfg = std::max(cfg, it.plan->tile_cfg);
            done[q] = true;
        }
        tab.per_xcd = (tab.total + 7) / 8;
        hipError_t e = launch_bp_batch(lead.plan->bz, cfg, lead.plan->g.weighting, lead.plan->g.grad_mode, tab,
                                       lead.phase == 1, s);
        for (int e2 = 0; e2 < tab.n && e == hipSuccess && lead.phase == 0; ++e2)
            e = launch_sum_chunks(tab.item[e2], s);
        if (e != hipSuccess) return hip_fail(e, "batched backprojection");
    }
    for (int32_t q = 0; q < n_items; ++q) {
        const gmc_work& it = items[q];
        if (it.phase != 1) continue;
        gmc_status st = gmc_bp_vjp_finish(it.plan, it.grad_theta, it.grad_P, it.workspace, hip_stream);
        if (st != GMC_OK) return st;
    }
    return GMC_OK;
}

gmc_status gmc_check(const gmc_plan* plan, void* workspace, void* hip_stream) {
    gmc_status st = check_plan_ws(plan, workspace);
    if (st != GMC_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    const WS w = carve(plan, workspace);
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, w.status, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "check");
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, s, w.status);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "check");
    if (flag) return fail(GMC_E_GEOMETRY, "some voxel projected with w <= 0 (at or behind the source)");
    return GMC_OK;
}

const char* gmc_status_string(gmc_status s) {
    switch (s) {
        case GMC_OK: return "GMC_OK";
        case GMC_E_INVALID: return "GMC_E_INVALID";
        case GMC_E_WORKSPACE: return "GMC_E_WORKSPACE";
        case GMC_E_HIP: return "GMC_E_HIP";
        case GMC_E_GEOMETRY: return "GMC_E_GEOMETRY";
        case GMC_E_UNSUPPORTED: return "GMC_E_UNSUPPORTED";
    }
    return "GMC_E_UNKNOWN";
}

const char* gmc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
