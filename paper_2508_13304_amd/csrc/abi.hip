// C ABI of libdiffproj.so (declared in include/diffproj.h): argument
// validation, workspace layout, kernel sequencing on the caller's stream,
// error reporting and optional per-kernel event timing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <vector>

#include "dp_internal.h"

namespace dp {
namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t views = 0;     // offset of ViewGeo[V]
    size_t buf = 0;       // offset of the padded volume / image copy
    size_t partials = 0;  // offset of the per-block partial sums
    size_t n_part = 0;    // partial blocks per view
    size_t total = 0;
};

size_t padded_volume_elems(const dp_geom& g)
{
    return (size_t)(g.nx + 2 * kPadV) * (g.ny + 2 * kPadV) * (g.nz + 2 * kPadV);
}

size_t padded_image_elems(const dp_geom& g)
{
    return (size_t)(g.nu + 2 * kPadD) * (g.nv + 2 * kPadD);
}

Layout layout(const dp_geom& g, int V, int op)
{
    Layout L;
    const GeoScalars s = make_scalars(g);
    size_t off = 0;
    L.views = off;
    off = align_up(off + sizeof(ViewGeo) * (size_t)V);
    L.buf = off;
    switch (op) {
    case DP_OP_FWD:
        off = align_up(off + padded_volume_elems(g) * sizeof(float));
        break;
    case DP_OP_FWD_GRAD:
        off = align_up(off + 3 * padded_volume_elems(g) * sizeof(float));
        L.n_part = (size_t)rd_tiles(s);
        L.partials = off;
        off = align_up(off + (size_t)V * L.n_part * kRdChannels * sizeof(float));
        break;
    case DP_OP_BP:
        off = align_up(off + (size_t)V * padded_image_elems(g) * sizeof(float));
        break;
    case DP_OP_BP_GRAD:
        off = align_up(off + (size_t)V * padded_image_elems(g) * sizeof(float4));
        L.n_part = (size_t)vd_blocks(s, kVdGradCol);
        L.partials = off;
        off = align_up(off + (size_t)V * L.n_part * kVdChannels * sizeof(float));
        break;
    default:
        break;
    }
    L.total = off;
    return L;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

int check_geom(const dp_geom* g, int32_t V)
{
    if (!g) return fail(DP_ERR_ARG, "geometry pointer is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0)
        return fail(DP_ERR_ARG, "volume size must be positive (got %d x %d x %d)", g->nx, g->ny, g->nz);
    if (g->nu <= 0 || g->nv <= 0)
        return fail(DP_ERR_ARG, "detector size must be positive (got %d x %d)", g->nu, g->nv);
    if (!finite_pos(g->vx) || !finite_pos(g->vy) || !finite_pos(g->vz))
        return fail(DP_ERR_ARG, "voxel size must be finite and positive");
    if (!finite_pos(g->du) || !finite_pos(g->dv))
        return fail(DP_ERR_ARG, "pixel pitch must be finite and positive");
    if (!isfinite(g->off_u) || !isfinite(g->off_v))
        return fail(DP_ERR_ARG, "detector offsets must be finite");
    if (!finite_pos(g->sad) || !isfinite(g->sdd) || !(g->sdd > g->sad))
        return fail(DP_ERR_ARG, "need 0 < sad < sdd (got sad=%g sdd=%g)", g->sad, g->sdd);
    if (!finite_pos(g->step)) return fail(DP_ERR_ARG, "ray step must be finite and positive");
    if (V <= 0) return fail(DP_ERR_ARG, "n_views must be positive (got %d)", V);
    if (V > 65535) return fail(DP_ERR_UNSUPPORTED, "n_views above 65535 (got %d)", V);
    if (padded_volume_elems(*g) >= (size_t)1 << 31 || g->ny + 2 * kPadV > 65535 ||
        g->nz + 2 * kPadV > 65535)
        return fail(DP_ERR_UNSUPPORTED, "volume too large for 32-bit voxel indexing");
    if (g->nu > 16384 || g->nv > 16384)
        return fail(DP_ERR_UNSUPPORTED, "detector larger than 16384 pixels per side");
    // The sample of the ray march is fixed by the world-anchored grid; the
    // trilinear positions stay accurate in FP32 only for moderate extents.
    if ((g->nx + g->ny + g->nz) * 1.0 > 1.0e5) return fail(DP_ERR_UNSUPPORTED, "volume extent too large");
    return DP_OK;
}

int check_ws(const dp_geom* g, int32_t V, int op, void* ws, size_t ws_bytes)
{
    const size_t need = layout(*g, V, op).total;
    if (ws_bytes < need)
        return fail(DP_ERR_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    if (!ws) return fail(DP_ERR_ARG, "workspace pointer is NULL");
    if ((uintptr_t)ws % kAlign != 0) return fail(DP_ERR_ARG, "workspace must be 256-byte aligned");
    return DP_OK;
}

int check_launch(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return DP_OK;
}

// ---------------------------------------------------------------------------
// Profiling (events on the caller's stream around each launch)
// ---------------------------------------------------------------------------
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> ev;          // pairs (start, stop)
    std::vector<int> kern;               // kernel id of each pair
    size_t used = 0;
    double total_ms[DP_K_COUNT] = {0};
    int64_t count[DP_K_COUNT] = {0};
};
Prof g_prof;
constexpr size_t kProfPairs = 4096;

}  // namespace

void prof_begin(int kernel, hipStream_t st)
{
    if (!g_prof.on || g_prof.used >= kProfPairs) return;
    hipEventRecord(g_prof.ev[2 * g_prof.used], st);
    g_prof.kern[g_prof.used] = kernel;
}

void prof_end(int kernel, hipStream_t st)
{
    (void)kernel;
    if (!g_prof.on || g_prof.used >= kProfPairs) return;
    hipEventRecord(g_prof.ev[2 * g_prof.used + 1], st);
    ++g_prof.used;
}

}  // namespace dp

using namespace dp;

extern "C" {

const char* dp_last_error(void) { return g_err; }

int32_t dp_version(void) { return 10000; }

size_t dp_workspace_bytes(const dp_geom* g, int32_t n_views, int32_t op)
{
    if (op < DP_OP_FWD || op > DP_OP_BP_GRAD) return 0;
    if (check_geom(g, n_views) != DP_OK) return 0;
    return layout(*g, n_views, op).total;
}

int dp_project_fwd(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                   const float* vol, float* proj, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (!angles || !poses || !vol || !proj) return fail(DP_ERR_ARG, "NULL array argument");
    if ((rc = check_ws(g, V, DP_OP_FWD, ws, ws_bytes))) return rc;
    const Layout L = layout(*g, V, DP_OP_FWD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    ViewGeo* views = (ViewGeo*)(base + L.views);
    float* volp = (float*)(base + L.buf);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_vol_pad(s, vol, volp, st);
    launch_rd_fwd(s, V, views, volp, proj, st);
    return check_launch("dp_project_fwd");
}

int dp_project_fwd_grad_pose(const dp_geom* g, int32_t V, const double* angles,
                             const double* poses, const float* vol, const float* grad_proj,
                             double* grad_pose, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (!angles || !poses || !vol || !grad_proj || !grad_pose)
        return fail(DP_ERR_ARG, "NULL array argument");
    if ((rc = check_ws(g, V, DP_OP_FWD_GRAD, ws, ws_bytes))) return rc;
    const Layout L = layout(*g, V, DP_OP_FWD_GRAD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    ViewGeo* views = (ViewGeo*)(base + L.views);
    float* vol3 = (float*)(base + L.buf);
    float* part = (float*)(base + L.partials);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_vol_grad(s, vol, vol3, st);
    launch_rd_grad(s, V, views, vol3, grad_proj, part, st);
    launch_finalize_fwd(s, V, views, part, (int)L.n_part, grad_pose, st);
    return check_launch("dp_project_fwd_grad_pose");
}

int dp_backproject(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                   const float* proj, float* vol, int32_t weight_mode, void* ws, size_t ws_bytes,
                   void* stream)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (!angles || !poses || !proj || !vol) return fail(DP_ERR_ARG, "NULL array argument");
    if (weight_mode != DP_W_NONE && weight_mode != DP_W_FDK)
        return fail(DP_ERR_ARG, "unknown weight_mode %d", weight_mode);
    if ((rc = check_ws(g, V, DP_OP_BP, ws, ws_bytes))) return rc;
    const Layout L = layout(*g, V, DP_OP_BP);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    ViewGeo* views = (ViewGeo*)(base + L.views);
    float* projp = (float*)(base + L.buf);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_det_pad(s, V, proj, projp, st);
    launch_vd_bp(s, V, views, projp, vol, weight_mode, st);
    return check_launch("dp_backproject");
}

int dp_backproject_grad_pose(const dp_geom* g, int32_t V, const double* angles,
                             const double* poses, const float* proj, const float* grad_vol,
                             double* grad_pose, int32_t weight_mode, void* ws, size_t ws_bytes,
                             void* stream)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (!angles || !poses || !proj || !grad_vol || !grad_pose)
        return fail(DP_ERR_ARG, "NULL array argument");
    if (weight_mode != DP_W_NONE && weight_mode != DP_W_FDK)
        return fail(DP_ERR_ARG, "unknown weight_mode %d", weight_mode);
    if ((rc = check_ws(g, V, DP_OP_BP_GRAD, ws, ws_bytes))) return rc;
    const Layout L = layout(*g, V, DP_OP_BP_GRAD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    ViewGeo* views = (ViewGeo*)(base + L.views);
    float4* proj4 = (float4*)(base + L.buf);
    float* part = (float*)(base + L.partials);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_det_grad(s, V, proj, proj4, st);
    launch_vd_grad(s, V, views, proj4, grad_vol, part, weight_mode, st);
    launch_finalize_bp(s, V, views, part, (int)L.n_part, grad_pose, st);
    return check_launch("dp_backproject_grad_pose");
}

int dp_profile_enable(int32_t on)
{
    if (on && g_prof.ev.empty()) {
        g_prof.ev.resize(2 * kProfPairs);
        g_prof.kern.resize(kProfPairs);
        for (auto& e : g_prof.ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(DP_ERR_HIP, "hipEventCreate failed");
    }
    g_prof.on = on != 0;
    return DP_OK;
}

int dp_profile_collect(void)
{
    for (size_t i = 0; i < g_prof.used; ++i) {
        float ms = 0.0f;
        if (hipEventSynchronize(g_prof.ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess)
            return fail(DP_ERR_HIP, "event timing failed");
        g_prof.total_ms[g_prof.kern[i]] += ms;
        g_prof.count[g_prof.kern[i]] += 1;
    }
    g_prof.used = 0;
    return DP_OK;
}

int dp_profile_read(int32_t kernel, double* total_ms, int64_t* launches)
{
    if (kernel < 0 || kernel >= DP_K_COUNT || !total_ms || !launches)
        return fail(DP_ERR_ARG, "bad profile query");
    *total_ms = g_prof.total_ms[kernel];
    *launches = g_prof.count[kernel];
    g_prof.total_ms[kernel] = 0.0;
    g_prof.count[kernel] = 0;
    return DP_OK;
}

}  // extern "C"
