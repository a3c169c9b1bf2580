// C ABI of libdiffproj.so (declared in include/diffproj.h): argument
// validation, workspace layout, kernel sequencing on the caller's stream,
// error reporting and optional per-kernel event timing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
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
    size_t buf = 0;       // offset of the detector image copy (back-projection ops)
    size_t partials = 0;  // offset of the per-block partial sums
    size_t n_part = 0;    // partial blocks per view
    size_t spare = 0;     // FWD_SSD: [V][6] f64 pose-gradient slot used by the autotuner
    size_t flags = 0;     // BP_GRAD: [V] int, "a column of this view has no usable anchor"
    size_t inter = 0;     // FWD_GRAD, FWD_SSD of sparse-ray geometries: padded (mu, G) float4
    bool has_inter = false;
    int chunk = 0;        // back-projection ops: views per detector-image chunk
    size_t total = 0;
};

size_t padded_volume_elems(const dp_geom& g)
{
    return (size_t)(g.nx + 2 * kPadV) * (g.ny + 2 * kPadV) * (g.nz + 2 * kPadV);
}

size_t volume_elems(const dp_geom& g) { return (size_t)g.nx * g.ny * g.nz; }


size_t padded_image_elems(const dp_geom& g)
{
    return (size_t)(g.nu + 2 * kPadD) * (g.nv + 2 * kPadD);
}

// Views whose detector-image copies (bytes_per_px per padded pixel) fit the
// chunk budget, at least one and at most min(V, vmax).
int det_chunk(const dp_geom& g, int V, size_t bytes_per_px, int vmax)
{
    const size_t per_view = padded_image_elems(g) * bytes_per_px;
    size_t c = kDetChunkBytes / std::max<size_t>(per_view, 1);
    c = std::min(c, (size_t)std::min(V, vmax));
    return (int)std::max<size_t>(c, 1);
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
    // The ray-driven kernels read the caller's volume directly and form the
    // volume gradient while staging it: no volume-sized workspace.
    case DP_OP_FWD:
        break;
    case DP_OP_FWD_GRAD:
        // per-block partials, sized for the tile shape with the most tiles
        L.n_part = (size_t)rd_tiles_max(s);
        L.partials = off;
        off = align_up(off + (size_t)V * L.n_part * kRdChannels * sizeof(float));
        if (sparse_rays(s)) {  // tiles that cannot stage a box gather from this copy
            L.has_inter = true;
            L.inter = off;
            off = align_up(off + padded_volume_elems(g) * sizeof(float4));
        }
        break;
    case DP_OP_FWD_SSD:
        if (sparse_rays(s)) {
            L.has_inter = true;
            L.inter = off;
            off = align_up(off + padded_volume_elems(g) * sizeof(float4));
        }
        L.n_part = (size_t)rd_tiles_max(s);
        L.partials = off;
        off = align_up(off + (size_t)V * L.n_part * kRdChannelsGN * sizeof(float));
        L.spare = off;
        off = align_up(off + (size_t)V * 6 * sizeof(double));
        break;
    case DP_OP_BP:
        L.chunk = det_chunk(g, V, sizeof(float4), V);
        off = align_up(off + (size_t)L.chunk * padded_image_elems(g) * sizeof(float4));
        break;
    case DP_OP_FP_FWD:
    case DP_OP_FP_BP:
        break;
    case DP_OP_FP_FWD_GRAD:
        L.n_part = (size_t)sf_blocks(s);
        L.partials = off;
        off = align_up(off + (size_t)V * L.n_part * kRdChannels * sizeof(float));
        break;
    case DP_OP_FP_BP_GRAD:
        L.chunk = det_chunk(g, V, sizeof(float4), V);
        off = align_up(off + (size_t)L.chunk * padded_image_elems(g) * sizeof(float4));
        L.n_part = (size_t)sf_blocks(s);
        L.partials = off;
        off = align_up(off + (size_t)V * L.n_part * kVdChannels * sizeof(float));
        break;
    case DP_OP_BP_GRAD:
        L.chunk = det_chunk(g, V, sizeof(DetTap3), kVdMaxChunk);
        off = align_up(off + (size_t)L.chunk * padded_image_elems(g) * sizeof(DetTap3));
        L.n_part = (size_t)vd_grad_grid(s).blocks;  // one partial set per block
        L.partials = off;
        // partials, then one int per view: "a column of this view has no usable anchor"
        L.flags = off + (size_t)V * L.n_part * kVdChannels * sizeof(float);
        off = align_up(L.flags + (size_t)V * sizeof(int));
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
    // LDS box origins and extents are stored as 16-bit values per axis
    // the ray-driven kernels address the volume with 32-bit byte offsets
    if (padded_volume_elems(*g) >= (size_t)1 << 31 || volume_elems(*g) > (size_t)1 << 30 ||
        g->nx + 2 * kPadV > 65535 ||
        g->ny + 2 * kPadV > 65535 || g->nz + 2 * kPadV > 65535)
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
// Kernel variants: a process-wide cache of autotuned choices per shape class
// ---------------------------------------------------------------------------
struct VariantKey {
    int op, nx, ny, nz, nu, nv, vbucket, ratio;
    bool operator<(const VariantKey& o) const
    {
        const int a[8] = {op, nx, ny, nz, nu, nv, vbucket, ratio};
        const int b[8] = {o.op, o.nx, o.ny, o.nz, o.nu, o.nv, o.vbucket, o.ratio};
        return std::lexicographical_compare(a, a + 8, b, b + 8);
    }
};
std::mutex g_var_mu;
std::map<VariantKey, int> g_var_cache;
int g_var_force[5] = {-1, -1, -1, -1, -1};
constexpr int kDefaultVariant = 1;

// Shape class: grid and detector sizes, view-count octave and the ratio of
// the pixel footprint at the isocentre to the voxel size (in eighths).
VariantKey variant_key(int op, const dp_geom& g, int V)
{
    VariantKey k;
    k.op = op; k.nx = g.nx; k.ny = g.ny; k.nz = g.nz; k.nu = g.nu; k.nv = g.nv;
    int vb = 0;
    while ((1 << vb) < V && vb < 30) ++vb;
    k.vbucket = vb;
    const double hmin = std::min(g.vx, std::min(g.vy, g.vz));
    k.ratio = (int)lround(8.0 * std::min(g.du, g.dv) * g.sad / g.sdd / hmin);
    return k;
}

int variant_for(int op, const dp_geom& g, int V)
{
    std::lock_guard<std::mutex> lk(g_var_mu);
    if (g_var_force[op] >= 0) return g_var_force[op];
    auto it = g_var_cache.find(variant_key(op, g, V));
    return it == g_var_cache.end() ? kDefaultVariant : it->second;
}

// ---------------------------------------------------------------------------
// Profiling (events on the caller's stream around each launch)
// ---------------------------------------------------------------------------
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> ev;          // pairs (start, stop)
    std::vector<int> kern;               // kernel id of each pair
    size_t used = 0;
    bool open = false;                   // a start event of pair `used` was recorded
    double total_ms[DP_K_COUNT] = {0};
    int64_t count[DP_K_COUNT] = {0};
};
Prof g_prof;
constexpr size_t kProfPairs = 4096;

}  // namespace

// Best effort: a pair whose events could not be recorded is dropped.
void prof_begin(int kernel, hipStream_t st)
{
    g_prof.open = false;
    if (!g_prof.on || g_prof.used >= kProfPairs) return;
    if (hipEventRecord(g_prof.ev[2 * g_prof.used], st) != hipSuccess) return;
    g_prof.kern[g_prof.used] = kernel;
    g_prof.open = true;
}

void prof_end(int kernel, hipStream_t st)
{
    (void)kernel;
    if (!g_prof.on || !g_prof.open) return;
    g_prof.open = false;
    if (hipEventRecord(g_prof.ev[2 * g_prof.used + 1], st) == hipSuccess) ++g_prof.used;
}

}  // namespace dp

using namespace dp;

extern "C" {

const char* dp_last_error(void) { return g_err; }

int32_t dp_version(void) { return 10000; }

size_t dp_workspace_bytes(const dp_geom* g, int32_t n_views, int32_t op)
{
    if (op < DP_OP_FWD || op > DP_OP_FP_BP_GRAD) return 0;
    if (check_geom(g, n_views) != DP_OK) return 0;
    return layout(*g, n_views, op).total;
}

size_t dp_bp_grad_flags_offset(const dp_geom* g, int32_t n_views)
{
    if (check_geom(g, n_views) != DP_OK) return (size_t)-1;
    return layout(*g, n_views, DP_OP_BP_GRAD).flags;
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
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_rd_fwd(s, V, views, vol, proj, variant_for(DP_OP_FWD, *g, V), st);
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
    float* part = (float*)(base + L.partials);
    float4* inter = L.has_inter ? (float4*)(base + L.inter) : nullptr;
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    if (inter) launch_vol_inter(s, vol, inter, st);
    const int var = variant_for(DP_OP_FWD_GRAD, *g, V);
    launch_rd_grad(s, V, views, vol, inter, grad_proj, part, var, st);
    launch_finalize_fwd(s, V, views, part, rd_tiles(s, rd_variant_shape(var)), grad_pose, st);
    return check_launch("dp_project_fwd_grad_pose");
}

static int fwd_ssd(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                   const float* vol, const float* target, float* proj, double* loss,
                   double* grad_pose, double* hess, void* ws, size_t ws_bytes, void* stream,
                   const char* name)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (!angles || !poses || !vol || !target || !proj || !grad_pose)
        return fail(DP_ERR_ARG, "NULL array argument");
    if ((rc = check_ws(g, V, DP_OP_FWD_SSD, ws, ws_bytes))) return rc;
    const Layout L = layout(*g, V, DP_OP_FWD_SSD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    ViewGeo* views = (ViewGeo*)(base + L.views);
    float* part = (float*)(base + L.partials);
    float4* inter = L.has_inter ? (float4*)(base + L.inter) : nullptr;
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    if (inter) launch_vol_inter(s, vol, inter, st);
    const int var = variant_for(DP_OP_FWD_SSD, *g, V);
    launch_rd_fused(s, V, views, vol, inter, target, proj, part, hess != nullptr, var, st);
    launch_finalize_fwd_ssd(s, V, views, part, rd_tiles(s, rd_variant_shape(var)), grad_pose,
                            loss, hess, st);
    return check_launch(name);
}

// ---------------------------------------------------------------------------
// Allocation-free variant of dp_project_fwd_ssd_grad_pose: its workspace is a
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never uses the array's name as an address: the device address is
// taken once per device with hipGetSymbolAddress and kept per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of its scratch

static int scratch_for_current_device(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(DP_ERR_HIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DP_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return DP_OK;
}

int dp_project_fwd_ssd_grad_pose(const dp_geom* g, int32_t V, const double* angles,
                                 const double* poses, const float* vol, const float* target,
                                 float* proj, double* loss, double* grad_pose, void* ws,
                                 size_t ws_bytes, void* stream)
{
    return fwd_ssd(g, V, angles, poses, vol, target, proj, loss, grad_pose, nullptr, ws, ws_bytes,
                   stream, "dp_project_fwd_ssd_grad_pose");
}

int dp_project_fwd_ssd_grad_pose_noalloc(const dp_geom* g, int32_t V, const double* angles,
                                         const double* poses, const float* vol,
                                         const float* target, float* proj, double* loss,
                                         double* grad_pose, void* stream)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    const size_t need = layout(*g, V, DP_OP_FWD_SSD).total;
    if (need > kScratchBytes)
        return fail(DP_ERR_UNSUPPORTED,
                    "dp_project_fwd_ssd_grad_pose_noalloc: needs %zu bytes of scratch, the "
                    "library holds %zu (fewer views or a smaller detector per call)",
                    need, kScratchBytes);
    void* ws = nullptr;
    if ((rc = scratch_for_current_device(&ws))) return rc;
    return fwd_ssd(g, V, angles, poses, vol, target, proj, loss, grad_pose, nullptr, ws,
                   kScratchBytes, stream, "dp_project_fwd_ssd_grad_pose_noalloc");
}

int dp_project_fwd_ssd_gauss_newton(const dp_geom* g, int32_t V, const double* angles,
                                    const double* poses, const float* vol, const float* target,
                                    float* proj, double* loss, double* grad_pose, double* hess,
                                    void* ws, size_t ws_bytes, void* stream)
{
    if (!hess) return fail(DP_ERR_ARG, "NULL array argument");
    return fwd_ssd(g, V, angles, poses, vol, target, proj, loss, grad_pose, hess, ws, ws_bytes,
                   stream, "dp_project_fwd_ssd_gauss_newton");
}

// --- footprint projector pairs (SF, DD) --------------------------------------------

static int sf_common(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                     const void* a, const void* b, int op, int kind, void* ws, size_t ws_bytes)
{
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (kind != DP_FP_SF && kind != DP_FP_DD) return fail(DP_ERR_ARG, "unknown footprint kind %d", kind);
    if (!angles || !poses || !a || !b) return fail(DP_ERR_ARG, "NULL array argument");
    return check_ws(g, V, op, ws, ws_bytes);
}

int dp_fp_project(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                  const float* vol, float* proj, int32_t kind, void* ws, size_t ws_bytes,
                  void* stream)
{
    int rc = sf_common(g, V, angles, poses, vol, proj, DP_OP_FP_FWD, kind, ws, ws_bytes);
    if (rc) return rc;
    const Layout L = layout(*g, V, DP_OP_FP_FWD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    ViewGeo* views = (ViewGeo*)((char*)ws + L.views);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_sf_fwd(s, V, views, vol, proj, kind, st);
    return check_launch("dp_fp_project");
}

int dp_fp_backproject(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                      const float* proj, float* vol, int32_t kind, void* ws, size_t ws_bytes,
                      void* stream)
{
    int rc = sf_common(g, V, angles, poses, proj, vol, DP_OP_FP_BP, kind, ws, ws_bytes);
    if (rc) return rc;
    const Layout L = layout(*g, V, DP_OP_FP_BP);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    ViewGeo* views = (ViewGeo*)((char*)ws + L.views);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_sf_bp(s, V, views, proj, vol, kind, st);
    return check_launch("dp_fp_backproject");
}

int dp_fp_project_grad_pose(const dp_geom* g, int32_t V, const double* angles, const double* poses,
                            const float* vol, const float* grad_proj, double* grad_pose,
                            int32_t kind, void* ws, size_t ws_bytes, void* stream)
{
    int rc = sf_common(g, V, angles, poses, vol, grad_proj, DP_OP_FP_FWD_GRAD, kind, ws, ws_bytes);
    if (rc) return rc;
    if (!grad_pose) return fail(DP_ERR_ARG, "NULL array argument");
    const Layout L = layout(*g, V, DP_OP_FP_FWD_GRAD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    ViewGeo* views = (ViewGeo*)((char*)ws + L.views);
    float* part = (float*)((char*)ws + L.partials);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_sf_fwd_grad(s, V, views, vol, grad_proj, part, kind, st);
    launch_finalize_fwd(s, V, views, part, (int)L.n_part, grad_pose, st);
    return check_launch("dp_fp_project_grad_pose");
}

int dp_fp_backproject_grad_pose(const dp_geom* g, int32_t V, const double* angles,
                                const double* poses, const float* proj, const float* grad_vol,
                                double* grad_pose, int32_t kind, void* ws, size_t ws_bytes,
                                void* stream)
{
    int rc = sf_common(g, V, angles, poses, proj, grad_vol, DP_OP_FP_BP_GRAD, kind, ws, ws_bytes);
    if (rc) return rc;
    if (!grad_pose) return fail(DP_ERR_ARG, "NULL array argument");
    const Layout L = layout(*g, V, DP_OP_FP_BP_GRAD);
    const GeoScalars s = make_scalars(*g);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    ViewGeo* views = (ViewGeo*)(base + L.views);
    float4* proj4 = (float4*)(base + L.buf);
    float* part = (float*)(base + L.partials);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    const size_t img = (size_t)g->nu * g->nv;
    for (int v0 = 0; v0 < V; v0 += L.chunk) {
        const int vc = std::min(L.chunk, V - v0);
        launch_det_grad(s, vc, proj + v0 * img, proj4, st);
        launch_sf_bp_grad(s, v0, vc, views, proj4, grad_vol, part, kind, st);
    }
    launch_finalize_bp(s, V, views, part, (int)L.n_part, grad_pose, st);
    return check_launch("dp_fp_backproject_grad_pose");
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
    float4* projq = (float4*)(base + L.buf);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    // views in chunks: the column sums are carried in vol between chunks
    const size_t img = (size_t)g->nu * g->nv;
    for (int v0 = 0; v0 < V; v0 += L.chunk) {
        const int vc = std::min(L.chunk, V - v0);
        launch_det_pad(s, vc, proj + v0 * img, projq, st);
        launch_vd_bp(s, v0, vc, views, projq, vol, weight_mode, v0 == 0, v0 + vc == V, st);
    }
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
    DetTap3* det = (DetTap3*)(base + L.buf);
    float* part = (float*)(base + L.partials);
    int* flags = (int*)(base + L.flags);
    (void)hipGetLastError();
    launch_view_setup(s, V, angles, poses, views, st);
    launch_vd_flags_clear(V, flags, st);
    const size_t img = (size_t)g->nu * g->nv;
    for (int v0 = 0; v0 < V; v0 += L.chunk) {
        const int vc = std::min(L.chunk, V - v0);
        launch_det_tap3(s, vc, proj + v0 * img, det, st);
        launch_vd_grad(s, v0, vc, views, det, grad_vol, part, flags, weight_mode, st);
    }
    launch_finalize_bp(s, V, views, part, (int)L.n_part, grad_pose, st);
    return check_launch("dp_backproject_grad_pose");
}

// ---------------------------------------------------------------------------
// Variant control and autotuning
// ---------------------------------------------------------------------------

int dp_set_variant(int32_t op, int32_t variant)
{
    if (op != DP_OP_FWD && op != DP_OP_FWD_GRAD && op != DP_OP_FWD_SSD)
        return fail(DP_ERR_ARG, "op must be FWD, FWD_GRAD or FWD_SSD");
    if (variant < -1 || variant >= kRdVariants) return fail(DP_ERR_ARG, "variant out of range");
    std::lock_guard<std::mutex> lk(g_var_mu);
    g_var_force[op] = variant;
    return DP_OK;
}

int32_t dp_get_variant(const dp_geom* g, int32_t n_views, int32_t op)
{
    if (!g || (op != DP_OP_FWD && op != DP_OP_FWD_GRAD && op != DP_OP_FWD_SSD)) return -1;
    return variant_for(op, *g, n_views);
}

int dp_autotune(int32_t op, const dp_geom* g, int32_t V, const double* angles, const double* poses,
                const float* vol, const float* grad_proj, void* out, void* ws, size_t ws_bytes,
                void* stream, int32_t reps, int32_t* best, float* ms_per_variant)
{
    if (op != DP_OP_FWD && op != DP_OP_FWD_GRAD && op != DP_OP_FWD_SSD)
        return fail(DP_ERR_ARG, "op must be FWD, FWD_GRAD or FWD_SSD");
    if (reps <= 0 || reps > 100) return fail(DP_ERR_ARG, "reps must be in [1, 100]");
    int rc = check_geom(g, V);
    if (rc) return rc;
    if (!angles || !poses || !vol || !out || (op != DP_OP_FWD && !grad_proj))
        return fail(DP_ERR_ARG, "NULL array argument");
    if ((rc = check_ws(g, V, op, ws, ws_bytes))) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(DP_ERR_HIP, "hipEventCreate failed");
    int saved;
    {
        std::lock_guard<std::mutex> lk(g_var_mu);
        saved = g_var_force[op];
    }
    float times[kRdVariants];
    int arg = 0;
    for (int var = 0; var < kRdVariants && rc == DP_OK; ++var) {
        dp_set_variant(op, var);
        for (int r = 0; r <= reps && rc == DP_OK; ++r) {  // first call warms up
            if (r == 1 && hipEventRecord(e0, st) != hipSuccess) {
                rc = fail(DP_ERR_HIP, "hipEventRecord failed");
                break;
            }
            if (op == DP_OP_FWD)
                rc = dp_project_fwd(g, V, angles, poses, vol, (float*)out, ws, ws_bytes, stream);
            else if (op == DP_OP_FWD_GRAD)
                rc = dp_project_fwd_grad_pose(g, V, angles, poses, vol, grad_proj, (double*)out,
                                              ws, ws_bytes, stream);
            else  // out = proj; the pose gradient goes to the workspace's spare slot
                rc = dp_project_fwd_ssd_grad_pose(
                    g, V, angles, poses, vol, grad_proj, (float*)out, nullptr,
                    (double*)((char*)ws + layout(*g, V, DP_OP_FWD_SSD).spare), ws, ws_bytes, stream);
        }
        if (rc != DP_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&times[var], e0, e1) != hipSuccess) {
            rc = fail(DP_ERR_HIP, "event timing failed");
            break;
        }
        times[var] /= reps;
        if (times[var] < times[arg]) arg = var;
    }
    {
        std::lock_guard<std::mutex> lk(g_var_mu);
        g_var_force[op] = saved;
        if (rc == DP_OK) g_var_cache[variant_key(op, *g, V)] = arg;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best) *best = arg;
    if (ms_per_variant)
        for (int v = 0; v < kRdVariants; ++v) ms_per_variant[v] = times[v];
    return DP_OK;
}

// ---------------------------------------------------------------------------
// Uneven batches of ray-driven problems
// ---------------------------------------------------------------------------

static int check_batch(const dp_problem* pr, int32_t n, int op)
{
    if (!pr) return fail(DP_ERR_ARG, "problem array is NULL");
    if (n <= 0) return fail(DP_ERR_ARG, "batch size must be positive");
    if (n > kRdMaxBatch) return fail(DP_ERR_UNSUPPORTED, "at most %d problems per batch", kRdMaxBatch);
    for (int i = 0; i < n; ++i) {
        const int rc = check_geom(&pr[i].geom, pr[i].n_views);
        if (rc) {
            char msg[sizeof g_err];
            snprintf(msg, sizeof msg, "%s", g_err);
            return fail(rc, "problem %d: %s", i, msg);
        }
        const dp_problem& q = pr[i];
        if (!q.angles || !q.poses || !q.vol) return fail(DP_ERR_ARG, "problem %d: NULL input", i);
        if (op == DP_OP_FWD && !q.proj) return fail(DP_ERR_ARG, "problem %d: NULL proj", i);
        if (op == DP_OP_FWD_GRAD && (!q.grad_proj || !q.grad_pose))
            return fail(DP_ERR_ARG, "problem %d: NULL grad_proj / grad_pose", i);
        if (op == DP_OP_FWD_SSD && (!q.proj || !q.grad_proj || !q.grad_pose || !q.hess))
            return fail(DP_ERR_ARG, "problem %d: NULL proj / grad_proj (target) / grad_pose / hess", i);
    }
    return DP_OK;
}

size_t dp_batch_workspace_bytes(const dp_problem* pr, int32_t n, int32_t op)
{
    if ((op != DP_OP_FWD && op != DP_OP_FWD_GRAD && op != DP_OP_FWD_SSD) || !pr || n <= 0 ||
        n > kRdMaxBatch)
        return 0;
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (check_geom(&pr[i].geom, pr[i].n_views) != DP_OK) return 0;
        total += layout(pr[i].geom, pr[i].n_views, op).total;
    }
    return total;
}

static int run_batch(const dp_problem* pr, int32_t n, int op, void* ws, size_t ws_bytes,
                     int32_t variant, void* stream)
{
    int rc = check_batch(pr, n, op);
    if (rc) return rc;
    if (variant < -1 || variant >= kRdVariants) return fail(DP_ERR_ARG, "variant out of range");
    const size_t need = dp_batch_workspace_bytes(pr, n, op);
    if (ws_bytes < need)
        return fail(DP_ERR_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    if (!ws || (uintptr_t)ws % kAlign) return fail(DP_ERR_ARG, "workspace NULL or not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    // largest problems first: their blocks are dispatched first, shortening the tail
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](int i) {
        const dp_geom& g = pr[i].geom;
        return (double)pr[i].n_views * g.nu * g.nv * std::max(g.nx, std::max(g.ny, g.nz));
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    RdBatch bt;
    bt.n = n;
    size_t off = 0;
    long long blocks = 0;
    const int big = order[0];
    const int var = variant >= 0 ? variant : variant_for(op, pr[big].geom, pr[big].n_views);
    const int shape = rd_variant_shape(var);
    std::vector<size_t> offs(n);
    for (int i = 0; i < n; ++i) {
        offs[i] = off;
        off += layout(pr[i].geom, pr[i].n_views, op).total;
    }
    (void)hipGetLastError();
    for (int j = 0; j < n; ++j) {
        const int i = order[j];
        const dp_problem& q = pr[i];
        const Layout L = layout(q.geom, q.n_views, op);
        const GeoScalars s = make_scalars(q.geom);
        char* base = (char*)ws + offs[i];
        ViewGeo* views = (ViewGeo*)(base + L.views);
        launch_view_setup(s, q.n_views, q.angles, q.poses, views, st);
        float4* inter = op != DP_OP_FWD && L.has_inter ? (float4*)(base + L.inter) : nullptr;
        if (inter) launch_vol_inter(s, q.vol, inter, st);
        RdBatchItem& it = bt.it[j];
        it.s = s;
        it.views = views;
        it.vol = q.vol;
        it.inter = inter;
        it.gin = op == DP_OP_FWD ? nullptr : q.grad_proj;
        it.out = op == DP_OP_FWD ? q.proj : (float*)(base + L.partials);
        it.proj = op == DP_OP_FWD_SSD ? q.proj : nullptr;
        it.tiles = rd_tiles(s, shape);
        it.first = (int)blocks;
        blocks += (long long)it.tiles * q.n_views;
    }
    if (blocks >= (1LL << 31)) return fail(DP_ERR_UNSUPPORTED, "batch too large for one launch");
    if (op == DP_OP_FWD) {
        launch_rd_fwd_batch(bt, (int)blocks, var, st);
    } else {
        if (op == DP_OP_FWD_GRAD)
            launch_rd_grad_batch(bt, (int)blocks, var, st);
        else
            launch_rd_fused_batch(bt, (int)blocks, var, st);
        for (int j = 0; j < n; ++j) {
            const int i = order[j];
            const dp_problem& q = pr[i];
            const Layout L = layout(q.geom, q.n_views, op);
            char* base = (char*)ws + offs[i];
            const ViewGeo* views = (ViewGeo*)(base + L.views);
            const float* part = (float*)(base + L.partials);
            const GeoScalars s = make_scalars(q.geom);
            const int tiles = rd_tiles(s, shape);
            if (op == DP_OP_FWD_GRAD)
                launch_finalize_fwd(s, q.n_views, views, part, tiles, q.grad_pose, st);
            else
                launch_finalize_fwd_ssd(s, q.n_views, views, part, tiles, q.grad_pose, q.loss,
                                        q.hess, st);
        }
    }
    return check_launch(op == DP_OP_FWD        ? "dp_project_fwd_batch"
                        : op == DP_OP_FWD_GRAD ? "dp_project_fwd_grad_pose_batch"
                                               : "dp_project_fwd_ssd_gauss_newton_batch");
}

int dp_project_fwd_batch(const dp_problem* problems, int32_t n, void* ws, size_t ws_bytes,
                         int32_t variant, void* stream)
{
    return run_batch(problems, n, DP_OP_FWD, ws, ws_bytes, variant, stream);
}

int dp_project_fwd_grad_pose_batch(const dp_problem* problems, int32_t n, void* ws,
                                   size_t ws_bytes, int32_t variant, void* stream)
{
    return run_batch(problems, n, DP_OP_FWD_GRAD, ws, ws_bytes, variant, stream);
}

int dp_project_fwd_ssd_gauss_newton_batch(const dp_problem* problems, int32_t n, void* ws,
                                          size_t ws_bytes, int32_t variant, void* stream)
{
    return run_batch(problems, n, DP_OP_FWD_SSD, ws, ws_bytes, variant, stream);
}

int dp_lm_update(int32_t n, double* trial, const double* loss, const double* grad,
                 const double* hess, double* state_pose, double* state_f, double* state_g,
                 double* state_h, double* lam, int32_t* done, double tol, void* stream)
{
    if (n <= 0) return fail(DP_ERR_ARG, "number of views must be positive (got %d)", n);
    if (!trial || !loss || !grad || !hess || !state_pose || !state_f || !state_g || !state_h ||
        !lam || !done)
        return fail(DP_ERR_ARG, "NULL array argument");
    if (!(tol >= 0.0)) return fail(DP_ERR_ARG, "tol must be non-negative");
    (void)hipGetLastError();
    launch_lm_update(n, trial, loss, grad, hess, state_pose, state_f, state_g, state_h, lam,
                     (int*)done, tol, (hipStream_t)stream);
    return check_launch("dp_lm_update");
}

// ---------------------------------------------------------------------------
// Streaming-read probe (measurement only)
// ---------------------------------------------------------------------------

}  // extern "C"

namespace dp {
void launch_read_probe(const void* buf, uint32_t n_vec, int reps, bool shared, int n_blocks,
                       float* out, hipStream_t st);
void launch_lds_probe(int reps, int n_blocks, float* out, hipStream_t st);
}

extern "C" {

int dp_read_probe(const void* buf, int64_t n_vec, int32_t reps, int32_t shared, int32_t n_blocks,
                  float* out, void* stream)
{
    if (!buf || !out) return fail(DP_ERR_ARG, "read probe: NULL pointer");
    if (((uintptr_t)buf & 15) != 0) return fail(DP_ERR_ARG, "read probe: buf must be 16-byte aligned");
    if (n_vec <= 0 || reps <= 0 || n_blocks <= 0)
        return fail(DP_ERR_ARG, "read probe: n_vec, reps and n_blocks must be positive");
    if (n_blocks > (1 << 20)) return fail(DP_ERR_UNSUPPORTED, "read probe: more than 2^20 blocks");
    if (shared) {
        if ((n_vec & (n_vec - 1)) != 0 || n_vec < 2048 || n_vec > ((int64_t)1 << 30))
            return fail(DP_ERR_ARG, "read probe: shared footprint must be a power of two in [2048, 2^30] float4");
    } else if (n_vec + (int64_t)n_blocks * 256 >= ((int64_t)1 << 32)) {
        return fail(DP_ERR_UNSUPPORTED, "read probe: buffer beyond the kernel's 32-bit index range");
    }
    (void)hipGetLastError();
    launch_read_probe(buf, (uint32_t)n_vec, reps, shared != 0, n_blocks, out, (hipStream_t)stream);
    return check_launch("dp_read_probe");
}

int dp_lds_probe(int32_t reps, int32_t n_blocks, float* out, void* stream)
{
    if (!out) return fail(DP_ERR_ARG, "lds probe: NULL pointer");
    if (reps <= 0 || n_blocks <= 0) return fail(DP_ERR_ARG, "lds probe: reps and n_blocks must be positive");
    if (n_blocks > (1 << 20)) return fail(DP_ERR_UNSUPPORTED, "lds probe: more than 2^20 blocks");
    (void)hipGetLastError();
    launch_lds_probe(reps, n_blocks, out, (hipStream_t)stream);
    return check_launch("dp_lds_probe");
}

// ---------------------------------------------------------------------------
// Learned-proposal CNN primitives (BF16 MFMA GEMM and conv helpers)
// ---------------------------------------------------------------------------

int dp_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K, const void* A,
                 int32_t lda, const void* B, int32_t ldb, float* C, int32_t ldc,
                 int32_t accumulate, void* stream)
{
    if (M <= 0 || N <= 0 || K <= 0) return fail(DP_ERR_ARG, "gemm sizes must be positive");
    if (!A || !B || !C) return fail(DP_ERR_ARG, "gemm: NULL operand");
    if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N) || ldc < N)
        return fail(DP_ERR_ARG, "gemm: leading dimension too small");
    if ((size_t)M * ldc >= ((size_t)1 << 40)) return fail(DP_ERR_UNSUPPORTED, "gemm too large");
    if ((N + 63) / 64 > 65535) return fail(DP_ERR_UNSUPPORTED, "gemm: N above 65535 tiles of 64");
    (void)hipGetLastError();
    launch_gemm_bf16(trans_a != 0, trans_b != 0, M, N, K, A, lda, B, ldb, C, ldc, accumulate != 0,
                     nullptr, 0, (hipStream_t)stream);
    return check_launch("dp_gemm_bf16");
}

size_t dp_gemm_bf16_ws_bytes(int32_t M, int32_t N, int32_t K)
{
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    return gemm_ws_bytes(M, N, K);
}

int dp_gemm_bf16_ws(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                    const void* A, int32_t lda, const void* B, int32_t ldb, float* C, int32_t ldc,
                    int32_t accumulate, void* ws, size_t ws_bytes, void* stream)
{
    if (M <= 0 || N <= 0 || K <= 0) return fail(DP_ERR_ARG, "gemm sizes must be positive");
    if (!A || !B || !C) return fail(DP_ERR_ARG, "gemm: NULL operand");
    if (lda < (trans_a ? M : K) || ldb < (trans_b ? K : N) || ldc < N)
        return fail(DP_ERR_ARG, "gemm: leading dimension too small");
    if ((size_t)M * ldc >= ((size_t)1 << 40)) return fail(DP_ERR_UNSUPPORTED, "gemm too large");
    if ((N + 63) / 64 > 65535) return fail(DP_ERR_UNSUPPORTED, "gemm: N above 65535 tiles of 64");
    const size_t need = gemm_ws_bytes(M, N, K);
    if (need && (!ws || ws_bytes < need))
        return fail(DP_ERR_ARG, "gemm: workspace of %zu bytes needed, %zu given", need, ws_bytes);
    (void)hipGetLastError();
    launch_gemm_bf16(trans_a != 0, trans_b != 0, M, N, K, A, lda, B, ldb, C, ldc, accumulate != 0,
                     (float*)ws, ws_bytes, (hipStream_t)stream);
    return check_launch("dp_gemm_bf16_ws");
}

int dp_gemm_bias_act_bf16(int32_t M, int32_t N, int32_t K, const void* A, int32_t lda,
                          const void* B, int32_t ldb, const float* bias, int32_t bias_stride,
                          int32_t relu, void* Y, int32_t ldy, void* stream)
{
    if (M <= 0 || N <= 0 || K <= 0) return fail(DP_ERR_ARG, "gemm sizes must be positive");
    if (!A || !B || !bias || !Y) return fail(DP_ERR_ARG, "gemm_bias_act: NULL pointer");
    if (lda < K || ldb < K || ldy < N || bias_stride < 1)
        return fail(DP_ERR_ARG, "gemm_bias_act: leading dimension or bias stride too small");
    if ((size_t)M * ldy >= ((size_t)1 << 40)) return fail(DP_ERR_UNSUPPORTED, "gemm too large");
    if ((N + 63) / 64 > 65535) return fail(DP_ERR_UNSUPPORTED, "gemm: N above 65535 tiles of 64");
    (void)hipGetLastError();
    launch_gemm_bias_act(M, N, K, A, lda, B, ldb, bias, bias_stride, relu != 0, Y, ldy,
                         (hipStream_t)stream);
    return check_launch("dp_gemm_bias_act_bf16");
}

static int conv_dims(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride)
{
    if (N <= 0 || H <= 0 || W <= 0 || C <= 0 || stride <= 0)
        return fail(DP_ERR_ARG, "conv sizes must be positive");
    // the im2col / col2im kernels index with 32 bits
    const int64_t Ho = (H - 1) / stride + 1, Wo = (W - 1) / stride + 1;
    if ((int64_t)N * Ho * Wo * 9 * C >= ((int64_t)1 << 31) || (int64_t)N * H * W * C >= ((int64_t)1 << 31))
        return fail(DP_ERR_UNSUPPORTED, "conv: N x H x W x 9 C exceeds 2^31 elements; split the batch");
    return DP_OK;
}

int dp_im2col3x3_bf16(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride, const void* x,
                      void* col, void* stream)
{
    int rc = conv_dims(N, H, W, C, stride);
    if (rc) return rc;
    if (!x || !col) return fail(DP_ERR_ARG, "im2col: NULL pointer");
    const int Ho = (H - 1) / stride + 1, Wo = (W - 1) / stride + 1;
    (void)hipGetLastError();
    launch_im2col(N, H, W, C, stride, Ho, Wo, x, col, 9 * C, false, (hipStream_t)stream);
    return check_launch("dp_im2col3x3_bf16");
}

int dp_im2col3x3_ld_bf16(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride,
                         const void* x, void* col, int32_t ld, int32_t ones, void* stream)
{
    int rc = conv_dims(N, H, W, C, stride);
    if (rc) return rc;
    if (!x || !col) return fail(DP_ERR_ARG, "im2col: NULL pointer");
    if (ld < 9 * C + (ones ? 1 : 0)) return fail(DP_ERR_ARG, "im2col: row stride %d too small", ld);
    const int Ho = (H - 1) / stride + 1, Wo = (W - 1) / stride + 1;
    if ((int64_t)N * Ho * Wo * ld >= ((int64_t)1 << 31))
        return fail(DP_ERR_UNSUPPORTED, "im2col: N x Ho x Wo x ld exceeds 2^31 elements; split the batch");
    (void)hipGetLastError();
    launch_im2col(N, H, W, C, stride, Ho, Wo, x, col, ld, ones != 0, (hipStream_t)stream);
    return check_launch("dp_im2col3x3_ld_bf16");
}

int dp_col2im3x3(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride, const float* dcol,
                 float* dx, void* stream)
{
    int rc = conv_dims(N, H, W, C, stride);
    if (rc) return rc;
    if (!dcol || !dx) return fail(DP_ERR_ARG, "col2im: NULL pointer");
    const int Ho = (H - 1) / stride + 1, Wo = (W - 1) / stride + 1;
    (void)hipGetLastError();
    launch_col2im(N, H, W, C, stride, Ho, Wo, dcol, dx, nullptr, false, nullptr, (hipStream_t)stream);
    return check_launch("dp_col2im3x3");
}

int dp_col2im3x3_act_bf16(int32_t N, int32_t H, int32_t W, int32_t C, int32_t stride,
                          const float* dcol, const void* y, int32_t relu, void* dz, void* stream)
{
    int rc = conv_dims(N, H, W, C, stride);
    if (rc) return rc;
    if (!dcol || !y || !dz) return fail(DP_ERR_ARG, "col2im_act: NULL pointer");
    const int Ho = (H - 1) / stride + 1, Wo = (W - 1) / stride + 1;
    (void)hipGetLastError();
    launch_col2im(N, H, W, C, stride, Ho, Wo, dcol, nullptr, y, relu != 0, dz, (hipStream_t)stream);
    return check_launch("dp_col2im3x3_act_bf16");
}

// Shared checks of the implicit-GEMM convolutions.
static int conv_igemm_args(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                           int32_t stride, int32_t ldw, int extra, const char* what)
{
    int rc = conv_dims(N, H, W, Ci, stride);
    if (rc) return rc;
    if (Co <= 0) return fail(DP_ERR_ARG, "%s: Co must be positive", what);
    if (Ci % 8 || Co % 8 || ldw % 8)
        return fail(DP_ERR_ARG, "%s: Ci, Co and ldw must be multiples of 8", what);
    if (ldw < 9 * Ci + extra) return fail(DP_ERR_ARG, "%s: ldw %d too small", what, ldw);
    const int64_t Ho = (H - 1) / stride + 1, Wo = (W - 1) / stride + 1;
    if ((int64_t)N * Ho * Wo * Co >= ((int64_t)1 << 31) || (int64_t)N * H * W * Co >= ((int64_t)1 << 31) ||
        (int64_t)Co * ldw >= ((int64_t)1 << 31))
        return fail(DP_ERR_UNSUPPORTED, "%s: tensor above 2^31 elements; split the batch", what);
    if ((N * Ho * Wo + 63) / 64 > 0x7FFFFFFF || (ldw + 63) / 64 > 65535 || (Ci + 63) / 64 > 65535 ||
        (Co + 63) / 64 > 65535)
        return fail(DP_ERR_UNSUPPORTED, "%s: too many tiles", what);
    return DP_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int dp_conv3x3_fwd_bf16(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co, int32_t stride,
                        const void* x, const void* w, int32_t ldw, const float* bias,
                        int32_t bias_stride, int32_t relu, void* y, void* stream)
{
    int rc = conv_igemm_args(N, H, W, Ci, Co, stride, ldw, 0, "conv3x3_fwd");
    if (rc) return rc;
    if (!x || !w || !bias || !y) return fail(DP_ERR_ARG, "conv3x3_fwd: NULL pointer");
    if (bias_stride < 1) return fail(DP_ERR_ARG, "conv3x3_fwd: bias_stride must be positive");
    if (!aligned16(x) || !aligned16(w) || !aligned16(y))
        return fail(DP_ERR_ARG, "conv3x3_fwd: pointers must be 16-byte aligned");
    (void)hipGetLastError();
    launch_conv_fwd(N, H, W, Ci, Co, stride, x, w, ldw, bias, bias_stride, relu != 0, y,
                    (hipStream_t)stream);
    return check_launch("dp_conv3x3_fwd_bf16");
}

size_t dp_conv3x3_wgrad_ws_bytes(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                                 int32_t stride, int32_t ldw)
{
    if (conv_igemm_args(N, H, W, Ci, Co, stride, ldw, 0, "conv3x3_wgrad_ws_bytes")) return 0;
    return conv_wgrad_ws_bytes(N, H, W, Ci, Co, stride, ldw);
}

int dp_conv3x3_wgrad_bf16(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                          int32_t stride, const void* x, const void* dz, int32_t ldw,
                          int32_t ones, float* dw, void* ws, size_t ws_bytes, void* stream)
{
    int rc = conv_igemm_args(N, H, W, Ci, Co, stride, ldw, ones ? 1 : 0, "conv3x3_wgrad");
    if (rc) return rc;
    if (!x || !dz || !dw) return fail(DP_ERR_ARG, "conv3x3_wgrad: NULL pointer");
    if (!aligned16(x) || !aligned16(dz))
        return fail(DP_ERR_ARG, "conv3x3_wgrad: x and dz must be 16-byte aligned");
    const size_t need = conv_wgrad_ws_bytes(N, H, W, Ci, Co, stride, ldw);
    if (need && (!ws || ws_bytes < need))
        return fail(DP_ERR_ARG, "conv3x3_wgrad: workspace of %zu bytes needed, %zu given", need,
                    ws_bytes);
    (void)hipGetLastError();
    launch_conv_wgrad(N, H, W, Ci, Co, stride, x, dz, ldw, ones != 0, dw, (float*)ws, ws_bytes,
                      (hipStream_t)stream);
    return check_launch("dp_conv3x3_wgrad_bf16");
}

int dp_conv3x3_dgrad_act_bf16(int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                              int32_t stride, const void* dz, const void* w, int32_t ldw,
                              const void* y, int32_t relu, void* out, void* stream)
{
    int rc = conv_igemm_args(N, H, W, Ci, Co, stride, ldw, 0, "conv3x3_dgrad_act");
    if (rc) return rc;
    if (!dz || !w || !out || (relu && !y)) return fail(DP_ERR_ARG, "conv3x3_dgrad_act: NULL pointer");
    if (!aligned16(dz) || !aligned16(w) || !aligned16(out))
        return fail(DP_ERR_ARG, "conv3x3_dgrad_act: pointers must be 16-byte aligned");
    (void)hipGetLastError();
    launch_conv_dgrad_act(N, H, W, Ci, Co, stride, dz, w, ldw, relu ? y : nullptr, relu != 0, out,
                          (hipStream_t)stream);
    return check_launch("dp_conv3x3_dgrad_act_bf16");
}

int dp_adam_f32(int64_t n, float* p, const float* g, float* m, float* v, void* p_bf16, float lr,
                float beta1, float beta2, float eps, float c1, float c2, void* stream)
{
    if (n <= 0 || !p || !g || !m || !v || !p_bf16) return fail(DP_ERR_ARG, "adam: bad argument");
    if (!(c1 > 0.0f) || !(c2 > 0.0f)) return fail(DP_ERR_ARG, "adam: bias corrections must be positive");
    (void)hipGetLastError();
    launch_adam((size_t)n, p, g, m, v, p_bf16, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream);
    return check_launch("dp_adam_f32");
}

int dp_bias_act_bf16(int64_t rows, int32_t C, const float* z, const float* bias, int32_t relu,
                     void* y, void* stream)
{
    if (rows <= 0 || C <= 0 || !z || !bias || !y) return fail(DP_ERR_ARG, "bias_act: bad argument");
    (void)hipGetLastError();
    launch_bias_relu((size_t)rows * C, C, z, bias, relu != 0, y, (hipStream_t)stream);
    return check_launch("dp_bias_act_bf16");
}

int dp_act_bwd_bf16(int64_t total, const float* dy, const void* y, int32_t relu, void* dz,
                    void* stream)
{
    if (total <= 0 || !dy || !y || !dz) return fail(DP_ERR_ARG, "act_bwd: bad argument");
    (void)hipGetLastError();
    launch_relu_bwd((size_t)total, dy, y, relu != 0, dz, (hipStream_t)stream);
    return check_launch("dp_act_bwd_bf16");
}

int dp_colsum_bf16(int32_t M, int32_t C, const void* dz, float* db, void* stream)
{
    if (M <= 0 || C <= 0 || !dz || !db) return fail(DP_ERR_ARG, "colsum: bad argument");
    (void)hipGetLastError();
    launch_colsum(M, C, dz, db, (hipStream_t)stream);
    return check_launch("dp_colsum_bf16");
}

int dp_fdk_filter(const dp_geom* g, int32_t n_views, const float* proj, float* out, double scale,
                  void* stream)
{
    int rc = check_geom(g, n_views);
    if (rc) return rc;
    if (!proj || !out) return fail(DP_ERR_ARG, "fdk_filter: NULL array argument");
    if (g->nu > fdk_max_nu())
        return fail(DP_ERR_UNSUPPORTED, "fdk_filter: detector rows longer than %d pixels (got %d)",
                    fdk_max_nu(), g->nu);
    if ((int64_t)n_views * g->nv > INT32_MAX) return fail(DP_ERR_ARG, "fdk_filter: too many rows");
    if (!std::isfinite(scale)) return fail(DP_ERR_ARG, "fdk_filter: scale must be finite");
    (void)hipGetLastError();
    const GeoScalars s = make_scalars(*g);
    prof_begin(DP_K_FDK_FILTER, (hipStream_t)stream);
    launch_fdk_filter(s, n_views, proj, out, scale, (hipStream_t)stream);
    prof_end(DP_K_FDK_FILTER, (hipStream_t)stream);
    return check_launch("dp_fdk_filter");
}

size_t dp_sharpness_workspace_bytes(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return 0;
    return (sharpness_partials(nx, ny, nz) * sizeof(double) + kAlign - 1) / kAlign * kAlign;
}

int dp_sharpness(int32_t nx, int32_t ny, int32_t nz, const float* vol, double* loss, float* grad,
                 void* ws, size_t ws_bytes, void* stream)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(DP_ERR_ARG, "sharpness: sizes must be positive");
    if ((int64_t)nx * ny * nz >= ((int64_t)1 << 31) * 256)
        return fail(DP_ERR_ARG, "sharpness: volume too large");
    if (!vol || !loss) return fail(DP_ERR_ARG, "sharpness: NULL array argument");
    const size_t need = dp_sharpness_workspace_bytes(nx, ny, nz);
    if (!ws) return fail(DP_ERR_ARG, "workspace pointer is NULL");
    if ((uintptr_t)ws % kAlign != 0) return fail(DP_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(DP_ERR_WORKSPACE, "sharpness: workspace too small (%zu < %zu bytes)", ws_bytes, need);
    (void)hipGetLastError();
    prof_begin(DP_K_SHARPNESS, (hipStream_t)stream);
    launch_sharpness(nx, ny, nz, vol, grad, loss, (double*)ws, (hipStream_t)stream);
    prof_end(DP_K_SHARPNESS, (hipStream_t)stream);
    return check_launch("dp_sharpness");
}

size_t dp_gradient_entropy_workspace_bytes(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return 0;
    return (gradient_entropy_ws_doubles(nx, ny, nz) * sizeof(double) + kAlign - 1) / kAlign * kAlign;
}

int dp_gradient_entropy(int32_t nx, int32_t ny, int32_t nz, const float* vol, float eps,
                        double* loss, float* grad, void* ws, size_t ws_bytes, void* stream)
{
    if (nx <= 0 || ny <= 0 || nz <= 0)
        return fail(DP_ERR_ARG, "gradient_entropy: sizes must be positive");
    if ((int64_t)nx * ny * nz >= ((int64_t)1 << 31) * 256)
        return fail(DP_ERR_ARG, "gradient_entropy: volume too large");
    if (!vol || !loss) return fail(DP_ERR_ARG, "gradient_entropy: NULL array argument");
    if (!(eps > 0.0f) || !std::isfinite(eps))
        return fail(DP_ERR_ARG, "gradient_entropy: eps must be finite and positive");
    const size_t need = dp_gradient_entropy_workspace_bytes(nx, ny, nz);
    if (!ws) return fail(DP_ERR_ARG, "workspace pointer is NULL");
    if ((uintptr_t)ws % kAlign != 0) return fail(DP_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(DP_ERR_WORKSPACE, "gradient_entropy: workspace too small (%zu < %zu bytes)",
                    ws_bytes, need);
    (void)hipGetLastError();
    prof_begin(DP_K_SHARPNESS, (hipStream_t)stream);
    launch_gradient_entropy(nx, ny, nz, eps, vol, grad, loss, (double*)ws, (hipStream_t)stream);
    prof_end(DP_K_SHARPNESS, (hipStream_t)stream);
    return check_launch("dp_gradient_entropy");
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
