// Host side of the C ABI declared in include/fhgs.h: plan and workspace
// layout, argument checks, and the launch sequence of every call.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"

namespace fh {

// ---------------------------------------------------------------------------
static int ceil_log2(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b < 1 ? 1 : b;
}

static ViewTable view_table(const fh_plan& p) {
    ViewTable vt;
    memset(&vt, 0, sizeof(vt));
    vt.n_views = p.n_views;
    vt.n_tiles = (int)p.n_tiles;
    for (int v = 0; v < p.n_views; ++v) {
        vt.tiles_x[v] = p.tiles_x[v];
        vt.tiles_y[v] = p.tiles_y[v];
        vt.width[v] = p.cams[v].width;
        vt.height[v] = p.cams[v].height;
    }
    for (int v = 0; v <= p.n_views; ++v) {
        vt.tile_off[v] = (int)p.tile_off[v];
        vt.pix_off[v] = p.pix_off[v];
    }
    return vt;
}

static CamTable cam_table(const fh_plan& p) {
    CamTable ct;
    memset(&ct, 0, sizeof(ct));
    for (int v = 0; v < p.n_views; ++v) ct.cam[v] = p.cams[v];
    return ct;
}

template <typename T>
static T* buf(const fh_plan* p, void* ws, int which) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + p->off[which]);
}
template <typename T>
static const T* cbuf(const fh_plan* p, const void* ws, int which) {
    return reinterpret_cast<const T*>(static_cast<const char*>(ws) + p->off[which]);
}

static int inst_sort_passes(const fh_plan* p) { return (p->tile_bits + 7) / 8; }
static int final_keys_buf(const fh_plan* p) { return (inst_sort_passes(p) % 2) ? WS_KEYS_B : WS_KEYS_A; }
static int final_vals_buf(const fh_plan* p) { return (inst_sort_passes(p) % 2) ? WS_VALS_B : WS_VALS_A; }

static fh_status launch_status() {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FH_OK : FH_E_HIP;
}

// Benchmark hook (fh_set_kernel_events): events around the next n launches of one kernel.
static struct {
    int which = -1;
    hipEvent_t* start = nullptr;
    hipEvent_t* stop = nullptr;
    int n = 0, i = 0;
} g_prof;

static void prof_begin(int which, hipStream_t s) {
    if (g_prof.which == which && g_prof.i < g_prof.n) (void)hipEventRecord(g_prof.start[g_prof.i], s);
}
static void prof_end(int which, hipStream_t s) {
    if (g_prof.which == which && g_prof.i < g_prof.n) (void)hipEventRecord(g_prof.stop[g_prof.i++], s);
}

static bool gaussians_ok(const fh_plan* p, const fh_gaussians* g) {
    if (!g) return false;
    if (g->n != p->n || g->sh_degree != p->sh_degree || g->d != p->d) return false;
    // (an empty scene may pass NULL arrays: nothing is read from them)
    if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacity || !g->sh)) return false;
    if (g->n > 0 && p->d > 0 && !g->feat) return false;
    if (g->feat_dtype != p->feat_dtype) return false;
    return true;
}

__global__ void k_reset_bin_counters(Counters* c) {
    if (threadIdx.x == 0) {
        c->n_instances = 0;
        c->inst_overflow = 0;
        c->n_visited = 0;
        c->visit_overflow = 0;
    }
}

__global__ void k_reset_all_counters(Counters* c) {
    if (threadIdx.x == 0) {
        c->n_instances = 0;
        c->n_visited = 0;
        c->n_culled_nonfinite = 0;
        c->inst_overflow = 0;
        c->visit_overflow = 0;
    }
}

// Average duration of `reps` calls of f (after one warm-up), by HIP events on s.
template <typename Fn>
static fh_status time_calls(Fn f, int reps, hipStream_t s, float* ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FH_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FH_E_HIP;
    }
    fh_status st = f();
    if (st == FH_OK && hipEventRecord(e0, s) != hipSuccess) st = FH_E_HIP;
    for (int r = 0; r < reps && st == FH_OK; ++r) st = f();
    if (st == FH_OK && hipEventRecord(e1, s) != hipSuccess) st = FH_E_HIP;
    if (st == FH_OK && hipEventSynchronize(e1) != hipSuccess) st = FH_E_HIP;
    if (st == FH_OK && hipEventElapsedTime(ms, e0, e1) != hipSuccess) st = FH_E_HIP;
    if (st == FH_OK) *ms /= (float)reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Launch shapes (fh_tuning): defaults and validity.
// The MFMA forward serves the BF16 form, and the FP32 form with FP32 features
// at the widths its channel slices divide (the features enter as three BF16
// terms).  FP32-form runs with BF16-stored features keep the VALU forward: with
// only the weights split the error would reach ~0.8 of the FP32 rule.
// float4 per screen record and floats per per-instance partial row
static int rec_w(const fh_plan* p) { return p->primitive == FH_PRIM_SURFEL ? 4 : 3; }
static int geom_w(const fh_plan* p) { return p->primitive == FH_PRIM_SURFEL ? 16 : 12; }

// (Surfels take the MFMA forward in the BF16 form only; in the FP32 form they
// composite on the VALU forward.)
static bool mfma_forward(int d, int form, int feat_dtype, int prim) {
    if (prim == FH_PRIM_SURFEL) return form == FH_FORM_BF16;
    return form == FH_FORM_BF16 ||
           (feat_dtype == FH_F32 && (d == 32 || d == 64 || d == 96 || (d > 0 && d % 128 == 0)));
}

static fh_tuning default_tuning(int d, int form, int feat_dtype, int prim) {
    fh_tuning t;
    memset(&t, 0, sizeof(t));
    t.fwd_rows = 16;
    if (d > 0) {
        if (mfma_forward(d, form, feat_dtype, prim)) {
            if (d == 32 || d == 64 || d == 96) {
                t.fwd_slice = d;
            } else {
                t.fwd_slice = d % 256 == 0 ? 256 : 128;
                t.fwd_rows = 8;
            }
        } else {
            t.fwd_slice = d <= 8 ? 8 : (d <= 16 ? 16 : (d <= 32 ? 32 : 64));
        }
    }
    t.bwd_chunk = d <= 512 ? 32 : 16;
    t.schedule = 0;
    return t;
}

static bool fwd_shape_ok(int d, int form, int feat_dtype, int prim, int slice, int rows) {
    if (d == 0) return slice == 0 && rows == 16;
    // (FP32 features: 16 rows of 128 channels is not offered, it would spill)
    if (mfma_forward(d, form, feat_dtype, prim))
        return render_fwd_bf16_shape_ok(d, slice, rows) && !(form == FH_FORM_F32 && rows == 16 && slice == 128) &&
               !(form == FH_FORM_F32 && rows == 4);
    return rows == 16 && (slice == 8 || slice == 16 || slice == 32 || slice == 64);
}

static bool bwd_chunk_ok(int d, int chunk) { return chunk == 16 || (chunk == 32 && d <= 512); }

static bool tuning_ok(const fh_plan* p) {
    return fwd_shape_ok(p->d, p->form, p->feat_dtype, p->primitive, p->tuning.fwd_slice, p->tuning.fwd_rows) &&
           bwd_chunk_ok(p->d, p->tuning.bwd_chunk) && (p->tuning.schedule == 0 || p->tuning.schedule == 1);
}

// The work order of the MFMA walk kernels (fh_tuning.schedule): nullptr for
// tile index order; else the tiles sorted by cost, longest first (a stable
// sort of 16-bit keys, ties in index order), cost = the list length
// (by_range) or the traversal length.
static const uint32_t* tile_schedule(const fh_plan* p, void* ws, bool by_range, hipStream_t s) {
    if (p->tuning.schedule == 0 || p->n_tiles <= 0) return nullptr;
    uint32_t* ka = buf<uint32_t>(p, ws, WS_TORDER_KA);
    launch_tile_cost_keys(by_range ? cbuf<uint32_t>(p, ws, WS_RANGES) : nullptr,
                          by_range ? nullptr : cbuf<uint32_t>(p, ws, WS_TILE_NITER), p->n_tiles, ka, s);
    const int passes = radix_sort(ka, nullptr, ka, buf<uint32_t>(p, ws, WS_TORDER_VA), buf<uint32_t>(p, ws, WS_TORDER_KB),
                                  buf<uint32_t>(p, ws, WS_TORDER_VB), true, 1, p->n_tiles, nullptr, 0, 0, 16,
                                  buf<uint32_t>(p, ws, WS_HIST), buf<uint32_t>(p, ws, WS_SCAN_TMP), s);
    return cbuf<uint32_t>(p, ws, (passes % 2) ? WS_TORDER_VB : WS_TORDER_VA);
}

// depth sort, tiles per rank, their scan, the instance count and the overflow flag
static void bin_count_impl(const fh_plan* p, void* ws, hipStream_t s) {
    const int64_t total = (int64_t)p->n_views * p->n;
    Counters* c = buf<Counters>(p, ws, WS_COUNTERS);
    hipLaunchKernelGGL(k_reset_bin_counters, dim3(1), dim3(64), 0, s, c);
    if (total == 0) return;
    uint32_t* hist = buf<uint32_t>(p, ws, WS_HIST);
    uint32_t* scan_tmp = buf<uint32_t>(p, ws, WS_SCAN_TMP);
    radix_sort(cbuf<uint32_t>(p, ws, WS_DEPTH_KEY), nullptr, buf<uint32_t>(p, ws, WS_DKEY_TMP2),
               buf<uint32_t>(p, ws, WS_ORDER), buf<uint32_t>(p, ws, WS_DKEY_TMP), buf<uint32_t>(p, ws, WS_ORDER_TMP),
               true, p->n_views, p->n, nullptr, 0, 0, 32, hist, scan_tmp, s);
    uint32_t* ntiles = buf<uint32_t>(p, ws, WS_DKEY_TMP);
    launch_tiles_by_rank(cbuf<uint32_t>(p, ws, WS_ORDER), cbuf<int4>(p, ws, WS_RECT), p->n, total, ntiles, c, s);
    device_exclusive_scan(ntiles, buf<uint32_t>(p, ws, WS_INST_OFF), total, scan_tmp, 1, s);
    launch_check_capacity(c, p->inst_capacity, s);
    launch_rank_tables(cbuf<uint32_t>(p, ws, WS_ORDER), cbuf<float4>(p, ws, WS_REC), p->n, total,
                       buf<uint32_t>(p, ws, WS_RANK_OF), buf<float4>(p, ws, WS_RREC), rec_w(p), s);
}

// ---------------------------------------------------------------------------
// Static scratch of fh_render_fwd_static: the workspace of callers that cannot
// allocate, one copy per device, held until the process ends.  Host code uses
// the device address hipGetSymbolAddress gives for the current device, never
// the array's name.
static __device__ __align__(256) unsigned char scratch[FH_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES];

// The current device's scratch address (looked up once per device).
static fh_status static_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FH_E_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return FH_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FH_E_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FH_OK;
}

__global__ void k_export_counters(const Counters* c, fh_counters* out) {
    if (threadIdx.x == 0) {
        out->n_instances = (int64_t)c->n_instances;
        out->n_visited = (int64_t)c->n_visited;
        out->n_culled_nonfinite = (int64_t)c->n_culled_nonfinite;
        out->inst_overflow = (int32_t)c->inst_overflow;
        out->visit_overflow = (int32_t)c->visit_overflow;
    }
}

}  // namespace fh

using namespace fh;

extern "C" {

// Sizes and offsets of the workspace sub-buffers of a plan whose sizes and
// capacities are set.
static void plan_layout(fh_plan* plan) {
    const int64_t n = plan->n, total = (int64_t)n * plan->n_views, tiles = plan->n_tiles;
    const int64_t inst_capacity = plan->inst_capacity, visit_capacity = plan->visit_capacity;
    const int32_t n_views = plan->n_views, d = plan->d;
    size_t sz[WS_COUNT];
    memset(sz, 0, sizeof(sz));
    const size_t u4 = sizeof(uint32_t);
    sz[WS_COUNTERS] = 256;
    const size_t rw = (size_t)rec_w(plan), gw = (size_t)geom_w(plan);
    sz[WS_REC] = (size_t)total * rw * 16;
    sz[WS_DEPTH_KEY] = (size_t)total * u4;
    sz[WS_RECT] = (size_t)total * 16;
    sz[WS_ORDER] = sz[WS_ORDER_TMP] = sz[WS_DKEY_TMP] = sz[WS_DKEY_TMP2] = (size_t)total * u4;
    sz[WS_INST_OFF] = (size_t)(total + 1) * u4;
    const size_t hist_depth = radix_hist_u32(n_views, n);
    const size_t hist_inst = radix_hist_u32(1, inst_capacity);
    const size_t hist_visit = radix_hist_u32(1, visit_capacity);
    const size_t hist_tiles = radix_hist_u32(1, tiles);
    const size_t hist = std::max(std::max(std::max(hist_depth, hist_inst), hist_visit), hist_tiles);
    sz[WS_HIST] = hist * u4;
    sz[WS_SCAN_TMP] = scan_scratch_u32(std::max<int64_t>({(int64_t)hist, total + 1, tiles + 1})) * u4;
    sz[WS_RANGES] = (size_t)tiles * 2 * u4;
    sz[WS_TILE_NITER] = (size_t)tiles * u4;
    sz[WS_TILE_VOFF] = (size_t)(tiles + 1) * u4;
    sz[WS_GRAD2D] = (size_t)total * gw * sizeof(float);
    sz[WS_RANK_OF] = (size_t)total * u4;
    sz[WS_KEYS_A] = sz[WS_KEYS_B] = (size_t)inst_capacity * u4;
    sz[WS_VALS_A] = sz[WS_VALS_B] = plan->packed_keys ? 0 : (size_t)inst_capacity * u4;
    sz[WS_VSEG] = (size_t)total * 2 * u4;
    sz[WS_LONG] = (size_t)(total + 3 * n) * u4;
    sz[WS_VKEY_A] = sz[WS_VKEY_B] = sz[WS_VVAL_A] = sz[WS_VVAL_B] = (size_t)visit_capacity * u4;
    sz[WS_PART_GEOM] = (size_t)visit_capacity * gw * sizeof(float);
    sz[WS_PART_FUSE] = (size_t)visit_capacity * d * sizeof(float);
    sz[WS_VREC] = (size_t)visit_capacity * rw * 16;
    sz[WS_VGID] = (size_t)visit_capacity * u4;
    sz[WS_RREC] = (size_t)total * rw * 16;
    sz[WS_UNIT_OWNER] = (size_t)fuse_unit_capacity(visit_capacity) * u4;
    sz[WS_UPART] = (size_t)fuse_unit_capacity(visit_capacity) * (2 * (size_t)d + 2) * sizeof(float);
    // NDFD gradient storage (fh_plan_set_ndfd): per-part partials and the
    // forward sweep's (sigma, prefix term) of every visited (position, pixel)
    sz[WS_PART_NDFD] = plan->ndfd ? (size_t)visit_capacity * 2 * ndfd_part_floats(plan->primitive) * sizeof(float) : 0;
    sz[WS_NDFD_SC] = plan->ndfd ? (size_t)visit_capacity * TILE_PIX * 2 * sizeof(float) : 0;
    sz[WS_TORDER_KA] = sz[WS_TORDER_KB] = sz[WS_TORDER_VA] = sz[WS_TORDER_VB] = (size_t)tiles * u4;
    // the BF16 gradient kernel records w for the fusion kernel of the same call
    sz[WS_WREC] = (plan->form == FH_FORM_BF16 && d > 0 && render_bwd_bf16_supported(d))
                      ? (size_t)visit_capacity * TILE_PIX * sizeof(float) : 0;
    sz[WS_GREC] = (plan->form == FH_FORM_BF16 && d > 0 && render_bwd_bf16_sliced(d))
                      ? (size_t)visit_capacity * TILE_PIX * sizeof(float) : 0;
    static_assert(WS_COUNT <= FH_WS_SLOTS, "fh_plan.off holds the offset of every workspace sub-buffer");
    size_t off = 0;
    plan->n_ws = WS_COUNT;
    for (int i = 0; i < WS_COUNT; ++i) {
        plan->off[i] = off;
        off += (sz[i] + 255) & ~(size_t)255;
    }
    plan->ws_bytes = off;
}

fh_status fh_plan_init(fh_plan* plan, int64_t n, int32_t sh_degree, int32_t d, fh_dtype feat_dtype, fh_form form,
                       const fh_camera* cams, int32_t n_views, int64_t inst_capacity, int64_t visit_capacity) {
    if (!plan || !cams || n < 0 || d < 0 || n_views < 1 || inst_capacity < 0 || visit_capacity < 0)
        return FH_E_INVALID;
    if (sh_degree < 0 || sh_degree > 3 || n_views > FH_MAX_VIEWS || d > 1024) return FH_E_UNSUPPORTED;
    if (feat_dtype != FH_F32 && feat_dtype != FH_BF16) return FH_E_INVALID;
    if (form != FH_FORM_F32 && form != FH_FORM_BF16) return FH_E_INVALID;
    if (form == FH_FORM_BF16 && feat_dtype != FH_BF16) return FH_E_UNSUPPORTED;
    // the MFMA form tiles channels by 32 (and by 128 beyond 96)
    if (form == FH_FORM_BF16 && !(d == 32 || d == 64 || d == 96 || (d > 0 && d % 128 == 0))) return FH_E_UNSUPPORTED;
    if (inst_capacity > 0xFFFFFFFFll || visit_capacity > 0xFFFFFFFFll) return FH_E_UNSUPPORTED;
    if ((int64_t)n * n_views >= ((int64_t)1 << 32)) return FH_E_UNSUPPORTED;
    memset(plan, 0, sizeof(*plan));
    plan->n = n;
    plan->n_views = n_views;
    plan->d = d;
    plan->sh_degree = sh_degree;
    plan->feat_dtype = feat_dtype;
    plan->form = form;
    plan->inst_capacity = inst_capacity;
    plan->visit_capacity = visit_capacity;
    int64_t pix = 0, tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        const fh_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384) return FH_E_INVALID;
        plan->cams[v] = c;
        plan->pix_off[v] = pix;
        plan->tile_off[v] = tiles;
        plan->tiles_x[v] = (c.width + FH_TILE - 1) / FH_TILE;
        plan->tiles_y[v] = (c.height + FH_TILE - 1) / FH_TILE;
        pix += (int64_t)c.width * c.height;
        tiles += (int64_t)plan->tiles_x[v] * plan->tiles_y[v];
    }
    plan->pix_off[n_views] = pix;
    plan->tile_off[n_views] = tiles;
    plan->n_pixels = pix;
    plan->n_tiles = tiles;
    if (tiles >= ((int64_t)1 << 31)) return FH_E_UNSUPPORTED;
    const int64_t total = (int64_t)n * n_views;
    plan->rank_bits = ceil_log2(total > 1 ? total : 2);
    plan->tile_bits = ceil_log2(tiles > 1 ? tiles : 2);
    plan->packed_keys = (plan->rank_bits + plan->tile_bits) <= 32 ? 1 : 0;
    plan->tuning = default_tuning(d, form, feat_dtype, FH_PRIM_GAUSSIAN);

    plan_layout(plan);
    return FH_OK;
}

fh_status fh_plan_set_ndfd(fh_plan* plan, int32_t enable) {
    if (!plan) return FH_E_INVALID;
    plan->ndfd = enable ? 1 : 0;
    plan_layout(plan);
    return FH_OK;
}

fh_status fh_plan_set_primitive(fh_plan* plan, int32_t primitive) {
    if (!plan) return FH_E_INVALID;
    if (primitive != FH_PRIM_GAUSSIAN && primitive != FH_PRIM_SURFEL) return FH_E_INVALID;
    plan->primitive = primitive;
    plan->tuning = default_tuning(plan->d, plan->form, plan->feat_dtype, primitive);
    plan_layout(plan);
    return FH_OK;
}

fh_status fh_project(const fh_plan* p, const fh_gaussians* g, void* ws, hipStream_t s) {
    if (!p || !ws || !gaussians_ok(p, g)) return FH_E_INVALID;
    if (p->bin_rule != FH_BIN_BOX && p->bin_rule != FH_BIN_OPACITY) return FH_E_INVALID;
    Counters* c = buf<Counters>(p, ws, WS_COUNTERS);
    hipLaunchKernelGGL(k_reset_all_counters, dim3(1), dim3(64), 0, s, c);
    if (p->n == 0) return launch_status();
    ProjectArgs a;
    a.means = g->means;
    a.scales = g->scales;
    a.quats = g->quats;
    a.opacity = g->opacity;
    a.sh = g->sh;
    a.n = (int)p->n;
    a.sh_degree = p->sh_degree;
    a.bin_rule = p->bin_rule;
    a.prim = p->primitive;
    a.rec = buf<float4>(p, ws, WS_REC);
    a.depth_key = buf<uint32_t>(p, ws, WS_DEPTH_KEY);
    a.rect = buf<int4>(p, ws, WS_RECT);
    a.counters = c;
    prof_begin(FH_K_PROJECT, s);
    if (p->n > 0) launch_project(a, cam_table(*p), view_table(*p), p->n_views, s);
    prof_end(FH_K_PROJECT, s);
    return launch_status();
}

fh_status fh_bin_count(const fh_plan* p, void* ws, hipStream_t s) {
    if (!p || !ws) return FH_E_INVALID;
    bin_count_impl(p, ws, s);
    return launch_status();
}

fh_status fh_bin_sort(const fh_plan* p, void* ws, hipStream_t s) {
    if (!p || !ws) return FH_E_INVALID;
    if (p->inst_capacity <= 0) return FH_E_INVALID;
    prof_begin(FH_K_BIN, s);
    bin_count_impl(p, ws, s);
    const int64_t total = (int64_t)p->n_views * p->n;
    const Counters* c = cbuf<Counters>(p, ws, WS_COUNTERS);
    uint32_t* ranges = buf<uint32_t>(p, ws, WS_RANGES);
    launch_fill_u32(ranges, p->n_tiles * 2, 0u, s);
    if (total == 0) {
        prof_end(FH_K_BIN, s);
        return launch_status();
    }
    DupArgs da;
    da.inst_off = cbuf<uint32_t>(p, ws, WS_INST_OFF);
    da.order = cbuf<uint32_t>(p, ws, WS_ORDER);
    da.rect = cbuf<int4>(p, ws, WS_RECT);
    da.n = p->n;
    da.total_ranks = total;
    da.cap = p->inst_capacity;
    da.counters = c;
    da.keys = buf<uint32_t>(p, ws, WS_KEYS_A);
    da.vals = p->packed_keys ? nullptr : buf<uint32_t>(p, ws, WS_VALS_A);
    da.rank_bits = p->rank_bits;
    da.packed = p->packed_keys;
    da.vt = view_table(*p);
    launch_duplicate(da, s);
    const int lo = p->packed_keys ? p->rank_bits : 0;
    radix_sort(buf<uint32_t>(p, ws, WS_KEYS_A), p->packed_keys ? nullptr : buf<uint32_t>(p, ws, WS_VALS_A),
               buf<uint32_t>(p, ws, WS_KEYS_A), p->packed_keys ? nullptr : buf<uint32_t>(p, ws, WS_VALS_A),
               buf<uint32_t>(p, ws, WS_KEYS_B), p->packed_keys ? nullptr : buf<uint32_t>(p, ws, WS_VALS_B),
               !p->packed_keys, 1, 0, &c->n_instances, p->inst_capacity, lo, lo + p->tile_bits,
               buf<uint32_t>(p, ws, WS_HIST), buf<uint32_t>(p, ws, WS_SCAN_TMP), s);
    launch_ranges(cbuf<uint32_t>(p, ws, final_keys_buf(p)), c, p->inst_capacity, p->rank_bits, p->packed_keys, ranges,
                  s);
    prof_end(FH_K_BIN, s);
    return launch_status();
}

fh_status fh_bin_keys(const fh_plan* p, const void* ws, uint64_t* keys_out, uint32_t* gid_out, int64_t n_inst,
                      hipStream_t s) {
    if (!p || !ws || n_inst < 0 || n_inst > p->inst_capacity) return FH_E_INVALID;
    launch_bin_keys(cbuf<uint32_t>(p, ws, final_keys_buf(p)),
                    p->packed_keys ? nullptr : cbuf<uint32_t>(p, ws, final_vals_buf(p)),
                    cbuf<uint32_t>(p, ws, WS_ORDER), cbuf<uint32_t>(p, ws, WS_DEPTH_KEY), n_inst, p->n, p->rank_bits,
                    p->packed_keys, keys_out, gid_out, s);
    return launch_status();
}

fh_status fh_render_fwd(const fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* out, hipStream_t s) {
    if (!p || !ws || !out || !gaussians_ok(p, g)) return FH_E_INVALID;
    if (!out->C || !out->T || !out->n_iter || (p->d > 0 && !out->F)) return FH_E_INVALID;
    if (p->inst_capacity <= 0) return FH_E_INVALID;
    if (!tuning_ok(p)) return FH_E_UNSUPPORTED;
    RenderArgs a;
    a.rec = cbuf<float4>(p, ws, WS_REC);
    a.rrec = cbuf<float4>(p, ws, WS_RREC);
    a.order = cbuf<uint32_t>(p, ws, WS_ORDER);
    a.keys = cbuf<uint32_t>(p, ws, final_keys_buf(p));
    a.vals = p->packed_keys ? nullptr : cbuf<uint32_t>(p, ws, final_vals_buf(p));
    a.ranges = cbuf<uint32_t>(p, ws, WS_RANGES);
    a.counters = cbuf<Counters>(p, ws, WS_COUNTERS);
    a.rank_bits = p->rank_bits;
    a.packed = p->packed_keys;
    a.n = p->n;
    a.feat = g->feat;
    a.d = p->d;
    a.feat_bf16 = p->feat_dtype == FH_BF16;
    a.C = out->C;
    a.F = out->F;
    a.T = out->T;
    a.n_iter = out->n_iter;
    uint32_t* tile_niter = buf<uint32_t>(p, ws, WS_TILE_NITER);
    a.tile_niter = tile_niter;
    a.tile_order = nullptr;
    a.prim = p->primitive;
    // several row groups of a tile combine their traversal lengths with atomicMax
    launch_fill_u32(tile_niter, p->n_tiles, 0u, s);
    const ViewTable vt = view_table(*p);
    if (mfma_forward(p->d, p->form, p->feat_dtype, p->primitive)) a.tile_order = tile_schedule(p, ws, true, s);
    prof_begin(FH_K_RENDER_FWD, s);
    if (mfma_forward(p->d, p->form, p->feat_dtype, p->primitive))
        launch_render_fwd_bf16(a, vt, (int)p->n_tiles, p->tuning.fwd_slice, p->tuning.fwd_rows, !a.feat_bf16, s);
    else
        launch_render_fwd_f32(a, vt, (int)p->n_tiles, p->tuning.fwd_slice, s);
    prof_end(FH_K_RENDER_FWD, s);
    uint32_t* voff = buf<uint32_t>(p, ws, WS_TILE_VOFF);
    device_exclusive_scan(tile_niter, voff, p->n_tiles, buf<uint32_t>(p, ws, WS_SCAN_TMP), 1, s);
    launch_check_visits(voff, (int)p->n_tiles, buf<Counters>(p, ws, WS_COUNTERS), p->visit_capacity, s);
    return launch_status();
}

static void fill_bwd_args(const fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* fwd, BwdArgs& a) {
    a.rec = cbuf<float4>(p, ws, WS_REC);
    a.order = cbuf<uint32_t>(p, ws, WS_ORDER);
    a.keys = cbuf<uint32_t>(p, ws, final_keys_buf(p));
    a.vals = p->packed_keys ? nullptr : cbuf<uint32_t>(p, ws, final_vals_buf(p));
    a.ranges = cbuf<uint32_t>(p, ws, WS_RANGES);
    a.tile_niter = cbuf<uint32_t>(p, ws, WS_TILE_NITER);
    a.tile_voff = cbuf<uint32_t>(p, ws, WS_TILE_VOFF);
    a.counters = cbuf<Counters>(p, ws, WS_COUNTERS);
    a.rank_bits = p->rank_bits;
    a.packed = p->packed_keys;
    a.n = p->n;
    a.feat = g->feat;
    a.d = p->d;
    a.feat_bf16 = p->feat_dtype == FH_BF16;
    a.T_final = fwd->T;
    a.n_iter = fwd->n_iter;
    a.dC = nullptr;
    a.dF = nullptr;
    a.dT = nullptr;
    a.target = nullptr;
    a.target_bf16 = 0;
    a.vrec = cbuf<float4>(p, ws, WS_VREC);
    a.vgid = cbuf<uint32_t>(p, ws, WS_VGID);
    a.part_geom = buf<float>(p, ws, WS_PART_GEOM);
    a.part_fuse = buf<float>(p, ws, WS_PART_FUSE);
    a.tile_order = nullptr;
    a.wrec = nullptr;
    a.d0 = 0;
    a.g_in = nullptr;
    a.g_out = nullptr;
    a.prim = p->primitive;
}

static int visit_sort_passes(const fh_plan* p) { return (p->rank_bits + 7) / 8; }

// The BF16-MFMA backward covers d <= 256; wider features use the FP32-VALU
// backward with BF16 feature loads.
static void launch_bwd(const fh_plan* p, void* ws, const BwdArgs& a0, const ViewTable& vt, bool fuse, hipStream_t s) {
    if (p->form == FH_FORM_BF16 && render_bwd_bf16_supported(p->d)) {
        BwdArgs a = a0;
        a.tile_order = tile_schedule(p, ws, false, s);
        // the gradient kernel records w when the fusion kernel follows it
        a.wrec = (fuse && a.dC != nullptr) ? buf<float>(p, ws, WS_WREC) : nullptr;
        if (render_bwd_bf16_sliced(p->d)) a.g_out = buf<float>(p, ws, WS_GREC);
        launch_render_bwd_bf16(a, vt, (int)p->n_tiles, a.dC != nullptr, fuse, s);
    } else {
        const BwdArgs& a = a0;
        launch_render_bwd_f32(a, vt, (int)p->n_tiles, fuse, p->tuning.bwd_chunk, s);
    }
}

// Rank, Gaussian and record of every visited instance, in visit order.
static void visit_stage(const fh_plan* p, void* ws, hipStream_t s) {
    VisitStageArgs a;
    a.ranges = cbuf<uint32_t>(p, ws, WS_RANGES);
    a.tile_niter = cbuf<uint32_t>(p, ws, WS_TILE_NITER);
    a.tile_voff = cbuf<uint32_t>(p, ws, WS_TILE_VOFF);
    a.keys = cbuf<uint32_t>(p, ws, final_keys_buf(p));
    a.vals = p->packed_keys ? nullptr : cbuf<uint32_t>(p, ws, final_vals_buf(p));
    a.rank_bits = p->rank_bits;
    a.packed = p->packed_keys;
    a.order = cbuf<uint32_t>(p, ws, WS_ORDER);
    a.rrec = cbuf<float4>(p, ws, WS_RREC);
    a.counters = buf<Counters>(p, ws, WS_COUNTERS);
    a.vkey = buf<uint32_t>(p, ws, WS_VKEY_A);
    a.vgid = buf<uint32_t>(p, ws, WS_VGID);
    a.vrec = buf<float4>(p, ws, WS_VREC);
    a.rw = rec_w(p);
    launch_visit_stage(a, (int)p->n_tiles, s);
}

// Visited instances sorted stably by rank (the keys visit_stage wrote): each
// (view, Gaussian) gets a contiguous segment of visit indices in row-major
// tile order.
static void visit_sort(const fh_plan* p, void* ws, hipStream_t s) {
    Counters* c = buf<Counters>(p, ws, WS_COUNTERS);
    const int64_t total = (int64_t)p->n * p->n_views;
    uint32_t* vka = buf<uint32_t>(p, ws, WS_VKEY_A);
    radix_sort(vka, nullptr, vka, buf<uint32_t>(p, ws, WS_VVAL_A), buf<uint32_t>(p, ws, WS_VKEY_B),
               buf<uint32_t>(p, ws, WS_VVAL_B), true, 1, 0, &c->n_visited, p->visit_capacity, 0, p->rank_bits,
               buf<uint32_t>(p, ws, WS_HIST), buf<uint32_t>(p, ws, WS_SCAN_TMP), s);
    const bool odd = visit_sort_passes(p) % 2;
    uint32_t* vseg = buf<uint32_t>(p, ws, WS_VSEG);
    launch_fill_u32(vseg, total * 2, 0u, s);
    launch_vseg(cbuf<uint32_t>(p, ws, odd ? WS_VKEY_B : WS_VKEY_A), c, p->visit_capacity, vseg, s);
}

static void fill_reduce_args(const fh_plan* p, void* ws, ReduceArgs& r) {
    r.order = cbuf<uint32_t>(p, ws, WS_ORDER);
    r.vseg = cbuf<uint32_t>(p, ws, WS_VSEG);
    r.vsorted = cbuf<uint32_t>(p, ws, (visit_sort_passes(p) % 2) ? WS_VVAL_B : WS_VVAL_A);
    r.counters = buf<Counters>(p, ws, WS_COUNTERS);
    r.long_list = buf<uint32_t>(p, ws, WS_LONG);
    r.unit_owner = buf<uint32_t>(p, ws, WS_UNIT_OWNER);
    r.upart = buf<float>(p, ws, WS_UPART);
    r.unit_cap = fuse_unit_capacity(p->visit_capacity);
    r.n = p->n;
    r.total = (int64_t)p->n * p->n_views;
    r.part_geom = cbuf<float>(p, ws, WS_PART_GEOM);
    r.wslot = p->primitive == FH_PRIM_SURFEL ? 13 : 9;
    r.grad2d = buf<float>(p, ws, WS_GRAD2D);
    r.rank_of = cbuf<uint32_t>(p, ws, WS_RANK_OF);
    r.part_fuse = cbuf<float>(p, ws, WS_PART_FUSE);
    r.d = p->d;
    r.n_views = p->n_views;
    r.acc_sum = r.acc_comp = r.acc_wsum = r.acc_wcomp = nullptr;
}

// NDFD walk over the staged visits (visit_stage must have run)
static NdfdArgs ndfd_args(const fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* fwd, const void* gt) {
    NdfdArgs n;
    n.tile_niter = cbuf<uint32_t>(p, ws, WS_TILE_NITER);
    n.tile_voff = cbuf<uint32_t>(p, ws, WS_TILE_VOFF);
    n.counters = cbuf<Counters>(p, ws, WS_COUNTERS);
    n.vrec = cbuf<float4>(p, ws, WS_VREC);
    n.vgid = cbuf<uint32_t>(p, ws, WS_VGID);
    n.feat = static_cast<const uint16_t*>(g->feat);
    n.d = p->d;
    n.T_final = fwd->T;
    n.n_iter = fwd->n_iter;
    n.gt = static_cast<const uint16_t*>(gt);
    n.a = n.b = nullptr;
    n.lam = 0.5f;
    n.kk = 20.0f;
    n.Lgt = n.Lcf = nullptr;
    n.part = buf<float>(p, ws, WS_PART_NDFD);
    n.sc = buf<float2>(p, ws, WS_NDFD_SC);
    n.prim = p->primitive;
    return n;
}

static bool ndfd_ok(const fh_plan* p) { return p->feat_dtype == FH_BF16 && ndfd_supported(p->d); }

fh_status fh_render_bwd(const fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* fwd, const fh_upstream* up,
                        const void* fusion_target, fh_dtype target_dtype, const fh_fusion* acc, const fh_grads* out,
                        hipStream_t s) {
    if (!p || !ws || !fwd || !up || !out || !gaussians_ok(p, g)) return FH_E_INVALID;
    if (!fwd->T || !fwd->n_iter || !up->dC) return FH_E_INVALID;
    // (per-Gaussian arrays may be NULL for an empty scene)
    if (p->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh)) return FH_E_INVALID;
    const bool fuse = fusion_target != nullptr;
    if (fuse && (!acc || p->d == 0)) return FH_E_INVALID;
    if (fuse && p->n > 0 && (!acc->sum || !acc->comp || !acc->wsum || !acc->wcomp)) return FH_E_INVALID;
    // the BF16 form feeds the target to the MFMA as is: it must be BF16
    if (fuse && p->form == FH_FORM_BF16 && target_dtype != FH_BF16) return FH_E_UNSUPPORTED;
    if (p->inst_capacity <= 0 || p->visit_capacity <= 0) return FH_E_INVALID;
    if (!tuning_ok(p)) return FH_E_UNSUPPORTED;
    const bool ndfd = up->ndfd_gt != nullptr;
    if (ndfd && !ndfd_ok(p)) return FH_E_UNSUPPORTED;
    if (ndfd && !p->ndfd) return FH_E_INVALID;   // the plan holds no NDFD gradient storage
    BwdArgs a;
    fill_bwd_args(p, g, ws, fwd, a);
    a.dC = up->dC;
    a.dF = p->d > 0 ? up->dF : nullptr;
    a.dT = up->dT;
    a.target = fusion_target;
    a.target_bf16 = target_dtype == FH_BF16;
    const ViewTable vt = view_table(*p);
    prof_begin(FH_K_RENDER_BWD, s);
    visit_stage(p, ws, s);
    launch_bwd(p, ws, a, vt, fuse, s);
    prof_end(FH_K_RENDER_BWD, s);
    if (ndfd) {
        // the NDFD terms of the same walk, added to the gradient kernel's partials
        NdfdArgs n = ndfd_args(p, g, ws, fwd, up->ndfd_gt);
        n.a = up->ndfd_a;
        n.b = up->ndfd_b;
        n.lam = up->ndfd_lambda;
        n.kk = up->ndfd_k;
        n.Lgt = up->ndfd_Lgt;
        n.Lcf = up->ndfd_Lcf;
        prof_begin(FH_K_NDFD, s);
        launch_ndfd(n, vt, (int)p->n_tiles, true, s);
        prof_end(FH_K_NDFD, s);
        launch_ndfd_combine(n.part, buf<float>(p, ws, WS_PART_GEOM), n.counters, p->visit_capacity, p->primitive, s);
    }
    ReduceArgs r;
    fill_reduce_args(p, ws, r);
    prof_begin(FH_K_REDUCE, s);
    visit_sort(p, ws, s);
    if (p->n > 0) launch_reduce_geom(r, geom_w(p), s);
    if (fuse) {
        r.acc_sum = acc->sum;
        r.acc_comp = acc->comp;
        r.acc_wsum = acc->wsum;
        r.acc_wcomp = acc->wcomp;
        launch_reduce_fuse(r, s);
    }
    prof_end(FH_K_REDUCE, s);
    ProjectBwdArgs pb;
    pb.prim = p->primitive;
    pb.means = g->means;
    pb.scales = g->scales;
    pb.quats = g->quats;
    pb.opacity = g->opacity;
    pb.sh = g->sh;
    pb.n = (int)p->n;
    pb.sh_degree = p->sh_degree;
    pb.grad2d = r.grad2d;
    pb.depth_key = cbuf<uint32_t>(p, ws, WS_DEPTH_KEY);
    pb.counters = cbuf<Counters>(p, ws, WS_COUNTERS);
    pb.g_means = out->means;
    pb.g_scales = out->scales;
    pb.g_quats = out->quats;
    pb.g_opacity = out->opacity;
    pb.g_sh = out->sh;
    prof_begin(FH_K_PROJECT_BWD, s);
    if (p->n > 0) launch_project_bwd(pb, cam_table(*p), p->n_views, s);
    prof_end(FH_K_PROJECT_BWD, s);
    return launch_status();
}

fh_status fh_ndfd_losses(const fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* fwd, const void* gt,
                         float lambda, float k, float* Lgt, float* Lcf, hipStream_t s) {
    if (!p || !ws || !fwd || !gt || !gaussians_ok(p, g)) return FH_E_INVALID;
    if (!fwd->T || !fwd->n_iter) return FH_E_INVALID;
    if (p->inst_capacity <= 0 || p->visit_capacity <= 0) return FH_E_INVALID;
    if (!ndfd_ok(p)) return FH_E_UNSUPPORTED;
    NdfdArgs n = ndfd_args(p, g, ws, fwd, gt);
    n.lam = lambda;
    n.kk = k;
    n.Lgt = Lgt;
    n.Lcf = Lcf;
    const ViewTable vt = view_table(*p);
    visit_stage(p, ws, s);
    prof_begin(FH_K_NDFD, s);
    launch_ndfd(n, vt, (int)p->n_tiles, false, s);
    prof_end(FH_K_NDFD, s);
    return launch_status();
}

fh_status fh_fuse_features(const fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* fwd, const void* target,
                           fh_dtype target_dtype, const fh_fusion* acc, hipStream_t s) {
    if (!p || !ws || !fwd || !target || !acc || !gaussians_ok(p, g)) return FH_E_INVALID;
    if (!fwd->T || !fwd->n_iter || p->d == 0) return FH_E_INVALID;
    if (p->n > 0 && (!acc->sum || !acc->comp || !acc->wsum || !acc->wcomp)) return FH_E_INVALID;
    if (p->form == FH_FORM_BF16 && target_dtype != FH_BF16) return FH_E_UNSUPPORTED;
    if (p->inst_capacity <= 0 || p->visit_capacity <= 0) return FH_E_INVALID;
    if (!tuning_ok(p)) return FH_E_UNSUPPORTED;
    BwdArgs a;
    fill_bwd_args(p, g, ws, fwd, a);
    a.target = target;
    a.target_bf16 = target_dtype == FH_BF16;
    const ViewTable vt = view_table(*p);
    prof_begin(FH_K_RENDER_BWD, s);
    visit_stage(p, ws, s);
    launch_bwd(p, ws, a, vt, true, s);
    prof_end(FH_K_RENDER_BWD, s);
    ReduceArgs r;
    fill_reduce_args(p, ws, r);
    r.acc_sum = acc->sum;
    r.acc_comp = acc->comp;
    r.acc_wsum = acc->wsum;
    r.acc_wcomp = acc->wcomp;
    prof_begin(FH_K_REDUCE, s);
    visit_sort(p, ws, s);
    launch_reduce_fuse(r, s);
    prof_end(FH_K_REDUCE, s);
    return launch_status();
}

fh_status fh_render_fwd_static(const fh_plan* p, const fh_gaussians* g, const fh_image* out, fh_counters* counters,
                               hipStream_t s) {
    if (!p || !out || !gaussians_ok(p, g)) return FH_E_INVALID;
    if (p->inst_capacity <= 0) return FH_E_INVALID;
    if (p->ws_bytes > (size_t)FH_STATIC_SCRATCH_BYTES) return FH_E_SCRATCH;
    void* ws = nullptr;
    fh_status st = static_scratch(&ws);
    if (st != FH_OK) return st;
    if ((st = fh_project(p, g, ws, s)) != FH_OK) return st;
    if ((st = fh_bin_sort(p, ws, s)) != FH_OK) return st;
    if ((st = fh_render_fwd(p, g, ws, out, s)) != FH_OK) return st;
    if (counters) hipLaunchKernelGGL(k_export_counters, dim3(1), dim3(64), 0, s, cbuf<Counters>(p, ws, WS_COUNTERS),
                                     counters);
    return launch_status();
}

fh_status fh_tuning_candidates(const fh_plan* p, int32_t which, fh_tuning* out, int32_t max, int32_t* count) {
    if (!p || !out || !count || max < 1) return FH_E_INVALID;
    int n = 0;
    if (which == FH_K_RENDER_FWD && p->d > 0) {
        static const int slices[] = {8, 16, 32, 64, 96, 128, 256};
        // (the MFMA forward also takes the two work orders)
        const int nsched = mfma_forward(p->d, p->form, p->feat_dtype, p->primitive) ? 2 : 1;
        for (int sc = 0; sc < nsched; ++sc)
            for (int rows : {16, 8, 4})
                for (int sl : slices)
                    if (fwd_shape_ok(p->d, p->form, p->feat_dtype, p->primitive, sl, rows) &&
                        (p->form == FH_FORM_BF16 || sl < 2 * p->d) && n < max) {
                        out[n] = p->tuning;
                        out[n].fwd_slice = sl;
                        out[n].fwd_rows = rows;
                        out[n++].schedule = sc;
                    }
    } else if (which == FH_K_RENDER_BWD && p->form == FH_FORM_F32) {
        static const int chunks[] = {16, 32};
        for (int ch : chunks)
            if (bwd_chunk_ok(p->d, ch) && n < max) {
                out[n] = p->tuning;
                out[n++].bwd_chunk = ch;
            }
    } else if (which == FH_K_RENDER_BWD && p->form == FH_FORM_BF16 && render_bwd_bf16_supported(p->d)) {
        for (int sc : {0, 1})
            if (n < max) {
                out[n] = p->tuning;
                out[n++].schedule = sc;
            }
    }
    if (n == 0) {
        out[0] = p->tuning;
        n = 1;
    }
    *count = n;
    return FH_OK;
}

fh_status fh_autotune(fh_plan* p, const fh_gaussians* g, void* ws, const fh_image* fwd, const fh_upstream* up,
                      const void* target, fh_dtype target_dtype, const fh_fusion* acc, const fh_grads* grads,
                      int32_t reps, hipStream_t s) {
    if (!p || !ws || !fwd || reps < 1) return FH_E_INVALID;
    fh_tuning cand[32];
    int32_t nc = 0;
    for (int which : {(int)FH_K_RENDER_FWD, (int)FH_K_RENDER_BWD}) {
        if (which == FH_K_RENDER_BWD && (!up || !grads)) break;
        fh_status st = fh_tuning_candidates(p, which, cand, 32, &nc);
        if (st != FH_OK) return st;
        if (nc < 2) continue;
        int best = -1;
        float best_ms = 0.0f;
        for (int c = 0; c < nc; ++c) {
            fh_plan q = *p;
            q.tuning = cand[c];
            float ms = 0.0f;
            if (which == FH_K_RENDER_FWD)
                st = time_calls([&] { return fh_render_fwd(&q, g, ws, fwd, s); }, reps, s, &ms);
            else
                st = time_calls([&] { return fh_render_bwd(&q, g, ws, fwd, up, target, target_dtype, acc, grads, s); },
                                reps, s, &ms);
            if (st != FH_OK) return st;
            if (best < 0 || ms < best_ms) {
                best = c;
                best_ms = ms;
            }
        }
        p->tuning = cand[best];
    }
    return FH_OK;
}

fh_status fh_set_kernel_events(fh_kernel which, hipEvent_t* start, hipEvent_t* stop, int32_t n) {
    if (n < 0 || (n > 0 && (!start || !stop))) return FH_E_INVALID;
    if ((int)which < FH_K_PROJECT || (int)which > FH_K_NDFD) return FH_E_INVALID;
    g_prof.which = n > 0 ? (int)which : -1;
    g_prof.start = start;
    g_prof.stop = stop;
    g_prof.n = n;
    g_prof.i = 0;
    return FH_OK;
}

fh_status fh_fuse_finalize(const fh_fusion* acc, int64_t n, int32_t d, const void* feat_in, void* feat_out,
                           fh_dtype dtype, hipStream_t s) {
    if (!acc || n < 0 || d <= 0) return FH_E_INVALID;
    if (n > 0 && (!acc->sum || !acc->comp || !acc->wsum || !acc->wcomp || !feat_out)) return FH_E_INVALID;
    if (dtype != FH_F32 && dtype != FH_BF16) return FH_E_INVALID;
    launch_fuse_finalize(acc->sum, acc->comp, acc->wsum, acc->wcomp, n, d, feat_in, feat_out, dtype == FH_BF16, s);
    return launch_status();
}

fh_status fh_read_counters(const fh_plan* p, const void* ws, fh_counters* out, hipStream_t s) {
    if (!p || !ws || !out) return FH_E_INVALID;
    Counters c;
    if (hipStreamSynchronize(s) != hipSuccess) return FH_E_HIP;
    if (hipMemcpy(&c, cbuf<Counters>(p, ws, WS_COUNTERS), sizeof(c), hipMemcpyDeviceToHost) != hipSuccess)
        return FH_E_HIP;
    out->n_instances = (int64_t)c.n_instances;
    out->n_visited = (int64_t)c.n_visited;
    out->n_culled_nonfinite = (int64_t)c.n_culled_nonfinite;
    out->inst_overflow = (int32_t)c.inst_overflow;
    out->visit_overflow = (int32_t)c.visit_overflow;
    return FH_OK;
}

fh_status fh_get_status(const fh_plan* p, const void* ws, fh_counters* out, hipStream_t s) {
    if (!p || !ws || !out) return FH_E_INVALID;
    hipLaunchKernelGGL(k_export_counters, dim3(1), dim3(64), 0, s, cbuf<Counters>(p, ws, WS_COUNTERS), out);
    return launch_status();
}

fh_status fh_get_buffer(const fh_plan* p, void* ws, fh_buffer which, void** ptr, int64_t* count) {
    if (!p || !ws || !ptr || !count) return FH_E_INVALID;
    const int64_t total = (int64_t)p->n * p->n_views;
    switch (which) {
        case FH_BUF_RECORDS: *ptr = buf<void>(p, ws, WS_REC); *count = total * rec_w(p); break;
        case FH_BUF_DEPTH_KEY: *ptr = buf<void>(p, ws, WS_DEPTH_KEY); *count = total; break;
        case FH_BUF_RECT: *ptr = buf<void>(p, ws, WS_RECT); *count = total * 4; break;
        case FH_BUF_DEPTH_ORDER: *ptr = buf<void>(p, ws, WS_ORDER); *count = total; break;
        case FH_BUF_RANGES: *ptr = buf<void>(p, ws, WS_RANGES); *count = p->n_tiles * 2; break;
        case FH_BUF_TILE_NITER: *ptr = buf<void>(p, ws, WS_TILE_NITER); *count = p->n_tiles; break;
        case FH_BUF_GRAD2D: *ptr = buf<void>(p, ws, WS_GRAD2D); *count = total * geom_w(p); break;
        default: return FH_E_INVALID;
    }
    return FH_OK;
}

const char* fh_status_string(fh_status s) {
    switch (s) {
        case FH_OK: return "ok";
        case FH_E_INVALID: return "invalid argument";
        case FH_E_UNSUPPORTED: return "unsupported configuration";
        case FH_E_HIP: return "HIP runtime or launch error";
        case FH_E_CAPACITY: return "capacity exceeded";
        case FH_E_SCRATCH: return "the plan's workspace exceeds the static scratch (FH_STATIC_SCRATCH_BYTES)";
        default: break;
    }
    return "unknown status";
}

int32_t fh_version(void) { return FH_VERSION; }

}  // extern "C"
