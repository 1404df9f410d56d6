// Device-side definitions shared by the HIP kernels of the rasterizer.
// gfx950 (CDNA4): 64-lane wavefronts, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fhgs.h"

namespace fh {

// ---------------------------------------------------------------------------
// Method constants.  The paper fixes the 16x16 tile and the (tile, depth) key
// (Appendix A, "Details of the Rasterizer"); the rest are the 3DGS rules the
// paper's rasterizer inherits without restating them.
constexpr int TILE = FH_TILE;
constexpr int TILE_PIX = TILE * TILE;
constexpr float Z_NEAR = 0.2f;          // near-plane cull on float32 camera depth
constexpr float LOWPASS = 0.3f;         // px^2 added to the 2D covariance diagonal
constexpr double LOWPASS_D = 0.3;
constexpr float ALPHA_MAX = 0.99f;      // alpha clamp
constexpr float ALPHA_MIN = 1.0f / 255.0f;  // blends below are skipped
constexpr float T_MIN = 1e-4f;          // a pixel stops before T would drop below this
constexpr float KAPPA = 11.1f;          // binning box: sqrt(KAPPA * Sigma2_ii) > 2 ln 255
constexpr uint32_t CULLED_KEY = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Workspace sub-buffers (indices into fh_plan::off).
enum WsBuf {
    WS_COUNTERS = 0,   // Counters
    WS_REC,            // float4 [V*N*3]
    WS_DEPTH_KEY,      // u32 [V*N]
    WS_RECT,           // int4 [V*N]
    WS_ORDER,          // u32 [V*N]  depth-sorted Gaussian index per view
    WS_ORDER_TMP,      // u32 [V*N]
    WS_DKEY_TMP,       // u32 [V*N]  radix ping-pong for the depth keys
    WS_DKEY_TMP2,      // u32 [V*N]
    WS_INST_OFF,       // u32 [V*N + 1] exclusive scan of tiles per rank
    WS_SCAN_TMP,       // u32 scratch for multi-level scans
    WS_HIST,           // u32 radix histograms
    WS_RANGES,         // u32 [tiles*2]
    WS_TILE_NITER,     // u32 [tiles]
    WS_TILE_VOFF,      // u32 [tiles+1]
    WS_GRAD2D,         // float [V*N*12]
    WS_RANK_OF,        // u32 [V*N]  depth rank of every (view, Gaussian)
    WS_KEYS_A,         // u32 [cap]
    WS_KEYS_B,         // u32 [cap]
    WS_VALS_A,         // u32 [cap] (unpacked keys only)
    WS_VALS_B,         // u32 [cap]
    WS_VSEG,           // u32 [V*N*2] per-rank [start, end) into the rank-sorted visits
    WS_PART_GEOM,      // float [visit_cap * 12]
    WS_PART_FUSE,      // float [visit_cap * d]
    WS_VKEY_A,         // u32 [visit_cap] rank of each visited instance (ping-pong)
    WS_VKEY_B,
    WS_VVAL_A,         // u32 [visit_cap] visit index, sorted by rank
    WS_VVAL_B,
    WS_LONG,           // u32 [V*N + 3N] lists of long reduction segments (+ unit bases), short fusion list
    WS_VREC,           // float4 [visit_cap * 3] screen record of each visited instance
    WS_VGID,           // u32 [visit_cap] Gaussian of each visited instance
    WS_RREC,           // float4 [V*N*3] screen records in depth-rank order
    WS_UNIT_OWNER,     // u32 [unit_cap] long-fusion slot of each unit
    WS_UPART,          // float [unit_cap * (2 d + 2)] compensated partial sums of each unit
    WS_PART_NDFD,      // float [visit_cap * 2 * 8] NDFD screen-space partials of the two half-tiles (plan.ndfd)
    WS_NDFD_SC,        // float2 [visit_cap * 256] NDFD (sigma, prefix term) per visited (position, pixel) (plan.ndfd)
    WS_TORDER_KA,      // u32 [tiles] tile schedule: sort keys (ping-pong)
    WS_TORDER_KB,
    WS_TORDER_VA,      // u32 [tiles] tile schedule: tile ids (ping-pong; the order ends here)
    WS_TORDER_VB,
    WS_WREC,           // float [visit_cap * 256] w per visited (position, pixel), BF16 form (gradient -> fusion)
    WS_GREC,           // float [visit_cap * 256] f . dF of earlier channel slices, BF16 form above 256 channels
    WS_COUNT
};

struct Counters {
    unsigned long long n_instances;
    unsigned long long n_visited;
    unsigned long long n_culled_nonfinite;
    unsigned int inst_overflow;
    unsigned int visit_overflow;
    unsigned int n_long_geom;   // ranks whose visit segment goes to the workgroup-wide reduction
    unsigned int n_long_fuse;   // Gaussians whose fusion goes to the unit-wise reduction
    unsigned int n_fuse_units;  // units (runs of consecutive visits) of those Gaussians
    unsigned int n_short_fuse;  // Gaussians whose fusion is summed by one wavefront
    unsigned int pad[4];
};

// Per-view constants passed by value to kernels.
struct ViewTable {
    int n_views;
    int n_tiles;
    int tiles_x[FH_MAX_VIEWS];
    int tiles_y[FH_MAX_VIEWS];
    int width[FH_MAX_VIEWS];
    int height[FH_MAX_VIEWS];
    int tile_off[FH_MAX_VIEWS + 1];
    long long pix_off[FH_MAX_VIEWS + 1];
};

struct CamTable {
    fh_camera cam[FH_MAX_VIEWS];
};

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int t) {
    int v = 0;
    while (v + 1 < vt.n_views && t >= vt.tile_off[v + 1]) ++v;
    return v;
}

// ---------------------------------------------------------------------------
// Screen-space record of one (view, Gaussian), three float4:
//   r0 = (u_hi, v_hi, u_lo, v_lo)      mean, as an unevaluated float pair
//   r1 = (e_x, e_y, q1, q2)            eigenframe of the conic: unit e1 and
//                                      q_i = -lambda_i log2(e) / 2
//   r2 = (opacity, r, g, b)
// The screen density is G = exp2(q1 a^2 + q2 b^2) with a = e1 . d,
// b = e1 x d, d = pixel - mean; this equals exp(-1/2 d^T Sigma2^-1 d).
struct Rec {
    float4 r0, r1, r2;
};
static_assert(sizeof(Rec) == 48, "records are read and written as 12 consecutive dwords");

// A chunk's records staged in LDS as float4 triples with one float4 of padding
// after every G records.  Lanes that read records G apart at the same time (one
// per 16-lane row) then start 3G + 1 float4s apart, i.e. in different groups
// of four banks, instead of all in the same one (records are 12 dwords).
template <int G>
__device__ __forceinline__ int rec_slot(int k) {
    return 3 * k + k / G;
}
template <int G>
__device__ __forceinline__ Rec lds_rec(const float4* base, int k) {
    const float4* p = base + rec_slot<G>(k);
    Rec r;
    r.r0 = p[0];
    r.r1 = p[1];
    r.r2 = p[2];
    return r;
}
template <int G>
__device__ __forceinline__ void lds_put_rec(float4* base, int k, const Rec& r) {
    float4* p = base + rec_slot<G>(k);
    p[0] = r.r0;
    p[1] = r.r1;
    p[2] = r.r2;
}

// alpha = min(ALPHA_MAX, o G) at pixel centre (x, y), evaluated with explicit
// fused operations so that every kernel gets the same bits.
struct AlphaEval {
    float dx, dy, a, b, G, raw, alpha;
};

__device__ __forceinline__ AlphaEval eval_alpha(const Rec& r, float x, float y) {
#pragma clang fp contract(off)
    AlphaEval e;
    e.dx = (x - r.r0.x) - r.r0.z;
    e.dy = (y - r.r0.y) - r.r0.w;
    const float ex = r.r1.x, ey = r.r1.y;
    e.a = __builtin_fmaf(ex, e.dx, ey * e.dy);
    e.b = __builtin_fmaf(ex, e.dy, -(ey * e.dx));
    const float p2 = __builtin_fmaf(r.r1.z, e.a * e.a, r.r1.w * (e.b * e.b));
    e.G = __builtin_amdgcn_exp2f(p2);
    e.raw = r.r2.x * e.G;
    e.alpha = fminf(ALPHA_MAX, e.raw);
    return e;
}

// ---------------------------------------------------------------------------
// Surfel record of one (view, surfel) (Section 3.1), four float4:
//   r0 = (x_c hi, y_c hi, x_c lo, y_c lo)   projected centre, a float pair
//   r1 = (a0, a1, b0, b1)                   plane map rows: pixel offsets
//   r3 = (D, e1, e2, 0)                     (dx w, dy w) = (a0 u + a1 v, b0 u + b1 v),
//                                           w = 1 + c0 u + c1 v, D = a0 b1 - a1 b0,
//                                           e1 = a0 c1 - a1 c0, e2 = c0 b1 - c1 b0
//   r2 = (opacity, r, g, b)                 (the same slot as a Gaussian's)
struct SRec {
    float4 r0, r1, r2, r3;
};
static_assert(sizeof(SRec) == 64, "surfel records are read and written as 16 consecutive dwords");

// The plane point (u, v) = (k0, k1) / k2 that the ray of pixel offsets
// (dx, dy) meets: k0 = dx b1 - dy a1, k1 = dy a0 - dx b0, k2 = D - dy e1 - dx e2;
// ik2 = 1 / k2 by the hardware reciprocal, 0 for a ray parallel to the plane.
struct SurfPlane {
    float u, v, ik2;
    bool hit;
};
__device__ __forceinline__ SurfPlane surfel_plane(const SRec& r, float dx, float dy) {
#pragma clang fp contract(off)
    SurfPlane s;
    const float a0 = r.r1.x, a1 = r.r1.y, b0 = r.r1.z, b1 = r.r1.w;
    const float k0 = __builtin_fmaf(dx, b1, -(dy * a1));
    const float k1 = __builtin_fmaf(dy, a0, -(dx * b0));
    const float k2 = __builtin_fmaf(-dx, r.r3.z, __builtin_fmaf(-dy, r.r3.y, r.r3.x));
    s.hit = k2 != 0.0f;
    s.ik2 = s.hit ? __builtin_amdgcn_rcpf(k2) : 0.0f;
    s.u = k0 * s.ik2;
    s.v = k1 * s.ik2;
    return s;
}

// A surfel at pixel centre (x, y): pixel offsets from the projected centre,
// the plane point its ray meets, G = exp(-(u^2 + v^2)/2) (0 for a ray parallel
// to the plane), alpha = min(0.99, o G).  Every kernel evaluates alpha with
// this function, so forward and backward take the same decisions.
struct SurfEval {
    float dx, dy, u, v, ik2, raw, alpha;
};
__device__ __forceinline__ SurfEval eval_surfel(const SRec& r, float x, float y) {
#pragma clang fp contract(off)
    SurfEval e;
    e.dx = (x - r.r0.x) - r.r0.z;
    e.dy = (y - r.r0.y) - r.r0.w;
    const SurfPlane sp = surfel_plane(r, e.dx, e.dy);
    e.ik2 = sp.ik2;
    e.u = sp.u;
    e.v = sp.v;
    // exp(-r2 / 2) = exp2(-(log2 e / 2) r2)
    const float G = sp.hit ? __builtin_amdgcn_exp2f(-0.72134752044448170f * (e.u * e.u + e.v * e.v)) : 0.0f;
    e.raw = r.r2.x * G;
    e.alpha = fminf(ALPHA_MAX, e.raw);
    return e;
}

// Per-primitive record type, width and per-instance partial row:
// NQ terms in rows of GP floats, the weight sum at WSLOT.
template <bool SURF>
struct PrimRec {
    using T = Rec;
    static constexpr int RW = 3;
    static constexpr int NQ = 10, GP = 12, WSLOT = 9;
};
template <>
struct PrimRec<true> {
    using T = SRec;
    static constexpr int RW = 4;
    static constexpr int NQ = 14, GP = 16, WSLOT = 13;
};
template <bool SURF>
__device__ __forceinline__ typename PrimRec<SURF>::T load_rec(const float4* base, int64_t j) {
    typename PrimRec<SURF>::T r;
    r.r0 = base[PrimRec<SURF>::RW * j];
    r.r1 = base[PrimRec<SURF>::RW * j + 1];
    r.r2 = base[PrimRec<SURF>::RW * j + 2];
    if constexpr (SURF) r.r3 = base[PrimRec<SURF>::RW * j + 3];
    return r;
}
// A record that never blends (opacity 0), for the padding positions of a chunk.
template <bool SURF>
__device__ __forceinline__ typename PrimRec<SURF>::T pad_rec() {
    typename PrimRec<SURF>::T r;
    r.r0 = make_float4(0.f, 0.f, 0.f, 0.f);
    r.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (SURF) {
        r.r1 = make_float4(0.f, 0.f, 0.f, 0.f);
        r.r3 = make_float4(1.f, 0.f, 0.f, 0.f);
    } else {
        r.r1 = make_float4(1.f, 0.f, -1.f, -1.f);
    }
    return r;
}
template <bool SURF>
__device__ __forceinline__ float prim_alpha(const typename PrimRec<SURF>::T& r, float x, float y) {
    if constexpr (SURF)
        return eval_surfel(r, x, y).alpha;
    else
        return eval_alpha(r, x, y).alpha;
}

// Chunk records staged in LDS as RW float4 each, with one float4 of padding
// after every G records (as rec_slot for the three-float4 records).
template <bool SURF, int G>
__device__ __forceinline__ int prec_slot(int k) {
    return PrimRec<SURF>::RW * k + k / G;
}
template <bool SURF, int G>
__device__ __forceinline__ typename PrimRec<SURF>::T lds_prec(const float4* base, int k) {
    const float4* p = base + prec_slot<SURF, G>(k);
    typename PrimRec<SURF>::T r;
    r.r0 = p[0];
    r.r1 = p[1];
    r.r2 = p[2];
    if constexpr (SURF) r.r3 = p[3];
    return r;
}
template <bool SURF, int G>
__device__ __forceinline__ void lds_put_prec(float4* base, int k, const typename PrimRec<SURF>::T& r) {
    float4* p = base + prec_slot<SURF, G>(k);
    p[0] = r.r0;
    p[1] = r.r1;
    p[2] = r.r2;
    if constexpr (SURF) p[3] = r.r3;
}

// ---------------------------------------------------------------------------
// Wavefront helpers (64 lanes).
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned int wave_max_u32(unsigned int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned int o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// A wave's four 16-lane rows: every lane gets the values of lanes xi, xi + 16,
// xi + 32 and xi + 48 (xi = lane % 16) from three cross-row swaps (gfx950
// v_permlane16_swap / v_permlane32_swap, VALU) instead of four LDS permutes.
// All 64 lanes must be active.
struct Rows4 {
    float r0, r1, r2, r3;
};
__device__ __forceinline__ Rows4 rows4(float v) {
    const unsigned u = __float_as_uint(v);
    // odd rows of one copy trade places with even rows of the other:
    // a[0] = (row 0, row 0, row 2, row 2), a[1] = (row 1, row 1, row 3, row 3)
    const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    // upper half of one copy with lower half of the other:
    // b = (row 0 everywhere, row 2 everywhere), c = (row 1 ..., row 3 ...)
    const auto b = __builtin_amdgcn_permlane32_swap(a[0], a[0], false, false);
    const auto c = __builtin_amdgcn_permlane32_swap(a[1], a[1], false, false);
    return Rows4{__uint_as_float(b[0]), __uint_as_float(c[0]), __uint_as_float(b[1]), __uint_as_float(c[1])};
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Neumaier compensated addition: (s, c) += x.
__device__ __forceinline__ void neumaier_add(float& s, float& c, float x) {
#pragma clang fp contract(off)
    const float t = s + x;
    if (fabsf(s) >= fabsf(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

template <typename T>
__device__ __forceinline__ T* ws_ptr(const fh_plan& p, void* ws, int which) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + p.off[which]);
}

}  // namespace fh
