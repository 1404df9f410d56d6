// Kernel argument structs and launchers shared by the HIP translation units.
#pragma once

#include "common.hpp"

namespace fh {
// project.hip
struct ProjectArgs {
    const float *means, *scales, *quats, *opacity, *sh;
    int n, sh_degree;
    int bin_rule;       // fh_bin_rule
    int prim;           // fh_primitive (surfel records: 4 float4)
    float4* rec;
    uint32_t* depth_key;
    int4* rect;
    Counters* counters;
};
struct ProjectBwdArgs {
    const float *means, *scales, *quats, *opacity, *sh;
    int n, sh_degree;
    const float* grad2d;
    const uint32_t* depth_key;
    const Counters* counters;   // an instance or visit overflow leaves the (zero-filled) outputs zero
    float *g_means, *g_scales, *g_quats, *g_opacity, *g_sh;
    int prim;                   // fh_primitive (surfel adjoint rows: 16 floats)
};
void launch_project(const ProjectArgs&, const CamTable&, const ViewTable&, int, hipStream_t);
void launch_project_bwd(const ProjectBwdArgs&, const CamTable&, int, hipStream_t);
// sort.hip
size_t scan_scratch_u32(int64_t n);
void device_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch, int write_total,
                           hipStream_t s);
int radix_sort(const uint32_t* keys_src, const uint32_t* vals_src, uint32_t* ka, uint32_t* va, uint32_t* kb,
               uint32_t* vb, bool with_vals, int64_t segs, int64_t seg_len, const unsigned long long* dev_len,
               int64_t cap, int lo, int hi, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s);
size_t radix_hist_u32(int64_t segs, int64_t span);
struct DupArgs {
    const uint32_t* inst_off;
    const uint32_t* order;
    const int4* rect;
    int64_t n, total_ranks;
    int64_t cap;
    const Counters* counters;
    uint32_t* keys;
    uint32_t* vals;
    int rank_bits;
    int packed;
    ViewTable vt;
};
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// tile schedule keys: 0xFFFF - min(cost, 0xFFFF), cost = the list length
// (ranges) or the traversal length (tile_niter)
void launch_tile_cost_keys(const uint32_t* ranges, const uint32_t* tile_niter, int64_t n_tiles, uint32_t* keys,
                           hipStream_t s);
void launch_tiles_by_rank(const uint32_t* order, const int4* rect, int64_t n, int64_t total, uint32_t* ntiles,
                          Counters* c, hipStream_t s);
void launch_check_capacity(Counters* c, int64_t cap, hipStream_t s);
void launch_duplicate(const DupArgs& a, hipStream_t s);
void launch_ranges(const uint32_t* keys, const Counters* c, int64_t cap, int rank_bits, int packed, uint32_t* ranges,
                   hipStream_t s);
void launch_bin_keys(const uint32_t* keys, const uint32_t* vals, const uint32_t* order, const uint32_t* depth_key,
                     int64_t n_inst, int64_t n, int rank_bits, int packed, uint64_t* ko, uint32_t* go, hipStream_t s);
// render_f32.hip
struct RenderArgs {
    const float4* rec;
    const float4* rrec;       // [V*N*3] records in depth-rank order
    const uint32_t* order;
    const uint32_t* keys;
    const uint32_t* vals;
    const uint32_t* ranges;
    const Counters* counters;
    int rank_bits, packed;
    int64_t n;
    const void* feat;
    int d, feat_bf16;
    float* C;
    float* F;
    float* T;
    uint32_t* n_iter;
    uint32_t* tile_niter;
    const uint32_t* tile_order;   // nullable: work item i takes tile tile_order[i]
    int prim;                     // fh_primitive (FP32 VALU kernels)
};
struct BwdArgs {
    const float4* rec;
    const uint32_t* order;
    const uint32_t* keys;
    const uint32_t* vals;
    const uint32_t* ranges;
    const uint32_t* tile_niter;
    const uint32_t* tile_voff;
    const Counters* counters;
    int rank_bits, packed;
    int64_t n;
    const void* feat;
    int d, feat_bf16;
    const float* T_final;
    const uint32_t* n_iter;
    const float* dC;
    const float* dF;
    const float* dT;
    const void* target;
    int target_bf16;
    const float4* vrec;        // [visits * 3] staged records, in visit order
    const uint32_t* vgid;      // [visits] staged Gaussians
    float* part_geom;
    float* part_fuse;
    const uint32_t* tile_order;   // nullable: work item i takes tile tile_order[i]
    float* wrec;                  // nullable: [visits][256] w of every visited (position, pixel), recorded by the
                                  // BF16 gradient kernel for the fusion kernel of the same call
    // BF16 kernels at feature widths above 256 work in channel slices: the
    // slice starts at channel d0 (rows of feat, dF, target and the fusion
    // partials keep the stride d); g = f . dF of the earlier slices is carried
    // between launches in [visits][256] rows (g_in added, g_out written)
    int d0;
    const float* g_in;
    float* g_out;
    int prim;                     // fh_primitive (FP32 VALU kernels)
};
struct VisitStageArgs {
    const uint32_t* ranges;
    const uint32_t* tile_niter;
    const uint32_t* tile_voff;
    const uint32_t* keys;
    const uint32_t* vals;
    int rank_bits, packed;
    const uint32_t* order;
    const float4* rrec;
    Counters* counters;
    uint32_t* vkey;     // [visits] rank of the visited instance
    uint32_t* vgid;     // [visits] its Gaussian
    float4* vrec;       // [visits * rw] its screen record
    int rw;             // float4 per record: 3 (Gaussians) or 4 (surfels)
};
struct ReduceArgs {
    const uint32_t* order;
    const uint32_t* vseg;      // [V*N][2] per-rank [start, end) into vsorted
    const uint32_t* vsorted;   // visit indices sorted by rank (stable: row-major tiles)
    Counters* counters;
    uint32_t* long_list;       // [total] ranks (geometry), [n] long Gaussians (fusion), [n] their first unit,
                               // [n] short Gaussians (fusion)
    uint32_t* unit_owner;      // [unit_cap] long-fusion slot of each unit
    float* upart;              // [unit_cap][2 d + 2] unit partials (sum, compensation per channel; weight pair)
    int64_t unit_cap;
    int64_t n, total;
    const float* part_geom;
    float* grad2d;
    const uint32_t* rank_of;
    const float* part_fuse;
    int d;
    int n_views;
    float *acc_sum, *acc_comp, *acc_wsum, *acc_wcomp;
    int wslot;                 // per-instance partial row (12 floats, surfels 16): weight sum at entry 9 (surfels 13)
};
// slice: channels per workgroup (8, 16, 32 or 64)
void launch_render_fwd_f32(const RenderArgs& a, const ViewTable& vt, int n_tiles, int slice, hipStream_t s);
// slice: channels per workgroup; rows: pixel rows per workgroup (16 or 8)
bool render_fwd_bf16_shape_ok(int d, int slice, int rows);
void launch_render_fwd_bf16(const RenderArgs& a, const ViewTable& vt, int n_tiles, int slice, int rows, bool fsplit,
                            hipStream_t s);
bool render_bwd_bf16_supported(int d);
bool render_bwd_bf16_sliced(int d);   // above 256 channels: sliced, with a carry of f . dF between slices
void launch_render_bwd_bf16(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool grads, bool fuse,
                            hipStream_t s);
void launch_visit_stage(const VisitStageArgs& a, int n_tiles, hipStream_t s);
void launch_vseg(const uint32_t* skeys, const Counters* c, int64_t cap, uint32_t* vseg, hipStream_t s);
void launch_check_visits(const uint32_t* tile_voff, int n_tiles, Counters* c, int64_t cap, hipStream_t s);
// chunk: Gaussians per back-to-front chunk (16, or 32 when d <= 512)
void launch_render_bwd_f32(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool fuse, int chunk, hipStream_t s);
// gp: floats per partial row, 12 (Gaussians: 10 used) or 16 (surfels: 14 used)
void launch_reduce_geom(const ReduceArgs& a, int gp, hipStream_t s);
void launch_reduce_fuse(const ReduceArgs& a, hipStream_t s);
// units available for the long fusion reduction at a visit capacity (see reduce.hip)
int64_t fuse_unit_capacity(int64_t visit_capacity);
// rw: float4 per record (3, surfels 4)
void launch_rank_tables(const uint32_t* order, const float4* rec, int64_t n, int64_t total, uint32_t* rank_of,
                        float4* rrec, int rw, hipStream_t s);
// ndfd.hip
struct NdfdArgs {
    const uint32_t* tile_niter;
    const uint32_t* tile_voff;
    const Counters* counters;
    const float4* vrec;         // [visits * rw] staged records, in visit order
    const uint32_t* vgid;       // [visits] staged Gaussians
    const uint16_t* feat;       // [n, d] BF16 features
    int d;
    const float* T_final;
    const uint32_t* n_iter;
    const uint16_t* gt;         // [P, d] BF16 ground-truth feature map
    const float* a;             // [P] dL/dL_gt (nullable: 0)
    const float* b;             // [P] dL/dL_cf (nullable: 0)
    float lam, kk;              // sigmoid threshold and slope
    float* Lgt;                 // [P] (nullable)
    float* Lcf;                 // [P] (nullable)
    float* part;                // [visits][2 halves][ndfd_part_floats] screen-space partials (gradient)
    float2* sc;                 // [visits][256 pixels] (sigma, prefix term) of the forward sweep (gradient)
    int prim;                   // fh_primitive (surfel records: 4 float4)
};
bool ndfd_supported(int d);
int ndfd_part_floats(int prim);   // floats per (visit, half) partial: 8 (Gaussians), 16 (surfels)
void launch_ndfd(const NdfdArgs& a, const ViewTable& vt, int n_tiles, bool grad, hipStream_t s);
void launch_ndfd_combine(const float* part, float* part_geom, const Counters* c, int64_t cap, int prim,
                         hipStream_t s);
void launch_fuse_finalize(const float* sum, const float* comp, const float* wsum, const float* wcomp, int64_t n, int d,
                          const void* feat_in, void* feat_out, int bf16, hipStream_t s);

}  // namespace fh
