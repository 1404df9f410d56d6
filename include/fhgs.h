/*
 * fhgs.h -- C ABI of the MI355X (gfx950) tile-based Gaussian-splatting
 * rasterizer with w-weighted feature fusion (FHGS, arXiv 2505.19154).
 *
 * The path, in the order of Algorithm 2 of the paper:
 *   fh_project        screen-space Gaussians (EWA projection, conic, SH colour,
 *                     depth key and tile rectangle) for every (view, Gaussian)
 *   fh_bin_sort       DuplicateWithKeys + SortByKeys + IdentifyTileRanges: one
 *                     instance per (Gaussian, overlapped 16x16 tile), ordered by
 *                     (tile, depth, Gaussian index), and each tile's [start, end)
 *   fh_render_fwd     front-to-back alpha compositing of colour and of the
 *                     D-channel feature (Section 3.1: c = sum_i c_i w_i,
 *                     w_i = alpha_i T_i)
 *   fh_render_bwd     the adjoint through w (Appendix A.2, dL/dalpha_k), chained
 *                     to means, scales, rotations, opacities and SH; optionally
 *                     fused with feature fusion
 *   fh_fuse_features  w-weighted scatter of a per-pixel target map into
 *                     per-Gaussian accumulators (compensated FP32 sums)
 *   fh_fuse_finalize  accumulators -> fused per-Gaussian features
 *
 * Conventions
 *   - Every data pointer is a DEVICE pointer unless its comment says host.
 *     The caller allocates every buffer (inputs, outputs, accumulators and the
 *     workspace); the library never allocates or frees device memory and keeps
 *     no device state between calls.
 *   - All calls are asynchronous on the given HIP stream (NULL = the default
 *     stream) and never synchronise the host, except fh_read_counters, which
 *     waits for the stream (fh_get_status copies the same counters on the
 *     stream without waiting).  Calls that only launch kernels can be captured
 *     into a HIP graph.
 *   - Return value: FH_OK, or a negative fh_status for errors detected on the
 *     host (bad arguments, launch failure).  Conditions only known on the
 *     device (instance capacity exceeded, non-finite Gaussians culled) are
 *     recorded in the workspace and read back by fh_read_counters or
 *     fh_get_status.
 *   - Cameras: pinhole, OpenCV axes (x right, y down, z forward);
 *     p_cam = R p_world + t with R row-major.  Pixel (px, py) samples the
 *     point (px + 1/2, py + 1/2).
 *   - Views are concatenated: per-pixel arrays of view v start at pixel
 *     offset sum_{u<v} W_u H_u, row-major within the view.
 */
#ifndef FHGS_H
#define FHGS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FH_VERSION 1
#define FH_MAX_VIEWS 32
#define FH_WS_SLOTS 48   /* capacity of fh_plan.off (workspace sub-buffers in use: fh_plan.n_ws) */
#define FH_TILE 16

/* Every enum of this interface spans the whole int32 range (its two _RANGE_
 * enumerators are bounds, not values): callers pass enums as plain integers,
 * and the library's rejection of an unknown one (FH_E_INVALID, or "unknown"
 * from fh_status_string) is then well defined in C and C++ alike. */
#define FH_ENUM_RANGE(P) P##_RANGE_MIN_ = -0x7fffffff - 1, P##_RANGE_MAX_ = 0x7fffffff

typedef enum {
    FH_OK = 0,
    FH_E_INVALID = -1,      /* null pointer, size or layout error */
    FH_E_UNSUPPORTED = -2,  /* e.g. sh_degree > 3, too many views */
    FH_E_HIP = -3,          /* a HIP launch or runtime call failed */
    FH_E_CAPACITY = -4,     /* device-side: instance or visit capacity exceeded */
    FH_E_SCRATCH = -5,      /* the plan's workspace exceeds FH_STATIC_SCRATCH_BYTES (fh_render_fwd_static) */
    FH_ENUM_RANGE(FH_STATUS)
} fh_status;

typedef enum { FH_F32 = 0, FH_BF16 = 1, FH_ENUM_RANGE(FH_DTYPE) } fh_dtype;

/* Footprint rule of the tile binning (fh_plan.bin_rule).  Both rules give
 * every tile holding a pixel where alpha = o G can reach 1/255, so no
 * composited value depends on the rule; only the instance lists (and n_iter,
 * a list position) do.
 *   FH_BIN_BOX      half-extents sqrt(11.1 Sigma2_ii) for every Gaussian
 *                   (11.1 > 2 ln 255)
 *   FH_BIN_OPACITY  half-extents sqrt(kappa_i Sigma2_ii) with
 *                   kappa_i = min(11.1, 2 ln(255 o_i) + 1/256): alpha reaches
 *                   1/255 only where d^T Sigma2^-1 d <= 2 ln(255 o_i);
 *                   Gaussians with 255 o_i <= 1 get no instances.  ln is a
 *                   fixed sequence of float32 operations (range reduction
 *                   to [sqrt(1/2), sqrt 2) and the atanh series to s^9). */
typedef enum { FH_BIN_BOX = 0, FH_BIN_OPACITY = 1, FH_ENUM_RANGE(FH_BIN) } fh_bin_rule;

/* Primitive (fh_plan.primitive, set by fh_plan_set_primitive).
 *   FH_PRIM_GAUSSIAN  3D Gaussians with the EWA screen-space projection
 *   FH_PRIM_SURFEL    the paper's planar primitives (Section 3.1): centre
 *                     (means), tangents t_u, t_v = the first two columns of
 *                     the quaternion's rotation, planar scales s_u, s_v =
 *                     scales[:, 0:2] (scales[:, 2] takes no part and gets a
 *                     zero gradient); a pixel takes the density
 *                     exp(-(u^2 + v^2)/2) of the point (u, v) of the
 *                     surfel's plane that its ray meets (the ray-plane
 *                     intersection x = W H (u, v, 1, 1)^T); depth order by
 *                     the centre's camera depth; tile rects bound the image
 *                     of the disc u^2 + v^2 <= kappa_i (the opacity-aware
 *                     kappa_i of FH_BIN_OPACITY, whatever bin_rule says),
 *                     and surfels whose disc reaches the camera plane are
 *                     culled.  Both arithmetic forms and the NDFD branch. */
typedef enum { FH_PRIM_GAUSSIAN = 0, FH_PRIM_SURFEL = 1, FH_ENUM_RANGE(FH_PRIM) } fh_primitive;

/* Arithmetic form of the compositing kernels. */
typedef enum {
    FH_FORM_F32 = 0,        /* FP32 blending; the adjoint and fusion on the FP32 VALU; the forward on MFMA with
                               three-term BF16 splits of w and f for FP32 features where d allows, else on the VALU */
    FH_FORM_BF16 = 1,       /* BF16 features, (pixels x K)(K x D) blends on MFMA, FP32 accumulation */
    FH_ENUM_RANGE(FH_FORM)
} fh_form;

/* The Gaussians theta_i (Section 3.1), structure of arrays, activated values.
 * means [n,3], scales [n,3] (> 0), quats [n,4] (w, x, y, z; normalised inside,
 * gradients include the normalisation), opacity [n] in (0, 1),
 * sh [n, (sh_degree+1)^2, 3], feat [n, d] (FP32 or BF16 per feat_dtype; the
 * frozen semantic feature f_i, never differentiated).  With n = 0 (an empty
 * scene: every pixel keeps C = 0, T = 1, n_iter = 0, F = 0) these arrays, and
 * the per-Gaussian gradient and fusion accumulator arrays of fh_render_bwd,
 * fh_fuse_features and fh_fuse_finalize, may be NULL. */
typedef struct {
    const float *means;
    const float *scales;
    const float *quats;
    const float *opacity;
    const float *sh;
    const void *feat;
    int64_t n;
    int32_t sh_degree;      /* 0..3 */
    int32_t d;              /* feature channels, 0..1024 */
    int32_t feat_dtype;     /* fh_dtype */
    int32_t reserved;
} fh_gaussians;

/* One pinhole camera (the world-to-camera transform W of Section 3.1). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];             /* row-major world->camera rotation */
    float t[3];
} fh_camera;

/* Launch shape of the compositing kernels.  No result depends on it: every
 * pixel's walk and every instance's partial sums are computed in the same
 * order for every setting.
 *   fwd_slice  channels per forward workgroup (the feature dimension is cut
 *              into ceil(d / fwd_slice) slices, each re-walking the tile).
 *              BF16 form, and FP32 form with FP32 features and d = 32, 64,
 *              96 or a multiple of 128 (the MFMA forward; the features enter
 *              it as three BF16 terms): dividing d, and 32, 64, 96 or 128 (BF16 form only) with
 *              fwd_rows 16, 64, 128 or 256 with fwd_rows 8, or 128 or 256
 *              with fwd_rows 4 (BF16 form only).  Other FP32-form widths: 8,
 *              16, 32 or 64.  0 when d == 0.
 *   fwd_rows   pixel rows per forward workgroup (BF16 form: 16, 8 for two
 *              workgroups per tile with twice the registers each, or 4 for
 *              four workgroups per tile, several resident per CU, each with
 *              its own barriers; the FP32 VALU forward: 16).
 *   bwd_chunk  Gaussians per back-to-front chunk of the FP32-form adjoint:
 *              16 or 32 (32 needs d <= 512).  The BF16-form adjoint always
 *              takes 32 (the MFMA k).
 *   schedule   order in which the MFMA walk kernels take the (view, tile)
 *              work items: 0 tile index order; 1 longest first (tiles sorted
 *              by their list length for the forward, by their traversal
 *              length for the adjoint and fusion; ties in index order), so
 *              that the heaviest tiles of all views start first and the light
 *              ones fill the tail.
 * fh_plan_init fills defaults; fh_autotune picks the fastest by timing. */
typedef struct {
    int32_t fwd_slice;
    int32_t bwd_chunk;
    int32_t fwd_rows;
    int32_t schedule;
} fh_tuning;

/* Host-side description of one batch of views: sizes, capacities and the
 * workspace layout.  Filled by fh_plan_init; plain data, may be copied. */
typedef struct {
    int64_t n;                       /* Gaussians */
    int32_t n_views, d, sh_degree, feat_dtype;
    int32_t form;                    /* fh_form */
    int32_t rank_bits, tile_bits;    /* key layout of the instance sort */
    int32_t packed_keys;             /* 1: one u32 key (tile << rank_bits | rank); 0: u32 tile + u32 rank */
    int32_t bin_rule;                /* fh_bin_rule; fh_plan_init sets FH_BIN_BOX, callers may change it */
    int32_t ndfd;                    /* 1: the workspace holds the NDFD gradient storage (fh_plan_set_ndfd) */
    int32_t primitive;               /* fh_primitive; fh_plan_init sets FH_PRIM_GAUSSIAN (fh_plan_set_primitive) */
    int64_t inst_capacity;           /* max (Gaussian, tile) instances over all views */
    int64_t visit_capacity;          /* max instances visited by the backward (per-instance partials) */
    int64_t n_pixels, n_tiles;
    fh_camera cams[FH_MAX_VIEWS];
    int64_t pix_off[FH_MAX_VIEWS + 1];
    int64_t tile_off[FH_MAX_VIEWS + 1];
    int32_t tiles_x[FH_MAX_VIEWS], tiles_y[FH_MAX_VIEWS];
    fh_tuning tuning;                /* launch shape (see fh_tuning) */
    /* workspace layout: byte offsets of the n_ws sub-buffers (each 256-byte
     * aligned, ascending, the last one ending at or before ws_bytes), the total */
    int32_t n_ws;
    size_t off[FH_WS_SLOTS];
    size_t ws_bytes;
} fh_plan;

/* Per-pixel outputs of fh_render_fwd (caller-owned, FP32 unless noted).
 * C [P,3], F [P,d] (may be NULL when d == 0), T [P] (final transmittance),
 * n_iter [P] (u32: 1 + position within the tile's list of the last
 * contributing Gaussian, 0 if none). */
typedef struct {
    float *C;
    float *F;
    float *T;
    uint32_t *n_iter;
} fh_image;

/* Upstream adjoints for fh_render_bwd: dC [P,3], dF [P,d] (NULL = 0),
 * dT [P] (NULL = 0). FP32.
 *
 * Optional NDFD feature branch (Section 3.3, Appendix A.1-A.2; ndfd_gt NULL:
 * off).  With unit features fh_i and gh = F_gt(p) / |F_gt(p)|, along each
 * pixel's walk sigma_i = 1 / (1 + exp(ndfd_k (fh_i . gh - ndfd_lambda))),
 * L_gt = sum_i w_i sigma_i and L_cf = sum_i sigma_i w_i (W_{i-1} -
 * F_{i-1} . fh_i) with W, F the running weight and unit-feature sums; the
 * derivative of sum_p (ndfd_a[p] L_gt(p) + ndfd_b[p] L_cf(p)) through the
 * blend weights joins the adjoint (sigma is a constant of the frozen
 * features).  ndfd_gt [P,d] BF16; ndfd_a, ndfd_b [P] FP32 (NULL = 0);
 * ndfd_Lgt, ndfd_Lcf [P] FP32 outputs of the same sweep (NULL: not written).
 * Needs BF16 features and d in {32, 64, 96, 128, 256} (FH_E_UNSUPPORTED
 * otherwise) and a plan with the NDFD storage (fh_plan_set_ndfd; FH_E_INVALID
 * otherwise). */
typedef struct {
    const float *dC;
    const float *dF;
    const float *dT;
    const void *ndfd_gt;
    const float *ndfd_a;
    const float *ndfd_b;
    float *ndfd_Lgt;
    float *ndfd_Lcf;
    float ndfd_lambda;
    float ndfd_k;
} fh_upstream;

/* Gradients written by fh_render_bwd (caller-owned, FP32, overwritten):
 * means [n,3], scales [n,3], quats [n,4], opacity [n], sh [n,B,3]. */
typedef struct {
    float *means;
    float *scales;
    float *quats;
    float *opacity;
    float *sh;
} fh_grads;

/* Fusion accumulators (caller-owned, FP32, persistent across calls and views;
 * zero them once before the first view).  Neumaier-compensated pairs:
 * the running value is sum + comp.  sum, comp [n,d]; wsum, wcomp [n]. */
typedef struct {
    float *sum;
    float *comp;
    float *wsum;
    float *wcomp;
} fh_fusion;

/* Device-side counters, read back by fh_read_counters (host struct). */
typedef struct {
    int64_t n_instances;     /* instances the binning produced (may exceed capacity) */
    int64_t n_visited;       /* instances the forward traversal reached (backward partials) */
    int64_t n_culled_nonfinite;
    int32_t inst_overflow;   /* 1 if n_instances > inst_capacity: bin_sort results invalid */
    int32_t visit_overflow;  /* 1 if n_visited > visit_capacity: render_bwd results invalid */
} fh_counters;

/* Buffers inside the workspace that callers may inspect (fh_get_buffer). */
typedef enum {
    FH_BUF_RECORDS = 0,      /* float4 [V*n*3] screen-space records (surfels: [V*n*4]) */
    FH_BUF_DEPTH_KEY = 1,    /* u32 [V*n] float32 depth bits, 0xFFFFFFFF if culled */
    FH_BUF_RECT = 2,         /* i32 [V*n*4] tile rect x0, y0, x1, y1 (inclusive; x0 > x1 if culled) */
    FH_BUF_DEPTH_ORDER = 3,  /* u32 [V*n] Gaussian index, per view sorted by (depth, index) */
    FH_BUF_RANGES = 4,       /* u32 [tiles,2] [start, end) into the sorted instances */
    FH_BUF_TILE_NITER = 5,   /* u32 [tiles] max n_iter over the tile's pixels (after render_fwd) */
    FH_BUF_GRAD2D = 6,       /* float [V*n,12] per-(view, Gaussian) screen-space adjoints (after render_bwd;
                                surfels: [V*n,16]) */
    FH_ENUM_RANGE(FH_BUF)
} fh_buffer;

/* Fill `plan` for n Gaussians and n_views cameras (host array `cams`).
 * inst_capacity / visit_capacity bound the data-dependent instance counts;
 * pass 0 to get a plan whose workspace holds only the projection and the
 * counters (enough for fh_project + fh_bin_count).  Errors: FH_E_INVALID for
 * null/negative sizes, FH_E_UNSUPPORTED for sh_degree > 3, n_views >
 * FH_MAX_VIEWS, d > 1024, or a BF16 form with FP32 features. */
fh_status fh_plan_init(fh_plan *plan, int64_t n, int32_t sh_degree, int32_t d, fh_dtype feat_dtype,
                       fh_form form, const fh_camera *cams, int32_t n_views,
                       int64_t inst_capacity, int64_t visit_capacity);

/* Add (enable = 1) or drop (0) the workspace storage of the NDFD gradient
 * (the ndfd_* fields of fh_upstream in fh_render_bwd): two floats per visited
 * (position, pixel) and the per-half-tile partials, 2 KB + 64 B (surfels:
 * 2 KB + 128 B) per unit of visit_capacity.  Recomputes the workspace layout (ws_bytes); set it before
 * allocating the workspace.  fh_ndfd_losses needs no storage. */
fh_status fh_plan_set_ndfd(fh_plan *plan, int32_t enable);

/* Choose the primitive (fh_primitive; Section 3.1's surfels or 3D Gaussians)
 * of a plan from fh_plan_init.  Surfel records take 64 B per
 * (view, primitive) and their per-instance partials 64 B per visited
 * instance.  Resets the launch shape to the primitive's default and
 * recomputes the workspace layout; set it before allocating the workspace. */
fh_status fh_plan_set_primitive(fh_plan *plan, int32_t primitive);

/* Project every (view, Gaussian) (Algorithm 2: Homogenization and
 * 2DScreenGaussians; the screen-space Gaussian of Section 3.1).  Writes the
 * records, depth keys and tile rects into the workspace and clears the
 * counters.  Gaussians with float32 depth <= 0.2 or a non-finite projection
 * are culled. */
fh_status fh_project(const fh_plan *plan, const fh_gaussians *g, void *ws, hipStream_t stream);

/* Count the instances (sum of tile-rect areas) after fh_project, so that the
 * caller can size inst_capacity; the count is read with fh_read_counters. */
fh_status fh_bin_count(const fh_plan *plan, void *ws, hipStream_t stream);

/* Tile binning (Appendix A, "Details of the Rasterizer"; Algorithm 2:
 * CreateTiles, DuplicateWithKeys, SortByKeys, IdentifyTileRanges).  Produces
 * the instances in (tile, depth, Gaussian index) order and every tile's
 * range.  Requires inst_capacity > 0; if the instance count exceeds it the
 * overflow counter is set and the ranges are left empty. */
fh_status fh_bin_sort(const fh_plan *plan, void *ws, hipStream_t stream);

/* The paper's 64-bit keys of the sorted instances, (global tile << 32) | depth
 * bits, and the Gaussian index of each: keys_out u64 [n_inst], gid_out u32
 * [n_inst] (either may be NULL), n_inst = the instance count (<= capacity). */
fh_status fh_bin_keys(const fh_plan *plan, const void *ws, uint64_t *keys_out, uint32_t *gid_out,
                      int64_t n_inst, hipStream_t stream);

/* Front-to-back compositing of every pixel of every view (Section 3.1).
 * Reads the projection and the binning from the workspace and feat from g.
 * Also records per-tile traversal lengths for the backward pass. */
fh_status fh_render_fwd(const fh_plan *plan, const fh_gaussians *g, void *ws, const fh_image *out,
                        hipStream_t stream);

/* Adjoint of fh_render_fwd (Appendix A.2) chained through the projection.
 * Recomputes transmittance back to front from T and n_iter of `fwd`.
 * If fusion_target (per-pixel [P,d], dtype target_dtype) and acc are given,
 * the same sweep also accumulates feature fusion into acc.  In the BF16 form
 * the target must be BF16 (FH_E_UNSUPPORTED otherwise): it is an MFMA
 * operand as stored.  BF16 form above 256 channels: the feature contractions
 * run in channel slices of 256 (or 128 when 256 does not divide d), the part
 * f_k . dF of the earlier slices carried between launches in the workspace.
 * Gradients are written (not accumulated) into `out`.  After an instance or
 * visit overflow (fh_read_counters) the gradients are all zero and acc is
 * left unchanged. */
fh_status fh_render_bwd(const fh_plan *plan, const fh_gaussians *g, void *ws, const fh_image *fwd,
                        const fh_upstream *up, const void *fusion_target, fh_dtype target_dtype,
                        const fh_fusion *acc, const fh_grads *out, hipStream_t stream);

/* The NDFD losses alone (Section 3.3): L_gt [P] and L_cf [P] of every pixel
 * (either may be NULL) for the ground-truth map gt [P,d] (BF16), with the
 * sigmoid's threshold lambda and slope k; needs fh_render_fwd's T and n_iter
 * for the same views.  BF16 features, d in {32, 64, 96, 128, 256}. */
fh_status fh_ndfd_losses(const fh_plan *plan, const fh_gaussians *g, void *ws, const fh_image *fwd, const void *gt,
                         float lambda, float k, float *Lgt, float *Lcf, hipStream_t stream);

/* Feature fusion alone: acc.sum += sum_p w_g(p) target(p), acc.wsum += sum_p
 * w_g(p) for every Gaussian g, Neumaier-compensated; needs fh_render_fwd's
 * T and n_iter for the same views.  BF16 form: target must be BF16. */
fh_status fh_fuse_features(const fh_plan *plan, const fh_gaussians *g, void *ws, const fh_image *fwd,
                           const void *target, fh_dtype target_dtype, const fh_fusion *acc,
                           hipStream_t stream);

/* feat_out[g] = (sum + comp) / (wsum + wcomp) where wsum + wcomp > 0, else
 * feat_in[g] (NULL feat_in: 0).  feat_in, feat_out [n,d] of dtype. */
fh_status fh_fuse_finalize(const fh_fusion *acc, int64_t n, int32_t d, const void *feat_in, void *feat_out,
                           fh_dtype dtype, hipStream_t stream);

/* Wait for `stream` and copy the device counters into *out (host). */
fh_status fh_read_counters(const fh_plan *plan, const void *ws, fh_counters *out, hipStream_t stream);

/* The device counters (the status word of the calls so far on `stream`:
 * instance and visit counts, overflow flags, non-finite culls) copied by a
 * kernel on `stream` into *out, a DEVICE-accessible pointer (device memory or
 * pinned host memory), without synchronising the host; capturable in a HIP
 * graph.  The values are there once `stream` has reached the copy.
 * FH_E_INVALID for a null argument. */
fh_status fh_get_status(const fh_plan *plan, const void *ws, fh_counters *out, hipStream_t stream);

/* Device pointer and element count of a workspace buffer (no device access). */
fh_status fh_get_buffer(const fh_plan *plan, void *ws, fh_buffer which, void **ptr, int64_t *count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): fh_project +
 * fh_bin_sort + fh_render_fwd of `plan` with the workspace taken from a static
 * device array of FH_STATIC_SCRATCH_BYTES that the library holds on every GPU
 * it runs on until the process ends, instead of a caller allocation.  No
 * hipMalloc or other allocating call is made.  The caller passes the inputs
 * (g) and the outputs (out, as for fh_render_fwd) and, optionally, counters: a
 * DEVICE pointer that receives the call's fh_counters (instance count and
 * overflow flags) on the stream.  Results equal those of the three calls with
 * a caller workspace.  Errors: FH_E_SCRATCH when plan->ws_bytes exceeds
 * FH_STATIC_SCRATCH_BYTES (use a plan with smaller capacities, or the calls
 * with a workspace), and those of the three calls.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * threads or processes' graphs) race, and the array keeps the last call's
 * contents. */
#define FH_STATIC_SCRATCH_BYTES (64ull << 20)
fh_status fh_render_fwd_static(const fh_plan *plan, const fh_gaussians *g, const fh_image *out, fh_counters *counters,
                               hipStream_t stream);

/* Valid launch shapes for this plan: writes up to `max` settings into out
 * (host array) and their number into *count (host).  Each differs from
 * plan->tuning in the field that the kernel `which` uses (FH_K_RENDER_FWD:
 * fwd_slice; FH_K_RENDER_BWD: bwd_chunk); for other kernels, or when only one
 * setting is valid, the one entry is plan->tuning.  For FH_K_RENDER_FWD the
 * entries differ in fwd_slice and fwd_rows.  Host only. */
fh_status fh_tuning_candidates(const fh_plan *plan, int32_t which, fh_tuning *out, int32_t max, int32_t *count);

/* Autotuner (the batched form picks its launch shape on the real workload):
 * times every candidate of fh_tuning_candidates for FH_K_RENDER_FWD, then for
 * FH_K_RENDER_BWD, `reps` calls each after one warm-up, with HIP events on
 * `stream`, and writes the fastest into plan->tuning.  Needs the state of a
 * completed fh_project + fh_bin_sort + fh_render_fwd in ws with no capacity
 * overflow.  fwd, grads and acc are written as by the calls they time (acc is
 * accumulated into: pass a scratch accumulator, or NULL to time without
 * fusion); up, target as for fh_render_bwd (up may be NULL to tune only the
 * forward).  Synchronises the stream.  Errors: those of the timed calls, and
 * FH_E_HIP if an event call fails. */
fh_status fh_autotune(fh_plan *plan, const fh_gaussians *g, void *ws, const fh_image *fwd,
                      const fh_upstream *up, const void *target, fh_dtype target_dtype, const fh_fusion *acc,
                      const fh_grads *grads, int32_t reps, hipStream_t stream);

/* Kernels that fh_set_kernel_events can bracket with events. */
typedef enum {
    FH_K_PROJECT = 0,       /* the projection kernel of fh_project */
    FH_K_BIN = 1,           /* all of fh_bin_sort */
    FH_K_RENDER_FWD = 2,    /* the compositing kernel of fh_render_fwd */
    FH_K_RENDER_BWD = 3,    /* the adjoint (+ fusion) compositing kernel of fh_render_bwd / fh_fuse_features */
    FH_K_REDUCE = 4,        /* the per-Gaussian reductions of the per-instance partials */
    FH_K_PROJECT_BWD = 5,   /* the projection adjoint of fh_render_bwd */
    FH_K_NDFD = 6,          /* the NDFD walk of fh_render_bwd / fh_ndfd_losses */
    FH_ENUM_RANGE(FH_K)
} fh_kernel;

/* Profiling hook for benchmarks: for the next n launches of `which`, record
 * start[i] before and stop[i] after the i-th launch, on the launch's stream.
 * start/stop are host arrays of n caller-created HIP events and must stay
 * valid until those launches are issued; n = 0 switches the hook off.
 * Process-wide host state, not thread-safe. */
fh_status fh_set_kernel_events(fh_kernel which, hipEvent_t *start, hipEvent_t *stop, int32_t n);

/* ------------------------------------------------------------------------
 * The training step around the rasterizer (Algorithm 1 of the paper:
 * photometric loss, Adam update of the Gaussians, and periodic adaptive
 * density control).  Elementwise kernels over pixels or Gaussians; all calls
 * asynchronous on `stream`, no allocation, no host synchronisation.
 * ------------------------------------------------------------------------ */

/* Raw trainable parameters (device, FP32, structure of arrays): means [n,3],
 * log_scales [n,3] (scale = exp), quats [n,4] (raw, normalised inside the
 * projection), logit_opacity [n] (opacity = sigmoid), sh [n,(L+1)^2,3].  The
 * same layout holds Adam's first and second moments. */
typedef struct {
    float *means;
    float *log_scales;
    float *quats;
    float *logit_opacity;
    float *sh;
} fh_params;

/* Adam (Kingma and Ba): per element with raw gradient g at step t >= 1,
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * x -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * lr per group in fh_params order (means, log_scales, quats, logit, sh). */
typedef struct {
    float lr[5];
    float beta1, beta2, eps;
    int32_t step;
} fh_adam;

/* One Adam step of every group, in place on `param`, `m` and `v`.  `grads`
 * are fh_render_bwd's gradients of the ACTIVATED parameters; the raw
 * gradients are taken through the activations at the rendering values held
 * in `scales` [n,3] and `opacity` [n] (dL/dlog s = s dL/ds, dL/dlogit =
 * o (1 - o) dL/do), which are then overwritten with the activations of the
 * updated raw values, ready for the next fh_project.  Errors: FH_E_INVALID for
 * null pointers, n < 0, sh_degree outside 0..3, step < 1, betas outside
 * [0, 1) or eps < 0. */
fh_status fh_adam_step(int64_t n, int32_t sh_degree, const fh_params *param, const fh_params *m,
                       const fh_params *v, const fh_grads *grads, const fh_adam *cfg, float *scales,
                       float *opacity, hipStream_t stream);

/* The activated values rendering reads: scales [n,3] = exp(log_scales),
 * opacity [n] = 1 / (1 + exp(-logit_opacity)). */
fh_status fh_activate(int64_t n, const float *log_scales, const float *logit_opacity, float *scales, float *opacity,
                      hipStream_t stream);

/* Densification statistics (Algorithm 1, Densification), accumulated after
 * each fh_render_bwd of `plan`: for every Gaussian and every view that binned
 * it (at least one tile instance), grad_sum [n] += |dL/d(u, v)| (the norm of
 * the screen-space mean gradient of that view) and count [n] += 1, views in
 * order, FP32.  Caller-owned accumulators, zeroed at each refinement.  After an
 * instance or visit overflow nothing is added. */
fh_status fh_densify_stats(const fh_plan *plan, const void *ws, float *grad_sum, int32_t *count, hipStream_t stream);

/* Thresholds of the adaptive density control.  With avg = grad_sum / count
 * (0 if count = 0) and lmax the largest log-scale, all in float32:
 * avg >= grad_threshold and lmax <= log_scale_threshold: clone;
 * avg >= grad_threshold and lmax > log_scale_threshold: split into two;
 * then every Gaussian (with its clone or second child) whose logit is below
 * prune_logit is removed. */
typedef struct {
    float grad_threshold;
    float log_scale_threshold;
    float prune_logit;
} fh_densify_config;

/* Bytes of the caller workspace fh_densify_plan / fh_densify_apply use for n
 * Gaussians. */
size_t fh_densify_workspace_size(int64_t n);

/* Decide every Gaussian's action and its output positions, and write
 * counts[0] = n_out (kept Gaussians + appended copies) and counts[1] = n_keep
 * (kept originals) to `counts` (device int64[2]); the caller reads them (a
 * synchronising read) to allocate the outputs of fh_densify_apply.  dws:
 * fh_densify_workspace_size(n) bytes, kept until fh_densify_apply. */
fh_status fh_densify_plan(int64_t n, const float *grad_sum, const int32_t *count, const float *log_scales,
                          const float *logit_opacity, const fh_densify_config *cfg, void *dws, int64_t *counts,
                          hipStream_t stream);

/* Write the densified set: the kept Gaussians in index order (a split one
 * replaced by its first child), then the clones and second children in the
 * index order of their parents.  Split children: means mu + R(q) diag(s) z_j
 * (z [n,2,3]: standard normal draws, j = 0, 1; only split Gaussians' rows are
 * read), log-scales log s - ln 1.6, other parameters copied.  Moments: kept
 * originals keep theirs, split parents and new Gaussians start at zero.
 * Outputs hold n_out rows (counts[0] of fh_densify_plan); n_keep = counts[1];
 * n_out = 0 writes nothing (outputs may then be NULL).  scales_out [n_out,3],
 * opacity_out [n_out]: the activated values.  Outputs must not alias the
 * inputs. */
fh_status fh_densify_apply(int64_t n, int32_t sh_degree, const void *dws, const fh_params *in, const fh_params *m_in,
                           const fh_params *v_in, const float *z, int64_t n_out, int64_t n_keep, const fh_params *out,
                           const fh_params *m_out, const fh_params *v_out, float *scales_out, float *opacity_out,
                           hipStream_t stream);

/* Densify any other per-Gaussian attribute (the frozen features f, which
 * Algorithm 1's densification carries along): out row k receives the row of
 * the parent of output Gaussian k, in the order of fh_densify_apply.  in [n,
 * row_bytes], out [n_out, row_bytes]; dws as left by fh_densify_plan. */
fh_status fh_densify_copy_rows(int64_t n, const void *dws, const void *in, void *out, int64_t row_bytes,
                               int64_t n_out, int64_t n_keep, hipStream_t stream);

/* Bytes of the caller workspace fh_photometric_loss uses for n_pixels. */
size_t fh_loss_workspace_size(int64_t n_pixels);

/* Photometric loss of a rendered image against its target (Algorithm 1,
 * Photometric Loss; the paper leaves the function open, here the mean squared
 * error over pixels and channels): *loss (device) = sum (C - C_target)^2 /
 * (3 P), dC [P,3] = 2 (C - C_target) / (3 P), the upstream adjoint of
 * fh_render_bwd.  Summed in a fixed order (reproducible). */
fh_status fh_photometric_loss(int64_t n_pixels, const float *C, const float *C_target, float *dC, float *loss,
                              void *lws, hipStream_t stream);

const char *fh_status_string(fh_status s);
int32_t fh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FHGS_H */
