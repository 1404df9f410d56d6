// The training step around the rasterizer (Algorithm 1: photometric loss,
// Adam update, adaptive density control), on the GPU.
//
// Parameters are held raw and activated for rendering: scale = exp(log-scale),
// opacity = sigmoid(logit); means, the raw quaternion and the SH coefficients
// are rendered as stored.  Every kernel here is elementwise over pixels or
// Gaussians (HBM-bound); reductions run in a fixed order (bitwise
// reproducible), and the densification decisions are taken in float32 on
// float32 values, so they are integers that any float32 evaluation in the same
// order reproduces.
#include <cmath>

#include "kernels.hpp"

namespace fh {

constexpr int TB = 256;

// ---------------------------------------------------------------------------
// Adam (Kingma and Ba) on one parameter group, with the activation's chain
// rule folded in: the raw gradient is g * dact/draw, evaluated at the
// activated value used for rendering (act), and the new activated value is
// written back.  kind: 0 identity, 1 exp (log-scales), 2 sigmoid (logits).
struct AdamGroup {
    float* x;
    float* m;
    float* v;
    const float* g;
    float* act;       // kinds 1, 2: activated values (read: rendering value; written: the updated one)
    int64_t count;
    float lr;
    int kind;
};
struct AdamArgs {
    AdamGroup grp[5];
    float b1, b2, eps, bc1, bc2;   // bc1 = 1 / (1 - b1^t), bc2 = 1 / (1 - b2^t)
};

__global__ __launch_bounds__(TB) void k_adam(AdamArgs a) {
    const AdamGroup& G = a.grp[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * TB;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < G.count; i += stride) {
        float g = G.g[i];
        float act = 0.0f;
        if (G.kind == 1) {
            act = G.act[i];
            g *= act;                       // d exp(l) / dl = exp(l)
        } else if (G.kind == 2) {
            act = G.act[i];
            g *= act * (1.0f - act);        // d sigmoid(z) / dz = o (1 - o)
        }
        const float m = a.b1 * G.m[i] + (1.0f - a.b1) * g;
        const float v = a.b2 * G.v[i] + (1.0f - a.b2) * (g * g);
        const float mh = m * a.bc1, vh = v * a.bc2;
        const float x = G.x[i] - G.lr * mh / (sqrtf(vh) + a.eps);
        G.m[i] = m;
        G.v[i] = v;
        G.x[i] = x;
        if (G.kind == 1)
            G.act[i] = expf(x);
        else if (G.kind == 2)
            G.act[i] = 1.0f / (1.0f + expf(-x));
    }
}

// Activations of raw values: scales = exp(log-scales), opacity = sigmoid(logit).
__global__ __launch_bounds__(TB) void k_activate(int64_t n, const float* __restrict__ log_scales,
                                                 const float* __restrict__ logit, float* __restrict__ scales,
                                                 float* __restrict__ opacity) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i < 3 * n) scales[i] = expf(log_scales[i]);
    if (i < n) opacity[i] = 1.0f / (1.0f + expf(-logit[i]));
}

// ---------------------------------------------------------------------------
// Densification statistics: per Gaussian, over the views that binned it (at
// least one tile instance), the norm of the screen-space mean gradient
// |dL/d(u, v)| is added (in view order) and the views counted.
__global__ __launch_bounds__(TB) void k_densify_stats(const float* __restrict__ grad2d, const int4* __restrict__ rect,
                                                      const Counters* c, int64_t n, int n_views,
                                                      float* __restrict__ gsum, int32_t* __restrict__ cnt) {
    const int64_t g = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (g >= n) return;
    // after an instance or visit overflow the screen-space adjoints are stale
    if (c->inst_overflow || c->visit_overflow) return;
    float s = gsum[g];
    int k = cnt[g];
    for (int v = 0; v < n_views; ++v) {
        const int64_t j = (int64_t)v * n + g;
        const int4 r = rect[j];
        if (r.x > r.z || r.y > r.w) continue;
        const float du = grad2d[j * 12], dv = grad2d[j * 12 + 1];
        s += sqrtf(du * du + dv * dv);
        ++k;
    }
    gsum[g] = s;
    cnt[g] = k;
}

// ---------------------------------------------------------------------------
// Densification decisions: 0 keep, 1 clone (small and hot), 2 split (large and
// hot); a Gaussian below the opacity threshold is pruned together with its
// copies (they share its logit).  keep[g] = 1 if it survives (its first copy
// stays at its place in index order), extra[g] = 1 if it also appends one.
struct DensifyCfg {
    float grad_thr, log_scale_thr, prune_logit;
};

__global__ __launch_bounds__(TB) void k_densify_classify(int64_t n, const float* __restrict__ gsum,
                                                         const int32_t* __restrict__ cnt,
                                                         const float* __restrict__ log_scales,
                                                         const float* __restrict__ logit, DensifyCfg cfg,
                                                         uint32_t* __restrict__ action, uint32_t* __restrict__ keep,
                                                         uint32_t* __restrict__ extra) {
    const int64_t g = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (g >= n) return;
    const int32_t k = cnt[g];
    const float avg = k > 0 ? gsum[g] / (float)k : 0.0f;
    const float lmax = fmaxf(fmaxf(log_scales[3 * g], log_scales[3 * g + 1]), log_scales[3 * g + 2]);
    const bool hot = avg >= cfg.grad_thr;
    const uint32_t act = hot ? (lmax <= cfg.log_scale_thr ? 1u : 2u) : 0u;
    const bool kept = logit[g] >= cfg.prune_logit;
    action[g] = act;
    keep[g] = kept ? 1u : 0u;
    extra[g] = (kept && act != 0u) ? 1u : 0u;
}

// counts[0] = kept + appended (the two scans' totals), counts[1] = kept
__global__ void k_densify_total(const uint32_t* keep_off, const uint32_t* extra_off, int64_t n, int64_t* counts) {
    if (threadIdx.x == 0) {
        counts[0] = (int64_t)keep_off[n] + (int64_t)extra_off[n];
        counts[1] = (int64_t)keep_off[n];
    }
}

// Rotation matrix of the normalised quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(const float* q, float R[9]) {
    const float nn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] * nn, x = q[1] * nn, y = q[2] * nn, z = q[3] * nn;
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

struct ParamSet {
    float *means, *log_scales, *quats, *logit, *sh;
};
struct DensifyApplyArgs {
    int64_t n, n_keep;
    int nsh;                    // SH floats per Gaussian
    const uint32_t *action, *keep_off, *extra_off, *keep;
    ParamSet in, m_in, v_in;    // (const in use)
    const float* z;             // [n, 2, 3] standard normal draws (used by split Gaussians)
    ParamSet out, m_out, v_out;
    float *scales_out, *opacity_out;
};

__device__ __forceinline__ void copy_row(float* dst, const float* src, int k) {
    for (int i = 0; i < k; ++i) dst[i] = src[i];
}
__device__ __forceinline__ void zero_row(float* dst, int k) {
    for (int i = 0; i < k; ++i) dst[i] = 0.0f;
}

// One thread per parent: the kept original (or first child) at keep_off[g],
// the clone or second child at n_keep + extra_off[g].  Split children: means
// mu + R(q) diag(s) z_j, log-scales log s - ln 1.6, other parameters copied.
// Moments: a kept original keeps its own, split parents and new Gaussians start
// at zero.
__global__ __launch_bounds__(TB) void k_densify_apply(DensifyApplyArgs a) {
    const int64_t g = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (g >= a.n || !a.keep[g]) return;
    const uint32_t act = a.action[g];
    const int64_t dst[2] = {(int64_t)a.keep_off[g], a.n_keep + (int64_t)a.extra_off[g]};
    const int ncopy = act != 0u ? 2 : 1;
    const float* mu = a.in.means + 3 * g;
    const float* ls = a.in.log_scales + 3 * g;
    const float* q = a.in.quats + 4 * g;
    float child[2][3];
    float lsc[3];
    if (act == 2u) {
        float R[9];
        quat_rot(q, R);
        const float s[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
        for (int j = 0; j < 2; ++j) {
            const float* zj = a.z + 6 * g + 3 * j;
            const float t[3] = {s[0] * zj[0], s[1] * zj[1], s[2] * zj[2]};
            for (int r = 0; r < 3; ++r)
                child[j][r] = mu[r] + (R[3 * r] * t[0] + R[3 * r + 1] * t[1] + R[3 * r + 2] * t[2]);
        }
        const float ln16 = 0.47000362924573558f;   // ln 1.6
        for (int r = 0; r < 3; ++r) lsc[r] = ls[r] - ln16;
    }
    for (int c = 0; c < ncopy; ++c) {
        const int64_t o = dst[c];
        if (act == 2u) {
            copy_row(a.out.means + 3 * o, child[c], 3);
            copy_row(a.out.log_scales + 3 * o, lsc, 3);
        } else {
            copy_row(a.out.means + 3 * o, mu, 3);
            copy_row(a.out.log_scales + 3 * o, ls, 3);
        }
        copy_row(a.out.quats + 4 * o, q, 4);
        a.out.logit[o] = a.in.logit[g];
        copy_row(a.out.sh + (int64_t)a.nsh * o, a.in.sh + (int64_t)a.nsh * g, a.nsh);
        const float* lso = a.out.log_scales + 3 * o;
        for (int r = 0; r < 3; ++r) a.scales_out[3 * o + r] = expf(lso[r]);
        a.opacity_out[o] = 1.0f / (1.0f + expf(-a.in.logit[g]));
        const ParamSet* ms[2] = {&a.m_out, &a.v_out};
        const ParamSet* mi[2] = {&a.m_in, &a.v_in};
        for (int k = 0; k < 2; ++k) {
            const ParamSet& d = *ms[k];
            if (c == 0 && act != 2u) {
                const ParamSet& sI = *mi[k];
                copy_row(d.means + 3 * o, sI.means + 3 * g, 3);
                copy_row(d.log_scales + 3 * o, sI.log_scales + 3 * g, 3);
                copy_row(d.quats + 4 * o, sI.quats + 4 * g, 4);
                d.logit[o] = sI.logit[g];
                copy_row(d.sh + (int64_t)a.nsh * o, sI.sh + (int64_t)a.nsh * g, a.nsh);
            } else {
                zero_row(d.means + 3 * o, 3);
                zero_row(d.log_scales + 3 * o, 3);
                zero_row(d.quats + 4 * o, 4);
                d.logit[o] = 0.0f;
                zero_row(d.sh + (int64_t)a.nsh * o, a.nsh);
            }
        }
    }
}

// Rows of any other per-Gaussian attribute (the frozen features): the same
// positions as k_densify_apply, every copy the parent's row.  16-byte units
// when the row allows, else bytes.
__global__ __launch_bounds__(TB) void k_densify_copy_rows(int64_t n, int64_t n_keep, const uint32_t* __restrict__ action,
                                                          const uint32_t* __restrict__ keep,
                                                          const uint32_t* __restrict__ keep_off,
                                                          const uint32_t* __restrict__ extra_off,
                                                          const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                          int64_t row_bytes) {
    const int64_t g = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (g >= n || !keep[g]) return;
    const int64_t dst[2] = {(int64_t)keep_off[g], n_keep + (int64_t)extra_off[g]};
    const int ncopy = action[g] != 0u ? 2 : 1;
    for (int c = 0; c < ncopy; ++c) {
        if (row_bytes % 16 == 0) {
            const uint4* s4 = reinterpret_cast<const uint4*>(in + g * row_bytes);
            uint4* d4 = reinterpret_cast<uint4*>(out + dst[c] * row_bytes);
            for (int64_t i = 0; i < row_bytes / 16; ++i) d4[i] = s4[i];
        } else {
            for (int64_t i = 0; i < row_bytes; ++i) out[dst[c] * row_bytes + i] = in[g * row_bytes + i];
        }
    }
}

// ---------------------------------------------------------------------------
// Photometric loss (mean squared error over pixels and channels) and its
// gradient dC = 2 (C - C_target) / (3 P).  Block b sums elements
// [b * LOSS_CHUNK, (b + 1) * LOSS_CHUNK) by a fixed tree; one block then adds
// the partials in block order.
constexpr int LOSS_CHUNK = 8192;

__device__ __forceinline__ float block_sum_256(float v, float* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    float t = 0.0f;
    if (threadIdx.x == 0) t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(TB) void k_loss_partial(const float* __restrict__ C, const float* __restrict__ Ct,
                                                     int64_t count, float scale, float* __restrict__ dC,
                                                     float* __restrict__ part) {
    __shared__ float sh[4];
    const int64_t b0 = (int64_t)blockIdx.x * LOSS_CHUNK;
    const int64_t b1 = b0 + LOSS_CHUNK < count ? b0 + LOSS_CHUNK : count;
    float acc = 0.0f;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += TB) {
        const float e = C[i] - Ct[i];
        acc += e * e;
        dC[i] = (2.0f * scale) * e;
    }
    const float t = block_sum_256(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(TB) void k_loss_final(const float* __restrict__ part, int nb, float scale,
                                                   float* __restrict__ loss) {
    __shared__ float sh[4];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < nb; i += TB) acc += part[i];
    const float t = block_sum_256(acc, sh);
    if (threadIdx.x == 0) loss[0] = t * scale;
}

// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n) {
    const int64_t b = (n + TB - 1) / TB;
    return (unsigned)(b < 1 ? 1 : b);
}

void launch_adam(const AdamArgs& a, int64_t max_count, hipStream_t s) {
    int64_t b = (max_count + TB - 1) / TB;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)b, 5), dim3(TB), 0, s, a);
}

void launch_densify_stats(const float* grad2d, const int4* rect, const Counters* c, int64_t n, int n_views,
                          float* gsum, int32_t* cnt, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_densify_stats, dim3(grid_for(n)), dim3(TB), 0, s, grad2d, rect, c, n, n_views, gsum, cnt);
}

}  // namespace fh

using namespace fh;

namespace {
// densify workspace: action, keep, extra [n]; keep_off, extra_off [n + 1]; scan scratch
struct DensifyWs {
    uint32_t *action, *keep, *extra, *keep_off, *extra_off, *scratch;
};
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t densify_ws_layout(int64_t n, char* base, DensifyWs* w) {
    const size_t u = sizeof(uint32_t);
    const size_t sizes[6] = {n * u, n * u, n * u, (n + 1) * u, (n + 1) * u, scan_scratch_u32(n + 1) * u};
    size_t off = 0;
    uint32_t* at[6];
    for (int i = 0; i < 6; ++i) {
        at[i] = base ? reinterpret_cast<uint32_t*>(base + off) : nullptr;
        off += al256(sizes[i]);
    }
    if (w) *w = DensifyWs{at[0], at[1], at[2], at[3], at[4], at[5]};
    return off;
}
bool params_ok(const fh_params* p) {
    return p && p->means && p->log_scales && p->quats && p->logit_opacity && p->sh;
}
ParamSet to_set(const fh_params* p) {
    return ParamSet{p->means, p->log_scales, p->quats, p->logit_opacity, p->sh};
}
fh_status status_of_launch() { return hipGetLastError() == hipSuccess ? FH_OK : FH_E_HIP; }
}  // namespace

extern "C" {

fh_status fh_adam_step(int64_t n, int32_t sh_degree, const fh_params* param, const fh_params* m, const fh_params* v,
                       const fh_grads* grads, const fh_adam* cfg, float* scales, float* opacity, hipStream_t s) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3) return FH_E_INVALID;
    if (!params_ok(param) || !params_ok(m) || !params_ok(v) || !grads || !cfg || !scales || !opacity)
        return FH_E_INVALID;
    if (!grads->means || !grads->scales || !grads->quats || !grads->opacity || !grads->sh) return FH_E_INVALID;
    if (cfg->step < 1 || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->eps >= 0.0f))
        return FH_E_INVALID;
    if (n == 0) return FH_OK;
    const int64_t nsh = 3 * (int64_t)(sh_degree + 1) * (sh_degree + 1);
    AdamArgs a;
    a.b1 = cfg->beta1;
    a.b2 = cfg->beta2;
    a.eps = cfg->eps;
    a.bc1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, (double)cfg->step)));
    a.bc2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, (double)cfg->step)));
    a.grp[0] = AdamGroup{param->means, m->means, v->means, grads->means, nullptr, 3 * n, cfg->lr[0], 0};
    a.grp[1] = AdamGroup{param->log_scales, m->log_scales, v->log_scales, grads->scales, scales, 3 * n, cfg->lr[1], 1};
    a.grp[2] = AdamGroup{param->quats, m->quats, v->quats, grads->quats, nullptr, 4 * n, cfg->lr[2], 0};
    a.grp[3] = AdamGroup{param->logit_opacity, m->logit_opacity, v->logit_opacity, grads->opacity, opacity, n,
                         cfg->lr[3], 2};
    a.grp[4] = AdamGroup{param->sh, m->sh, v->sh, grads->sh, nullptr, nsh * n, cfg->lr[4], 0};
    launch_adam(a, nsh * n > 4 * n ? nsh * n : 4 * n, s);
    return status_of_launch();
}

fh_status fh_activate(int64_t n, const float* log_scales, const float* logit_opacity, float* scales, float* opacity,
                      hipStream_t s) {
    if (n < 0) return FH_E_INVALID;
    if (n == 0) return FH_OK;
    if (!log_scales || !logit_opacity || !scales || !opacity) return FH_E_INVALID;
    hipLaunchKernelGGL(k_activate, dim3(grid_for(3 * n)), dim3(TB), 0, s, n, log_scales, logit_opacity, scales,
                       opacity);
    return status_of_launch();
}

fh_status fh_densify_stats(const fh_plan* p, const void* ws, float* grad_sum, int32_t* count, hipStream_t s) {
    if (!p || !ws || !grad_sum || !count) return FH_E_INVALID;
    const char* b = static_cast<const char*>(ws);
    launch_densify_stats(reinterpret_cast<const float*>(b + p->off[WS_GRAD2D]),
                         reinterpret_cast<const int4*>(b + p->off[WS_RECT]),
                         reinterpret_cast<const Counters*>(b + p->off[WS_COUNTERS]), p->n, p->n_views, grad_sum, count,
                         s);
    return status_of_launch();
}

size_t fh_densify_workspace_size(int64_t n) { return n < 0 ? 0 : densify_ws_layout(n, nullptr, nullptr); }

fh_status fh_densify_plan(int64_t n, const float* grad_sum, const int32_t* count, const float* log_scales,
                          const float* logit_opacity, const fh_densify_config* cfg, void* dws, int64_t* counts,
                          hipStream_t s) {
    if (n < 0 || !cfg || !dws || !counts) return FH_E_INVALID;
    if (n > 0 && (!grad_sum || !count || !log_scales || !logit_opacity)) return FH_E_INVALID;
    DensifyWs w;
    densify_ws_layout(n, static_cast<char*>(dws), &w);
    if (n > 0) {
        const DensifyCfg c{cfg->grad_threshold, cfg->log_scale_threshold, cfg->prune_logit};
        hipLaunchKernelGGL(k_densify_classify, dim3(grid_for(n)), dim3(TB), 0, s, n, grad_sum, count, log_scales,
                           logit_opacity, c, w.action, w.keep, w.extra);
        device_exclusive_scan(w.keep, w.keep_off, n, w.scratch, 1, s);
        device_exclusive_scan(w.extra, w.extra_off, n, w.scratch, 1, s);
    } else {
        launch_fill_u32(w.keep_off, 1, 0u, s);
        launch_fill_u32(w.extra_off, 1, 0u, s);
    }
    hipLaunchKernelGGL(k_densify_total, dim3(1), dim3(64), 0, s, w.keep_off, w.extra_off, n, counts);
    return status_of_launch();
}

fh_status fh_densify_apply(int64_t n, int32_t sh_degree, const void* dws, const fh_params* in, const fh_params* m_in,
                           const fh_params* v_in, const float* z, int64_t n_out, int64_t n_keep, const fh_params* out,
                           const fh_params* m_out, const fh_params* v_out, float* scales_out, float* opacity_out,
                           hipStream_t s) {
    if (n < 0 || n_keep < 0 || n_keep > n || n_out < n_keep || n_out > n_keep + n || sh_degree < 0 ||
        sh_degree > 3 || !dws)
        return FH_E_INVALID;
    if (n_out == 0) return FH_OK;   // every Gaussian pruned: nothing to write
    if (!params_ok(in) || !params_ok(m_in) || !params_ok(v_in) || !z || !params_ok(out) || !params_ok(m_out) ||
        !params_ok(v_out) || !scales_out || !opacity_out)
        return FH_E_INVALID;
    DensifyWs w;
    densify_ws_layout(n, static_cast<char*>(const_cast<void*>(dws)), &w);
    DensifyApplyArgs a;
    a.n = n;
    a.n_keep = n_keep;
    a.nsh = 3 * (sh_degree + 1) * (sh_degree + 1);
    a.action = w.action;
    a.keep = w.keep;
    a.keep_off = w.keep_off;
    a.extra_off = w.extra_off;
    a.in = to_set(in);
    a.m_in = to_set(m_in);
    a.v_in = to_set(v_in);
    a.z = z;
    a.out = to_set(out);
    a.m_out = to_set(m_out);
    a.v_out = to_set(v_out);
    a.scales_out = scales_out;
    a.opacity_out = opacity_out;
    hipLaunchKernelGGL(k_densify_apply, dim3(grid_for(n)), dim3(TB), 0, s, a);
    return status_of_launch();
}

fh_status fh_densify_copy_rows(int64_t n, const void* dws, const void* in, void* out, int64_t row_bytes,
                               int64_t n_out, int64_t n_keep, hipStream_t s) {
    if (n < 0 || row_bytes < 0 || n_keep < 0 || n_keep > n || n_out < n_keep || n_out > n_keep + n || !dws)
        return FH_E_INVALID;
    if (n_out == 0 || row_bytes == 0) return FH_OK;
    if (!in || !out) return FH_E_INVALID;
    DensifyWs w;
    densify_ws_layout(n, static_cast<char*>(const_cast<void*>(dws)), &w);
    hipLaunchKernelGGL(k_densify_copy_rows, dim3(grid_for(n)), dim3(TB), 0, s, n, n_keep, (const uint32_t*)w.action,
                       (const uint32_t*)w.keep, (const uint32_t*)w.keep_off, (const uint32_t*)w.extra_off,
                       static_cast<const uint8_t*>(in), static_cast<uint8_t*>(out), row_bytes);
    return status_of_launch();
}

size_t fh_loss_workspace_size(int64_t n_pixels) {
    if (n_pixels < 0) return 0;
    const int64_t nb = (3 * n_pixels + LOSS_CHUNK - 1) / LOSS_CHUNK;
    return al256((size_t)(nb < 1 ? 1 : nb) * sizeof(float));
}

fh_status fh_photometric_loss(int64_t n_pixels, const float* C, const float* C_target, float* dC, float* loss,
                              void* lws, hipStream_t s) {
    if (n_pixels < 1 || !C || !C_target || !dC || !loss || !lws) return FH_E_INVALID;
    const int64_t count = 3 * n_pixels;
    const int64_t nb = (count + LOSS_CHUNK - 1) / LOSS_CHUNK;
    if (nb > 0x7fffffff) return FH_E_UNSUPPORTED;
    const float scale = (float)(1.0 / (double)count);
    float* part = static_cast<float*>(lws);
    hipLaunchKernelGGL(k_loss_partial, dim3((unsigned)nb), dim3(TB), 0, s, C, C_target, count, scale, dC, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(TB), 0, s, (const float*)part, (int)nb, scale, loss);
    return status_of_launch();
}

}  // extern "C"
