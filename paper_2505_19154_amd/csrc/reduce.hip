// Deterministic per-Gaussian reductions of the backward pass's per-instance
// partials (no atomics on values).
//
// After the forward pass every tile knows how far its pixels walked; the
// visited instances of all tiles get consecutive visit indices (tile-major).
// Sorting the visits stably by rank gives every (view, Gaussian) a contiguous
// segment of visit indices in row-major tile order.  Short segments are summed
// by one thread (geometry) or one wavefront (fusion, lanes over channels).
// Gaussians visited in many tiles (large splats near the camera) are queued:
// a long geometry segment is summed by a whole workgroup with a fixed-order
// tree; a long fusion segment is cut into units of consecutive visits, each
// summed by a wavefront with compensation, and the units are combined in
// order.  So one long segment does not serialise the launch, and every sum
// has a fixed order: the results are bitwise reproducible.
#include "kernels.hpp"

namespace fh {

constexpr uint32_t LONG_GEOM = 64;    // visits above which a rank goes to the workgroup reduction
constexpr uint32_t LONG_FUSE = 32;    // same for fusion (per Gaussian, all views)
constexpr uint32_t FUSE_UNIT = 64;    // visits per unit of the long fusion reduction

__device__ __forceinline__ uint32_t rank_of_inst(const uint32_t* keys, const uint32_t* vals, int64_t i, int rank_bits,
                                                 int packed) {
    return packed ? (keys[i] & ((1u << rank_bits) - 1u)) : vals[i];
}

// Visit staging, one workgroup per tile, run once the forward pass has fixed
// every tile's traversal length: for visit index vo + pos (position pos of
// tile t's list, pos < tile_niter[t]) it writes the instance's rank (the key
// of the visit sort), its Gaussian and its screen record.  The backward
// kernels then read a chunk's records and Gaussians with one contiguous load
// each instead of a chain of dependent gathers (list -> rank -> record).
__global__ __launch_bounds__(256) void k_visit_stage(VisitStageArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.counters->n_long_geom = 0;
        a.counters->n_long_fuse = 0;
        a.counters->n_fuse_units = 0;
        a.counters->n_short_fuse = 0;
    }
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = blockIdx.x;
    const uint32_t nt = a.tile_niter[t];
    const uint32_t s = a.ranges[2 * t], vo = a.tile_voff[t];
    for (uint32_t pos = threadIdx.x; pos < nt; pos += 256) {
        const uint32_t j = rank_of_inst(a.keys, a.vals, (int64_t)s + pos, a.rank_bits, a.packed);
        const int64_t vi = (int64_t)vo + pos;
        a.vkey[vi] = j;
        a.vgid[vi] = a.order[j];
        for (int k = 0; k < a.rw; ++k) a.vrec[a.rw * vi + k] = a.rrec[a.rw * (int64_t)j + k];
    }
}

// vseg[2j], vseg[2j+1] = [first, end) of rank j in the rank-sorted visits.
__global__ __launch_bounds__(256) void k_vseg(const uint32_t* __restrict__ skeys, const Counters* counters,
                                              int64_t cap, uint32_t* __restrict__ vseg) {
    if (counters->inst_overflow || counters->visit_overflow) return;
    const int64_t m = (int64_t)counters->n_visited;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m || k >= cap) return;
    const uint32_t j = skeys[k];
    if (k == 0 || skeys[k - 1] != j) vseg[2 * (int64_t)j] = (uint32_t)k;
    if (k == m - 1 || skeys[k + 1] != j) vseg[2 * (int64_t)j + 1] = (uint32_t)(k + 1);
}

// Queue slots for a wave: lanes with `take` get consecutive slots of *counter
// (in lane order) from one atomic per wave.  All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_slot(unsigned int* counter, bool take) {
    const uint64_t m = ballot64(take);
    if (m == 0) return 0u;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0u;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned int)__builtin_popcountll(m));
    base = (uint32_t)__shfl((int)base, leader, 64);
    return base + (uint32_t)__builtin_popcountll(m & lanemask_lt());
}

// The same for n slots per lane (n = 0 takes none): the lane's first slot.
__device__ __forceinline__ uint32_t wave_slots(unsigned int* counter, uint32_t n) {
    const int lane = lane_id();
    uint32_t incl = n;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, off, 64);
        if (lane >= off) incl += y;
    }
    const uint32_t tot = (uint32_t)__shfl((int)incl, 63, 64);
    if (tot == 0) return 0u;
    uint32_t base = 0u;
    if (lane == 63) base = atomicAdd(counter, tot);
    base = (uint32_t)__shfl((int)base, 63, 64);
    return base + incl - n;
}

// Partial rows of GP floats (Gaussians 12, 10 used; surfels 16, 14 used).
template <int GP>
__device__ __forceinline__ void add_geom(float* acc, const float* part_geom, uint32_t idx) {
    constexpr int NV = GP - 2;
    const float4* pg = reinterpret_cast<const float4*>(part_geom + (int64_t)idx * GP);
    float4 q[GP / 4];
#pragma unroll
    for (int k = 0; k < GP / 4; ++k) q[k] = pg[k];
    const float* f = reinterpret_cast<const float*>(q);
#pragma unroll
    for (int m = 0; m < NV; ++m) acc[m] += f[m];
}

// acc += the partials of visits k0, k0 + st, k0 + 2 st, ... below k1 (of the
// rank-sorted list), added in that order; their indices and rows are loaded
// four at a time, so that the loads do not wait for one another.
template <int GP>
__device__ __forceinline__ void add_geom_run(float* acc, const ReduceArgs& a, uint32_t k0, uint32_t k1, uint32_t st) {
    constexpr int NV = GP - 2;
    uint32_t k = k0;
    for (; k + 3 * st < k1; k += 4 * st) {
        uint32_t idx[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) idx[i] = a.vsorted[k + (uint32_t)i * st];
        float4 r[4][GP / 4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4* pg = reinterpret_cast<const float4*>(a.part_geom + (int64_t)idx[i] * GP);
#pragma unroll
            for (int c = 0; c < GP / 4; ++c) r[i][c] = pg[c];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float* f = reinterpret_cast<const float*>(r[i]);
#pragma unroll
            for (int m = 0; m < NV; ++m) acc[m] += f[m];
        }
    }
    for (; k < k1; k += st) add_geom<GP>(acc, a.part_geom, a.vsorted[k]);
}

template <int GP>
__device__ __forceinline__ void store_geom(float* grad2d, int64_t row, const float* acc) {
    constexpr int NV = GP - 2;
    float4* o = reinterpret_cast<float4*>(grad2d + row * GP);
#pragma unroll
    for (int c = 0; c < GP / 4; ++c) {
        const int m = 4 * c;
        o[c] = make_float4(m < NV ? acc[m] : 0.0f, m + 1 < NV ? acc[m + 1] : 0.0f, m + 2 < NV ? acc[m + 2] : 0.0f,
                           m + 3 < NV ? acc[m + 3] : 0.0f);
    }
}

// One thread per (view, rank): the screen-space adjoint of that (view, Gaussian).
template <int GP>
__global__ __launch_bounds__(256) void k_reduce_geom(ReduceArgs a) {
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;   // (uniform)
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = j < a.total;
    // every lane stays active for the wave-wide slot allocation
    const uint32_t b0 = valid ? a.vseg[2 * j] : 0u, b1 = valid ? a.vseg[2 * j + 1] : 0u;
    const bool is_long = b1 - b0 > LONG_GEOM;
    const uint32_t slot = wave_slot(&a.counters->n_long_geom, is_long);
    if (!valid) return;
    if (is_long) {
        a.long_list[slot] = (uint32_t)j;
        return;
    }
    const int64_t v = j / a.n;
    const uint32_t g = a.order[j];
    float acc[GP];
#pragma unroll
    for (int m = 0; m < GP; ++m) acc[m] = 0.0f;
    add_geom_run<GP>(acc, a, b0, b1, 1u);
    store_geom<GP>(a.grad2d, v * a.n + g, acc);
}

// One workgroup per long rank (grid-stride over the queue): thread t sums
// entries t, t + 256, ... of the segment, then a fixed-order tree.
template <int GP>
__global__ __launch_bounds__(256) void k_reduce_geom_long(ReduceArgs a) {
    constexpr int NV = GP - 2;
    __shared__ float red[256][NV + 1];
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const uint32_t nlong = a.counters->n_long_geom;
    for (uint32_t li = blockIdx.x; li < nlong; li += gridDim.x) {
        const int64_t j = a.long_list[li];
        const uint32_t b0 = a.vseg[2 * j], b1 = a.vseg[2 * j + 1];
        float acc[GP];
#pragma unroll
        for (int m = 0; m < GP; ++m) acc[m] = 0.0f;
        add_geom_run<GP>(acc, a, b0 + threadIdx.x, b1, 256u);
#pragma unroll
        for (int m = 0; m < NV; ++m) red[threadIdx.x][m] = acc[m];
        __syncthreads();
        for (int st = 128; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st)
#pragma unroll
                for (int m = 0; m < NV; ++m) red[threadIdx.x][m] += red[threadIdx.x + st][m];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int m = 0; m < NV; ++m) acc[m] = red[0][m];
            store_geom<GP>(a.grad2d, (j / a.n) * a.n + a.order[j], acc);
        }
        __syncthreads();
    }
}

// Visits k0 .. k1-1 of the rank-sorted list, in order, Neumaier-added into
// the lane's channels c = lane + 64 m (m < NC) and the weight pair.  Loads are
// issued B visits at a time (visit indices first, then their rows), and the
// additions then run in visit order, so batching changes no result.
template <int NC, int B>
__device__ __forceinline__ void accumulate_span(const ReduceArgs& a, int lane, uint32_t k0, uint32_t k1, float* sm,
                                                float* cp, float& ws, float& wc) {
    const int D = a.d;
    for (uint32_t kb = k0; kb < k1; kb += B) {
        // visit indices of the batch: lane l < B loads the l-th
        int64_t my = -1;
        float myw = 0.0f;
        if (lane < B) {
            const uint32_t k = kb + (uint32_t)lane;
            if (k < k1) {
                my = a.vsorted[k];
                myw = a.part_geom[my * (a.wslot == 9 ? 12 : 16) + a.wslot];
            }
        }
        float rows[B][NC];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t idx = __shfl(my, b, 64);
#pragma unroll
            for (int m = 0; m < NC; ++m) {
                const int c = lane + 64 * m;
                rows[b][m] = (idx >= 0 && c < D) ? a.part_fuse[idx * D + c] : 0.0f;
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t idx = __shfl(my, b, 64);
            const float wb = __shfl(myw, b, 64);
            if (idx >= 0) {
#pragma unroll
                for (int m = 0; m < NC; ++m) neumaier_add(sm[m], cp[m], rows[b][m]);
                neumaier_add(ws, wc, wb);
            }
        }
    }
}

// Positions p0 .. p1-1 of the concatenation of a Gaussian's per-view visit
// segments (views ascending, tiles row-major within a view).
template <int NC, int B>
__device__ __forceinline__ void accumulate_positions(const ReduceArgs& a, int64_t g, int lane, uint32_t p0,
                                                     uint32_t p1, float* sm, float* cp, float& ws, float& wc) {
    uint32_t off = 0;   // visits of earlier views
    for (int v = 0; v < a.n_views && off < p1; ++v) {
        const int64_t j = (int64_t)v * a.n + a.rank_of[(int64_t)v * a.n + g];
        const uint32_t b0 = a.vseg[2 * j], b1 = a.vseg[2 * j + 1];
        const uint32_t len = b1 - b0;
        const uint32_t lo = p0 > off ? p0 : off, hi = p1 < off + len ? p1 : off + len;
        if (lo < hi) accumulate_span<NC, B>(a, lane, b0 + (lo - off), b0 + (hi - off), sm, cp, ws, wc);
        off += len;
    }
}

__device__ __forceinline__ uint32_t fuse_visit_total(const ReduceArgs& a, int64_t g) {
    uint32_t total = 0;
    for (int v = 0; v < a.n_views; ++v) {
        const int64_t j = (int64_t)v * a.n + a.rank_of[(int64_t)v * a.n + g];
        total += a.vseg[2 * j + 1] - a.vseg[2 * j];
    }
    return total;
}

// One thread per Gaussian: its visit count over all views decides the
// reduction.  Up to LONG_FUSE visits it is queued for one wavefront; beyond,
// it is queued with its run of units of FUSE_UNIT consecutive visits.  (Queue
// order does not matter: each Gaussian's sums depend on its own visits only.)
__global__ __launch_bounds__(256) void k_fuse_classify(ReduceArgs a) {
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;   // (uniform)
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // every lane stays active for the wave-wide slot allocation
    const uint32_t total = g < a.n ? fuse_visit_total(a, g) : 0u;
    const bool is_short = total > 0 && total <= LONG_FUSE, is_long = total > LONG_FUSE;
    const uint32_t nu = is_long ? (total + FUSE_UNIT - 1) / FUSE_UNIT : 0u;
    const uint32_t sslot = wave_slot(&a.counters->n_short_fuse, is_short);
    const uint32_t slot = wave_slot(&a.counters->n_long_fuse, is_long);
    const uint32_t ub = wave_slots(&a.counters->n_fuse_units, nu);
    if (is_short) a.long_list[a.total + 2 * a.n + sslot] = (uint32_t)g;
    if (!is_long) return;
    a.long_list[a.total + slot] = (uint32_t)g;
    a.long_list[a.total + a.n + slot] = ub;
    // (cannot happen: the units never exceed the capacity that the visit
    // capacity implies; flagged as a visit overflow if they did)
    if ((int64_t)ub + nu > a.unit_cap) {
        a.counters->visit_overflow = 1u;
        return;
    }
    for (uint32_t i = 0; i < nu; ++i) a.unit_owner[ub + i] = slot;
}

// One wavefront per queued short Gaussian: Neumaier-add its partials of every
// view, views ascending and tiles row-major, into the persistent accumulators.
template <int NC, int B>
__global__ __launch_bounds__(256) void k_reduce_fuse_short(ReduceArgs a) {
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int lane = threadIdx.x & 63;
    const int D = a.d;
    const uint32_t ns = a.counters->n_short_fuse;
    for (uint32_t si = blockIdx.x * 4 + (threadIdx.x >> 6); si < ns; si += gridDim.x * 4) {
        const int64_t g = a.long_list[a.total + 2 * a.n + si];
        const uint32_t total = fuse_visit_total(a, g);
        float sm[NC], cp[NC];
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int c = lane + 64 * m;
            sm[m] = c < D ? a.acc_sum[g * D + c] : 0.0f;
            cp[m] = c < D ? a.acc_comp[g * D + c] : 0.0f;
        }
        float ws = a.acc_wsum[g], wc = a.acc_wcomp[g];
        accumulate_positions<NC, B>(a, g, lane, 0u, total, sm, cp, ws, wc);
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int c = lane + 64 * m;
            if (c < D) {
                a.acc_sum[g * D + c] = sm[m];
                a.acc_comp[g * D + c] = cp[m];
            }
        }
        if (lane == 0) {
            a.acc_wsum[g] = ws;
            a.acc_wcomp[g] = wc;
        }
    }
}

// One wavefront per unit: the compensated sums (from zero) of the unit's
// FUSE_UNIT visits, written to the unit's partial row.
template <int NC, int B>
__global__ __launch_bounds__(256) void k_reduce_fuse_units(ReduceArgs a) {
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int lane = threadIdx.x & 63;
    const int D = a.d;
    const uint32_t nlong = a.counters->n_long_fuse;
    const uint32_t nu = (int64_t)a.counters->n_fuse_units < a.unit_cap ? a.counters->n_fuse_units : (uint32_t)a.unit_cap;
    for (uint32_t u = blockIdx.x * 4 + (threadIdx.x >> 6); u < nu; u += gridDim.x * 4) {
        const uint32_t slot = a.unit_owner[u];
        if (slot >= nlong) continue;
        const int64_t g = a.long_list[a.total + slot];
        const uint32_t i = u - a.long_list[a.total + a.n + slot];
        float sm[NC], cp[NC];
#pragma unroll
        for (int m = 0; m < NC; ++m) sm[m] = cp[m] = 0.0f;
        float ws = 0.0f, wc = 0.0f;
        accumulate_positions<NC, B>(a, g, lane, i * FUSE_UNIT, (i + 1) * FUSE_UNIT, sm, cp, ws, wc);
        float* row = a.upart + (int64_t)u * (2 * D + 2);
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int c = lane + 64 * m;
            if (c < D) {
                row[c] = sm[m];
                row[D + c] = cp[m];
            }
        }
        if (lane == 0) {
            row[2 * D] = ws;
            row[2 * D + 1] = wc;
        }
    }
}

// One wavefront per long Gaussian: its units' sums and compensations are
// Neumaier-added into the accumulators, units in order.
template <int NC, int UB>
__global__ __launch_bounds__(256) void k_reduce_fuse_combine(ReduceArgs a) {
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int lane = threadIdx.x & 63;
    const int D = a.d;
    const uint32_t nlong = a.counters->n_long_fuse;
    for (uint32_t li = blockIdx.x * 4 + (threadIdx.x >> 6); li < nlong; li += gridDim.x * 4) {
        const int64_t g = a.long_list[a.total + li];
        const uint32_t ub = a.long_list[a.total + a.n + li];
        const uint32_t nu = (fuse_visit_total(a, g) + FUSE_UNIT - 1) / FUSE_UNIT;
        if ((int64_t)ub + nu > a.unit_cap) continue;
        float sm[NC], cp[NC];
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int c = lane + 64 * m;
            sm[m] = c < D ? a.acc_sum[g * D + c] : 0.0f;
            cp[m] = c < D ? a.acc_comp[g * D + c] : 0.0f;
        }
        float ws = a.acc_wsum[g], wc = a.acc_wcomp[g];
        // units are read UB at a time (all loads issued, then the additions in unit order)
        for (uint32_t i0 = 0; i0 < nu; i0 += UB) {
            float us[UB][NC], uc[UB][NC], uw[UB][2];
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                const bool have = i0 + b < nu;
                const float* row = a.upart + (int64_t)(ub + i0 + (have ? b : 0)) * (2 * D + 2);
#pragma unroll
                for (int m = 0; m < NC; ++m) {
                    const int c = lane + 64 * m;
                    us[b][m] = c < D ? row[c] : 0.0f;
                    uc[b][m] = c < D ? row[D + c] : 0.0f;
                }
                uw[b][0] = row[2 * D];
                uw[b][1] = row[2 * D + 1];
            }
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                if (i0 + b < nu) {
#pragma unroll
                    for (int m = 0; m < NC; ++m) {
                        if (lane + 64 * m < D) {
                            neumaier_add(sm[m], cp[m], us[b][m]);
                            neumaier_add(sm[m], cp[m], uc[b][m]);
                        }
                    }
                    neumaier_add(ws, wc, uw[b][0]);
                    neumaier_add(ws, wc, uw[b][1]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int c = lane + 64 * m;
            if (c < D) {
                a.acc_sum[g * D + c] = sm[m];
                a.acc_comp[g * D + c] = cp[m];
            }
        }
        if (lane == 0) {
            a.acc_wsum[g] = ws;
            a.acc_wcomp[g] = wc;
        }
    }
}

// Upper bound of the units: a long Gaussian has more than LONG_FUSE visits, so
// sum ceil(len / FUSE_UNIT) <= V / FUSE_UNIT + V / (LONG_FUSE + 1) <= 3 V / 64.
int64_t fuse_unit_capacity(int64_t visit_capacity) {
    static_assert(FUSE_UNIT == 64 && LONG_FUSE == 32, "capacity bound below assumes these");
    return visit_capacity * 3 / 64 + 1;
}

void launch_visit_stage(const VisitStageArgs& a, int n_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_visit_stage, dim3(n_tiles), dim3(256), 0, s, a);
}

void launch_vseg(const uint32_t* skeys, const Counters* c, int64_t cap, uint32_t* vseg, hipStream_t s) {
    if (cap > 0) hipLaunchKernelGGL(k_vseg, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, skeys, c, cap, vseg);
}

void launch_reduce_geom(const ReduceArgs& a, int gp, hipStream_t s) {
    // (long ranks are few: at 500k Gaussians at 1080p about 1,900, one per workgroup)
    if (gp == 16) {
        hipLaunchKernelGGL(k_reduce_geom<16>, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_reduce_geom_long<16>, dim3(4096), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_reduce_geom<12>, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_reduce_geom_long<12>, dim3(4096), dim3(256), 0, s, a);
    }
}

template <int NC, int B>
static void launch_reduce_fuse_nc(const ReduceArgs& a, hipStream_t s) {
    if (a.n == 0) return;
    hipLaunchKernelGGL(k_fuse_classify, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_reduce_fuse_short<NC, B>), dim3(2048), dim3(256), 0, s, a);
    // one wavefront per unit where the capacity allows (the unit count is only
    // known on the device; waves past it exit at once), so that the hardware
    // balances the units instead of a fixed stride over a smaller grid
    const int64_t ub = (a.unit_cap + 3) / 4;
    const unsigned ugrid = (unsigned)(ub < 2048 ? 2048 : (ub > 32768 ? 32768 : ub));
    hipLaunchKernelGGL((k_reduce_fuse_units<NC, B>), dim3(ugrid), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_reduce_fuse_combine<NC, B>), dim3(512), dim3(256), 0, s, a);
}

// channels per lane NC = ceil(d / 64); visits per batch B keep B * NC <= 32 registers of rows
void launch_reduce_fuse(const ReduceArgs& a, hipStream_t s) {
    const int nc = (a.d + 63) / 64;
    if (nc <= 1) launch_reduce_fuse_nc<1, 8>(a, s);
    else if (nc <= 2) launch_reduce_fuse_nc<2, 8>(a, s);
    else if (nc <= 4) launch_reduce_fuse_nc<4, 8>(a, s);
    else if (nc <= 8) launch_reduce_fuse_nc<8, 4>(a, s);
    else launch_reduce_fuse_nc<16, 2>(a, s);
}

}  // namespace fh
