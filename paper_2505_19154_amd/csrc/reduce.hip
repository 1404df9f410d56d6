// Deterministic per-Gaussian reductions of the backward pass's per-instance
// partials (no atomics on values).
//
// After the forward pass every tile knows how far its pixels walked; the
// visited instances of all tiles get consecutive visit indices (tile-major).
// Sorting the visits stably by rank gives every (view, Gaussian) a contiguous
// segment of visit indices in row-major tile order.  Short segments are summed
// by one thread (geometry) or one wavefront (fusion, lanes over channels);
// Gaussians visited in many tiles (large splats near the camera) are queued and
// summed by a whole workgroup with a fixed-order tree, so that one long
// segment does not serialise the launch.  Every sum has a fixed order, so the
// results are bitwise reproducible.
#include "kernels.hpp"

namespace fh {

constexpr uint32_t LONG_GEOM = 64;    // visits above which a rank goes to the workgroup reduction
constexpr uint32_t LONG_FUSE = 32;    // same for fusion (per Gaussian, all views)

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
        a.vrec[3 * vi] = a.rrec[3 * (int64_t)j];
        a.vrec[3 * vi + 1] = a.rrec[3 * (int64_t)j + 1];
        a.vrec[3 * vi + 2] = a.rrec[3 * (int64_t)j + 2];
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

__device__ __forceinline__ void add_geom(float* acc, const float* part_geom, uint32_t idx) {
    const float4* pg = reinterpret_cast<const float4*>(part_geom + (int64_t)idx * 12);
    const float4 q0 = pg[0], q1 = pg[1], q2 = pg[2];
    acc[0] += q0.x; acc[1] += q0.y; acc[2] += q0.z; acc[3] += q0.w;
    acc[4] += q1.x; acc[5] += q1.y; acc[6] += q1.z; acc[7] += q1.w;
    acc[8] += q2.x; acc[9] += q2.y;
}

__device__ __forceinline__ void store_geom(float* grad2d, int64_t row, const float* acc) {
    float4* o = reinterpret_cast<float4*>(grad2d + row * 12);
    o[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    o[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    o[2] = make_float4(acc[8], acc[9], 0.0f, 0.0f);
}

// One thread per (view, rank): the screen-space adjoint of that (view, Gaussian).
__global__ __launch_bounds__(256) void k_reduce_geom(ReduceArgs a) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.total) return;
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int64_t v = j / a.n;
    const uint32_t g = a.order[j];
    const uint32_t b0 = a.vseg[2 * j], b1 = a.vseg[2 * j + 1];
    if (b1 - b0 > LONG_GEOM) {
        const uint32_t slot = atomicAdd(&a.counters->n_long_geom, 1u);
        a.long_list[slot] = (uint32_t)j;
        return;
    }
    float acc[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) acc[m] = 0.0f;
    for (uint32_t k = b0; k < b1; ++k) add_geom(acc, a.part_geom, a.vsorted[k]);
    store_geom(a.grad2d, v * a.n + g, acc);
}

// One workgroup per long rank (grid-stride over the queue): thread t sums
// entries t, t + 256, ... of the segment, then a fixed-order tree.
__global__ __launch_bounds__(256) void k_reduce_geom_long(ReduceArgs a) {
    __shared__ float red[256][11];
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const uint32_t nlong = a.counters->n_long_geom;
    for (uint32_t li = blockIdx.x; li < nlong; li += gridDim.x) {
        const int64_t j = a.long_list[li];
        const uint32_t b0 = a.vseg[2 * j], b1 = a.vseg[2 * j + 1];
        float acc[12];
#pragma unroll
        for (int m = 0; m < 12; ++m) acc[m] = 0.0f;
        for (uint32_t k = b0 + threadIdx.x; k < b1; k += 256) add_geom(acc, a.part_geom, a.vsorted[k]);
#pragma unroll
        for (int m = 0; m < 10; ++m) red[threadIdx.x][m] = acc[m];
        __syncthreads();
        for (int st = 128; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st)
#pragma unroll
                for (int m = 0; m < 10; ++m) red[threadIdx.x][m] += red[threadIdx.x + st][m];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int m = 0; m < 10; ++m) acc[m] = red[0][m];
            store_geom(a.grad2d, (j / a.n) * a.n + a.order[j], acc);
        }
        __syncthreads();
    }
}

// The visits of one wavefront, in its fixed order, Neumaier-added into the
// lane's channels c = lane + 64 m (m < NC) and the weight pair.  `stride` and
// `phase` select the wavefront's share: positions phase, phase + stride, ... of
// the concatenation of the per-view segments (views ascending).  Loads are
// issued B visits at a time (visit indices first, then their rows), and the
// additions then run in visit order, so batching changes no result.
template <int NC, int B>
__device__ __forceinline__ void accumulate_visits(const ReduceArgs& a, int64_t g, int lane, uint32_t stride,
                                                  uint32_t phase, float* sm, float* cp, float& ws, float& wc) {
    const int D = a.d;
    uint32_t off = 0;   // visits of earlier views
    for (int v = 0; v < a.n_views; ++v) {
        const int64_t j = (int64_t)v * a.n + a.rank_of[(int64_t)v * a.n + g];
        const uint32_t b0 = a.vseg[2 * j], b1 = a.vseg[2 * j + 1];
        // first k in [b0, b1) whose position in the concatenation is phase mod stride
        const uint32_t first = b0 + (phase + stride - off % stride) % stride;
        for (uint32_t k0 = first; k0 < b1; k0 += stride * B) {
            // visit indices of the batch: lane l < B loads the l-th
            int64_t my = -1;
            float myw = 0.0f;
            if (lane < B) {
                const uint32_t k = k0 + stride * (uint32_t)lane;
                if (k < b1) {
                    my = a.vsorted[k];
                    myw = a.part_geom[my * 12 + 9];
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
        off += b1 - b0;
    }
}

// One wavefront per Gaussian: Neumaier-add its partials of every view, views
// ascending and tiles row-major, into the persistent accumulators.
template <int NC, int B>
__global__ __launch_bounds__(256) void k_reduce_fuse(ReduceArgs a) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= a.n) return;
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    uint32_t total = 0;
    for (int v = 0; v < a.n_views; ++v) {
        const int64_t j = (int64_t)v * a.n + a.rank_of[(int64_t)v * a.n + g];
        total += a.vseg[2 * j + 1] - a.vseg[2 * j];
    }
    if (total == 0) return;
    if (total > LONG_FUSE) {
        if (lane == 0) {
            const uint32_t slot = atomicAdd(&a.counters->n_long_fuse, 1u);
            a.long_list[a.total + slot] = (uint32_t)g;
        }
        return;
    }
    const int D = a.d;
    float sm[NC], cp[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        const int c = lane + 64 * m;
        sm[m] = c < D ? a.acc_sum[g * D + c] : 0.0f;
        cp[m] = c < D ? a.acc_comp[g * D + c] : 0.0f;
    }
    float ws = a.acc_wsum[g], wc = a.acc_wcomp[g];
    accumulate_visits<NC, B>(a, g, lane, 1u, 0u, sm, cp, ws, wc);
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

// One 1024-thread workgroup per long Gaussian: wave w takes every 16th visit
// of the concatenated per-view segments, keeping its own compensated sums;
// the 16 waves are then added into the accumulators in wave order.
template <int NC, int B>
__global__ __launch_bounds__(1024) void k_reduce_fuse_long(ReduceArgs a) {
    extern __shared__ float sred[];   // [16][2][d] then [16][2] for the weights
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int D = a.d;
    const uint32_t nlong = a.counters->n_long_fuse;
    float* sw = sred + 16 * 2 * D;
    for (uint32_t li = blockIdx.x; li < nlong; li += gridDim.x) {
        const int64_t g = a.long_list[a.total + li];
        float sm[NC], cp[NC];
#pragma unroll
        for (int m = 0; m < NC; ++m) sm[m] = cp[m] = 0.0f;
        float ws = 0.0f, wc = 0.0f;
        accumulate_visits<NC, B>(a, g, lane, 16u, (uint32_t)w, sm, cp, ws, wc);
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int c = lane + 64 * m;
            if (c < D) {
                sred[(w * 2) * D + c] = sm[m];
                sred[(w * 2 + 1) * D + c] = cp[m];
            }
        }
        if (lane == 0) {
            sw[2 * w] = ws;
            sw[2 * w + 1] = wc;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < D; c += 1024) {
            float s = a.acc_sum[g * D + c], cc = a.acc_comp[g * D + c];
            for (int k = 0; k < 16; ++k) {
                neumaier_add(s, cc, sred[(k * 2) * D + c]);
                neumaier_add(s, cc, sred[(k * 2 + 1) * D + c]);
            }
            a.acc_sum[g * D + c] = s;
            a.acc_comp[g * D + c] = cc;
        }
        if (threadIdx.x == 0) {
            float s = a.acc_wsum[g], cc = a.acc_wcomp[g];
            for (int k = 0; k < 16; ++k) {
                neumaier_add(s, cc, sw[2 * k]);
                neumaier_add(s, cc, sw[2 * k + 1]);
            }
            a.acc_wsum[g] = s;
            a.acc_wcomp[g] = cc;
        }
        __syncthreads();
    }
}

void launch_visit_stage(const VisitStageArgs& a, int n_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_visit_stage, dim3(n_tiles), dim3(256), 0, s, a);
}

void launch_vseg(const uint32_t* skeys, const Counters* c, int64_t cap, uint32_t* vseg, hipStream_t s) {
    if (cap > 0) hipLaunchKernelGGL(k_vseg, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, skeys, c, cap, vseg);
}

void launch_reduce_geom(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_geom, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_reduce_geom_long, dim3(512), dim3(256), 0, s, a);
}

template <int NC, int B>
static void launch_reduce_fuse_nc(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_reduce_fuse<NC, B>), dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, s, a);
    const size_t lds = sizeof(float) * (16 * 2 * (size_t)a.d + 32);
    hipLaunchKernelGGL((k_reduce_fuse_long<NC, B>), dim3(512), dim3(1024), lds, s, a);
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
