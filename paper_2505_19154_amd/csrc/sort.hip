// Tile binning: depth sort, instance generation, radix sort by tile, ranges.
//
// The paper's method (Appendix A, "Details of the Rasterizer"; Algorithm 2)
// duplicates every Gaussian once per overlapped tile, keys each copy with
// (tile << 32 | depth bits) and radix-sorts the keys.  This implementation
// reaches the same order with less traffic: the visible Gaussians of each view
// are first sorted by (depth, index) -- N keys instead of M instances -- and
// the instances are then generated in that order, so that a stable sort on
// the tile bits alone yields (tile, depth, index) order.  The instance key is
// (tile << rank_bits | rank), one u32 when it fits, else a u32 tile key with
// a u32 rank payload.
//
// Radix sort: LSD, 8-bit digits, reduce-then-scan (upsweep digit histograms,
// device-wide scan, downsweep scatter).  Each 256-thread block owns 4096 keys;
// the four wavefronts rank their keys with ballot-based digit matching, which
// is stable (positions are visited in order) and needs no LDS atomics.
#include "kernels.hpp"

namespace fh {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;   // 4096
constexpr int RADIX_BLOCK = 256;
constexpr int RADIX_ITEMS = 16;
constexpr int RADIX_TILE = RADIX_BLOCK * RADIX_ITEMS; // 4096
constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one u32 per thread (256 threads = 4 waves).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* total, uint32_t* sh_wave) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, WAVE);
        if (lane >= off) incl += y;
    }
    if (lane == WAVE - 1) sh_wave[w] = incl;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int k = 0; k < SCAN_BLOCK / WAVE; ++k) {
        const uint32_t s = sh_wave[k];
        if (k < w) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + incl - x;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t sh_wave[SCAN_BLOCK / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    uint32_t tot;
    block_exclusive_scan(s, &tot, sh_wave);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// out[i] = offsets[block] + exclusive prefix within the block; optionally
// out[n] = total (when total_out is set, written by the last block).
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down(const uint32_t* __restrict__ in, int64_t n,
                                                          const uint32_t* __restrict__ block_offsets,
                                                          uint32_t* __restrict__ out, int write_total) {
    __shared__ uint32_t sh_wave[SCAN_BLOCK / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot, sh_wave) + (block_offsets ? block_offsets[blockIdx.x] : 0u);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) out[n] = run;
}

// Scratch (in u32) needed by device_exclusive_scan for n items.
size_t scan_scratch_u32(int64_t n) {
    size_t tot = 0;
    int64_t m = n;
    while (m > SCAN_TILE) {
        m = (m + SCAN_TILE - 1) / SCAN_TILE;
        tot += (size_t)m + 64;
        tot += (size_t)m + 64;  // offsets of that level
    }
    return tot + 64;
}

// Exclusive scan of n u32 into out (out[n] = total if write_total).
void device_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch, int write_total,
                           hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(SCAN_BLOCK), 0, s, in, n, (const uint32_t*)nullptr, out,
                           write_total);
        return;
    }
    uint32_t* sums = scratch;
    uint32_t* offs = scratch + nb + 64;
    uint32_t* next = offs + nb + 64;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    device_exclusive_scan(sums, offs, nb, next, 0, s);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, (const uint32_t*)offs, out,
                       write_total);
}

// ---------------------------------------------------------------------------
// Radix sort pass over equal-length segments laid out back to back.
// The valid length of every segment is seg_len, or min(*dev_len, cap) for a
// single segment whose length is only known on the device.
struct RadixPass {
    const uint32_t* keys_in;
    const uint32_t* vals_in;   // nullptr: payload = position within the segment
    uint32_t* keys_out;
    uint32_t* vals_out;        // nullptr: keys only
    uint32_t* hist;            // [(seg * radix + digit) * blocks_per_seg + block]
    const unsigned long long* dev_len;
    int64_t seg_len;
    int64_t cap;
    int blocks_per_seg;
    int shift, bits;
};

__device__ __forceinline__ int64_t seg_valid_len(const RadixPass& p) {
    if (p.dev_len) {
        const unsigned long long m = *p.dev_len;
        return (int64_t)(m < (unsigned long long)p.cap ? m : (unsigned long long)p.cap);
    }
    return p.seg_len;
}

// Lanes of this wave whose digit equals mine (among lanes with valid = true).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int bits) {
    uint64_t m = ballot64(valid);
    for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = ballot64(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(RADIX_BLOCK) void k_radix_upsweep(RadixPass p) {
    __shared__ uint32_t cnt[RADIX_BLOCK / WAVE][256];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int seg = blockIdx.x / p.blocks_per_seg, blk = blockIdx.x % p.blocks_per_seg;
    const int radix = 1 << p.bits;
    const uint32_t mask = (uint32_t)radix - 1u;
    for (int t = threadIdx.x; t < (RADIX_BLOCK / WAVE) * 256; t += RADIX_BLOCK) (&cnt[0][0])[t] = 0u;
    __syncthreads();
    const int64_t len = seg_valid_len(p);
    const int64_t seg_base = (int64_t)seg * p.seg_len;
    const int64_t wbase = (int64_t)blk * RADIX_TILE + (int64_t)w * (RADIX_ITEMS * WAVE);
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        const int64_t pos = wbase + (int64_t)i * WAVE + lane;
        const bool valid = pos < len;
        if (!__any(valid)) break;
        const uint32_t d = valid ? ((p.keys_in[seg_base + pos] >> p.shift) & mask) : 0u;
        const uint64_t m = match_digit(d, valid, p.bits);
        if (valid && lane == (int)__builtin_ctzll(m)) cnt[w][d] += (uint32_t)__builtin_popcountll(m);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < radix; t += RADIX_BLOCK) {
        uint32_t s = 0;
        for (int k = 0; k < RADIX_BLOCK / WAVE; ++k) s += cnt[k][t];
        p.hist[((int64_t)seg * radix + t) * p.blocks_per_seg + blk] = s;
    }
}

__global__ __launch_bounds__(RADIX_BLOCK) void k_radix_downsweep(RadixPass p) {
    __shared__ uint32_t cnt[RADIX_BLOCK / WAVE][256];
    __shared__ uint32_t gbase[256];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int seg = blockIdx.x / p.blocks_per_seg, blk = blockIdx.x % p.blocks_per_seg;
    const int radix = 1 << p.bits;
    const uint32_t mask = (uint32_t)radix - 1u;
    const int64_t len = seg_valid_len(p);
    if ((int64_t)blk * RADIX_TILE >= len) return;   // whole block past the end: nothing to move
    for (int t = threadIdx.x; t < (RADIX_BLOCK / WAVE) * 256; t += RADIX_BLOCK) (&cnt[0][0])[t] = 0u;
    for (int t = threadIdx.x; t < radix; t += RADIX_BLOCK)
        gbase[t] = p.hist[((int64_t)seg * radix + t) * p.blocks_per_seg + blk];
    __syncthreads();
    const int64_t seg_base = (int64_t)seg * p.seg_len;
    const int64_t wbase = (int64_t)blk * RADIX_TILE + (int64_t)w * (RADIX_ITEMS * WAVE);
    uint32_t key[RADIX_ITEMS], val[RADIX_ITEMS], rank[RADIX_ITEMS];
#pragma unroll
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        const int64_t pos = wbase + (int64_t)i * WAVE + lane;
        const bool valid = pos < len;
        key[i] = valid ? p.keys_in[seg_base + pos] : 0u;
        if (p.vals_out) val[i] = valid ? (p.vals_in ? p.vals_in[seg_base + pos] : (uint32_t)pos) : 0u;
        const uint32_t d = (key[i] >> p.shift) & mask;
        const uint64_t m = match_digit(d, valid, p.bits);
        uint32_t before = 0;
        if (valid) before = cnt[w][d];
        rank[i] = before + (uint32_t)__builtin_popcountll(m & lanemask_lt());
        if (valid && lane == (int)__builtin_ctzll(m)) cnt[w][d] = before + (uint32_t)__builtin_popcountll(m);
    }
    __syncthreads();
    // per-digit exclusive prefix over the block's waves, folded into rank
    __shared__ uint32_t wpre[RADIX_BLOCK / WAVE][256];
    for (int t = threadIdx.x; t < radix; t += RADIX_BLOCK) {
        uint32_t run = gbase[t];
        for (int k = 0; k < RADIX_BLOCK / WAVE; ++k) {
            wpre[k][t] = run;
            run += cnt[k][t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RADIX_ITEMS; ++i) {
        const int64_t pos = wbase + (int64_t)i * WAVE + lane;
        if (pos < len) {
            const uint32_t d = (key[i] >> p.shift) & mask;
            // the scanned histogram already holds absolute positions (earlier
            // segments are counted in full before this one)
            const int64_t dst = (int64_t)wpre[w][d] + rank[i];
            p.keys_out[dst] = key[i];
            if (p.vals_out) p.vals_out[dst] = val[i];
        }
    }
}

// Sort `segs` segments of seg_len keys (or one segment of min(*dev_len, cap)
// keys) by bits [lo, hi).  Buffers alternate (a -> b -> a ...); returns the
// number of passes (the result is in b if odd, in a if even, except that the
// first pass reads from keys_src/vals_src).
int radix_sort(const uint32_t* keys_src, const uint32_t* vals_src, uint32_t* ka, uint32_t* va, uint32_t* kb,
               uint32_t* vb, bool with_vals, int64_t segs, int64_t seg_len, const unsigned long long* dev_len,
               int64_t cap, int lo, int hi, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s) {
    const int64_t span = dev_len ? cap : seg_len;
    const int bps = (int)((span + RADIX_TILE - 1) / RADIX_TILE);
    if (bps == 0 || segs == 0) return 0;
    int pass = 0;
    for (int shift = lo; shift < hi; shift += 8, ++pass) {
        const int bits = (hi - shift) < 8 ? (hi - shift) : 8;
        RadixPass p;
        const bool first = (pass == 0);
        const bool to_b = (pass % 2 == 0);
        p.keys_in = first ? keys_src : (to_b ? ka : kb);
        p.vals_in = with_vals ? (first ? vals_src : (to_b ? va : vb)) : nullptr;
        p.keys_out = to_b ? kb : ka;
        p.vals_out = with_vals ? (to_b ? vb : va) : nullptr;
        p.hist = hist;
        p.dev_len = dev_len;
        p.seg_len = seg_len;
        p.cap = cap;
        p.blocks_per_seg = bps;
        p.shift = shift;
        p.bits = bits;
        const unsigned nblk = (unsigned)(segs * bps);
        hipLaunchKernelGGL(k_radix_upsweep, dim3(nblk), dim3(RADIX_BLOCK), 0, s, p);
        const int64_t nh = segs * (int64_t)(1 << bits) * bps;
        device_exclusive_scan(hist, hist, nh, scan_tmp, 0, s);
        hipLaunchKernelGGL(k_radix_downsweep, dim3(nblk), dim3(RADIX_BLOCK), 0, s, p);
    }
    return pass;
}

size_t radix_hist_u32(int64_t segs, int64_t span) {
    const int64_t bps = (span + RADIX_TILE - 1) / RADIX_TILE;
    return (size_t)(segs * 256 * (bps > 0 ? bps : 1)) + 64;
}

// ---------------------------------------------------------------------------
// Tiles per rank: ntiles[j] for j = v*N + r, the r-th Gaussian of view v in
// depth order (0 when culled), and the u64 total.
__global__ __launch_bounds__(256) void k_tiles_by_rank(const uint32_t* __restrict__ order,
                                                       const int4* __restrict__ rect, int64_t n, int64_t total,
                                                       uint32_t* __restrict__ ntiles, Counters* counters) {
    __shared__ unsigned long long red[4];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t c = 0;
    if (j < total) {
        const int64_t v = j / n;
        const int4 r = rect[v * n + order[j]];
        if (r.x <= r.z && r.y <= r.w) c = (uint32_t)((r.z - r.x + 1) * (r.w - r.y + 1));
        ntiles[j] = c;
    }
    unsigned long long s = c;
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(&counters->n_instances, t);
    }
}

__global__ void k_check_capacity(Counters* counters, int64_t cap) {
    if (threadIdx.x == 0) counters->inst_overflow = counters->n_instances > (unsigned long long)cap ? 1u : 0u;
}

// Instance generation.  Each workgroup writes a fixed range of 2048 output
// instances (so that the few huge Gaussians at the front of the depth order
// spread over many workgroups); the ranks covering the range are found by a
// binary search of the tiles-per-rank scan staged in LDS.  Every binned rank
// owns at least one instance, so within one view a range spans at most 2048
// ranks and the LDS window always holds them; only a range that crosses a
// view boundary with culled (zero-instance) ranks can need more, and then
// searches the scan in global memory.
constexpr int DUP_TILE = 2048;
constexpr int DUP_WIN = 2048;

// largest r in [lo, hi] with off[r] <= i (off non-decreasing, off[lo] <= i)
__device__ __forceinline__ int64_t last_le(const uint32_t* off, int64_t lo, int64_t hi, uint32_t i) {
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_duplicate(DupArgs a) {
    __shared__ uint32_t offs[DUP_WIN + 1];
    __shared__ int4 rects[DUP_WIN];
    __shared__ long long s_r0;
    __shared__ int s_win;
    if (a.counters->inst_overflow) return;   // uniform over the block
    const int64_t m = (int64_t)a.counters->n_instances;
    const int64_t ib = (int64_t)blockIdx.x * DUP_TILE;
    if (ib >= m) return;                      // uniform over the block
    const int64_t ie = ib + DUP_TILE < m ? ib + DUP_TILE : m;
    if (threadIdx.x == 0) {
        const int64_t r0 = last_le(a.inst_off, 0, a.total_ranks - 1, (uint32_t)ib);
        const int64_t r1 = last_le(a.inst_off, r0, a.total_ranks - 1, (uint32_t)(ie - 1));
        s_r0 = r0;
        s_win = (r1 - r0 + 1 <= DUP_WIN) ? (int)(r1 - r0 + 1) : -1;
    }
    __syncthreads();
    const int64_t r0 = s_r0;
    const int win = s_win;
    if (win > 0) {
        for (int k = threadIdx.x; k <= win; k += 256) offs[k] = a.inst_off[r0 + k];
        for (int k = threadIdx.x; k < win; k += 256) {
            const int64_t j = r0 + k;
            rects[k] = a.rect[(j / a.n) * a.n + a.order[j]];
        }
    }
    __syncthreads();
    for (int64_t ii = ib + threadIdx.x; ii < ie; ii += 256) {
        const uint32_t i = (uint32_t)ii;
        int64_t j;
        int4 r;
        uint32_t local;
        if (win > 0) {
            int lo = 0, hi = win - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (offs[mid] <= i) lo = mid; else hi = mid - 1;
            }
            j = r0 + lo;
            r = rects[lo];
            local = i - offs[lo];
        } else {
            j = last_le(a.inst_off, r0, a.total_ranks - 1, i);
            r = a.rect[(j / a.n) * a.n + a.order[j]];
            local = i - a.inst_off[j];
        }
        const int v = (int)(j / a.n);
        const uint32_t wdt = (uint32_t)(r.z - r.x + 1);
        const uint32_t tx = (uint32_t)r.x + local % wdt;
        const uint32_t ty = (uint32_t)r.y + local / wdt;
        const uint32_t tile = (uint32_t)a.vt.tile_off[v] + ty * (uint32_t)a.vt.tiles_x[v] + tx;
        if (a.packed) {
            a.keys[i] = (tile << a.rank_bits) | (uint32_t)j;
        } else {
            a.keys[i] = tile;
            a.vals[i] = (uint32_t)j;
        }
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ uint32_t inst_tile(const uint32_t* keys, int64_t i, int rank_bits, int packed) {
    return packed ? (keys[i] >> rank_bits) : keys[i];
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, const Counters* counters,
                                                int64_t cap, int rank_bits, int packed, uint32_t* ranges) {
    if (counters->inst_overflow) return;
    const int64_t m = (int64_t)counters->n_instances;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m || i >= cap) return;
    const uint32_t t = inst_tile(keys, i, rank_bits, packed);
    if (i == 0 || inst_tile(keys, i - 1, rank_bits, packed) != t) ranges[2 * t] = (uint32_t)i;
    if (i == m - 1 || inst_tile(keys, i + 1, rank_bits, packed) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
}

// The paper's 64-bit keys of the sorted instances.
__global__ __launch_bounds__(256) void k_bin_keys(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                  const uint32_t* __restrict__ order,
                                                  const uint32_t* __restrict__ depth_key, int64_t n_inst, int64_t n,
                                                  int rank_bits, int packed, uint64_t* keys_out, uint32_t* gid_out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_inst) return;
    const uint32_t tile = packed ? (keys[i] >> rank_bits) : keys[i];
    const uint32_t j = packed ? (keys[i] & ((1u << rank_bits) - 1u)) : vals[i];
    const int64_t v = (int64_t)j / n;
    const uint32_t g = order[j];
    if (keys_out) keys_out[i] = ((uint64_t)tile << 32) | (uint64_t)depth_key[v * n + g];
    if (gid_out) gid_out[i] = g;
}

// ---------------------------------------------------------------------------
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

void launch_tiles_by_rank(const uint32_t* order, const int4* rect, int64_t n, int64_t total, uint32_t* ntiles,
                          Counters* c, hipStream_t s) {
    hipLaunchKernelGGL(k_tiles_by_rank, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, order, rect, n, total,
                       ntiles, c);
}

void launch_check_capacity(Counters* c, int64_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_check_capacity, dim3(1), dim3(64), 0, s, c, cap);
}

void launch_duplicate(const DupArgs& a, hipStream_t s) {
    if (a.cap <= 0 || a.total_ranks <= 0) return;
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)((a.cap + DUP_TILE - 1) / DUP_TILE)), dim3(256), 0, s, a);
}

void launch_ranges(const uint32_t* keys, const Counters* c, int64_t cap, int rank_bits, int packed, uint32_t* ranges,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, keys, c, cap, rank_bits, packed,
                       ranges);
}

void launch_bin_keys(const uint32_t* keys, const uint32_t* vals, const uint32_t* order, const uint32_t* depth_key,
                     int64_t n_inst, int64_t n, int rank_bits, int packed, uint64_t* ko, uint32_t* go,
                     hipStream_t s) {
    if (n_inst <= 0) return;
    hipLaunchKernelGGL(k_bin_keys, dim3((unsigned)((n_inst + 255) / 256)), dim3(256), 0, s, keys, vals, order, depth_key,
                       n_inst, n, rank_bits, packed, ko, go);
}

}  // namespace fh
