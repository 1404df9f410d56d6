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

// The same, with the block's offset formed in place: the sum of the block sums
// before it (integer sums, so the order of the additions does not matter).
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down_sums(const uint32_t* __restrict__ in, int64_t n,
                                                               const uint32_t* __restrict__ block_sums,
                                                               uint32_t* __restrict__ out, int write_total) {
    __shared__ uint32_t sh_wave[SCAN_BLOCK / WAVE];
    uint32_t part = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += SCAN_BLOCK) part += block_sums[k];
    uint32_t offset;
    block_exclusive_scan(part, &offset, sh_wave);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot, sh_wave) + offset;
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
    if (nb <= 16 * SCAN_BLOCK) {
        // few blocks: each adds up the sums before it (two launches instead of three)
        hipLaunchKernelGGL(k_scan_down_sums, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, (const uint32_t*)sums,
                           out, write_total);
        return;
    }
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
    int tiles_per_block;       // consecutive RADIX_TILE-key tiles one workgroup handles, in order
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

// Digit counts of a workgroup's tiles (LDS atomics; counts are exact whatever
// their order), one histogram entry per (segment, digit, workgroup).
__global__ __launch_bounds__(RADIX_BLOCK) void k_radix_upsweep(RadixPass p) {
    __shared__ uint32_t cnt[256];
    const int seg = blockIdx.x / p.blocks_per_seg, blk = blockIdx.x % p.blocks_per_seg;
    const int radix = 1 << p.bits;
    const uint32_t mask = (uint32_t)radix - 1u;
    for (int t = threadIdx.x; t < 256; t += RADIX_BLOCK) cnt[t] = 0u;
    __syncthreads();
    const int64_t len = seg_valid_len(p);
    const int64_t seg_base = (int64_t)seg * p.seg_len;
    const int64_t b0 = (int64_t)blk * p.tiles_per_block * RADIX_TILE;
    const int64_t b1 = b0 + (int64_t)p.tiles_per_block * RADIX_TILE < len ? b0 + (int64_t)p.tiles_per_block * RADIX_TILE
                                                                         : len;
    for (int64_t pos = b0 + threadIdx.x; pos < b1; pos += RADIX_BLOCK)
        atomicAdd(&cnt[(p.keys_in[seg_base + pos] >> p.shift) & mask], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < radix; t += RADIX_BLOCK)
        p.hist[((int64_t)seg * radix + t) * p.blocks_per_seg + blk] = cnt[t];
}

// Scatter of a workgroup's tiles, in order.  Per tile: stable ranks within
// each wave by ballot matching, per-digit prefixes over the waves and over the
// digits, the keys placed in LDS in digit order, then written out so that
// consecutive threads write consecutive positions of each digit's run.
__global__ __launch_bounds__(RADIX_BLOCK, 4) void k_radix_downsweep(RadixPass p) {
    __shared__ uint32_t cnt[RADIX_BLOCK / WAVE][256];
    __shared__ uint32_t gbase[256];     // global position of the next key of each digit
    __shared__ uint32_t lstart[256];    // block-local position of the tile's first key of each digit
    __shared__ uint32_t wsum[RADIX_BLOCK / WAVE];
    __shared__ uint32_t skey[RADIX_TILE];
    __shared__ uint32_t sval[RADIX_TILE];
    static_assert(RADIX_BLOCK == 256, "one thread per digit");
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int seg = blockIdx.x / p.blocks_per_seg, blk = blockIdx.x % p.blocks_per_seg;
    const int radix = 1 << p.bits;
    const uint32_t mask = (uint32_t)radix - 1u;
    const int64_t len = seg_valid_len(p);
    const int64_t seg_base = (int64_t)seg * p.seg_len;
    if ((int64_t)blk * p.tiles_per_block * RADIX_TILE >= len) return;   // nothing to move (uniform)
    if ((int)threadIdx.x < radix) gbase[threadIdx.x] = p.hist[((int64_t)seg * radix + threadIdx.x) * p.blocks_per_seg + blk];
    for (int tt = 0; tt < p.tiles_per_block; ++tt) {
        const int64_t tb = ((int64_t)blk * p.tiles_per_block + tt) * RADIX_TILE;
        if (tb >= len) break;                                          // uniform over the block
        for (int t = threadIdx.x; t < (RADIX_BLOCK / WAVE) * 256; t += RADIX_BLOCK) (&cnt[0][0])[t] = 0u;
        __syncthreads();
        const int64_t wbase = tb + (int64_t)w * (RADIX_ITEMS * WAVE);
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
        // per digit (one thread each): the waves' counts become exclusive
        // prefixes in place; the tile's count of the digit is scanned over digits
        uint32_t tot = 0;
        if ((int)threadIdx.x < radix) {
            for (int k = 0; k < RADIX_BLOCK / WAVE; ++k) {
                const uint32_t c = cnt[k][threadIdx.x];
                cnt[k][threadIdx.x] = tot;
                tot += c;
            }
        }
        uint32_t incl = tot;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, off, WAVE);
            if (lane >= off) incl += t;
        }
        if (lane == WAVE - 1) wsum[w] = incl;
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += wsum[k];
        if ((int)threadIdx.x < radix) lstart[threadIdx.x] = before + incl - tot;
        __syncthreads();
        // keys to LDS in digit order (stable: waves, then items and lanes, in order)
#pragma unroll
        for (int i = 0; i < RADIX_ITEMS; ++i) {
            const int64_t pos = wbase + (int64_t)i * WAVE + lane;
            if (pos < len) {
                const uint32_t d = (key[i] >> p.shift) & mask;
                const uint32_t lp = lstart[d] + cnt[w][d] + rank[i];
                skey[lp] = key[i];
                if (p.vals_out) sval[lp] = val[i];
            }
        }
        __syncthreads();
        const int64_t nvalid = len - tb;
        const int nb = nvalid < RADIX_TILE ? (int)nvalid : RADIX_TILE;
        for (int lp = threadIdx.x; lp < nb; lp += RADIX_BLOCK) {
            const uint32_t k = skey[lp];
            const uint32_t d = (k >> p.shift) & mask;
            // the scanned histogram holds absolute positions (earlier segments
            // are counted in full before this one)
            const int64_t dst = (int64_t)gbase[d] + (uint32_t)(lp - (int)lstart[d]);
            p.keys_out[dst] = k;
            if (p.vals_out) p.vals_out[dst] = sval[lp];
        }
        __syncthreads();
        if ((int)threadIdx.x < radix) gbase[threadIdx.x] += tot;
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
    const int64_t tiles = (span + RADIX_TILE - 1) / RADIX_TILE;
    if (tiles == 0 || segs == 0) return 0;
    // several tiles per workgroup once there are more than ~2048 workgroups'
    // worth: fewer histogram entries, which are written and read scattered
    const int tpb = (int)std::min<int64_t>(8, std::max<int64_t>(1, (segs * tiles + 2047) / 2048));
    const int bps = (int)((tiles + tpb - 1) / tpb);
    // digits of at most 8 bits, as even as the bit count allows (13 bits: 7 + 6,
    // so that each digit's run per tile is long enough to fill whole lines)
    const int npass = (hi - lo + 7) / 8;
    const int width = npass > 0 ? (hi - lo + npass - 1) / npass : 8;
    int pass = 0;
    for (int shift = lo; shift < hi; shift += width, ++pass) {
        const int bits = (hi - shift) < width ? (hi - shift) : width;
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
        p.tiles_per_block = tpb;
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
// spread over many workgroups).  The ranks covering the range are staged in
// LDS with their first instance; every rank marks the position where its
// instances start (the largest rank wins: a rank with no instance starts where
// the next one does), and a prefix maximum over the range gives every
// instance its rank.  Every binned rank owns at least one instance, so within
// one view a range spans at most 2048 ranks and the LDS window holds them;
// only a range that crosses a view boundary with culled (zero-instance) ranks
// can need more, and then searches the scan in global memory.
constexpr int DUP_TILE = 2048;
constexpr int DUP_WIN = 1024;

// largest r in [lo, hi] with off[r] <= i (off non-decreasing, off[lo] <= i)
__device__ __forceinline__ int64_t last_le(const uint32_t* off, int64_t lo, int64_t hi, uint32_t i) {
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same search by all 256 threads of a workgroup (uniform arguments): each
// round probes 256 evenly spaced entries and keeps the interval after the last
// one <= i (the probes' test is true for a prefix of the threads), so a search
// over R entries takes log_256(R) rounds of parallel loads instead of log2(R)
// dependent ones.
__device__ __forceinline__ int64_t block_last_le(const uint32_t* off, int64_t lo, int64_t hi, uint32_t i) {
    while (hi - lo >= 256) {
        const int64_t step = (hi - lo + 256) / 256;
        const int64_t pr = lo + (int64_t)threadIdx.x * step;
        const int cnt = __syncthreads_count(pr <= hi && off[pr] <= i);
        lo += (int64_t)(cnt - 1) * step;
        hi = lo + step - 1 < hi ? lo + step - 1 : hi;
    }
    const int64_t pr = lo + (int64_t)threadIdx.x;
    const int cnt = __syncthreads_count(pr <= hi && off[pr] <= i);
    return lo + cnt - 1;
}

// q = a / b, r = a % b for a < 2^22, 1 <= b < 2^12: the float estimate is
// within one of the quotient (relative error below 2^-22), then corrected.
__device__ __forceinline__ void divmod_small(uint32_t a, uint32_t b, uint32_t& q, uint32_t& r) {
    uint32_t qq = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
    int32_t rr = (int32_t)a - (int32_t)(qq * b);
    if (rr < 0) {
        qq -= 1u;
        rr += (int32_t)b;
    }
    if (rr >= (int32_t)b) {
        qq += 1u;
        rr -= (int32_t)b;
    }
    q = qq;
    r = (uint32_t)rr;
}

__global__ __launch_bounds__(256) void k_duplicate(DupArgs a) {
    constexpr int PER = DUP_TILE / 256;   // positions per thread in the prefix maximum
    // (20 KB of LDS per workgroup, so that eight are resident per CU)
    __shared__ uint32_t offs[DUP_WIN + 1];
    __shared__ uint2 rects[DUP_WIN];      // tile rect origin (x0 | y0 << 16: views are at most 1024 tiles wide) and width
    __shared__ uint32_t owner[DUP_TILE];  // window index + 1 of the rank owning each position
    __shared__ uint32_t wmax[4];
    __shared__ long long s_r0;
    __shared__ int s_win;
    if (a.counters->inst_overflow) return;   // uniform over the block
    const int64_t m = (int64_t)a.counters->n_instances;
    const int64_t ib = (int64_t)blockIdx.x * DUP_TILE;
    if (ib >= m) return;                      // uniform over the block
    const int64_t ie = ib + DUP_TILE < m ? ib + DUP_TILE : m;
    {
        const int64_t q0 = block_last_le(a.inst_off, 0, a.total_ranks - 1, (uint32_t)ib);
        const int64_t q1 = block_last_le(a.inst_off, q0, a.total_ranks - 1, (uint32_t)(ie - 1));
        if (threadIdx.x == 0) {
            s_r0 = q0;
            s_win = (q1 - q0 + 1 <= DUP_WIN) ? (int)(q1 - q0 + 1) : -1;
        }
    }
    for (int k = threadIdx.x; k < DUP_TILE; k += 256) owner[k] = 0u;
    __syncthreads();
    const int64_t r0 = s_r0;
    const int win = s_win;
    if (win > 0) {
        for (int k = threadIdx.x; k <= win; k += 256) offs[k] = a.inst_off[r0 + k];
        for (int k = threadIdx.x; k < win; k += 256) {
            const int64_t j = r0 + k;
            const int4 rc = a.rect[(j / a.n) * a.n + a.order[j]];
            rects[k] = make_uint2((uint32_t)rc.x | ((uint32_t)rc.y << 16), (uint32_t)(rc.z - rc.x + 1));
        }
        __syncthreads();
        for (int k = threadIdx.x; k < win; k += 256) {
            const uint32_t st = offs[k];
            if (st >= (uint64_t)ib && st < (uint64_t)ie) atomicMax(&owner[st - (uint32_t)ib], (uint32_t)k + 1u);
        }
        if (threadIdx.x == 0) atomicMax(&owner[0], 1u);   // the first rank owns the range's first instance
        __syncthreads();
        // inclusive prefix maximum: PER consecutive positions per thread, then over threads
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        uint32_t run = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) run = max(run, owner[threadIdx.x * PER + e]);
        uint32_t incl = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, off, 64);
            if (lane >= off) incl = max(incl, t);
        }
        if (lane == 63) wmax[w] = incl;
        uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, 64);
        if (lane == 0) excl = 0u;
        __syncthreads();
        for (int k = 0; k < w; ++k) excl = max(excl, wmax[k]);
        uint32_t cur = excl;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            cur = max(cur, owner[threadIdx.x * PER + e]);
            owner[threadIdx.x * PER + e] = cur;
        }
    }
    __syncthreads();
    for (int64_t ii = ib + threadIdx.x; ii < ie; ii += 256) {
        const uint32_t i = (uint32_t)ii;
        int64_t j;
        uint32_t x0, y0, wdt, local;
        if (win > 0) {
            const int wi = (int)owner[ii - ib] - 1;
            j = r0 + wi;
            const uint2 r = rects[wi];
            x0 = r.x & 0xFFFFu;
            y0 = r.x >> 16;
            wdt = r.y;
            local = i - offs[wi];
        } else {
            j = last_le(a.inst_off, r0, a.total_ranks - 1, i);
            const int4 r = a.rect[(j / a.n) * a.n + a.order[j]];
            x0 = (uint32_t)r.x;
            y0 = (uint32_t)r.y;
            wdt = (uint32_t)(r.z - r.x + 1);
            local = i - a.inst_off[j];
        }
        const int v = (int)(j / a.n);
        uint32_t qy, qx;
        divmod_small(local, wdt, qy, qx);
        const uint32_t tx = x0 + qx;
        const uint32_t ty = y0 + qy;
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

// the same for a 16-byte aligned p, four values per thread
__global__ __launch_bounds__(256) void k_fill_u32x4(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i + 4 <= n) {
        *reinterpret_cast<uint4*>(p + i) = make_uint4(v, v, v, v);
    } else {
        for (int64_t k = i; k < n; ++k) p[k] = v;
    }
}

__device__ __forceinline__ uint32_t inst_tile(const uint32_t* keys, int64_t i, int rank_bits, int packed) {
    return packed ? (keys[i] >> rank_bits) : keys[i];
}

// [start, end) of every non-empty tile's run in the sorted instances; each
// thread checks 8 consecutive instances against their neighbours.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, const Counters* counters,
                                                int64_t cap, int rank_bits, int packed, uint32_t* ranges) {
    if (counters->inst_overflow) return;
    const int64_t n_inst = (int64_t)counters->n_instances;
    const int64_t m = n_inst < cap ? n_inst : cap;
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
    if (i0 >= m) return;
    uint32_t t[8];
    if (i0 + 8 <= m) {
        const uint4 a0 = *reinterpret_cast<const uint4*>(keys + i0);
        const uint4 a1 = *reinterpret_cast<const uint4*>(keys + i0 + 4);
        t[0] = a0.x; t[1] = a0.y; t[2] = a0.z; t[3] = a0.w;
        t[4] = a1.x; t[5] = a1.y; t[6] = a1.z; t[7] = a1.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = i0 + e < m ? keys[i0 + e] : 0u;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = packed ? (t[e] >> rank_bits) : t[e];
    uint32_t prev = i0 > 0 ? inst_tile(keys, i0 - 1, rank_bits, packed) : 0xFFFFFFFFu;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t i = i0 + e;
        if (i >= m) break;
        if (i == 0 || prev != t[e]) ranges[2 * t[e]] = (uint32_t)i;
        const uint32_t next = e < 7 ? (i + 1 < m ? t[e + 1] : 0xFFFFFFFFu)
                                    : (i + 1 < m ? inst_tile(keys, i + 1, rank_bits, packed) : 0xFFFFFFFFu);
        if (i == m - 1 || next != t[e]) ranges[2 * t[e] + 1] = (uint32_t)(i + 1);
        prev = t[e];
    }
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
__global__ __launch_bounds__(256) void k_tile_cost_keys(const uint32_t* __restrict__ ranges,
                                                      const uint32_t* __restrict__ tile_niter, int64_t n_tiles,
                                                      uint32_t* __restrict__ keys) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t cost = ranges ? ranges[2 * t + 1] - ranges[2 * t] : tile_niter[t];
    keys[t] = 0xFFFFu - (cost < 0xFFFFu ? cost : 0xFFFFu);
}

void launch_tile_cost_keys(const uint32_t* ranges, const uint32_t* tile_niter, int64_t n_tiles, uint32_t* keys,
                           hipStream_t s) {
    if (n_tiles <= 0) return;
    hipLaunchKernelGGL(k_tile_cost_keys, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, s, ranges, tile_niter,
                       n_tiles, keys);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    if (reinterpret_cast<uintptr_t>(p) % 16 == 0) {
        const int64_t threads = (n + 3) / 4;
        hipLaunchKernelGGL(k_fill_u32x4, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p, n, v);
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    }
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
    const int64_t threads = (cap + 7) / 8;
    if (threads > 0)
        hipLaunchKernelGGL(k_ranges, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, keys, c, cap, rank_bits,
                           packed, ranges);
}

void launch_bin_keys(const uint32_t* keys, const uint32_t* vals, const uint32_t* order, const uint32_t* depth_key,
                     int64_t n_inst, int64_t n, int rank_bits, int packed, uint64_t* ko, uint32_t* go,
                     hipStream_t s) {
    if (n_inst <= 0) return;
    hipLaunchKernelGGL(k_bin_keys, dim3((unsigned)((n_inst + 255) / 256)), dim3(256), 0, s, keys, vals, order, depth_key,
                       n_inst, n, rank_bits, packed, ko, go);
}

}  // namespace fh
