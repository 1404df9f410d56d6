// Compositing with BF16 features on MFMA (gfx950), FP32 accumulation.
//
// The feature part of the forward pass is a dense contraction per tile:
//   F[256 px x D] += W[256 px x K] . Feat[K x D]     (w = alpha T, Section 3.1)
// computed with v_mfma_f32_16x16x32_bf16.  W is split into two BF16 terms,
// W = hi + lo (hi = bf16(w), lo = bf16(w - hi)), so the product keeps about 16
// bits of w; the features are BF16 already.  Everything else (alpha, the
// transmittance walk, colour) stays on the VALU in FP32.
//
// SURF: the surfel primitive (Section 3.1): four-float4 records, alpha at the
// ray-plane intersection; the rest is the same.
//
// Work mapping: one workgroup per (tile, group of ROWS pixel rows, channel
// slice of DS); wave w is pixel row w of its group; lane l handles pixel
// x = l % 16 and Gaussians 8 (l / 16) .. 8 (l / 16) + 7 of each 32-Gaussian
// chunk.  The F accumulator takes DS / 4 registers per lane whatever ROWS is,
// so 8-row (512-thread) workgroups, with twice the register budget of 16-row
// ones, carry 256 channels and evaluate alpha once per pixel and Gaussian.  The lane's eight
// weights are exactly its MFMA A-operand (rows = pixels, k = Gaussians).  The
// four lanes of a pixel combine their transmittance with an exclusive product
// scan, which reproduces the sequential walk (skip rule, stop rule) up to
// rounding.
#include "kernels.hpp"

namespace fh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int FK = 32;        // Gaussians per chunk
constexpr int FKP = 40;       // padded k-stride of the transposed feature tile (80 B rows)

// Software pipeline over the tile's chunks of FK list positions.  While chunk
// c is composited, threads 0..FK-1 hold in registers the list entries (depth
// ranks) of chunk c+3 and the records and Gaussians of chunk c+2 (one load each,
// from the rank-ordered records), and every thread holds its share of chunk
// c+1's features.  All of them are requested at the top of the chunk and only
// stored to LDS at its end, so no global latency sits between two chunks.
// Records and Gaussians are triple-buffered in LDS, features double-buffered.
constexpr uint32_t BUF_DWORD3 = 0x00020000u;   // raw buffer, 32-bit data format

__device__ __forceinline__ uint32_t list_load(__amdgpu_buffer_rsrc_t rs, uint32_t pos) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(pos * 4u), 0, 0);
}

// FS: FP32 features (the FP32 form).  Weights and features are each split
// into three BF16 terms (x = h + m + l, h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m)) and F takes the six products hh, hm, mh, hl, lh, mm:
// what is left out is below 2^-24 of w f, so F keeps FP32 accuracy on MFMA.
template <int DS, int ROWS, bool FS, bool SURF>
// (8-row shapes up to 128 channels keep four waves per SIMD: two workgroups per
// CU; 4-row shapes are two or four workgroups per CU, each with its own barriers)
__global__ __launch_bounds__(64 * ROWS, (ROWS <= 8 && DS <= 128 && !FS) ? 4 : (ROWS == 4 ? (SURF ? 3 : 2) : 1)) void k_render_fwd_bf16(
    RenderArgs a, ViewTable vt) {
    constexpr int NB = DS / 16;
    static_assert(NB % 2 == 0, "channel blocks are processed in pairs");
    constexpr int NT = 64 * ROWS;                        // threads
    constexpr int NIT = (FK * (DS / 8) + NT - 1) / NT;   // feature items per thread
    constexpr int RG = 8;                                 // record padding group (lanes read records 8 apart)
    using RecT = typename PrimRec<SURF>::T;
    constexpr int RW = PrimRec<SURF>::RW;                 // float4 per record
    __shared__ float4 srec4[3][RW * FK + FK / RG];
    __shared__ uint32_t sg[3][FK];
    constexpr int NFT = FS ? 3 : 1;                       // feature tiles: h (+ m, l)
    constexpr int NFR = FS ? 2 * NIT : NIT;               // 16-byte registers of one chunk's feature items
    __shared__ __attribute__((aligned(16))) __bf16 sft[2][NFT * DS * FKP];
    __shared__ uint32_t smax[ROWS];
    __shared__ __attribute__((aligned(16))) uint8_t sbusy[2][16];   // per wave: a pixel still walking
    if (a.counters->inst_overflow) return;
    constexpr int NG = TILE / ROWS;                      // row groups per tile
    const int t = a.tile_order ? (int)a.tile_order[blockIdx.x] : (int)blockIdx.x;
    const int grp = blockIdx.y % NG, slice = blockIdx.y / NG, d0 = slice * DS;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, xi = lane & 15;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int px = tx * TILE + xi, py = ty * TILE + grp * ROWS + w;
    const bool inside = px < vt.width[v] && py < vt.height[v];
    const float x = (float)px + 0.5f, y = (float)py + 0.5f;
    const uint32_t s = a.ranges[2 * t], e = a.ranges[2 * t + 1];
    const uint32_t len = e - s;
    const uint16_t* feat = static_cast<const uint16_t*>(a.feat);
    // the tile's list as a range-checked buffer: positions past its end read 0
    // (rank 0, a valid index; such positions become padding when stored)
    const uint32_t* list = a.packed ? a.keys : a.vals;
    const __amdgpu_buffer_rsrc_t list_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(list + s), (short)0, (int)(len < 0x1fffffffu ? len * 4u : 0x7ffffffcu), BUF_DWORD3);
    const uint32_t rmask = a.packed ? ((1u << a.rank_bits) - 1u) : 0xFFFFFFFFu;
    const int k = (int)threadIdx.x;   // list position within a chunk (threads 0..FK-1)

    auto put_rec = [&](int buf, uint32_t pos, const RecT& r, uint32_t g) {
        const bool real = pos < len;
        // padding: opacity 0 never blends
        const RecT o = real ? r : pad_rec<SURF>();
        lds_put_prec<SURF, RG>(srec4[buf], k, o);
        sg[buf][k] = real ? g : 0xFFFFFFFFu;
    };
    // e: a raw list entry (masked here, where it is used, so that its load is
    // not waited for where it is issued)
    auto get_rec = [&](uint32_t e, RecT& r, uint32_t& g) {
        const uint32_t j = e & rmask;
        r = load_rec<SURF>(a.rrec, j);
        g = a.order[j];
    };
    // feature items of one chunk: item = k + FK * dg, 8 channels each; padding
    // positions read Gaussian 0 and are zeroed when stored
    auto load_feats = [&](const uint32_t* gl, uint4* fr) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = (int)threadIdx.x + NT * it;
            if (idx < FK * (DS / 8)) {
                const int kk = idx % FK, dg = idx / FK;
                const uint32_t g = gl[kk];
                const uint32_t ga = g != 0xFFFFFFFFu ? g : 0u;
                if constexpr (FS) {
                    const uint4* src = reinterpret_cast<const uint4*>(static_cast<const float*>(a.feat) +
                                                                      (int64_t)ga * a.d + d0 + dg * 8);
                    fr[2 * it] = src[0];
                    fr[2 * it + 1] = src[1];
                } else {
                    fr[it] = *reinterpret_cast<const uint4*>(feat + (int64_t)ga * a.d + d0 + dg * 8);
                }
            }
        }
    };
    auto store_feats = [&](const uint32_t* gl, const uint4* fr, __bf16* dstb) {
        uint16_t* dst = reinterpret_cast<uint16_t*>(dstb);
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = (int)threadIdx.x + NT * it;
            if (idx < FK * (DS / 8)) {
                const int kk = idx % FK, dg = idx / FK;
                const bool pad = gl[kk] == 0xFFFFFFFFu;
                if constexpr (FS) {
                    const float4 f0 = __builtin_bit_cast(float4, fr[2 * it]);
                    const float4 f1 = __builtin_bit_cast(float4, fr[2 * it + 1]);
                    const float v[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        const float x = pad ? 0.0f : v[m];
                        const __bf16 hb = (__bf16)x;
                        const float r = x - (float)hb;
                        const __bf16 mb = (__bf16)r;
                        const __bf16 lb = (__bf16)(r - (float)mb);
                        const int o = (dg * 8 + m) * FKP + kk;
                        dst[o] = __builtin_bit_cast(uint16_t, hb);
                        dst[DS * FKP + o] = __builtin_bit_cast(uint16_t, mb);
                        dst[2 * DS * FKP + o] = __builtin_bit_cast(uint16_t, lb);
                    }
                } else {
                    uint4 f = fr[it];
                    if (pad) f = make_uint4(0, 0, 0, 0);
                    const uint16_t* h = reinterpret_cast<const uint16_t*>(&f);
#pragma unroll
                    for (int m = 0; m < 8; ++m) dst[(dg * 8 + m) * FKP + kk] = h[m];
                }
            }
        }
    };

    // prologue: chunks 0 and 1 into LDS, chunk 2's ranks into registers, then chunk 0's features
    uint32_t rk2 = 0u;
    if (k < FK && len > 0) {
        const uint32_t j0 = list_load(list_rs, (uint32_t)k);
        const uint32_t j1 = list_load(list_rs, (uint32_t)(FK + k));
        rk2 = list_load(list_rs, (uint32_t)(2 * FK + k));
        RecT r0, r1;
        uint32_t g0, g1;
        get_rec(j0, r0, g0);
        get_rec(j1, r1, g1);
        put_rec(0, (uint32_t)k, r0, g0);
        put_rec(1, (uint32_t)(FK + k), r1, g1);
    }
    if (threadIdx.x < 32) reinterpret_cast<uint8_t*>(sbusy)[threadIdx.x] = 0;
    __syncthreads();
    if (len > 0) {   // (an empty list stages nothing: sg holds no Gaussians then)
        uint4 fr[NFR];
        load_feats(sg[0], fr);
        store_feats(sg[0], fr, sft[0]);
    }
    __syncthreads();

    f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    bool done = !inside;
    uint32_t last = 0;

    int b3 = 0, b2 = 0;   // chunk index mod 3 and mod 2
    for (uint32_t cpos = 0; cpos < len; cpos += FK) {
        const int n3 = b3 == 2 ? 0 : b3 + 1, nn3 = n3 == 2 ? 0 : n3 + 1;
        // chunk c+2's records and Gaussians, chunk c+3's ranks, chunk c+1's features: all in flight now
        RecT r2;
        uint32_t g2 = 0u, rk3 = 0u;
        if (k < FK) {
            get_rec(rk2, r2, g2);
            rk3 = list_load(list_rs, cpos + (uint32_t)(3 * FK + k));
        }
        uint4 fr[NFR];
        load_feats(sg[n3], fr);

        // alpha of this lane's eight Gaussians and their transmittance product
        float al[8];
        float P = 1.0f;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const float alpha = prim_alpha<SURF>(lds_prec<SURF, RG>(srec4[b3], 8 * q + m), x, y);
            al[m] = alpha >= ALPHA_MIN ? alpha : 0.0f;
            P *= (1.0f - al[m]);
        }
        const Rows4 Pr = rows4(P);
        const float P0 = Pr.r0, P1 = Pr.r1, P2 = Pr.r2;
        const float excl = q == 0 ? 1.0f : (q == 1 ? P0 : (q == 2 ? P0 * P1 : (P0 * P1) * P2));
        float Tl = T * excl;
        bool dl = done || Tl < T_MIN;
        bool term = false;
        uint32_t mylast = 0;
        // W (this lane's 8 weights) goes straight into its MFMA A operand as BF16 hi + lo
        bf16x8 ahi, alo, amid;   // (amid: FS only; then alo holds the third term)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            // Both forms of the step give the same bits (colour by explicit
            // fused multiply-adds; a Gaussian that does not blend adds w = 0
            // exactly).  The branch-free form needs more registers than the
            // shapes that keep four waves per SIMD have.
            float wv = 0.0f;
            const float4 col = srec4[b3][prec_slot<SURF, RG>(8 * q + m) + 2];   // (opacity, r, g, b)
            if constexpr (ROWS == 8 && DS > 128) {
                const float Tn = Tl * (1.0f - al[m]);
                const bool act = !dl && al[m] > 0.0f;
                const bool stop = act && Tn < T_MIN;
                const bool blend = act && !stop;
                wv = blend ? al[m] * Tl : 0.0f;
                c0 = __builtin_fmaf(wv, col.y, c0);
                c1 = __builtin_fmaf(wv, col.z, c1);
                c2 = __builtin_fmaf(wv, col.w, c2);
                Tl = blend ? Tn : Tl;
                mylast = blend ? cpos + 8 * q + m + 1 : mylast;
                dl = dl || stop;
                term = term || stop;
            } else {
                if (!dl && al[m] > 0.0f) {
                    const float Tn = Tl * (1.0f - al[m]);
                    if (Tn < T_MIN) {
                        dl = true;
                        term = true;
                    } else {
                        wv = al[m] * Tl;
                        c0 = __builtin_fmaf(wv, col.y, c0);
                        c1 = __builtin_fmaf(wv, col.z, c1);
                        c2 = __builtin_fmaf(wv, col.w, c2);
                        Tl = Tn;
                        mylast = cpos + 8 * q + m + 1;
                    }
                }
            }
            const __bf16 h = (__bf16)wv;
            ahi[m] = h;
            if constexpr (FS) {
                const float r = wv - (float)h;
                const __bf16 mb = (__bf16)r;
                amid[m] = mb;
                alo[m] = (__bf16)(r - (float)mb);
            } else {
                alo[m] = (__bf16)(wv - (float)h);
            }
        }
        // pixel state after the chunk: the first lane that stopped, else lane 3
        const uint64_t tb = ballot64(term);
        const Rows4 Tr = rows4(Tl);
        const float Tq0 = Tr.r0, Tq1 = Tr.r1, Tq2 = Tr.r2, Tq3 = Tr.r3;
        const bool t0 = (tb >> xi) & 1, t1 = (tb >> (xi + 16)) & 1, t2 = (tb >> (xi + 32)) & 1,
                   t3 = (tb >> (xi + 48)) & 1;
        if (!done) {
            T = t0 ? Tq0 : (t1 ? Tq1 : (t2 ? Tq2 : Tq3));
            done = t0 || t1 || t2 || t3;
        }
        const Rows4 Lr = rows4(__uint_as_float(mylast));
        const uint32_t lm = max(max(__float_as_uint(Lr.r0), __float_as_uint(Lr.r1)),
                                max(__float_as_uint(Lr.r2), __float_as_uint(Lr.r3)));
        last = max(last, lm);

        // W times the feature chunk (channel blocks in pairs, so that the hi and
        // lo products of one block are not issued back to back)
#pragma unroll
        for (int j = 0; j < NB; j += 2) {
            const bf16x8 bv0 = *reinterpret_cast<const bf16x8*>(&sft[b2][(j * 16 + xi) * FKP + 8 * q]);
            const bf16x8 bv1 = *reinterpret_cast<const bf16x8*>(&sft[b2][((j + 1) * 16 + xi) * FKP + 8 * q]);
            if constexpr (FS) {
                // the six products, smallest first: lh, hl, mm, mh, hm, hh
                const bf16x8 bm0 = *reinterpret_cast<const bf16x8*>(&sft[b2][DS * FKP + (j * 16 + xi) * FKP + 8 * q]);
                const bf16x8 bm1 =
                    *reinterpret_cast<const bf16x8*>(&sft[b2][DS * FKP + ((j + 1) * 16 + xi) * FKP + 8 * q]);
                const bf16x8 bl0 =
                    *reinterpret_cast<const bf16x8*>(&sft[b2][2 * DS * FKP + (j * 16 + xi) * FKP + 8 * q]);
                const bf16x8 bl1 =
                    *reinterpret_cast<const bf16x8*>(&sft[b2][2 * DS * FKP + ((j + 1) * 16 + xi) * FKP + 8 * q]);
                f32x4 s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bv0, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                f32x4 s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bv1, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bl0, s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bl1, s1, 0, 0, 0);
                s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amid, bm0, s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amid, bm1, s1, 0, 0, 0);
                s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amid, bv0, s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amid, bv1, s1, 0, 0, 0);
                s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bm0, s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bm1, s1, 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bv0, acc[j] + s0, 0, 0, 0);
                acc[j + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bv1, acc[j + 1] + s1, 0, 0, 0);
            } else {
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bv0, acc[j], 0, 0, 0);
                acc[j + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bv1, acc[j + 1], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bv0, acc[j], 0, 0, 0);
                acc[j + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bv1, acc[j + 1], 0, 0, 0);
            }
        }
        // chunk c+1's features and chunk c+2's records to LDS
        store_feats(sg[n3], fr, sft[b2 ^ 1]);
        if (k < FK) {
            put_rec(nn3, cpos + (uint32_t)(2 * FK + k), r2, g2);
            rk2 = rk3;
        }
        // leave when every pixel of the workgroup has stopped (flags double-buffered by chunk parity)
        const bool wave_busy = ballot64(!done) != 0;   // (all lanes vote, outside the lane-0 store)
        if (lane == 0) sbusy[b2][w] = wave_busy ? 1 : 0;
        __syncthreads();
        const uint4 bz = *reinterpret_cast<const uint4*>(sbusy[b2]);
        if ((bz.x | bz.y | bz.z | bz.w) == 0u) break;
        b3 = n3;
        b2 ^= 1;
    }

    // colour: the four lanes of a pixel hold partial sums
    c0 += __shfl_xor(c0, 16, 64);
    c0 += __shfl_xor(c0, 32, 64);
    c1 += __shfl_xor(c1, 16, 64);
    c1 += __shfl_xor(c1, 32, 64);
    c2 += __shfl_xor(c2, 16, 64);
    c2 += __shfl_xor(c2, 32, 64);
    const int64_t rowp = vt.pix_off[v] + (int64_t)py * vt.width[v];
    if (slice == 0 && q == 0 && inside) {
        const int64_t p = rowp + px;
        a.C[3 * p] = c0;
        a.C[3 * p + 1] = c1;
        a.C[3 * p + 2] = c2;
        a.T[p] = T;
        a.n_iter[p] = last;
    }
    // F: lane holds F[pixel 4q + r of this row][channel 16 j + xi]
    if (py < vt.height[v]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pxr = tx * TILE + 4 * q + r;
            if (pxr < vt.width[v]) {
                float* fo = a.F + (rowp + pxr) * a.d + d0 + xi;
#pragma unroll
                for (int j = 0; j < NB; ++j) fo[16 * j] = acc[j][r];
            }
        }
    }
    if (slice == 0) {
        // the tile's traversal length: max over its row groups (tile_niter is
        // zeroed before the launch)
        const uint32_t m = wave_max_u32(last);
        if (lane == 0) smax[w] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t mm = 0;
            for (int k = 0; k < ROWS; ++k) mm = smax[k] > mm ? smax[k] : mm;
            if (NG == 1)
                a.tile_niter[t] = mm;
            else
                atomicMax(&a.tile_niter[t], mm);
        }
    }
}

bool render_fwd_bf16_shape_ok(int d, int slice, int rows) {
    if (rows == 16) return (slice == 32 || slice == 64 || slice == 96 || slice == 128) && d % slice == 0;
    if (rows == 8) return (slice == 64 || slice == 128 || slice == 256) && d % slice == 0;
    if (rows == 4) return (slice == 128 || slice == 256) && d % slice == 0;
    return false;
}

template <bool FS, bool SURF>
static void launch_fwd_mfma(const RenderArgs& a, const ViewTable& vt, int n_tiles, int slice, int rows, hipStream_t s) {
    // slice and rows form a valid shape for d (checked by the caller)
    const unsigned ns = (unsigned)(a.d / slice);
    const dim3 g16(n_tiles, ns), g8(n_tiles, 2 * ns), g4(n_tiles, 4 * ns);
    if (rows == 4) {
        // (BF16-stored features only)
        if constexpr (!FS) {
            if (slice == 128)
                hipLaunchKernelGGL((k_render_fwd_bf16<128, 4, false, SURF>), g4, dim3(256), 0, s, a, vt);
            else
                hipLaunchKernelGGL((k_render_fwd_bf16<256, 4, false, SURF>), g4, dim3(256), 0, s, a, vt);
        }
        return;
    }
    if (rows == 8) {
        switch (slice) {
            case 64: hipLaunchKernelGGL((k_render_fwd_bf16<64, 8, FS, SURF>), g8, dim3(512), 0, s, a, vt); break;
            case 128: hipLaunchKernelGGL((k_render_fwd_bf16<128, 8, FS, SURF>), g8, dim3(512), 0, s, a, vt); break;
            default: hipLaunchKernelGGL((k_render_fwd_bf16<256, 8, FS, SURF>), g8, dim3(512), 0, s, a, vt); break;
        }
        return;
    }
    switch (slice) {
        case 32: hipLaunchKernelGGL((k_render_fwd_bf16<32, 16, FS, SURF>), g16, dim3(1024), 0, s, a, vt); break;
        case 64: hipLaunchKernelGGL((k_render_fwd_bf16<64, 16, FS, SURF>), g16, dim3(1024), 0, s, a, vt); break;
        case 96: hipLaunchKernelGGL((k_render_fwd_bf16<96, 16, FS, SURF>), g16, dim3(1024), 0, s, a, vt); break;
        default:
            // (16 rows of 128 channels is not an FP32-feature shape: it would spill)
            if constexpr (!FS) hipLaunchKernelGGL((k_render_fwd_bf16<128, 16, false, SURF>), g16, dim3(1024), 0, s, a, vt);
            break;
    }
}

// BF16 features enter the MFMA as stored; FP32 features (fsplit) as three terms.
// Surfels (a.prim): BF16 features only.
void launch_render_fwd_bf16(const RenderArgs& a, const ViewTable& vt, int n_tiles, int slice, int rows, bool fsplit,
                            hipStream_t s) {
    if (a.prim == FH_PRIM_SURFEL)
        launch_fwd_mfma<false, true>(a, vt, n_tiles, slice, rows, s);
    else if (fsplit)
        launch_fwd_mfma<true, false>(a, vt, n_tiles, slice, rows, s);
    else
        launch_fwd_mfma<false, false>(a, vt, n_tiles, slice, rows, s);
}

}  // namespace fh
