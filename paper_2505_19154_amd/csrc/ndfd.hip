// NDFD feature branch (Section 3.3; Appendix A.1-A.2): along each pixel's
// front-to-back walk, with unit features fh_i = f_i / |f_i| and
// gh = F_gt / |F_gt| (a zero vector's unit vector taken as zero),
//   phi_i = fh_i . gh,   sigma_i = 1 / (1 + exp(k (phi_i - lambda))),
//   L_gt  = sum_i w_i sigma_i,
//   L_cf  = sum_i sigma_i w_i (W_{i-1} - x_i),  x_i = F_{i-1} . fh_i,
//   W_{i-1} = sum_{j<i} w_j,  F_{i-1} = sum_{j<i} w_j fh_j,
// and, for a per-pixel loss a L_gt + b L_cf, the derivative with respect to
// w_k (Appendix A.2; the prefix part sigma_k (W_{k-1} - x_k) and sigma_k are
// recorded per (position, pixel) by the front-to-back sweep, the suffix part
// is accumulated by a back-to-front sweep)
//   h_k = a sigma_k + b (sigma_k (W_{k-1} - x_k) + A_k - y_k),
//   A_k = sum_{i>k} sigma_i w_i,  y_k = sum_{i>k} sigma_i w_i fh_i . fh_k,
// which joins the adjoint through w: dL/dalpha_k = T_k h_k - (sum_{i>k} w_i
// h_i) / (1 - alpha_k), chained to the screen-space terms as in the gradient
// kernel.  sigma is a constant of the frozen features: no gradient flows
// through it.
//
// All per-(pixel, Gaussian) dot products are MFMA contractions
// (v_mfma_f32_16x16x32_bf16) over the chunk of 32 positions:
//   phi^T[k x px]  = Feat[k x D] . gh^T[D x px]          (F_gt BF16, resident)
//   x^T, y^T       = Feat . Q^T, Feat . R^T               (Q = F, R = the sigma-weighted
//                                                          suffix; FP32 accumulators fed
//                                                          back as BF16 hi + lo)
//   Q^T, R^T      += Feat^T[D x k] . (w / |f|)^T[k x px] (weights split hi + lo;
//                                                          sigma w / |f| for R)
//   within chunk  : Gh[k x j] . W^T[j x px]               (Gh = the chunk's unit Gram
//                                                          matrix, masked, hi + lo)
// Accumulator layout and operand layout agree up to a permutation of the
// contracted index, so the running vectors never leave registers: lane
// (xi, q) of a 16-lane row holds channels 16 m + 4 q + r of pixel xi, which is
// exactly the B operand of the slab 32 s .. 32 s + 31 when the A operand reads
// its channels in the order (32 s + 4 q + r, 32 s + 16 + 4 q + r); and it walks
// the positions 4 q + r and 16 + 4 q + r of the chunk, which are both the rows
// the contractions return to it and the k-slots of its weight operand.
//
// Work mapping: two workgroups per tile (pixel rows 0-7 and 8-15), 512
// threads, wave w = pixel row; pass 1 walks the tile's visited list front to
// back (losses, with the running F in the Q registers; for the gradient it
// records sigma_k and the prefix term of every (position, pixel)), pass 2
// back to front with the suffix R in registers: one D-channel running vector
// per pixel at a time, so two waves per SIMD.  Each half writes its own
// per-instance screen-space partial (u, v, A, B, C, sum dL/dpower); a second
// kernel adds both halves into the gradient kernel's partials in a fixed
// order.
//
// SURF: the surfel primitive (Section 3.1): four-float4 records, alpha at the
// ray-plane intersection, and per half the nine record entries' terms and
// sum dL/dpower (rows of 16 floats), from the sums of dL/dk and dL/dk dx
// along each row as in the gradient kernel.
#include "kernels.hpp"

namespace fh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NK = 32;                       // positions per chunk
constexpr int NJP = 40;                      // row stride (bf16) of the transposed features and the Gram operands
constexpr int NSK = NK + 3;                  // padded per-pixel stride of dL/dpower
constexpr int NRG = 4;                       // record padding group (lane rows read records 4 apart)
constexpr int NDFD_PARTS = 2;                // halves per visit in the partial array
// per primitive: terms of a (visit, part) partial, and floats per partial row
template <bool SURF>
struct NdfdPart {
    static constexpr int NQ = 6, W = 8;      // u, v, A, B, C, sum dL/dpower
};
template <>
struct NdfdPart<true> {
    static constexpr int NQ = 10, W = 16;    // the nine record entries, sum dL/dpower
};

__device__ __forceinline__ bf16x8 bf16x8_of(uint2 lo, uint2 hi) {
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

__device__ __forceinline__ void split8(const float* v, bf16x8& h, bf16x8& l) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const __bf16 hb = (__bf16)v[m];
        h[m] = hb;
        l[m] = (__bf16)(v[m] - (float)hb);
    }
}

template <int D, bool GRAD, bool SURF>
__global__ __launch_bounds__(512) void k_ndfd(NdfdArgs a, ViewTable vt) {
    using RecT = typename PrimRec<SURF>::T;
    constexpr int RW = PrimRec<SURF>::RW;
    constexpr int NRSLOTS = RW * NK + NK / NRG;
    constexpr int NQN = NdfdPart<SURF>::NQ, NDP = NdfdPart<SURF>::W;
    constexpr int ROWS = 8;                   // pixel rows (waves) per workgroup
    constexpr int NT = 64 * ROWS;             // threads
    constexpr int NS = D / 32;                // 32-channel slabs
    constexpr int NB = D / 16;                // 16-channel accumulator blocks
    constexpr int DP = D + 8;                 // row stride (bf16) of the feature tile
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16* sfeat = reinterpret_cast<__bf16*>(smem);          // [NK][DP]
    __bf16* sfeatT = sfeat + NK * DP;                          // [D][NJP]
    __bf16* sA = sfeatT + D * NJP;                             // [3 masks][hi, lo][NK][NJP]
    float* sG = reinterpret_cast<float*>(sA + 6 * NK * NJP);  // [NK][NK + 1]
    float* sinv = sG + NK * (NK + 1);                          // [NK]
    float* sdp = sinv + NK;                                    // [16 ROWS][NSK] dL/dpower (gradient)
    float* sred = sdp + TILE * ROWS * NSK;                     // [ROWS][NQN][NK] row sums (gradient)
    __shared__ float4 srec[NRSLOTS];

    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = blockIdx.x, half = blockIdx.y;
    const uint32_t nt = a.tile_niter[t];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, xi = lane & 15;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const uint32_t voff = a.tile_voff[t];
    const int ry = ROWS * half + w;
    const int px = tx * TILE + xi, py = ty * TILE + ry;
    const bool inside = px < W && py < H;
    const float x = (float)px + 0.5f, y = (float)py + 0.5f;
    const int64_t p = vt.pix_off[v] + (int64_t)(inside ? py : 0) * W + (inside ? px : 0);
    const uint32_t nit = inside ? a.n_iter[p] : 0u;
    const float ca = (GRAD && inside && a.a) ? a.a[p] : 0.0f;
    const float cb = (GRAD && inside && a.b) ? a.b[p] : 0.0f;
    const float LN2 = 0.69314718055994531f;
    if (nt == 0) {
        // no Gaussian reaches this tile: both losses are zero
        if (q == 0 && inside) {
            if (a.Lgt) a.Lgt[p] = 0.0f;
            if (a.Lcf) a.Lcf[p] = 0.0f;
        }
        return;
    }

    // F_gt of this lane's pixel, channels (32 s + 4 q + m, 32 s + 16 + 4 q + m):
    // the B operand of phi; its norm over the pixel's four lanes
    bf16x8 gto[NS];
    float gn2 = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        uint2 lo = make_uint2(0u, 0u), hi = make_uint2(0u, 0u);
        if (inside) {
            lo = *reinterpret_cast<const uint2*>(a.gt + p * D + 32 * s + 4 * q);
            hi = *reinterpret_cast<const uint2*>(a.gt + p * D + 32 * s + 16 + 4 * q);
        }
        gto[s] = bf16x8_of(lo, hi);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const float g = (float)gto[s][m];
            gn2 = __builtin_fmaf(g, g, gn2);
        }
    }
    const Rows4 gr = rows4(gn2);
    const float gsum = (gr.r0 + gr.r1) + (gr.r2 + gr.r3);
    const float ig = gsum > 0.0f ? 1.0f / sqrtf(gsum) : 0.0f;

    // ---- chunk staging: records, features (row-major and transposed) --------
    // Chunk i of a pass: front to back, positions 32 i .. ; back to front, the
    // 32 positions ending at nt - 32 i.  Pipelined: the Gaussian of this
    // thread's position (k = thread % NK, the same for all its items) two
    // chunks ahead, and the feature rows and one record dword of the next
    // chunk, are held in registers while the current chunk is processed, and
    // stored to LDS at the next chunk's staging point.
    constexpr int ITEMS = NK * (D / 8), NI = (ITEMS + NT - 1) / NT;
    constexpr int RD = 4 * RW;                // record dwords (one per thread, threads 0 .. RD NK - 1)
    static_assert(NT % NK == 0 && RD * NK <= NT, "staging layout");
    auto chunk = [&](bool fwd, int i, int& cs, int& cnt) -> bool {
        if (fwd) {
            cs = NK * i;
            cnt = (int)nt - cs < NK ? (int)nt - cs : NK;
            return cs < (int)nt;
        }
        const int ce = (int)nt - NK * i;
        cs = ce - NK > 0 ? ce - NK : 0;
        cnt = ce - cs;
        return ce > 0;
    };
    const int kk = (int)threadIdx.x % NK;     // this thread's position in every staged chunk
    const int rk = (int)threadIdx.x / RD, rj = (int)threadIdx.x % RD;   // its record and dword
    float pad_dw = 0.0f;                      // the padding record's dword rj
    {
        const RecT pr = pad_rec<SURF>();
        float4 f4[4] = {pr.r0, pr.r1, pr.r2, pr.r0};
        if constexpr (SURF) f4[3] = pr.r3;
#pragma unroll
        for (int i = 0; i < RD; ++i) {
            const float4 c = f4[i / 4];
            const float e = (i % 4) == 0 ? c.x : ((i % 4) == 1 ? c.y : ((i % 4) == 2 ? c.z : c.w));
            pad_dw = rj == i ? e : pad_dw;
        }
    }
    uint32_t pgid = 0xFFFFFFFFu;              // Gaussian at position kk of the chunk after the next one
    uint4 praw[NI];                           // feature rows of the next chunk
    float prec = 0.0f;                        // record dword of the next chunk
    auto fetch_gid = [&](bool fwd, int i) {
        int cs, cnt;
        pgid = 0xFFFFFFFFu;
        if (chunk(fwd, i, cs, cnt) && kk < cnt) pgid = a.vgid[(int64_t)voff + cs + kk];
    };
    auto fetch_data = [&](bool fwd, int i) {   // chunk i, whose Gaussians pgid holds
        int cs, cnt;
        const bool ok = chunk(fwd, i, cs, cnt);
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const int idx = threadIdx.x + NT * it;
            praw[it] = make_uint4(0u, 0u, 0u, 0u);
            if (ok && idx < ITEMS && pgid != 0xFFFFFFFFu)
                praw[it] = *reinterpret_cast<const uint4*>(a.feat + (int64_t)pgid * D + (idx / NK) * 8);
        }
        prec = pad_dw;
        if (ok && (int)threadIdx.x < RD * NK && rk < cnt)
            prec = reinterpret_cast<const float*>(a.vrec)[((int64_t)voff + cs + rk) * RD + rj];
    };
    auto commit = [&]() {
        if ((int)threadIdx.x < RD * NK) reinterpret_cast<float*>(srec)[4 * prec_slot<SURF, NRG>(rk) + rj] = prec;
        // item = (position k, 8-channel group dg), k fastest.  The transposed
        // tile is written in 4-byte words holding positions (2p, 2p + 1) of one
        // channel: the neighbouring lane (k ^ 1, same dg) passes its row, the
        // even lane writes channels 0-3 of the group and the odd lane 4-7, so
        // that a store's four lane groups (even / odd, two dg) meet disjoint
        // bank ranges (rows 8 channels apart are 160 words apart).
        uint16_t* f16 = reinterpret_cast<uint16_t*>(sfeat);
        uint32_t* ft32 = reinterpret_cast<uint32_t*>(sfeatT);
        const bool odd = (kk & 1) != 0;
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const int idx = threadIdx.x + NT * it;
            // (every lane of a wave takes part in the exchange; NT is a multiple of 64)
            const uint4 nb = make_uint4(__shfl_xor(praw[it].x, 1), __shfl_xor(praw[it].y, 1),
                                        __shfl_xor(praw[it].z, 1), __shfl_xor(praw[it].w, 1));
            if (idx < ITEMS) {
                const int dg = idx / NK;
                *reinterpret_cast<uint4*>(&f16[kk * DP + dg * 8]) = praw[it];
                // words of channels 2j, 2j + 1 (j = 0, 1 even lanes; 2, 3 odd lanes)
                const uint4 lo4 = odd ? nb : praw[it], hi4 = odd ? praw[it] : nb;   // positions 2p, 2p + 1
                const uint32_t wl0 = odd ? lo4.z : lo4.x, wl1 = odd ? lo4.w : lo4.y;
                const uint32_t wh0 = odd ? hi4.z : hi4.x, wh1 = odd ? hi4.w : hi4.y;
                const int m0 = odd ? 4 : 0;
                uint32_t* row = ft32 + (dg * 8 + m0) * (NJP / 2) + (kk >> 1);
                row[0 * (NJP / 2)] = (wl0 & 0xFFFFu) | (wh0 << 16);
                row[1 * (NJP / 2)] = (wl0 >> 16) | (wh0 & 0xFFFF0000u);
                row[2 * (NJP / 2)] = (wl1 & 0xFFFFu) | (wh1 << 16);
                row[3 * (NJP / 2)] = (wl1 >> 16) | (wh1 & 0xFFFF0000u);
            }
        }
    };
    // first chunk of a pass in flight, the second one's Gaussians requested
    auto pipeline_start = [&](bool fwd) {
        fetch_gid(fwd, 0);
        fetch_data(fwd, 0);
        fetch_gid(fwd, 1);
    };
    // chunk i to LDS (between the two barriers), chunk i + 1 in flight
    auto stage = [&](bool fwd, int i) {
        commit();
        fetch_data(fwd, i + 1);
        fetch_gid(fwd, i + 2);
    };
    // A operand of a contraction over channels: feature row `row`, slab s, in
    // the channel order of the accumulator layout
    auto featA = [&](int row, int s) -> bf16x8 {
        const uint2 lo = *reinterpret_cast<const uint2*>(&sfeat[row * DP + 32 * s + 4 * q]);
        const uint2 hi = *reinterpret_cast<const uint2*>(&sfeat[row * DP + 32 * s + 16 + 4 * q]);
        return bf16x8_of(lo, hi);
    };
    // A operand of a contraction over positions: channel row d, positions
    // (4 q + m, 16 + 4 q + m) -- this lane group's walked positions
    auto featTA = [&](int d) -> bf16x8 {
        const uint2 lo = *reinterpret_cast<const uint2*>(&sfeatT[d * NJP + 4 * q]);
        const uint2 hi = *reinterpret_cast<const uint2*>(&sfeatT[d * NJP + 16 + 4 * q]);
        return bf16x8_of(lo, hi);
    };
    // waves 0..3: the chunk's Gram matrix G[j][k] = f_j . f_k, one 16 x 16 block
    // each, and the inverse norms of the chunk's features
    auto gram = [&]() {
        if (w < 4) {
            const int jb = w >> 1, kb = w & 1;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < NS; ++s)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(featA(16 * jb + xi, s), featA(16 * kb + xi, s), acc, 0,
                                                              0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) sG[(16 * jb + 4 * q + r) * (NK + 1) + 16 * kb + xi] = acc[r];
            // 1 / |f_k| from the diagonal blocks' diagonal (row 4 q + r = column xi)
            if (jb == kb && (xi >> 2) == q) {
                const int r = xi & 3;
                const float gkk = r == 0 ? acc[0] : (r == 1 ? acc[1] : (r == 2 ? acc[2] : acc[3]));
                sinv[16 * jb + xi] = gkk > 0.0f ? 1.0f / sqrtf(gkk) : 0.0f;
            }
        }
    };
    // unit Gram operands: row k, slot 8 g + m <-> position j(g, m), masked by
    // mask 0: j < k, 1: j >= k, 2: j > k (after gram)
    auto build_masks = [&](int m0, int m1) {
        uint16_t* a16 = reinterpret_cast<uint16_t*>(sA);
        for (int e = threadIdx.x; e < NK * NK; e += NT) {
            const int k = e / NK, sl = e % NK, g = sl >> 3, m = sl & 7;
            const int j = m < 4 ? 4 * g + m : 16 + 4 * g + (m - 4);
            const float gh = (sG[j * (NK + 1) + k] * sinv[j]) * sinv[k];
            for (int mk = m0; mk <= m1; ++mk) {
                const bool keep = mk == 0 ? j < k : (mk == 1 ? j >= k : j > k);
                const float val = keep ? gh : 0.0f;
                const __bf16 hb = (__bf16)val;
                a16[((2 * mk) * NK + k) * NJP + sl] = __builtin_bit_cast(uint16_t, hb);
                a16[((2 * mk + 1) * NK + k) * NJP + sl] = __builtin_bit_cast(uint16_t, (__bf16)(val - (float)hb));
            }
        }
    };
    // out^T[k][px] += sum_j mask[k][j] V^T[j][px] for both 16-row blocks (V = hi + lo)
    auto masked = [&](int mk, const bf16x8& vh, const bf16x8& vl, f32x4* out) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const int row = 16 * kb + xi;
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sA[((2 * mk) * NK + row) * NJP + 8 * q]);
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(&sA[((2 * mk + 1) * NK + row) * NJP + 8 * q]);
            out[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, vh, out[kb], 0, 0, 0);
            out[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, vl, out[kb], 0, 0, 0);
            out[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, vh, out[kb], 0, 0, 0);
        }
    };
    // out^T[k][px] = sum_d f_k[d] Acc^T[d][px] (the accumulator as a BF16 hi + lo operand)
    auto contract_acc = [&](const f32x4* acc, f32x4* out) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float vals[8] = {acc[2 * s][0], acc[2 * s][1], acc[2 * s][2], acc[2 * s][3],
                                   acc[2 * s + 1][0], acc[2 * s + 1][1], acc[2 * s + 1][2], acc[2 * s + 1][3]};
            bf16x8 bh, bl;
            split8(vals, bh, bl);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 fa = featA(16 * kb + xi, s);
                out[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, bh, out[kb], 0, 0, 0);
                out[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, bl, out[kb], 0, 0, 0);
            }
        }
    };
    // Acc^T[d][px] += sign sum_j f_j[d] V^T[j][px] (V = hi + lo in the walk's slots)
    auto accumulate = [&](f32x4* acc, const bf16x8& vh, const bf16x8& vl) {
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) {
            const bf16x8 fa = featTA(16 * mb + xi);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, vh, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, vl, acc[mb], 0, 0, 0);
        }
    };
    // phi (raw f . F_gt) for the chunk's positions 16 kb + 4 q + r
    auto phi_raw = [&](f32x4* ph) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            ph[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < NS; ++s)
                ph[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(featA(16 * kb + xi, s), gto[s], ph[kb], 0, 0, 0);
        }
    };
    // sigma = 1 / (1 + e^{k (phi - lambda)}) by the hardware exp2 and
    // reciprocal (about one ulp each: far inside sigma's companion)
    const float LOG2E = 1.4426950408889634f;
    auto sigma_of = [&](float phr, int k) {
        const float phi = (phr * sinv[k]) * ig;
        return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f((a.kk * (phi - a.lam)) * LOG2E));
    };

    f32x4 Q[NB];   // pass 1: F = sum w fh (running)
#pragma unroll
    for (int mb = 0; mb < NB; ++mb) Q[mb] = f32x4{0.f, 0.f, 0.f, 0.f};

    // ---- pass 1: front to back, the losses ------------------------------------
    float T = 1.0f, Wacc = 0.0f, lgt = 0.0f, lcf = 0.0f;
    pipeline_start(true);
    for (int cs = 0; cs < (int)nt; cs += NK) {
        const int cnt = (int)nt - cs < NK ? (int)nt - cs : NK;
        __syncthreads();
        stage(true, cs / NK);
        __syncthreads();
        gram();
        f32x4 ph[2];
        phi_raw(ph);
        // walk: w, T_k and W_{k-1} of this lane's positions 16 kb + 4 q + r
        float wv[2][4], Wp[2][4];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            float al[4];
            bool on[4];
            float trel = 1.0f, Wr = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * kb + 4 * q + r;
                const float4* rp = srec + (4 * RW + 1) * q + (16 * RW + 4) * kb + RW * r;   // slot of k
                RecT rc;
                rc.r0 = rp[0];
                rc.r1 = rp[1];
                rc.r2 = rp[2];
                if constexpr (SURF) rc.r3 = rp[3];
                const float alpha = prim_alpha<SURF>(rc, x, y);
                on[r] = k < cnt && (uint32_t)(cs + k) < nit && alpha >= ALPHA_MIN;
                al[r] = alpha;
                Wr = on[r] ? __builtin_fmaf(al[r], trel, Wr) : Wr;
                trel = on[r] ? trel * (1.0f - al[r]) : trel;
            }
            const Rows4 Pr = rows4(trel), Wrr = rows4(Wr);
            const float Te0 = T, Te1 = Te0 * Pr.r0, Te2 = Te1 * Pr.r1, Te3 = Te2 * Pr.r2;
            const float We0 = Wacc, We1 = We0 + Te0 * Wrr.r0, We2 = We1 + Te1 * Wrr.r1, We3 = We2 + Te2 * Wrr.r2;
            float Tc = q == 0 ? Te0 : (q == 1 ? Te1 : (q == 2 ? Te2 : Te3));
            float Wc = q == 0 ? We0 : (q == 1 ? We1 : (q == 2 ? We2 : We3));
            T = Te3 * Pr.r3;
            Wacc = We3 + Te3 * Wrr.r3;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float wk = on[r] ? al[r] * Tc : 0.0f;
                wv[kb][r] = wk;
                Wp[kb][r] = Wc;
                Wc += wk;
                Tc = on[r] ? Tc * (1.0f - al[r]) : Tc;
            }
        }
        __syncthreads();
        build_masks(0, 0);
        __syncthreads();
        // within-chunk part of x, and the accumulators' part
        const float wflat[8] = {wv[0][0], wv[0][1], wv[0][2], wv[0][3], wv[1][0], wv[1][1], wv[1][2], wv[1][3]};
        bf16x8 wh, wl;
        split8(wflat, wh, wl);
        f32x4 xw[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        masked(0, wh, wl, xw);
        f32x4 xa[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        contract_acc(Q, xa);
        float wsc[8];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * kb + 4 * q + r;
                const float ik = sinv[k];
                const float sg = sigma_of(ph[kb][r], k);
                const float xk = xa[kb][r] * ik + xw[kb][r];
                const float wk = wv[kb][r];
                const float ck = sg * (Wp[kb][r] - xk);     // sigma_k (W_{k-1} - x_k)
                lgt = __builtin_fmaf(wk, sg, lgt);
                lcf = __builtin_fmaf(ck, wk, lcf);
                wsc[4 * kb + r] = wk * ik;
                // (the gradient sweep reads sigma_k and the prefix term back)
                if (GRAD && k < cnt)
                    a.sc[((int64_t)voff + cs + k) * TILE_PIX + ry * TILE + xi] =
                        inside ? make_float2(sg, ck) : make_float2(0.0f, 0.0f);
            }
        bf16x8 vh, vl;
        split8(wsc, vh, vl);
        accumulate(Q, vh, vl);
    }
    {
        const Rows4 a4 = rows4(lgt), b4 = rows4(lcf);
        if (q == 0 && inside) {
            if (a.Lgt) a.Lgt[p] = (a4.r0 + a4.r1) + (a4.r2 + a4.r3);
            if (a.Lcf) a.Lcf[p] = (b4.r0 + b4.r1) + (b4.r2 + b4.r3);
        }
    }
    if constexpr (!GRAD) return;

    // ---- pass 2: back to front, the gradient ---------------------------------
    // sigma_k and the prefix term c_k = sigma_k (W_{k-1} - x_k) come back from
    // pass 1; the back-to-front walk adds the suffix terms:
    //   h_k = a sigma_k + b (c_k + A_k - y_k)
    f32x4 R[NB];
#pragma unroll
    for (int mb = 0; mb < NB; ++mb) R[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    T = inside ? a.T_final[p] : 1.0f;
    float Asuf = 0.0f, Ssuf = 0.0f;
    __syncthreads();   // (pass 1's stores of sc are read back by the same lanes)
    pipeline_start(false);
    for (int ce = (int)nt; ce > 0; ce -= NK) {
        const int cs = ce - NK > 0 ? ce - NK : 0;
        const int cnt = ce - cs;
        __syncthreads();
        stage(false, ((int)nt - ce) / NK);
        __syncthreads();
        gram();
        float al[2][4], iv[2][4], wv[2][4], Tk[2][4], sg[2][4], ck[2][4];
        bool on[2][4];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * kb + 4 * q + r;
                float2 v2 = make_float2(0.0f, 0.0f);
                if (k < cnt && inside) v2 = a.sc[((int64_t)voff + cs + k) * TILE_PIX + ry * TILE + xi];
                sg[kb][r] = v2.x;
                ck[kb][r] = v2.y;
            }
#pragma unroll
        for (int kb = 1; kb >= 0; --kb) {
            float P = 1.0f, trel = 1.0f;
#pragma unroll
            for (int r = 3; r >= 0; --r) {
                const int k = 16 * kb + 4 * q + r;
                const float4* rp = srec + (4 * RW + 1) * q + (16 * RW + 4) * kb + RW * r;   // slot of k
                RecT rc;
                rc.r0 = rp[0];
                rc.r1 = rp[1];
                rc.r2 = rp[2];
                if constexpr (SURF) rc.r3 = rp[3];
                const float alpha = prim_alpha<SURF>(rc, x, y);
                on[kb][r] = k < cnt && (uint32_t)(cs + k) < nit && alpha >= ALPHA_MIN;
                al[kb][r] = alpha;
                iv[kb][r] = __builtin_amdgcn_rcpf(1.0f - al[kb][r]);
                const float tn = trel * iv[kb][r];
                P = on[kb][r] ? P * (1.0f - al[kb][r]) : P;
                trel = on[kb][r] ? tn : trel;
            }
            const Rows4 Pr = rows4(P);
            const float Te3 = T, Te2 = Te3 * __builtin_amdgcn_rcpf(Pr.r3), Te1 = Te2 * __builtin_amdgcn_rcpf(Pr.r2),
                        Te0 = Te1 * __builtin_amdgcn_rcpf(Pr.r1);
            float Tc = q == 3 ? Te3 : (q == 2 ? Te2 : (q == 1 ? Te1 : Te0));
            T = Te0 * __builtin_amdgcn_rcpf(Pr.r0);
#pragma unroll
            for (int r = 3; r >= 0; --r) {
                const float tk = Tc * iv[kb][r];
                Tk[kb][r] = tk;
                wv[kb][r] = on[kb][r] ? al[kb][r] * tk : 0.0f;
                Tc = on[kb][r] ? tk : Tc;
            }
        }
        __syncthreads();
        build_masks(2, 2);
        __syncthreads();
        float sw8[8], swsc[8];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * kb + 4 * q + r;
                sw8[4 * kb + r] = sg[kb][r] * wv[kb][r];
                swsc[4 * kb + r] = sw8[4 * kb + r] * sinv[k];
            }
        // y_k = R . fh_k + sum_{i > k, i in chunk} sigma_i w_i fh_i . fh_k
        bf16x8 sh, sl;
        split8(sw8, sh, sl);
        f32x4 yw[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        masked(2, sh, sl, yw);
        f32x4 ya[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        contract_acc(R, ya);
        // A_k = sum_{i > k} sigma_i w_i: suffix over the chunk's positions
        // (index order kb, q, r) plus the later chunks'
        float ls[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            ls[kb] = ((sw8[4 * kb + 3] + sw8[4 * kb + 2]) + sw8[4 * kb + 1]) + sw8[4 * kb];
        float hk[2][4];
        float baseA = Asuf;
#pragma unroll
        for (int kb = 1; kb >= 0; --kb) {
            const Rows4 LS = rows4(ls[kb]);
            const float as3 = 0.0f, as2 = LS.r3, as1 = LS.r3 + LS.r2, as0 = (LS.r3 + LS.r2) + LS.r1;
            float cs2 = baseA + (q == 3 ? as3 : (q == 2 ? as2 : (q == 1 ? as1 : as0)));
#pragma unroll
            for (int r = 3; r >= 0; --r) {
                const int k = 16 * kb + 4 * q + r;
                const float yk = ya[kb][r] * sinv[k] + yw[kb][r];
                hk[kb][r] = ca * sg[kb][r] + cb * ((ck[kb][r] + cs2) - yk);
                cs2 += sw8[4 * kb + r];                       // A_{k-1} = A_k + sigma_k w_k
            }
            baseA += as0 + LS.r0;
        }
        Asuf = baseA;
        // adjoint through w: dL/dalpha_k = T_k h_k - S_k / (1 - alpha_k),
        // S_k = sum_{i > k} w_i h_i
        float lh[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            lh[kb] = ((wv[kb][3] * hk[kb][3] + wv[kb][2] * hk[kb][2]) + wv[kb][1] * hk[kb][1]) + wv[kb][0] * hk[kb][0];
        float baseS = Ssuf;
        const int n = w * TILE + xi;
#pragma unroll
        for (int kb = 1; kb >= 0; --kb) {
            const Rows4 LH = rows4(lh[kb]);
            const float ah3 = 0.0f, ah2 = LH.r3, ah1 = LH.r3 + LH.r2, ah0 = (LH.r3 + LH.r2) + LH.r1;
            float Sc = baseS + (q == 3 ? ah3 : (q == 2 ? ah2 : (q == 1 ? ah1 : ah0)));
#pragma unroll
            for (int r = 3; r >= 0; --r) {
                const int k = 16 * kb + 4 * q + r;
                const float dalpha = Tk[kb][r] * hk[kb][r] - Sc * iv[kb][r];
                const float dpow = (on[kb][r] && al[kb][r] < ALPHA_MAX) ? dalpha * al[kb][r] : 0.0f;
                sdp[n * NSK + k] = dpow;
                Sc += wv[kb][r] * hk[kb][r];
            }
            baseS += ah0 + LH.r0;
        }
        Ssuf = baseS;
        // the suffix accumulator: R += sum sigma w fh
        {
            bf16x8 ah, alo;
            split8(swsc, ah, alo);
            accumulate(R, ah, alo);
        }
        __syncthreads();
        // Gaussian-parallel sums over this part's rows: wave w = row w, lane
        // = position k (lanes 32..63 the row's right half), moments of
        // dL/dpower along the row as in the gradient kernel
        if constexpr (!SURF) {
            const int k = lane & 31, hp = lane >> 5;
            const Rec rc = lds_rec<NRG>(srec, k);
            const float ex = rc.r1.x, ey = rc.r1.y, q1 = rc.r1.z, q2 = rc.r1.w;
            const float dy = (((float)(ty * TILE + ry) + 0.5f) - rc.r0.y) - rc.r0.w;
            const float dx0 = (((float)(tx * TILE + 8 * hp) + 0.5f) - rc.r0.x) - rc.r0.z;
            float s0 = 0.0f, sx = 0.0f, sxx = 0.0f;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const float dp = sdp[(w * TILE + 8 * hp + m) * NSK + k];
                const float dx = dx0 + (float)m;
                const float pdx = dp * dx;
                s0 += dp;
                sx += pdx;
                sxx = __builtin_fmaf(pdx, dx, sxx);
            }
            const float A = q1 * ex * ex + q2 * ey * ey, B = (q1 - q2) * ex * ey, C = q1 * ey * ey + q2 * ex * ex;
            const float sy = dy * s0;
            float qv[6];
            qv[0] = -2.0f * LN2 * (A * sx + B * sy);
            qv[1] = -2.0f * LN2 * (B * sx + C * sy);
            qv[2] = -0.5f * sxx;
            qv[3] = -dy * sx;
            qv[4] = -0.5f * dy * sy;
            qv[5] = s0;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const auto hv = __builtin_amdgcn_permlane32_swap(__float_as_uint(qv[m]), __float_as_uint(qv[m]),
                                                                 false, false);
                qv[m] = __uint_as_float(hv[0]) + __uint_as_float(hv[1]);
                if (lane < 32) sred[(w * 6 + m) * NK + k] = qv[m];
            }
        } else {
            // surfel: per pixel l = dL/dk = dp (-u/k2, -v/k2, (u^2 + v^2)/k2)
            // from the staged record, summed with l dx along the row (dy fixed)
            const int k = lane & 31, hp = lane >> 5;
            const SRec rc = lds_prec<true, NRG>(srec, k);
            const float dy = (((float)(ty * TILE + ry) + 0.5f) - rc.r0.y) - rc.r0.w;
            float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f, L0x = 0.0f, L1x = 0.0f, L2x = 0.0f, s0 = 0.0f;
#pragma unroll 2
            for (int m = 0; m < 8; ++m) {
                const float dp = sdp[(w * TILE + 8 * hp + m) * NSK + k];
                const float dx = (((float)(tx * TILE + 8 * hp + m) + 0.5f) - rc.r0.x) - rc.r0.z;
                const SurfPlane sp = surfel_plane(rc, dx, dy);
                const float pk = dp * sp.ik2;
                const float l0 = -(pk * sp.u), l1 = -(pk * sp.v);
                const float l2 = pk * __builtin_fmaf(sp.u, sp.u, sp.v * sp.v);
                L0 += l0;
                L1 += l1;
                L2 += l2;
                L0x = __builtin_fmaf(l0, dx, L0x);
                L1x = __builtin_fmaf(l1, dx, L1x);
                L2x = __builtin_fmaf(l2, dx, L2x);
                s0 += dp;
            }
            const float a0 = rc.r1.x, a1 = rc.r1.y, b0 = rc.r1.z, b1 = rc.r1.w, e1 = rc.r3.y, e2 = rc.r3.z;
            float qv[10];
            qv[0] = __builtin_fmaf(-b1, L0, __builtin_fmaf(b0, L1, e2 * L2));
            qv[1] = __builtin_fmaf(a1, L0, __builtin_fmaf(-a0, L1, e1 * L2));
            qv[2] = dy * L1;
            qv[3] = -dy * L0;
            qv[4] = -L1x;
            qv[5] = L0x;
            qv[6] = L2;
            qv[7] = -dy * L2;
            qv[8] = -L2x;
            qv[9] = s0;
#pragma unroll
            for (int m = 0; m < 10; ++m) {
                const auto hv = __builtin_amdgcn_permlane32_swap(__float_as_uint(qv[m]), __float_as_uint(qv[m]),
                                                                 false, false);
                qv[m] = __uint_as_float(hv[0]) + __uint_as_float(hv[1]);
                if (lane < 32) sred[(w * 10 + m) * NK + k] = qv[m];
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < NQN * NK) {
            const int k = threadIdx.x % NK, m = threadIdx.x / NK;
            float sum = 0.0f;
#pragma unroll
            for (int ww = 0; ww < ROWS; ++ww) sum += sred[(ww * NQN + m) * NK + k];
            if (k < cnt) a.part[(((int64_t)voff + cs + k) * NDFD_PARTS + half) * NDP + m] = sum;
        }
    }
}

// part_geom[v][m] += part[v][0][m] + ... + part[v][nparts - 1][m] for the
// screen-space terms of every visited instance (fixed order): six for a
// Gaussian (rows of 12), ten for a surfel (rows of 16), the first entries of
// the gradient kernel's partial row in both.
template <bool SURF>
__global__ __launch_bounds__(256) void k_ndfd_combine(const float* __restrict__ part, float* __restrict__ part_geom,
                                                      const Counters* c, int64_t cap, int nparts) {
    constexpr int NQN = NdfdPart<SURF>::NQ, NDP = NdfdPart<SURF>::W, GP = PrimRec<SURF>::GP;
    if (c->inst_overflow || c->visit_overflow) return;
    const int64_t nv = (int64_t)c->n_visited < cap ? (int64_t)c->n_visited : cap;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nv * NQN) return;
    const int64_t vi = i / NQN;
    const int m = (int)(i % NQN);
    float s = 0.0f;
    for (int h = 0; h < nparts; ++h) s += part[(vi * NDFD_PARTS + h) * NDP + m];
    part_geom[vi * GP + m] += s;
}

template <int D, bool SURF>
static void launch_ndfd_d(const NdfdArgs& a, const ViewTable& vt, int n_tiles, bool grad, hipStream_t s) {
    constexpr int ROWS = 8;
    const size_t lds = sizeof(__bf16) * ((size_t)NK * (D + 8) + (size_t)D * NJP + 6 * (size_t)NK * NJP) +
                       sizeof(float) * ((size_t)NK * (NK + 1) + NK + (size_t)TILE * ROWS * NSK +
                                        (size_t)ROWS * NdfdPart<SURF>::NQ * NK);
    if (grad)
        hipLaunchKernelGGL((k_ndfd<D, true, SURF>), dim3(n_tiles, TILE / ROWS), dim3(64 * ROWS), lds, s, a, vt);
    else
        hipLaunchKernelGGL((k_ndfd<D, false, SURF>), dim3(n_tiles, TILE / ROWS), dim3(64 * ROWS), lds, s, a, vt);
}

template <bool SURF>
static void launch_ndfd_p(const NdfdArgs& a, const ViewTable& vt, int n_tiles, bool grad, hipStream_t s) {
    switch (a.d) {
        case 32: launch_ndfd_d<32, SURF>(a, vt, n_tiles, grad, s); break;
        case 64: launch_ndfd_d<64, SURF>(a, vt, n_tiles, grad, s); break;
        case 96: launch_ndfd_d<96, SURF>(a, vt, n_tiles, grad, s); break;
        case 128: launch_ndfd_d<128, SURF>(a, vt, n_tiles, grad, s); break;
        default: launch_ndfd_d<256, SURF>(a, vt, n_tiles, grad, s); break;
    }
}

bool ndfd_supported(int d) { return d == 32 || d == 64 || d == 96 || d == 128 || d == 256; }

void launch_ndfd(const NdfdArgs& a, const ViewTable& vt, int n_tiles, bool grad, hipStream_t s) {
    if (n_tiles <= 0) return;
    if (a.prim == FH_PRIM_SURFEL)
        launch_ndfd_p<true>(a, vt, n_tiles, grad, s);
    else
        launch_ndfd_p<false>(a, vt, n_tiles, grad, s);
}

int ndfd_part_floats(int prim) { return prim == FH_PRIM_SURFEL ? NdfdPart<true>::W : NdfdPart<false>::W; }

void launch_ndfd_combine(const float* part, float* part_geom, const Counters* c, int64_t cap, int prim,
                         hipStream_t s) {
    const bool surf = prim == FH_PRIM_SURFEL;
    const int64_t n = cap * (surf ? NdfdPart<true>::NQ : NdfdPart<false>::NQ);
    if (n <= 0) return;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (surf)
        hipLaunchKernelGGL(k_ndfd_combine<true>, grid, dim3(256), 0, s, part, part_geom, c, cap, NDFD_PARTS);
    else
        hipLaunchKernelGGL(k_ndfd_combine<false>, grid, dim3(256), 0, s, part, part_geom, c, cap, NDFD_PARTS);
}

}  // namespace fh
