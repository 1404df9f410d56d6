// Adjoint and feature fusion of the compositing pass with BF16 features on
// MFMA (gfx950).
//
// Gradient kernel, per tile, back to front over the tile's visited list in
// chunks of 32 Gaussians (Appendix A.2: dL/dalpha_k = T_k g_k - (S_k + T_final
// dT)/(1 - alpha_k), S_k = sum_{i>k} w_i g_i, g_k = rgb_k . dC + f_k . dF):
//   1. the feature part of g for all (pixel, Gaussian) pairs of the chunk is
//      one MFMA contraction G^T[k x px] = Feat[k x D] . dF^T[D x px]; its result
//      lands in exactly the lanes that walk those (pixel, Gaussian) pairs;
//   2. each pixel's four lanes walk four consecutive positions each; the
//      back-to-front transmittance division and the suffix sum S are combined
//      across the lanes with a scan of (product of (1 - alpha), sum of w g
//      relative to the entry transmittance) pairs;
//   3. w and dL/dpower per (Gaussian, pixel) go to LDS, and a Gaussian-parallel
//      pass sums the ten screen-space adjoint terms over the tile's pixels
//      (fixed order) into one partial per instance: no atomics.
// dF enters the contraction as two BF16 terms, hi = bf16(dF), lo = bf16(dF - hi)
// (about 16 significant bits), both resident in registers for the whole tile.
//
// Fusion kernel: the same back-to-front walk needs only w = alpha T; the
// per-instance partial sum_p w(p) target(p) is the MFMA contraction
// W^T[k x px] . Target[px x D] with W split into BF16 hi + lo and the tile's
// target held in registers for the whole tile.  Kept apart from the gradient
// kernel so that each keeps its own per-tile operand (dF or the target)
// resident without spilling; when both run, the per-instance weight sums come
// from the gradient kernel alone.
//
// SURF: the surfel primitive (Section 3.1): four-float4 records, alpha at the
// ray-plane intersection, and 14 screen-space terms per instance (the nine
// record entries', sum dL/dpower, rgb, sum w) in rows of 16 floats.
#include "kernels.hpp"

namespace fh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;   // positions per chunk
// padded per-pixel stride of the (pixel, position) LDS arrays: the walk's stores
// (lane (xi, q) at 35 xi + 4 q + r) hit each bank at most 3 times, the
// Gaussian-parallel reads (consecutive positions per lane) twice
constexpr int SK = BK + 3;
constexpr int RG = 4;        // record padding group: the walk's lane rows read records 4 apart
// Row padding (bf16) of the LDS tiles that MFMA operands are read from as
// 16-byte rows, lane (xi, q) at row xi, column 8 q: rows of D + 16 (or 256 +
// 16) bf16 start an odd multiple of 8 dwords apart, so that the lanes served
// together (xi = 0..7 of two adjacent q) fall in distinct banks; with 8 bf16
// of padding (rows an odd multiple of 4 dwords apart) they meet in pairs,
// which measures 1.8x slower on this read pattern.
constexpr int OPAD = 16;
// float4 slots of one chunk's staged records
template <bool SURF>
constexpr int rslots() {
    return PrimRec<SURF>::RW * BK + BK / RG;
}

// Stage the chunk's records (threads 0..31) from the visit-ordered copies;
// padding records never blend.
template <bool SURF>
__device__ __forceinline__ void stage_records(const BwdArgs& a, uint32_t voff, int cs, int cnt, float4* srec,
                                              uint32_t* sg) {
    if (threadIdx.x < BK) {
        typename PrimRec<SURF>::T r;
        if ((int)threadIdx.x < cnt) {
            const int64_t vi = (int64_t)voff + cs + threadIdx.x;
            r = load_rec<SURF>(a.vrec, vi);
            if (sg) sg[threadIdx.x] = a.vgid[vi];
        } else {
            r = pad_rec<SURF>();
            if (sg) sg[threadIdx.x] = 0xFFFFFFFFu;
        }
        lds_put_prec<SURF, RG>(srec, threadIdx.x, r);
    }
}

// One chunk record (position cs + k of the tile's list, or padding past cnt).
template <bool SURF>
__device__ __forceinline__ typename PrimRec<SURF>::T fetch_record(const BwdArgs& a, uint32_t voff, int cs, int cnt,
                                                                  int k) {
    if (k < cnt) return load_rec<SURF>(a.vrec, (int64_t)voff + cs + k);
    return pad_rec<SURF>();
}

// ---------------------------------------------------------------------------
// Gradient kernel.  512 threads (8 waves; 256 VGPRs per lane so that dF (hi and
// lo) stays resident); wave w owns pixel rows 2w and 2w + 1; lane (xi, q) = pixel x = xi
// of both rows, positions 4q..4q+3 of each 16-position half-chunk.
// SL: one channel slice of a wider feature (rows of stride a.d from channel
// a.d0; a.g_in adds the earlier slices' part of f . dF)
template <int D, bool SL, bool SURF>
__global__ __launch_bounds__(512) void k_render_bwd_bf16(BwdArgs a, ViewTable vt) {
    using RecT = typename PrimRec<SURF>::T;
    constexpr int RW = PrimRec<SURF>::RW, NQ = PrimRec<SURF>::NQ, GP = PrimRec<SURF>::GP;
    constexpr int RSLOTS = rslots<SURF>();
    const int dstride = SL ? a.d : D, dofs = SL ? a.d0 : 0;
    constexpr int DP = D + OPAD;         // padded row stride (bf16) of the feature chunk
    constexpr int NS = D / 32;           // MFMA steps over channels
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16* sfeat2 = reinterpret_cast<__bf16*>(smem);                        // [2][BK][DP], double-buffered
    // per (pixel, position) values, pixel-major with a padded stride SK so that
    // the walk's stores and the Gaussian-parallel reads spread over the banks
    float* sw = reinterpret_cast<float*>(sfeat2 + 2 * BK * DP);              // [256][SK] w
    float* sdp = sw + TILE_PIX * SK;                                         // [256][SK] dL/dpower
    float* sdc = sdp + TILE_PIX * SK;                                        // [256][3] dC of the tile
    float* sred = sdc + 3 * TILE_PIX;                                        // [8 waves][NQ][BK] partial sums
    __shared__ float4 srecb[3][RSLOTS];   // chunk records and Gaussians, triple-buffered:
    __shared__ uint32_t sgb[3][BK];       // those two chunks ahead arrive during this one

    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = a.tile_order ? (int)a.tile_order[blockIdx.x] : (int)blockIdx.x;
    const uint32_t nt = a.tile_niter[t];
    if (nt == 0) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, xi = lane & 15;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const uint32_t voff = a.tile_voff[t];
    const uint16_t* feat = static_cast<const uint16_t*>(a.feat);
    const bool has_df = a.dF != nullptr;
    const float LN2 = 0.69314718055994531f;
    const int px = tx * TILE + xi;
    const float x = (float)px + 0.5f;

    // per-pixel state of this lane's two pixels (identical in the pixel's four lanes)
    float T[2], S[2], TdT[2], dCp[2][3];     // TdT = T_final dT
    uint32_t nit[2];
    bf16x8 dfh[2][NS], dfl[2][NS];     // dF = hi + lo, both BF16
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int py = ty * TILE + 2 * w + h;
        const bool inside = px < W && py < H;
        const int64_t p = vt.pix_off[v] + (int64_t)py * W + px;
        nit[h] = inside ? a.n_iter[p] : 0u;
        T[h] = inside ? a.T_final[p] : 1.0f;
        S[h] = 0.0f;
        dCp[h][0] = dCp[h][1] = dCp[h][2] = 0.0f;
        if (inside && a.dC) {
            dCp[h][0] = a.dC[3 * p];
            dCp[h][1] = a.dC[3 * p + 1];
            dCp[h][2] = a.dC[3 * p + 2];
        }
        TdT[h] = T[h] * ((inside && a.dT) ? a.dT[p] : 0.0f);
        if (q == 0) {
            const int n = (2 * w + h) * TILE + xi;
            sdc[3 * n] = dCp[h][0];
            sdc[3 * n + 1] = dCp[h][1];
            sdc[3 * n + 2] = dCp[h][2];
        }
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            float vals[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) vals[m] = 0.0f;
            if (has_df && inside) {
                const float4* src = reinterpret_cast<const float4*>(a.dF + p * dstride + dofs + 32 * st + 8 * q);
                const float4 lo4 = src[0], hi4 = src[1];
                vals[0] = lo4.x; vals[1] = lo4.y; vals[2] = lo4.z; vals[3] = lo4.w;
                vals[4] = hi4.x; vals[5] = hi4.y; vals[6] = hi4.z; vals[7] = hi4.w;
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const __bf16 hb = (__bf16)vals[m];
                dfh[h][st][m] = hb;
                dfl[h][st][m] = (__bf16)(vals[m] - (float)hb);
            }
        }
    }

    // all of a thread's feature rows of one chunk are requested before any is
    // stored; a padding position reads Gaussian 0 (its contraction row is only
    // used by positions that blend, which it never does)
    constexpr int ITEMS = BK * (D / 8), NI = (ITEMS + 511) / 512;
    auto load_feats = [&](const uint32_t* gl, uint4* raw) {
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const int idx = threadIdx.x + 512 * it;
            raw[it] = make_uint4(0, 0, 0, 0);
            if (idx < ITEMS) {
                const int k = idx / (D / 8), dg = idx % (D / 8);
                const uint32_t g = gl[k];
                const uint32_t ga = g != 0xFFFFFFFFu ? g : 0u;
                raw[it] = *reinterpret_cast<const uint4*>(feat + (int64_t)ga * dstride + dofs + dg * 8);
            }
        }
    };
    auto store_feats = [&](const uint4* raw, __bf16* dst) {
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const int idx = threadIdx.x + 512 * it;
            if (idx < ITEMS) {
                const int k = idx / (D / 8), dg = idx % (D / 8);
                *reinterpret_cast<uint4*>(&dst[k * DP + dg * 8]) = raw[it];
            }
        }
    };

    // prologue: records and Gaussians of the first two chunks, features of the first
    {
        const int cs0 = (int)nt - BK > 0 ? (int)nt - BK : 0;
        stage_records<SURF>(a, voff, cs0, (int)nt - cs0, srecb[0], sgb[0]);
        if (cs0 > 0) {
            const int cs1 = cs0 - BK > 0 ? cs0 - BK : 0;
            stage_records<SURF>(a, voff, cs1, cs0 - cs1, srecb[1], sgb[1]);
        }
    }
    __syncthreads();
    if (has_df) {
        uint4 raw[NI];
        load_feats(sgb[0], raw);
        store_feats(raw, sfeat2);
    }
    __syncthreads();
    int b3 = 0, f2 = 0;   // this chunk's record buffer (mod 3) and feature buffer (mod 2)
    for (int ce = (int)nt; ce > 0; ce -= BK) {
        const int cs = ce - BK > 0 ? ce - BK : 0;
        const int cnt = ce - cs;
        const int n3 = b3 == 2 ? 0 : b3 + 1, nn3 = n3 == 2 ? 0 : n3 + 1;
        const float4* srec = srecb[b3];
        const __bf16* sfeat = sfeat2 + f2 * BK * DP;
        // records (RD = 4 RW dwords each, threads 0..RD BK-1) and Gaussians
        // (threads RD BK..RD BK+BK-1, or for surfels, whose records take all
        // 512 threads, a second load of threads 0..BK-1) of the chunk after
        // next: one dword per load, stored after this chunk's walk; padding
        // positions get the padding record.  (Positions nncs .. nncs + BK - 1
        // all lie in this tile's visits: that chunk exists only when this one
        // and the next are full.)
        constexpr int RD = 4 * RW;
        const int ncs = cs - BK > 0 ? cs - BK : 0;
        const int nncs = ncs - BK > 0 ? ncs - BK : 0;
        const int nncnt = ncs - nncs;
        const bool pre_on = ncs > 0 && threadIdx.x < (SURF ? RD * BK : (RD + 1) * BK);
        const bool pre_g = !SURF && threadIdx.x >= RD * BK;
        const int pre_k = pre_g ? (int)threadIdx.x - RD * BK : (int)threadIdx.x / RD;
        uint32_t pre = 0u, pre_gid = 0u;
        if (pre_on) {
            const uint32_t* src = pre_g ? a.vgid + ((int64_t)voff + nncs)
                                        : reinterpret_cast<const uint32_t*>(a.vrec) + ((int64_t)voff + nncs) * RD;
            pre = src[pre_g ? pre_k : (int)threadIdx.x];
            if (SURF && threadIdx.x < BK) pre_gid = a.vgid[(int64_t)voff + nncs + threadIdx.x];
        }
        // the next chunk's features, stored after this chunk's walk
        uint4 fnext[NI];
        const bool fnext_on = has_df && cs > 0;
        if (fnext_on) load_feats(sgb[n3], fnext);

#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // keep the two rows' LDS reads apart (no hoisting of the chunk records
            // across the unrolled rows, which would pin them in registers)
            asm volatile("" ::: "memory");
            const float y = (float)(ty * TILE + 2 * w + h) + 0.5f;
            const int n = (2 * w + h) * TILE + xi;
            // 1. G^T[k][px] = f_k . dF(px): lane gets k = 16 kb + 4 q + r for its pixel
            // (the two half-chunks' accumulations are interleaved: two
            // independent MFMA chains instead of one chain twice as long)
            f32x4 gk[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
            if (has_df) {
#pragma unroll
                for (int st = 0; st < NS; ++st) {
                    const bf16x8 fa0 = *reinterpret_cast<const bf16x8*>(&sfeat[xi * DP + 32 * st + 8 * q]);
                    const bf16x8 fa1 = *reinterpret_cast<const bf16x8*>(&sfeat[(16 + xi) * DP + 32 * st + 8 * q]);
                    gk[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, dfh[h][st], gk[0], 0, 0, 0);
                    gk[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, dfh[h][st], gk[1], 0, 0, 0);
                    gk[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, dfl[h][st], gk[0], 0, 0, 0);
                    gk[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, dfl[h][st], gk[1], 0, 0, 0);
                }
            }
            // 2. back to front: half-chunk kb = 1 (positions 16..31), then kb = 0
#pragma unroll
            for (int kb = 1; kb >= 0; --kb) {
                asm volatile("" ::: "memory");
                float al[4], gg[4], iv[4];   // iv = 1 / (1 - alpha), by the hardware reciprocal
                bool on[4];
                float P = 1.0f, R = 0.0f, trel = 1.0f;
#pragma unroll
                for (int r = 3; r >= 0; --r) {
                    const int k = 16 * kb + 4 * q + r;
                    // (slot of k = 16 kb + 4 q + r: (16 RW + 4) kb + (4 RW + 1) q + RW r)
                    const float4* rp = srec + (4 * RW + 1) * q + (16 * RW + 4) * kb + RW * r;
                    RecT rc;
                    rc.r0 = rp[0];
                    rc.r1 = rp[1];
                    rc.r2 = rp[2];
                    if constexpr (SURF) rc.r3 = rp[3];
                    const float alpha = prim_alpha<SURF>(rc, x, y);
                    on[r] = k < cnt && (uint32_t)(cs + k) < nit[h] && alpha >= ALPHA_MIN;
                    al[r] = alpha;
                    gg[r] = rc.r2.y * dCp[h][0] + rc.r2.z * dCp[h][1] + rc.r2.w * dCp[h][2] + gk[kb][r];
                    // the earlier channel slices' part of f_k . dF (positions of the chunk only)
                    if (SL && a.g_in && k < cnt) gg[r] += a.g_in[((int64_t)voff + cs + k) * TILE_PIX + n];
                    iv[r] = __builtin_amdgcn_rcpf(1.0f - al[r]);
                    // (branch-free: a position that does not blend leaves the state as is)
                    const float tn = trel * iv[r];
                    R = on[r] ? __builtin_fmaf(al[r] * tn, gg[r], R) : R;
                    P = on[r] ? P * (1.0f - al[r]) : P;
                    trel = on[r] ? tn : trel;
                }
                // entry state of every lane, scanning from the back (lane q = 3 first)
                const Rows4 Pr = rows4(P), Rr = rows4(R);
                const float P0 = Pr.r0, P1 = Pr.r1, P2 = Pr.r2, P3 = Pr.r3;
                const float R0 = Rr.r0, R1 = Rr.r1, R2 = Rr.r2, R3 = Rr.r3;
                const float Te3 = T[h], Se3 = S[h];
                const float Te2 = Te3 * __builtin_amdgcn_rcpf(P3), Se2 = Se3 + Te3 * R3;
                const float Te1 = Te2 * __builtin_amdgcn_rcpf(P2), Se1 = Se2 + Te2 * R2;
                const float Te0 = Te1 * __builtin_amdgcn_rcpf(P1), Se0 = Se1 + Te1 * R1;
                float Tc = q == 3 ? Te3 : (q == 2 ? Te2 : (q == 1 ? Te1 : Te0));
                float Sc = q == 3 ? Se3 : (q == 2 ? Se2 : (q == 1 ? Se1 : Se0));
                T[h] = Te0 * __builtin_amdgcn_rcpf(P0);
                S[h] = Se0 + Te0 * R0;
#pragma unroll
                for (int r = 3; r >= 0; --r) {
                    const int k = 16 * kb + 4 * q + r;
                    const float inv = iv[r];
                    const float Tk = Tc * inv;
                    const float wb = al[r] * Tk;
                    const float dalpha = Tk * gg[r] - (Sc + TdT[h]) * inv;
                    const float wv = on[r] ? wb : 0.0f;
                    // alpha < ALPHA_MAX exactly when o G was not clamped
                    const float dpow = (on[r] && al[r] < ALPHA_MAX) ? dalpha * al[r] : 0.0f;
                    Sc = on[r] ? __builtin_fmaf(wb, gg[r], Sc) : Sc;
                    Tc = on[r] ? Tk : Tc;
                    sw[n * SK + k] = wv;
                    sdp[n * SK + k] = dpow;
                }
            }
        }
        // the next chunk's records and Gaussians go to the other buffer now,
        // before this chunk's partial stores are issued (a wait for the
        // prefetch placed after them would also wait for the stores)
        if (pre_on) {
            // padding dwords: the padding record (opacity 0; a Gaussian's unit
            // eigenframe, a surfel's D = 1) and no Gaussian
            const int j = (int)threadIdx.x % RD;
            const uint32_t pad = pre_g ? 0xFFFFFFFFu
                                 : SURF ? (j == 12 ? 0x3f800000u : 0u)
                                        : (j == 4 ? 0x3f800000u : ((j == 6 || j == 7) ? 0xbf800000u : 0u));
            const uint32_t val = pre_k < nncnt ? pre : pad;
            if (pre_g)
                sgb[nn3][pre_k] = val;
            else
                reinterpret_cast<uint32_t*>(srecb[nn3])[4 * prec_slot<SURF, RG>(pre_k) + j] = val;
            if (SURF && threadIdx.x < BK)
                sgb[nn3][threadIdx.x] = (int)threadIdx.x < nncnt ? pre_gid : 0xFFFFFFFFu;
        }
        if (fnext_on) store_feats(fnext, sfeat2 + (f2 ^ 1) * BK * DP);
        __syncthreads();

        // 3. Gaussian-parallel sums over the tile's pixels: lane = position k
        //    (consecutive lanes read consecutive addresses), each half-wave one
        //    pixel row; then the 16 rows are added in a fixed order (the two of
        //    a wave, then the waves in order).  The screen-space terms are
        //    moments of dL/dpower over the row: with a = e.d and b = e x d
        //    linear in d = (dx, dy), and dy fixed along a row,
        //      sum dp (q1 a e_x - q2 b e_y) = A Sx + B dy S0,
        //      sum dp (q1 a e_y + q2 b e_x) = B Sx + C dy S0,
        //    A = q1 e_x^2 + q2 e_y^2, B = (q1 - q2) e_x e_y, C = q1 e_y^2 + q2 e_x^2,
        //    S0 = sum dp, Sx = sum dp dx, Sxx = sum dp dx^2.
        if constexpr (!SURF) {
            const int k = lane & 31, pg = 2 * w + (lane >> 5);
            const Rec rc = lds_rec<RG>(srec, k);
            const float ex = rc.r1.x, ey = rc.r1.y, q1 = rc.r1.z, q2 = rc.r1.w;
            const float dy = (((float)(ty * TILE + pg) + 0.5f) - rc.r0.y) - rc.r0.w;
            const float dx0 = (((float)(tx * TILE) + 0.5f) - rc.r0.x) - rc.r0.z;
            float s0 = 0.0f, sx = 0.0f, sxx = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, ws = 0.0f;
#pragma unroll 4
            for (int m = 0; m < 16; ++m) {
                const int n = pg * 16 + m;
                const float dp = sdp[n * SK + k], wv = sw[n * SK + k];
                const float dx = dx0 + (float)m;
                const float pdx = dp * dx;
                s0 += dp;
                sx += pdx;
                sxx = __builtin_fmaf(pdx, dx, sxx);
                c0 = __builtin_fmaf(wv, sdc[3 * n], c0);
                c1 = __builtin_fmaf(wv, sdc[3 * n + 1], c1);
                c2 = __builtin_fmaf(wv, sdc[3 * n + 2], c2);
                ws += wv;
            }
            const float A = q1 * ex * ex + q2 * ey * ey, B = (q1 - q2) * ex * ey, C = q1 * ey * ey + q2 * ex * ex;
            const float sy = dy * s0;
            float qv[10];
            qv[0] = -2.0f * LN2 * (A * sx + B * sy);
            qv[1] = -2.0f * LN2 * (B * sx + C * sy);
            qv[2] = -0.5f * sxx;
            qv[3] = -dy * sx;
            qv[4] = -0.5f * dy * sy;
            qv[5] = s0;
            qv[6] = c0;
            qv[7] = c1;
            qv[8] = c2;
            qv[9] = ws;
#pragma unroll
            for (int m = 0; m < 10; ++m) {
                // (the two half-waves' values, added in the same order in both halves)
                const auto hv = __builtin_amdgcn_permlane32_swap(__float_as_uint(qv[m]), __float_as_uint(qv[m]),
                                                                 false, false);
                qv[m] = __uint_as_float(hv[0]) + __uint_as_float(hv[1]);
                if (lane < 32) sred[(w * 10 + m) * BK + k] = qv[m];
            }
        } else {
            // Surfel: dL/dk = dp (-u/k2, -v/k2, (u^2 + v^2)/k2) = (l0, l1, l2) per
            // pixel (the intersection recomputed from the record, as in the
            // walk); the nine record terms are linear in l with coefficients
            // from the record and (dx, dy), so along a row (dy fixed) they need
            // the sums of l and of l dx:
            //   dx_c: -b1 L0 + b0 L1 + e2 L2,  dy_c: a1 L0 - a0 L1 + e1 L2,
            //   a0: dy L1, a1: -dy L0, b0: -L1x, b1: L0x, D: L2, e1: -dy L2, e2: -L2x.
            const int k = lane & 31, pg = 2 * w + (lane >> 5);
            const SRec rc = lds_prec<true, RG>(srec, k);
            const float dy = (((float)(ty * TILE + pg) + 0.5f) - rc.r0.y) - rc.r0.w;
            float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f, L0x = 0.0f, L1x = 0.0f, L2x = 0.0f;
            float s0 = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, ws = 0.0f;
#pragma unroll 2
            for (int m = 0; m < 16; ++m) {
                const int n = pg * 16 + m;
                const float dp = sdp[n * SK + k], wv = sw[n * SK + k];
                const float dx = (((float)(tx * TILE + m) + 0.5f) - rc.r0.x) - rc.r0.z;
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
                c0 = __builtin_fmaf(wv, sdc[3 * n], c0);
                c1 = __builtin_fmaf(wv, sdc[3 * n + 1], c1);
                c2 = __builtin_fmaf(wv, sdc[3 * n + 2], c2);
                ws += wv;
            }
            const float a0 = rc.r1.x, a1 = rc.r1.y, b0 = rc.r1.z, b1 = rc.r1.w, e1 = rc.r3.y, e2 = rc.r3.z;
            float qv[14];
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
            qv[10] = c0;
            qv[11] = c1;
            qv[12] = c2;
            qv[13] = ws;
#pragma unroll
            for (int m = 0; m < 14; ++m) {
                const auto hv = __builtin_amdgcn_permlane32_swap(__float_as_uint(qv[m]), __float_as_uint(qv[m]),
                                                                 false, false);
                qv[m] = __uint_as_float(hv[0]) + __uint_as_float(hv[1]);
                if (lane < 32) sred[(w * 14 + m) * BK + k] = qv[m];
            }
        }
        // w of the chunk, recorded for the fusion kernel of the same call as
        // W^T [position][pixel]: consecutive lanes store consecutive pixels
        // (and read LDS at the odd stride SK: no bank conflicts)
        if (a.wrec) {
            float* dst = a.wrec + ((int64_t)voff + cs) * TILE_PIX;
            // (the thread index is made opaque here so that the addresses are
            // not hoisted out of the chunk loop into registers held across the walk)
            int tid = (int)threadIdx.x;
            asm volatile("" : "+v"(tid));
#pragma unroll 4
            for (int j = 0; j < BK * TILE_PIX / 512; ++j) {
                const int e = tid + 512 * j, k = e >> 8, n = e & 255;
                if (k < cnt) dst[e] = sw[n * SK + k];
            }
        }
        __syncthreads();
        if (threadIdx.x < GP * BK) {
            // terms NQ..GP-1 of a partial are padding: written as zero
            const int k = threadIdx.x % BK, m = threadIdx.x / BK;
            float sum = 0.0f;
            if (m < NQ) {
#pragma unroll
                for (int ww = 0; ww < 8; ++ww) sum += sred[(ww * NQ + m) * BK + k];
            }
            if (k < cnt) a.part_geom[((int64_t)voff + cs + k) * GP + m] = sum;
        }
        // No barrier here: the next chunk's LDS writes before its first
        // barrier (w and dL/dpower, the chunk after next's records and
        // Gaussians, the next features) go to arrays whose last readers all
        // passed the barrier above, and the partial sums (sred) are written
        // only after the next first barrier, which these threads reach last.
        b3 = n3;
        f2 ^= 1;
    }
}

// ---------------------------------------------------------------------------
// f_k . dF over one channel slice, for feature widths above 256 (whose dF does
// not fit in registers at once): the slice's dF (hi + lo) stays resident as in
// the gradient kernel, and g_out[visit][pixel] = g_in (earlier slices, when
// given) + this slice's contraction, for every visited position of the tile.
// 512 threads; wave w owns pixel rows 2w and 2w + 1; chunks of 32 positions
// front to back, the features staged in LDS.
template <int D>
__global__ __launch_bounds__(512) void k_gk_bf16(BwdArgs a, ViewTable vt) {
    constexpr int DP = D + OPAD;
    constexpr int NS = D / 32;
    __shared__ __attribute__((aligned(16))) __bf16 sfeat[BK * DP];
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = a.tile_order ? (int)a.tile_order[blockIdx.x] : (int)blockIdx.x;
    const uint32_t nt = a.tile_niter[t];
    if (nt == 0) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, xi = lane & 15;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const uint32_t voff = a.tile_voff[t];
    const uint16_t* feat = static_cast<const uint16_t*>(a.feat);
    const int px = tx * TILE + xi;
    bf16x8 dfh[2][NS], dfl[2][NS];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int py = ty * TILE + 2 * w + h;
        const bool inside = px < W && py < H;
        const int64_t p = vt.pix_off[v] + (int64_t)py * W + px;
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            float vals[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) vals[m] = 0.0f;
            if (inside) {
                const float4* src = reinterpret_cast<const float4*>(a.dF + p * a.d + a.d0 + 32 * st + 8 * q);
                const float4 lo4 = src[0], hi4 = src[1];
                vals[0] = lo4.x; vals[1] = lo4.y; vals[2] = lo4.z; vals[3] = lo4.w;
                vals[4] = hi4.x; vals[5] = hi4.y; vals[6] = hi4.z; vals[7] = hi4.w;
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const __bf16 hb = (__bf16)vals[m];
                dfh[h][st][m] = hb;
                dfl[h][st][m] = (__bf16)(vals[m] - (float)hb);
            }
        }
    }
    constexpr int ITEMS = BK * (D / 8), NI = (ITEMS + 511) / 512;
    for (int cs = 0; cs < (int)nt; cs += BK) {
        const int cnt = (int)nt - cs < BK ? (int)nt - cs : BK;
        __syncthreads();   // (the previous chunk's readers are done with sfeat)
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            const int idx = (int)threadIdx.x + 512 * it;
            if (idx < ITEMS) {
                const int k = idx / (D / 8), dg = idx % (D / 8);
                // positions past the chunk read Gaussian 0; their results are not stored
                const uint32_t g = k < cnt ? a.vgid[(int64_t)voff + cs + k] : 0u;
                *reinterpret_cast<uint4*>(&sfeat[k * DP + dg * 8]) =
                    *reinterpret_cast<const uint4*>(feat + (int64_t)g * a.d + a.d0 + dg * 8);
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n = (2 * w + h) * TILE + xi;
            f32x4 gk[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                const bf16x8 fa0 = *reinterpret_cast<const bf16x8*>(&sfeat[xi * DP + 32 * st + 8 * q]);
                const bf16x8 fa1 = *reinterpret_cast<const bf16x8*>(&sfeat[(16 + xi) * DP + 32 * st + 8 * q]);
                gk[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, dfh[h][st], gk[0], 0, 0, 0);
                gk[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, dfh[h][st], gk[1], 0, 0, 0);
                gk[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, dfl[h][st], gk[0], 0, 0, 0);
                gk[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, dfl[h][st], gk[1], 0, 0, 0);
            }
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * kb + 4 * q + r;
                    if (k < cnt) {
                        const int64_t o = ((int64_t)voff + cs + k) * TILE_PIX + n;
                        a.g_out[o] = (a.g_in ? a.g_in[o] : 0.0f) + gk[kb][r];
                    }
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Fusion kernel.  1024 threads; wave w = pixel row w; lane (xi, q) = pixel
// x = xi, positions 4q..4q+3 of each half-chunk; wave w < D/16 owns channel
// block w of the contraction and keeps that block of the tile's target in
// registers.  Writes the fusion partial row of every visited instance and,
// with WS, its weight sum (the tenth geometry partial; without WS the gradient
// kernel of the same call has written it).
template <int D, bool WS, bool SURF>
__global__ __launch_bounds__(1024) void k_fuse_bf16(BwdArgs a, ViewTable vt) {
    using RecT = typename PrimRec<SURF>::T;
    constexpr int RW = PrimRec<SURF>::RW;
    constexpr int PP = TILE_PIX + OPAD;  // padded row stride (bf16) of W^T
    constexpr int NDB = D / 16;
    // W^T and the weight sums are double-buffered by chunk parity, so that one
    // barrier per chunk suffices: a wave may walk chunk c + 1 while others
    // still contract chunk c
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16* swh2 = reinterpret_cast<__bf16*>(smem);                          // [2][BK][PP] W^T hi
    __bf16* swl2 = swh2 + 2 * BK * PP;                                       // [2][BK][PP] W^T lo
    __shared__ float swsum2[2][16][BK];   // per wave (pixel row): sum over its pixels of w, per position
    __shared__ float4 srecb[2][rslots<SURF>()];   // chunk records, double-buffered (the next chunk's fetched ahead)

    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = a.tile_order ? (int)a.tile_order[blockIdx.x] : (int)blockIdx.x;
    const uint32_t nt = a.tile_niter[t];
    if (nt == 0) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, xi = lane & 15;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const uint32_t voff = a.tile_voff[t];
    const int px = tx * TILE + xi, py = ty * TILE + w;
    const bool inside = px < W && py < H;
    const float x = (float)px + 0.5f, y = (float)py + 0.5f;
    const int64_t p = vt.pix_off[v] + (int64_t)py * W + px;
    const uint32_t nit = inside ? a.n_iter[p] : 0u;
    float T = inside ? a.T_final[p] : 1.0f;
    const int d0 = (int)blockIdx.y * D;   // channel slice (feature widths above 256)

    // target[px = 32 st + 8 q + m][16 w + xi]: B operands of this wave's block
    // (BF16 target).  All 64 loads are issued before any is used: addresses of
    // pixels outside the image are clamped into it and the values zeroed after.
    bf16x8 tgo[8];
    if (w < NDB) {
        const uint16_t* tg = static_cast<const uint16_t*>(a.target);
        u16x8 raw[8];
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int n0 = 32 * st + 8 * q;   // 8 consecutive pixels of one tile row
            const int qy = ty * TILE + (n0 >> 4), qx0 = tx * TILE + (n0 & 15);
            const int64_t row = vt.pix_off[v] + (int64_t)(qy < H ? qy : H - 1) * W;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int qx = qx0 + m < W ? qx0 + m : W - 1;
                raw[st][m] = tg[(row + qx) * a.d + d0 + 16 * w + xi];
            }
        }
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int n0 = 32 * st + 8 * q;
            const int qy = ty * TILE + (n0 >> 4), qx0 = tx * TILE + (n0 & 15);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (qy >= H || qx0 + m >= W) raw[st][m] = 0;
            tgo[st] = __builtin_bit_cast(bf16x8, raw[st]);
        }
    } else {
#pragma unroll
        for (int st = 0; st < 8; ++st) tgo[st] = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    }

    if (threadIdx.x < BK) {
        const int cs0 = (int)nt - BK > 0 ? (int)nt - BK : 0;
        lds_put_prec<SURF, RG>(srecb[0], threadIdx.x, fetch_record<SURF>(a, voff, cs0, (int)nt - cs0, threadIdx.x));
    }
    // the tile's staged records as a buffer (raw, dword data format): reads
    // past its nt visits return zero instead of touching other memory
    constexpr uint32_t RB = 16u * RW;   // bytes per record
    const __amdgpu_buffer_rsrc_t vrec_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float4*>(a.vrec + RW * (int64_t)voff), (short)0,
        (int)(nt < 0x7fffffffu / RB ? nt * RB : 0x7fffffffu), 0x00020000);
    // the pixel's state is complete before the loop (its loads are not
    // carried into the loop's waits)
    asm volatile("" ::"v"(nit), "v"(T));
    __syncthreads();
    int b = 0;
    for (int ce = (int)nt; ce > 0; ce -= BK, b ^= 1) {
        const int cs = ce - BK > 0 ? ce - BK : 0;
        const int cnt = ce - cs;
        const float4* srec = srecb[b];
        __bf16* swh = swh2 + b * BK * PP;
        __bf16* swl = swl2 + b * BK * PP;
        float(*swsum)[BK] = swsum2[b];
        // the next chunk's records, in flight during this chunk
        const int ncs = cs - BK > 0 ? cs - BK : 0;
        // (positions ncs .. ncs + BK - 1 all lie in this tile's visits when
        // there is a next chunk, as the current one is then full; padding is
        // selected when the record is stored)
        RecT nxt;
        if (threadIdx.x < BK && cs > 0) {
            // buffer loads: a uniform chunk offset and a fixed lane offset, so the
            // loop needs no address registers that could alias the pending loads
            const int lo = (int)threadIdx.x * (int)RB, so = ncs * (int)RB;
            nxt.r0 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(vrec_rs, lo, so, 0));
            nxt.r1 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(vrec_rs, lo + 16, so, 0));
            nxt.r2 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(vrec_rs, lo + 32, so, 0));
            if constexpr (SURF)
                nxt.r3 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(vrec_rs, lo + 48, so, 0));
        }
        const int n = w * TILE + xi;
#pragma unroll
        for (int kb = 1; kb >= 0; --kb) {
            float al[4];
            bool on[4];
            float P = 1.0f;
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
                on[r] = k < cnt && (uint32_t)(cs + k) < nit && alpha >= ALPHA_MIN;
                al[r] = alpha;
                P = on[r] ? P * (1.0f - al[r]) : P;
            }
            const Rows4 Pr = rows4(P);
            const float P0 = Pr.r0, P1 = Pr.r1, P2 = Pr.r2, P3 = Pr.r3;
            const float Te3 = T, Te2 = Te3 * __builtin_amdgcn_rcpf(P3), Te1 = Te2 * __builtin_amdgcn_rcpf(P2),
                        Te0 = Te1 * __builtin_amdgcn_rcpf(P1);
            float Tc = q == 3 ? Te3 : (q == 2 ? Te2 : (q == 1 ? Te1 : Te0));
            T = Te0 * __builtin_amdgcn_rcpf(P0);
#pragma unroll
            for (int r = 3; r >= 0; --r) {
                const int k = 16 * kb + 4 * q + r;
                const float Tk = Tc * __builtin_amdgcn_rcpf(1.0f - al[r]);
                const float wv = on[r] ? al[r] * Tk : 0.0f;
                Tc = on[r] ? Tk : Tc;
                const __bf16 hh = (__bf16)wv;
                swh[k * PP + n] = hh;
                swl[k * PP + n] = (__bf16)(wv - (float)hh);
                if (WS && d0 == 0) {
                    // the row's weight sum of position k: butterfly over the 16 pixels
                    float rs = wv;
#pragma unroll
                    for (int off = 1; off < 16; off <<= 1) rs += __shfl_xor(rs, off, 64);
                    if (xi == 0) swsum[w][k] = rs;
                }
            }
        }
        // the next chunk's records go to the other buffer before this chunk's
        // stores are issued (a wait placed after them would also wait for those)
        if (threadIdx.x < BK && cs > 0) {
            if ((int)threadIdx.x >= cs - ncs) nxt = pad_rec<SURF>();
            lds_put_prec<SURF, RG>(srecb[b ^ 1], threadIdx.x, nxt);
        }
        __syncthreads();
        // weight sums per instance: the 16 rows in order
        if (WS && d0 == 0 && threadIdx.x < BK) {
            const int k = threadIdx.x;
            float ws = 0.0f;
#pragma unroll
            for (int ww = 0; ww < 16; ++ww) ws += swsum[ww][k];
            if (k < cnt) a.part_geom[((int64_t)voff + cs + k) * PrimRec<SURF>::GP + PrimRec<SURF>::WSLOT] = ws;
        }
        // out[k][d] = sum_px W^T[k][px] target[px][d], W = hi + lo
        if (w < NDB) {
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int st = 0; st < 8; ++st) {
                    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&swh[(16 * kb + xi) * PP + 32 * st + 8 * q]);
                    const bf16x8 alo = *reinterpret_cast<const bf16x8*>(&swl[(16 * kb + xi) * PP + 32 * st + 8 * q]);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, tgo[st], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, tgo[st], acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * kb + 4 * q + r;
                    if (k < cnt) a.part_fuse[((int64_t)voff + cs + k) * a.d + d0 + 16 * w + xi] = acc[r];
                }
            }
        }
        // No barrier here: before its barrier the next chunk writes the other
        // W^T and weight-sum buffers and this chunk's record buffer, whose last
        // readers (the chunk before this one, and this chunk's walk) all
        // passed the barrier above.
    }
}

// ---------------------------------------------------------------------------
// Fusion from the weights the gradient kernel of the same call recorded
// (W^T [visit][pixel], FP32): no second walk.  1024 threads; wave w < D/16
// keeps channel block w of the tile's target in registers (as k_fuse_bf16);
// every thread loads its share of each chunk's W^T (coalesced float4 rows),
// splits it into BF16 hi + lo and stores it to LDS, double-buffered by chunk
// parity (one barrier per chunk; the next chunk's loads are in flight during
// this chunk's contraction).
template <int D>
__global__ __launch_bounds__(1024) void k_fuse_rec_bf16(BwdArgs a, ViewTable vt) {
    constexpr int PP = TILE_PIX + OPAD;  // padded row stride (bf16) of W^T
    constexpr int NDB = D / 16;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16* swh2 = reinterpret_cast<__bf16*>(smem);                          // [2][BK][PP] W^T hi
    __bf16* swl2 = swh2 + 2 * BK * PP;                                       // [2][BK][PP] W^T lo

    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = a.tile_order ? (int)a.tile_order[blockIdx.x] : (int)blockIdx.x;
    const uint32_t nt = a.tile_niter[t];
    if (nt == 0) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, xi = lane & 15;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int W = vt.width[v], H = vt.height[v];
    const uint32_t voff = a.tile_voff[t];
    const int d0 = (int)blockIdx.y * D;   // channel slice (feature widths above 256)

    // W^T rows of a chunk: 32 positions x 64 float4 (256 pixels); thread
    // handles items threadIdx.x and threadIdx.x + 1024 (position = item / 64)
    const float4* wrec4 = reinterpret_cast<const float4*>(a.wrec);
    auto load_w = [&](int cs, int cnt, float4* f) {
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = threadIdx.x + 1024 * it, k = idx >> 6, c4 = idx & 63;
            f[it] = k < cnt ? wrec4[((int64_t)voff + cs + k) * 64 + c4] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_w = [&](const float4* f, __bf16* swh, __bf16* swl) {
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = threadIdx.x + 1024 * it, k = idx >> 6, n0 = 4 * (idx & 63);
            const float vals[4] = {f[it].x, f[it].y, f[it].z, f[it].w};
            bf16x4 hv, lv;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                hv[m] = (__bf16)vals[m];
                lv[m] = (__bf16)(vals[m] - (float)hv[m]);
            }
            *reinterpret_cast<bf16x4*>(&swh[k * PP + n0]) = hv;
            *reinterpret_cast<bf16x4*>(&swl[k * PP + n0]) = lv;
        }
    };

    // target[px = 32 st + 8 q + m][16 w + xi]: B operands of this wave's block
    // (as in k_fuse_bf16: all 64 loads issued before any is used; addresses of
    // pixels outside the image clamped into it and the values zeroed after)
    bf16x8 tgo[8];
    if (w < NDB) {
        const uint16_t* tg = static_cast<const uint16_t*>(a.target);
        u16x8 raw[8];
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int n0 = 32 * st + 8 * q;
            const int qy = ty * TILE + (n0 >> 4), qx0 = tx * TILE + (n0 & 15);
            const int64_t row = vt.pix_off[v] + (int64_t)(qy < H ? qy : H - 1) * W;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int qx = qx0 + m < W ? qx0 + m : W - 1;
                raw[st][m] = tg[(row + qx) * a.d + d0 + 16 * w + xi];
            }
        }
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int n0 = 32 * st + 8 * q;
            const int qy = ty * TILE + (n0 >> 4), qx0 = tx * TILE + (n0 & 15);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (qy >= H || qx0 + m >= W) raw[st][m] = 0;
            tgo[st] = __builtin_bit_cast(bf16x8, raw[st]);
        }
    } else {
#pragma unroll
        for (int st = 0; st < 8; ++st) tgo[st] = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    }

    {
        float4 f[2];
        load_w(0, (int)nt < BK ? (int)nt : BK, f);
        store_w(f, swh2, swl2);
    }
    __syncthreads();
    int b = 0;
    for (int cs = 0; cs < (int)nt; cs += BK, b ^= 1) {
        const int cnt = (int)nt - cs < BK ? (int)nt - cs : BK;
        const __bf16* swh = swh2 + b * BK * PP;
        const __bf16* swl = swl2 + b * BK * PP;
        // the next chunk's weights, in flight during this chunk's contraction
        const int ncs = cs + BK, ncnt = (int)nt - ncs < BK ? (int)nt - ncs : BK;
        float4 fn[2];
        if (ncs < (int)nt) load_w(ncs, ncnt, fn);
        // out[k][d] = sum_px W^T[k][px] target[px][d], W = hi + lo
        if (w < NDB) {
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int st = 0; st < 8; ++st) {
                    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&swh[(16 * kb + xi) * PP + 32 * st + 8 * q]);
                    const bf16x8 alo = *reinterpret_cast<const bf16x8*>(&swl[(16 * kb + xi) * PP + 32 * st + 8 * q]);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, tgo[st], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, tgo[st], acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * kb + 4 * q + r;
                    if (k < cnt) a.part_fuse[((int64_t)voff + cs + k) * a.d + d0 + 16 * w + xi] = acc[r];
                }
            }
        }
        // the other buffer's last readers (the previous chunk's contraction)
        // passed the previous barrier
        if (ncs < (int)nt) store_w(fn, swh2 + (b ^ 1) * BK * PP, swl2 + (b ^ 1) * BK * PP);
        __syncthreads();
    }
}

template <int D, bool SURF>
static void launch_fuse_bf16(const BwdArgs& a0, const ViewTable& vt, int n_tiles, int ns, bool grads, bool fuse,
                             hipStream_t s) {
    if (!fuse) return;
    // one workgroup per (tile, channel slice)
    const size_t lds = sizeof(__bf16) * 4 * (size_t)BK * (TILE_PIX + OPAD);
    const dim3 grid(n_tiles, ns);
    if (grads && a0.wrec)
        hipLaunchKernelGGL(k_fuse_rec_bf16<D>, grid, dim3(1024), lds, s, a0, vt);
    else if (grads)
        hipLaunchKernelGGL((k_fuse_bf16<D, false, SURF>), grid, dim3(1024), lds, s, a0, vt);
    else
        hipLaunchKernelGGL((k_fuse_bf16<D, true, SURF>), grid, dim3(1024), lds, s, a0, vt);
}

// D: the channel slice width (the feature width itself up to 256; above it,
// 256 when it divides the width, else 128)
template <int D, bool SURF>
static void launch_bf16_d(const BwdArgs& a0, const ViewTable& vt, int n_tiles, bool grads, bool fuse, hipStream_t s) {
    const int ns = a0.d / D;   // channel slices
    if (grads) {
        const size_t lds = sizeof(__bf16) * 2 * (size_t)BK * (D + OPAD) +
                           sizeof(float) * (2 * (size_t)TILE_PIX * SK + 3 * TILE_PIX + 8 * PrimRec<SURF>::NQ * BK);
        BwdArgs a = a0;
        a.d0 = 0;
        a.g_in = nullptr;
        bool sliced = false;
        if constexpr (D == 128 || D == 256) {
            if (ns > 1) {
                // f . dF of every slice but the last, summed in a0.g_out; the
                // gradient kernel takes the last slice and adds the carry
                sliced = true;
                if (a0.dF) {
                    for (int sl = 0; sl + 1 < ns; ++sl) {
                        BwdArgs g = a0;
                        g.d0 = sl * D;
                        g.g_in = sl > 0 ? a0.g_out : nullptr;
                        hipLaunchKernelGGL(k_gk_bf16<D>, dim3(n_tiles), dim3(512), 0, s, g, vt);
                    }
                    a.g_in = a0.g_out;
                }
                a.d0 = (ns - 1) * D;
                hipLaunchKernelGGL((k_render_bwd_bf16<D, true, SURF>), dim3(n_tiles), dim3(512), lds, s, a, vt);
            }
        }
        if (!sliced) hipLaunchKernelGGL((k_render_bwd_bf16<D, false, SURF>), dim3(n_tiles), dim3(512), lds, s, a, vt);
    }
    launch_fuse_bf16<D, SURF>(a0, vt, n_tiles, ns, grads, fuse, s);
}

bool render_bwd_bf16_supported(int d) {
    return d == 32 || d == 64 || d == 96 || d == 128 || d == 256 || (d > 256 && d % 128 == 0);
}

bool render_bwd_bf16_sliced(int d) { return d > 256; }

// grads: the gradient kernel (needs dC); fuse: the fusion kernel (needs the
// target).  Above 256 channels, a.g_out is the [visits][256] carry of f . dF
// between channel slices (needed when dF is given).
template <bool SURF>
static void launch_bf16(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool grads, bool fuse, hipStream_t s) {
    switch (a.d) {
        case 32: launch_bf16_d<32, SURF>(a, vt, n_tiles, grads, fuse, s); break;
        case 64: launch_bf16_d<64, SURF>(a, vt, n_tiles, grads, fuse, s); break;
        case 96: launch_bf16_d<96, SURF>(a, vt, n_tiles, grads, fuse, s); break;
        case 128: launch_bf16_d<128, SURF>(a, vt, n_tiles, grads, fuse, s); break;
        case 256: launch_bf16_d<256, SURF>(a, vt, n_tiles, grads, fuse, s); break;
        default:
            if (a.d % 256 == 0)
                launch_bf16_d<256, SURF>(a, vt, n_tiles, grads, fuse, s);
            else
                launch_bf16_d<128, SURF>(a, vt, n_tiles, grads, fuse, s);
            break;
    }
}

void launch_render_bwd_bf16(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool grads, bool fuse, hipStream_t s) {
    if (a.prim == FH_PRIM_SURFEL)
        launch_bf16<true>(a, vt, n_tiles, grads, fuse, s);
    else
        launch_bf16<false>(a, vt, n_tiles, grads, fuse, s);
}

}  // namespace fh
