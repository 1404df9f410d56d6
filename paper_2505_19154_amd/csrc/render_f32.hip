// Front-to-back compositing (FP32 VALU form) and its adjoint.
//
// Forward (Section 3.1): for every pixel, walk its tile's depth-sorted list;
//   alpha = min(0.99, o G), skip if alpha < 1/255, stop before T drops below
//   1e-4, w = alpha T, C += w rgb, F += w f, T *= (1 - alpha).
// One 256-thread workgroup per (tile, feature slice); records and feature rows
// of 256 instances at a time are staged in LDS and read by every pixel.
//
// Backward (Appendix A.2): per tile, back to front from the tile's longest
// traversal, transmittance recovered by division from T_final,
//   dL/dalpha_k = T_k g_k - (S_k + T_final dT) / (1 - alpha_k),
//   g_k = rgb_k . dC + f_k . dF,  S_k = sum_{i>k} w_i g_i,
// reduced over the tile's pixels into per-instance partials (no atomics);
// optionally the fusion partials sum_p w(p) target(p) in the same sweep.
//
// Both kernels also take the surfel primitive (Section 3.1; SURF = true):
// four-float4 records (see k_project_surfel), the density at the ray-plane
// intersection, and 14 per-instance partials (the nine record entries' terms,
// sum dL/dpower, rgb, sum w) in rows of 16 floats.
#include "kernels.hpp"

namespace fh {


__device__ __forceinline__ uint32_t inst_rank(const uint32_t* keys, const uint32_t* vals, int64_t i, int rank_bits,
                                              int packed) {
    return packed ? (keys[i] & ((1u << rank_bits) - 1u)) : vals[i];
}

__device__ __forceinline__ float load_feat(const void* f, int bf16, int64_t idx) {
    return bf16 ? bf16_to_f32(static_cast<const uint16_t*>(f)[idx]) : static_cast<const float*>(f)[idx];
}

template <int DS, bool SURF>
__global__ __launch_bounds__(256) void k_render_fwd_f32(RenderArgs a, ViewTable vt) {
    using RecT = typename PrimRec<SURF>::T;
    __shared__ RecT srec[256];
    __shared__ float sfeat[256][DS > 0 ? DS : 1];
    __shared__ uint32_t smax[4];
    if (a.counters->inst_overflow) return;
    const int t = blockIdx.x, slice = blockIdx.y, d0 = slice * DS;
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int px = tx * TILE + (threadIdx.x % TILE), py = ty * TILE + (threadIdx.x / TILE);
    const bool inside = px < vt.width[v] && py < vt.height[v];
    const float x = (float)px + 0.5f, y = (float)py + 0.5f;
    const uint32_t s = a.ranges[2 * t], e = a.ranges[2 * t + 1];
    const int ds_here = (a.d - d0) < DS ? (a.d - d0) : DS;

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    float F[DS > 0 ? DS : 1];
#pragma unroll
    for (int c = 0; c < (DS > 0 ? DS : 1); ++c) F[c] = 0.0f;
    bool done = !inside;
    uint32_t last = 0;

    for (uint32_t base = s; base < e; base += 256) {
        const uint32_t cnt = (e - base) < 256u ? (e - base) : 256u;
        if (threadIdx.x < cnt) {
            const int64_t i = base + threadIdx.x;
            const uint32_t j = inst_rank(a.keys, a.vals, i, a.rank_bits, a.packed);
            const uint32_t g = a.order[j];
            srec[threadIdx.x] = load_rec<SURF>(a.rrec, j);
            if (DS > 0) {
#pragma unroll
                for (int c = 0; c < DS; ++c)
                    sfeat[threadIdx.x][c] = c < ds_here ? load_feat(a.feat, a.feat_bf16, (int64_t)g * a.d + d0 + c) : 0.0f;
            }
        }
        __syncthreads();
        if (!done) {
            for (uint32_t k = 0; k < cnt; ++k) {
                const RecT r = srec[k];
                const float alpha = prim_alpha<SURF>(r, x, y);
                if (alpha < ALPHA_MIN) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < T_MIN) {
                    done = true;
                    break;
                }
                const float w = alpha * T;
                c0 += w * r.r2.y;
                c1 += w * r.r2.z;
                c2 += w * r.r2.w;
#pragma unroll
                for (int c = 0; c < DS; ++c) F[c] += w * sfeat[k][c];
                T = Tn;
                last = base - s + k + 1;
            }
        }
        if (__syncthreads_count(!done) == 0) break;
    }

    const int64_t p = vt.pix_off[v] + (int64_t)py * vt.width[v] + px;
    if (inside) {
        if (slice == 0) {
            a.C[3 * p] = c0;
            a.C[3 * p + 1] = c1;
            a.C[3 * p + 2] = c2;
            a.T[p] = T;
            a.n_iter[p] = last;
        }
        if (DS > 0) {
#pragma unroll
            for (int c = 0; c < DS; ++c)
                if (c < ds_here) a.F[p * a.d + d0 + c] = F[c];
        }
    }
    if (slice == 0) {
        const uint32_t m = wave_max_u32(last);
        if ((threadIdx.x & 63) == 0) smax[threadIdx.x / 64] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t mm = smax[0];
            for (int k = 1; k < 4; ++k) mm = smax[k] > mm ? smax[k] : mm;
            a.tile_niter[t] = mm;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-tile traversal bookkeeping after the forward pass.
__global__ void k_check_visits(const uint32_t* tile_voff, int n_tiles, Counters* c, int64_t cap) {
    if (threadIdx.x == 0) {
        const unsigned long long tot = tile_voff[n_tiles];
        c->n_visited = tot;
        c->visit_overflow = tot > (unsigned long long)cap ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------

template <int K, bool FUSE, bool SURF>
__global__ __launch_bounds__(256) void k_render_bwd_f32(BwdArgs a, ViewTable vt) {
    using RecT = typename PrimRec<SURF>::T;
    constexpr int NQ = SURF ? 14 : 10;    // per-instance partial terms
    constexpr int GP = SURF ? 16 : 12;    // floats per partial row
    extern __shared__ float dyn[];
    __shared__ RecT srec[K];
    __shared__ uint32_t sg[K];
    __shared__ float sred[4][K][NQ];
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    const int t = blockIdx.x;
    const uint32_t nt = a.tile_niter[t];
    if (nt == 0) return;
    const int D = a.d;
    float* sfeat = dyn;                              // [K][D]
    float* sW = dyn + (size_t)K * (D > 0 ? D : 1);   // [256][K+1]
    const int v = view_of_tile(vt, t);
    const int lt = t - vt.tile_off[v];
    const int tx = lt % vt.tiles_x[v], ty = lt / vt.tiles_x[v];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int px = tx * TILE + (threadIdx.x % TILE), py = ty * TILE + (threadIdx.x / TILE);
    const bool inside = px < vt.width[v] && py < vt.height[v];
    const float x = (float)px + 0.5f, y = (float)py + 0.5f;
    const uint32_t voff = a.tile_voff[t];
    const int64_t p = vt.pix_off[v] + (int64_t)py * vt.width[v] + px;

    const uint32_t nit = inside ? a.n_iter[p] : 0u;
    float T = inside ? a.T_final[p] : 1.0f;
    const float Tfin = T;
    float dCp[3] = {0, 0, 0};
    if (inside && a.dC) {
        dCp[0] = a.dC[3 * p];
        dCp[1] = a.dC[3 * p + 1];
        dCp[2] = a.dC[3 * p + 2];
    }
    const float dTp = (inside && a.dT) ? a.dT[p] : 0.0f;
    float S = 0.0f;
    const float LN2 = 0.69314718055994531f;

    for (int ce = (int)nt; ce > 0; ce -= K) {
        const int cs = ce - K > 0 ? ce - K : 0;
        const int cnt = ce - cs;
        if (threadIdx.x < cnt) {
            const int64_t vi = (int64_t)voff + cs + threadIdx.x;
            srec[threadIdx.x] = load_rec<SURF>(a.vrec, vi);
            sg[threadIdx.x] = a.vgid[vi];
        }
        __syncthreads();
        if (D > 0 && (a.dF || FUSE)) {
            for (int idx = threadIdx.x; idx < cnt * D; idx += 256) {
                const int k = idx / D, c = idx - k * D;
                sfeat[k * D + c] = load_feat(a.feat, a.feat_bf16, (int64_t)sg[k] * D + c);
            }
        }
        __syncthreads();
        // g_k's feature part: f_k . dF(p)
        float gacc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) gacc[k] = 0.0f;
        if (a.dF && D > 0 && inside && (uint32_t)cs < nit) {
            const float* dfp = a.dF + p * D;
            if ((D & 3) == 0) {
                for (int c = 0; c < D; c += 4) {
                    const float4 df = *reinterpret_cast<const float4*>(dfp + c);
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (k < cnt) {
                            const float4 f = *reinterpret_cast<const float4*>(&sfeat[k * D + c]);
                            gacc[k] += f.x * df.x + f.y * df.y + f.z * df.z + f.w * df.w;
                        }
                }
            } else {
                for (int c = 0; c < D; ++c) {
                    const float df = dfp[c];
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (k < cnt) gacc[k] += sfeat[k * D + c] * df;
                }
            }
        }
        // back to front over the chunk
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            if (k >= cnt) continue;
            const int pos = cs + k;
            float q[NQ];
#pragma unroll
            for (int m = 0; m < NQ; ++m) q[m] = 0.0f;
            float w = 0.0f;
            bool contrib = false;
            if (inside && (uint32_t)pos < nit) {
                const RecT r = srec[k];
                float alpha, raw;
                [[maybe_unused]] AlphaEval ae;
                [[maybe_unused]] SurfEval se;
                if constexpr (SURF) {
                    se = eval_surfel(r, x, y);
                    alpha = se.alpha;
                    raw = se.raw;
                } else {
                    ae = eval_alpha(r, x, y);
                    alpha = ae.alpha;
                    raw = ae.raw;
                }
                if (alpha >= ALPHA_MIN) {
                    contrib = true;
                    const float inv = 1.0f / (1.0f - alpha);
                    const float Tk = T * inv;
                    w = alpha * Tk;
                    const float gk = r.r2.y * dCp[0] + r.r2.z * dCp[1] + r.r2.w * dCp[2] + gacc[k];
                    const float dalpha = Tk * gk - (S + Tfin * dTp) * inv;
                    S += w * gk;
                    T = Tk;
                    const float dpow = (raw < ALPHA_MAX) ? dalpha * alpha : 0.0f;
                    if constexpr (SURF) {
                        // dL/dk = dpow (-u / k2, -v / k2, (u^2 + v^2) / k2), k linear in the record
                        const float l0 = -dpow * se.u * se.ik2, l1 = -dpow * se.v * se.ik2;
                        const float l2 = dpow * (se.u * se.u + se.v * se.v) * se.ik2;
                        const float a0 = r.r1.x, a1 = r.r1.y, b0 = r.r1.z, b1 = r.r1.w;
                        const float e1 = r.r3.y, e2 = r.r3.z;
                        q[0] = -(l0 * b1 - l1 * b0 - l2 * e2);
                        q[1] = -(l1 * a0 - l0 * a1 - l2 * e1);
                        q[2] = l1 * se.dy;
                        q[3] = -l0 * se.dy;
                        q[4] = -l1 * se.dx;
                        q[5] = l0 * se.dx;
                        q[6] = l2;
                        q[7] = -l2 * se.dy;
                        q[8] = -l2 * se.dx;
                    } else {
                        // d power / d(u, v) = Sigma2^-1 d, from the eigenframe:
                        // Sigma2^-1 d = -2 ln2 (q1 a e1 + q2 b e2), e2 = (-e_y, e_x)
                        const float ex = r.r1.x, ey = r.r1.y;
                        const float qa = r.r1.z * ae.a, qb = r.r1.w * ae.b;
                        const float sdx = -2.0f * LN2 * (qa * ex - qb * ey);
                        const float sdy = -2.0f * LN2 * (qa * ey + qb * ex);
                        q[0] = dpow * sdx;
                        q[1] = dpow * sdy;
                        q[2] = dpow * (-0.5f * ae.dx * ae.dx);
                        q[3] = dpow * (-ae.dx * ae.dy);
                        q[4] = dpow * (-0.5f * ae.dy * ae.dy);
                    }
                    q[NQ - 5] = dpow;
                    q[NQ - 4] = w * dCp[0];
                    q[NQ - 3] = w * dCp[1];
                    q[NQ - 2] = w * dCp[2];
                    q[NQ - 1] = w;
                }
            }
            if (FUSE) sW[threadIdx.x * (K + 1) + k] = w;
            if (__any(contrib)) {
#pragma unroll
                for (int m = 0; m < NQ; ++m) {
                    const float r = wave_sum(q[m]);
                    if (lane == 0) sred[wv][k][m] = r;
                }
            } else if (lane == 0) {
#pragma unroll
                for (int m = 0; m < NQ; ++m) sred[wv][k][m] = 0.0f;
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt * GP; idx += 256) {
            const int k = idx / GP, m = idx - k * GP;
            const float val = m < NQ ? (sred[0][k][m] + sred[1][k][m]) + (sred[2][k][m] + sred[3][k][m]) : 0.0f;
            a.part_geom[((int64_t)voff + cs + k) * GP + m] = val;
        }
        if (FUSE && D > 0) {
            // sum_p w(p) target(p) for the chunk's instances; pixels outside the image have w = 0
            const int W = vt.width[v], H = vt.height[v];
            for (int c = threadIdx.x; c < D; c += 256) {
                float acc[K];
#pragma unroll
                for (int k = 0; k < K; ++k) acc[k] = 0.0f;
                // one tile row (16 pixels) of target values in flight at a time
                for (int row = 0; row < TILE; ++row) {
                    const int qy = ty * TILE + row;
                    float tv[TILE];
#pragma unroll
                    for (int m = 0; m < TILE; ++m) {
                        const int qx = tx * TILE + m;
                        tv[m] = (qx < W && qy < H)
                                    ? load_feat(a.target, a.target_bf16,
                                                (vt.pix_off[v] + (int64_t)qy * W + qx) * D + c)
                                    : 0.0f;
                    }
#pragma unroll
                    for (int m = 0; m < TILE; ++m) {
                        const int pp = row * TILE + m;
#pragma unroll
                        for (int k = 0; k < K; ++k) acc[k] += sW[pp * (K + 1) + k] * tv[m];
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k < cnt) a.part_fuse[((int64_t)voff + cs + k) * D + c] = acc[k];
            }
        }
        __syncthreads();
    }
}

// Per depth rank j (view v = j / n): the rank of each (view, Gaussian) and the
// screen records in rank order, so that a tile list entry (a rank) reaches its
// record with one load.
__global__ __launch_bounds__(256) void k_rank_tables(const uint32_t* __restrict__ order, const float4* __restrict__ rec,
                                                     int64_t n, int64_t total, uint32_t* __restrict__ rank_of,
                                                     float4* __restrict__ rrec, int rw) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= total) return;
    const int64_t v = j / n;
    const int64_t i = v * n + order[j];
    rank_of[i] = (uint32_t)(j - v * n);
    for (int k = 0; k < rw; ++k) rrec[rw * j + k] = rec[rw * i + k];
}

__global__ __launch_bounds__(256) void k_fuse_finalize(const float* sum, const float* comp, const float* wsum,
                                                       const float* wcomp, int64_t n, int d, const void* feat_in,
                                                       void* feat_out, int bf16) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n * d) return;
    const int64_t g = i / d;
    const float W = wsum[g] + wcomp[g];
    float val;
    if (W > 0.0f)
        val = (sum[i] + comp[i]) / W;
    else
        val = feat_in ? load_feat(feat_in, bf16, i) : 0.0f;
    if (bf16) {
        // round to nearest even
        uint32_t u = __float_as_uint(val);
        u += 0x7FFFu + ((u >> 16) & 1u);
        static_cast<uint16_t*>(feat_out)[i] = (uint16_t)(u >> 16);
    } else {
        static_cast<float*>(feat_out)[i] = val;
    }
}

// ---------------------------------------------------------------------------
template <bool SURF>
static void launch_fwd_f32(const RenderArgs& a, const ViewTable& vt, int n_tiles, int slice, hipStream_t s) {
    if (a.d == 0) {
        hipLaunchKernelGGL((k_render_fwd_f32<0, SURF>), dim3(n_tiles, 1), dim3(256), 0, s, a, vt);
        return;
    }
    const unsigned ns = (unsigned)((a.d + slice - 1) / slice);
    switch (slice) {
        case 8: hipLaunchKernelGGL((k_render_fwd_f32<8, SURF>), dim3(n_tiles, ns), dim3(256), 0, s, a, vt); break;
        case 16: hipLaunchKernelGGL((k_render_fwd_f32<16, SURF>), dim3(n_tiles, ns), dim3(256), 0, s, a, vt); break;
        case 32: hipLaunchKernelGGL((k_render_fwd_f32<32, SURF>), dim3(n_tiles, ns), dim3(256), 0, s, a, vt); break;
        default: hipLaunchKernelGGL((k_render_fwd_f32<64, SURF>), dim3(n_tiles, ns), dim3(256), 0, s, a, vt); break;
    }
}

void launch_render_fwd_f32(const RenderArgs& a, const ViewTable& vt, int n_tiles, int slice, hipStream_t s) {
    if (a.prim == FH_PRIM_SURFEL)
        launch_fwd_f32<true>(a, vt, n_tiles, slice, s);
    else
        launch_fwd_f32<false>(a, vt, n_tiles, slice, s);
}

void launch_check_visits(const uint32_t* tile_voff, int n_tiles, Counters* c, int64_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_check_visits, dim3(1), dim3(64), 0, s, tile_voff, n_tiles, c, cap);
}

template <int K, bool SURF>
static void launch_bwd_ks(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool fuse, hipStream_t s) {
    const size_t dyn = sizeof(float) * ((size_t)K * (a.d > 0 ? a.d : 1) + (fuse ? (size_t)256 * (K + 1) : 0));
    if (fuse)
        hipLaunchKernelGGL((k_render_bwd_f32<K, true, SURF>), dim3(n_tiles), dim3(256), dyn, s, a, vt);
    else
        hipLaunchKernelGGL((k_render_bwd_f32<K, false, SURF>), dim3(n_tiles), dim3(256), dyn, s, a, vt);
}

template <int K>
static void launch_bwd_k(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool fuse, hipStream_t s) {
    if (a.prim == FH_PRIM_SURFEL)
        launch_bwd_ks<K, true>(a, vt, n_tiles, fuse, s);
    else
        launch_bwd_ks<K, false>(a, vt, n_tiles, fuse, s);
}

void launch_render_bwd_f32(const BwdArgs& a, const ViewTable& vt, int n_tiles, bool fuse, int chunk, hipStream_t s) {
    if (chunk == 32 && a.d <= 512)
        launch_bwd_k<32>(a, vt, n_tiles, fuse, s);
    else
        launch_bwd_k<16>(a, vt, n_tiles, fuse, s);
}

void launch_rank_tables(const uint32_t* order, const float4* rec, int64_t n, int64_t total, uint32_t* rank_of,
                        float4* rrec, int rw, hipStream_t s) {
    hipLaunchKernelGGL(k_rank_tables, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, order, rec, n, total,
                       rank_of, rrec, rw);
}

void launch_fuse_finalize(const float* sum, const float* comp, const float* wsum, const float* wcomp, int64_t n, int d,
                          const void* feat_in, void* feat_out, int bf16, hipStream_t s) {
    const int64_t tot = n * d;
    if (tot > 0)
        hipLaunchKernelGGL(k_fuse_finalize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, sum, comp, wsum,
                           wcomp, n, d, feat_in, feat_out, bf16);
}

}  // namespace fh
