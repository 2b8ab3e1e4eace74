// BF16 split-precision matrix-core form for L_low in {48, 64}: the Ll x Ll
// score map of one (observation, component) is covered by 2 x 2 tiles of 32x32
// (tile (tb1, tb2) holds t1 in [32 tb1, 32 tb1 + 32), t2 likewise; for Ll = 48
// the t >= 48 rows and columns repeat t - 48 and are masked).
//
// A block works on ONE component and groups of 8 observations; wave w owns
// tile (tb1, tb2) = (w >> 1, w & 1) for all 8 of them.  The operands are those
// of the one-tile form (srmra_bf16_impl.h) with the tile offsets added:
//   score   A[t2][k] = y_i[r1][(b2 + t2) % Ll],  B[k][t1] = x_c[(r1 - t1) % Ll][b2],
//           k = (r1 slice jb, b2, 16 r1 of the slice), slices outermost;
//   back-projection (posterior from the score accumulators, k = (t2, o))
//           Z[q2][t1] = sum_{t2, o} y_o[a1][(q2 + t2) % Ll] * w_o[t1][t2],
//           folded into b_c[(a1 - t1) % Ll][q2] in the wave's LDS accumulator;
// the four waves' accumulators are summed in a fixed order at the end of the
// chunk.  The observation planes are staged through LDS in slices (16 r1 of
// every column for the score, 16 rows a1 for the back-projection), so a block
// needs about 116 KB of LDS at Ll = 64 instead of the 350 KB of whole planes.
//
// Pass 1 writes one (max, sum) partial per (observation, component, tile):
// n_part = 4 K^2.  Both passes accumulate every score in the same k order, so
// pass 2 recomputes exactly the scores of pass 1.
#pragma once
#include "srmra_bf16_impl.h"

namespace srmra {
namespace b16w {

using b16::acc_row;
using b16::split8;

constexpr int SP = 24;   // staged yT row pitch in bf16 (16 r1 + 8): 48 B, conflict-free b128 reads
constexpr int YR = 16;   // rows a1 per staged back-projection slice

template <int LL> struct Geo {
    static constexpr int JS = LL / 16;                 // r1 slices
    static constexpr int NK = LL * JS;                 // k-steps of one score tile
    static constexpr int BP = LL + 1;                  // b accumulator pitch (floats)
    static constexpr int YT_OBS = 2 * LL * LL;         // bf16 per observation (both planes)
    static constexpr int YO_GRP = 2 * LL * LL * 8;     // bf16 per 8-observation group
    static constexpr int ST_YT = 8 * 2 * LL * SP;      // bf16 of one staged yT slice
    static constexpr int ST_YO = 2 * YR * LL * 8;      // bf16 of one staged Yo slice
    static constexpr int ST = ST_YT > ST_YO ? ST_YT : ST_YO;
};

// prepared layouts:
//   yT [N][JS][plane][col = r2][16 r1 of slice jb]   (slice-major: one staged
//       slice of one observation is 4 contiguous KiB at Ll = 64)
//   Yo [ceil(N/8)][plane][r1][r2][8 observations]
struct Prep {
    const __bf16* yT;
    const __bf16* yo;
};

// x of component c (less mu) as B fragments of every k-step of t1-tile tb1:
// lane (t1 = 32 tb1 + (lane & 31), g = lane >> 5) of k-step (jb, b2) holds
// x_c[(16 jb + 8 g + e - t1) mod Ll][b2], e = 0..7, split into hi and lo.
// Layout [c][tb1][jb][b2][plane][lane] of 16-byte fragments.
template <int LL>
__device__ __forceinline__ void pack_xb_body(const StepArgs& p, const float* __restrict__ x, int c,
                                             int tb1, int ks, uint4* __restrict__ xb) {
    using G = Geo<LL>;
    const int lane = threadIdx.x & 63;
    const int c1 = c / p.K, c2 = c % p.K;
    const int jb = ks / LL, b2 = ks % LL;
    const int t1 = 32 * tb1 + (lane & 31), g = lane >> 5;
    const int t1e = t1 < LL ? t1 : t1 - LL;
    const float mu = centre_of(p.centre);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int r = 16 * jb + 8 * g + e - t1e;
        r = r < 0 ? r + LL : r;
        v[e] = x[(int64_t)(c1 + r * p.K) * p.Lh + (c2 + b2 * p.K)] - mu;
    }
    bf16x8 h, l;
    split8(v, h, l);
    uint4* dst = xb + ((int64_t)((c * 2 + tb1) * G::NK + ks) * 2) * 64;
    dst[lane] = __builtin_bit_cast(uint4, h);
    dst[64 + lane] = __builtin_bit_cast(uint4, l);
}

// slice jb of the yT planes of observations [o0, o0 + 8) into LDS
// st[o][plane][col][SP], zeros past N.
template <int LL>
__device__ __forceinline__ void stage_yT(const Prep& q, int64_t N, int64_t o0, int jb, __bf16* st) {
    using G = Geo<LL>;
    constexpr int CH = 2 * LL * 2;              // 16-byte chunks per observation and slice
    for (int e = threadIdx.x; e < 8 * CH; e += 256) {
        const int o = e / CH, r = e % CH;       // r = (plane * LL + col) * 2 + half
        uint4 v = make_uint4(0, 0, 0, 0);
        if (o0 + o < N)
            v = reinterpret_cast<const uint4*>(q.yT + ((o0 + o) * G::JS + jb) * (int64_t)(2 * LL * 16))[r];
        *reinterpret_cast<uint4*>(st + (o * 2 * LL + (r >> 1)) * SP + (r & 1) * 8) = v;
    }
}

// rows [a1s, a1s + YR) of both Yo planes of the group starting at o0 into LDS
// st[plane][row][col][8].
template <int LL>
__device__ __forceinline__ void stage_yo(const Prep& q, int64_t o0, int a1s, __bf16* st) {
    constexpr int CH = YR * LL;                 // 16-byte chunks per plane
    const uint4* src = reinterpret_cast<const uint4*>(q.yo + (o0 / 8) * (int64_t)Geo<LL>::YO_GRP);
    uint4* dst = reinterpret_cast<uint4*>(st);
    for (int e = threadIdx.x; e < 2 * CH; e += 256) {
        const int plane = e / CH, r = e % CH;
        dst[e] = src[(plane * LL + a1s) * LL + r];
    }
}

// Score tile (tb1, tb2) of component comp for the 8 observations [o0, o0 + 8).
// Every thread of the block calls it (it stages through LDS).
template <int LL, int NP>
__device__ __forceinline__ void score(const StepArgs& p, const Prep& q, __bf16* st, int comp,
                                      int tb1, int tb2, int64_t o0, floatx16 (&acc)[8]) {
    using G = Geo<LL>;
    const int lane = threadIdx.x & 63;
    const int i = lane & 31, g = lane >> 5;
    const int t2 = 32 * tb2 + i;
    const int t2e = t2 < LL ? t2 : t2 - LL;
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = floatx16{0};
    const uint4* bsrc = p.xb + (int64_t)(comp * 2 + tb1) * G::NK * 128 + lane;
    bf16x8 bh = __builtin_bit_cast(bf16x8, bsrc[0]);
    bf16x8 bl = __builtin_bit_cast(bf16x8, bsrc[64]);
    for (int jb = 0; jb < G::JS; ++jb) {
        __syncthreads();
        stage_yT<LL>(q, p.N, o0, jb, st);
        __syncthreads();
        for (int b2 = 0; b2 < LL; ++b2) {
            const int ks = jb * LL + b2;
            const int kn = ks + 1 < G::NK ? ks + 1 : ks;
            const bf16x8 nh = __builtin_bit_cast(bf16x8, bsrc[kn * 128]);
            const bf16x8 nl = __builtin_bit_cast(bf16x8, bsrc[kn * 128 + 64]);
            int col = b2 + t2e;
            col = col >= LL ? col - LL : col;
            const __bf16* arow = st + col * SP + 8 * g;
            bf16x8 ah[8], al[8];
            auto load = [&](int o) {
                ah[o] = *reinterpret_cast<const bf16x8*>(arow + (o * 2 * LL) * SP);
                al[o] = *reinterpret_cast<const bf16x8*>(arow + (o * 2 * LL + LL) * SP);
            };
            load(0);
            load(1);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int pr = 0; pr < 4; ++pr) {
                const int o = 2 * pr;
                if (pr < 3) {
                    load(o + 2);
                    load(o + 3);
                }
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o], bh, acc[o], 0, 0, 0);
                acc[o + 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o + 1], bh, acc[o + 1], 0, 0, 0);
                acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o], bl, acc[o], 0, 0, 0);
                acc[o + 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o + 1], bl, acc[o + 1], 0, 0, 0);
                acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], bh, acc[o], 0, 0, 0);
                acc[o + 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o + 1], bh, acc[o + 1], 0, 0, 0);
                if constexpr (NP == 4) {
                    acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], bl, acc[o], 0, 0, 0);
                    acc[o + 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o + 1], bl, acc[o + 1], 0, 0, 0);
                }
            }
            bh = nh;
            bl = nl;
        }
    }
}

// bias of a lane's 16 slots of tile (tb1, tb2); -inf where t1 or t2 >= Ll
template <int LL>
__device__ __forceinline__ void tile_bias(const StepArgs& p, int comp, int tb1, int tb2, float (&bet)[16]) {
    const int lane = threadIdx.x & 63;
    const int t1 = 32 * tb1 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int t2 = 32 * tb2 + acc_row(v, lane);
        bet[v] = (t1 < LL && t2 < LL) ? p.betaT[(int64_t)comp * (LL * LL) + t2 * LL + t1] : -INFINITY;
    }
}

// ============================================================================
// Pass 1: (max, sum of exp) of every observation over the wave's tile.
template <int LL, int NP>
__device__ __forceinline__ void pass1_body(const StepArgs& p, const Prep& q, int chunk, int comp,
                                           float* lds) {
    __bf16* st = reinterpret_cast<__bf16*>(lds);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tb1 = wave >> 1, tb2 = wave & 1;
    const int cc = comp < p.KK ? comp : p.KK - 1;
    float bet[16];
    tile_bias<LL>(p, cc, tb1, tb2, bet);
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += 8) {
        floatx16 acc[8];
        score<LL, NP>(p, q, st, cc, tb1, tb2, o0, acc);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            float mx = -INFINITY;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float a = acc[o][v] * p.inv_s2 + bet[v];
                acc[o][v] = a;
                mx = fmaxf(mx, a);
            }
            for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
            float s = 0.f;
            if (mx > -INFINITY) {
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    if (acc[o][v] > -INFINITY) s += fast_exp(acc[o][v] - mx);
            }
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            const int64_t oi = o0 + o;
            if (lane == 0 && oi < p.N && comp < p.KK)
                p.part[(int64_t)(comp * 4 + wave) * p.N + oi] = make_float2(mx, s);
        }
    }
}

// Z[q2][t1] of one row a1 (staged Yo row yrow) over the first NV accumulator
// rows v of the wave's w fragments: Z = sum_v A_v W_v, A_v[q2][(t2, o)] =
// y_o[a1][(q2 + t2) % Ll].  The A fragments (both planes) are requested PF rows
// v ahead of their products so that the LDS latency is covered.
template <int LL, int NP, int NV>
__device__ __forceinline__ floatx16 bp_rows(const __bf16* yrow, int q2e, int tb2, const bf16x8 (&wh)[16],
                                            const bf16x8 (&wl)[16]) {
    constexpr int PF = 4;
    const int lane = threadIdx.x & 63;
    bf16x8 ah[NV], al[NV];
    auto load_a = [&](int v) {
        const int t2 = 32 * tb2 + acc_row(v, lane);
        int col = q2e + t2;
        col = col >= LL ? col - LL : col;
        ah[v] = *reinterpret_cast<const bf16x8*>(yrow + col * 8);
        al[v] = *reinterpret_cast<const bf16x8*>(yrow + YR * LL * 8 + col * 8);
    };
#pragma unroll
    for (int v = 0; v < PF; ++v) load_a(v);
    floatx16 zp[2] = {floatx16{0}, floatx16{0}};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v + PF < NV) load_a(v + PF);
        // compiler-only barriers: the request stays PF rows ahead of its use
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        zp[v & 1] = b16::mfma_split<NP>(ah[v], al[v], wh[v], wl[v], zp[v & 1]);
    }
    floatx16 z;
#pragma unroll
    for (int e = 0; e < 16; ++e) z[e] = zp[0][e] + zp[1][e];
    return z;
}

// ============================================================================
// Pass 2: posterior weights of the wave's tile, back-projection and posterior
// mass; per-chunk partials of component comp.
template <int LL, int NP>
__device__ __forceinline__ void pass2_body(const StepArgs& p, const Prep& q, int chunk, int comp,
                                           float* lds) {
    using G = Geo<LL>;
    float* bacc = lds;                                                   // 4 x Ll x BP
    __bf16* st = reinterpret_cast<__bf16*>(bacc + 4 * LL * G::BP);       // staging
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 31;
    const int tb1 = wave >> 1, tb2 = wave & 1;
    const bool cok = comp < p.KK;
    const int cc = cok ? comp : p.KK - 1;
    const int t1 = 32 * tb1 + j;
    const bool t1ok = t1 < LL;
    float* bw = bacc + wave * LL * G::BP;
    for (int e = lane; e < LL * G::BP; e += 64) bw[e] = 0.f;
    float bet[16], cnt[16];
    tile_bias<LL>(p, cc, tb1, tb2, bet);
#pragma unroll
    for (int v = 0; v < 16; ++v) cnt[v] = 0.f;
    // rows t2 >= Ll of the second t2-tile (Ll = 48: v >= 8) carry no weight
    const int nv = (LL < 64 && tb2 == 1) ? 8 : 16;
    static_assert(LL == 48 || LL == 64, "two 32-wide tiles per axis");
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += 8) {
        floatx16 acc[8];
        score<LL, NP>(p, q, st, cc, tb1, tb2, o0, acc);
        float2 lse[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) lse[o] = (o0 + o < p.N) ? p.lse[o0 + o] : make_float2(0.f, 0.f);
        bf16x8 wh[16], wl[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            float w[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                float ww = 0.f;
                if (cok && o0 + o < p.N) {
                    const float a = acc[o][v] * p.inv_s2 + bet[v];
                    ww = a > -INFINITY ? fast_exp((a - lse[o].x) - lse[o].y) : 0.f;
                }
                w[o] = ww;
                cnt[v] += ww;
            }
            split8(w, wh[v], wl[v]);
        }
        for (int a1s = 0; a1s < LL; a1s += YR) {
            __syncthreads();
            stage_yo<LL>(q, o0, a1s, st);
            __syncthreads();
            for (int a1 = a1s; a1 < a1s + YR; ++a1) {
                const __bf16* yrow = st + (a1 - a1s) * LL * 8;
#pragma unroll
                for (int qb = 0; qb < 2; ++qb) {
                    const int q2 = 32 * qb + j;
                    const int q2e = q2 < LL ? q2 : q2 - LL;
                    const floatx16 z = nv == 16 ? bp_rows<LL, NP, 16>(yrow, q2e, tb2, wh, wl)
                                                : bp_rows<LL, NP, (LL < 64 ? 8 : 16)>(yrow, q2e, tb2, wh, wl);
                    // lane holds Z[q2 = 32 qb + acc_row(v)][t1]; b_c[(a1 - t1) % Ll][q2] += Z.
                    // LDS adds without return: the accumulator is private to the
                    // wave, the lanes of one add hit distinct words and one wave's
                    // LDS operations complete in order, so the sums are deterministic
                    if (t1ok) {
                        int q1 = a1 - t1;
                        q1 = q1 < 0 ? q1 + LL : q1;
                        float* brow = bw + q1 * G::BP;
#pragma unroll
                        for (int v = 0; v < 16; ++v) {
                            const int qq = 32 * qb + acc_row(v, lane);
                            if (qq < LL) brow[qq] += z[v];
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    if (cok) {
        // b: the four tiles' accumulators in a fixed order
        float* bo = p.bpart + ((int64_t)chunk * p.KK + comp) * (LL * LL);
        for (int e = threadIdx.x; e < LL * LL; e += 256) {
            const int r = (e / LL) * G::BP + (e % LL);
            bo[e] = ((bacc[r] + bacc[LL * G::BP + r]) + bacc[2 * LL * G::BP + r]) + bacc[3 * LL * G::BP + r];
        }
        // c: lane holds c[t1][t2 = 32 tb2 + acc_row(v)] of its tile
        float* co = p.cpart + ((int64_t)chunk * p.KK + comp) * (LL * LL);
        if (t1ok) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int t2 = 32 * tb2 + acc_row(v, lane);
                if (t2 < LL) co[t1 * LL + t2] = cnt[v];
            }
        }
    }
}

// ---- per-job preparation: both prepared layouts of y - mu and the FP64
// squared norms (same summation order as the FP32 forms).  One block per group
// of 8 observations, staged whole in dynamic LDS ([o][r1][r2], pitch Ll + 1).
template <int LL>
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ y, int64_t N,
                                              const double* __restrict__ centre,
                                              __bf16* __restrict__ yT, __bf16* __restrict__ yo,
                                              double* __restrict__ ynorm) {
    using G = Geo<LL>;
    constexpr int SPF = LL + 1;
    extern __shared__ float s[];
    const int64_t grp = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int P4 = LL * LL / 4;
    const float mu = centre_of(centre);
    for (int e = threadIdx.x; e < 8 * P4; e += 256) {
        const int o = e / P4, qq = e % P4;
        const int64_t oi = grp * 8 + o;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (oi < N) {
            v = reinterpret_cast<const float4*>(y + oi * (int64_t)(LL * LL))[qq];
            v.x -= mu; v.y -= mu; v.z -= mu; v.w -= mu;
        }
        const int r1 = (4 * qq) / LL, r2 = (4 * qq) % LL;
        float* d = s + (o * LL + r1) * SPF + r2;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
    }
    __syncthreads();
    for (int k = 0; k < 2; ++k) {
        const int o = 2 * wave + k;
        const int64_t oi = grp * 8 + o;
        double acc = 0.0;
        for (int pp = lane; pp < P4; pp += 64) {
            const int r1 = (4 * pp) / LL, r2 = (4 * pp) % LL;
            const float* d = s + (o * LL + r1) * SPF + r2;
#pragma unroll
            for (int e = 0; e < 4; ++e) acc += (double)d[e] * d[e];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0 && oi < N) ynorm[oi] = acc;
    }
    // yT[o][jb][plane][r2][16]: runs of 8 consecutive r1
    for (int e = threadIdx.x; e < 8 * G::JS * LL * 2; e += 256) {
        const int o = e / (G::JS * LL * 2), r = e % (G::JS * LL * 2);
        const int jb = r / (LL * 2), col = (r / 2) % LL, half = r & 1;
        const int64_t oi = grp * 8 + o;
        if (oi >= N) continue;
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = s[(o * LL + 16 * jb + 8 * half + k) * SPF + col];
        bf16x8 h, l;
        split8(v, h, l);
        uint4* t = reinterpret_cast<uint4*>(yT + (oi * G::JS + jb) * (int64_t)(2 * LL * 16));
        t[col * 2 + half] = __builtin_bit_cast(uint4, h);
        t[LL * 2 + col * 2 + half] = __builtin_bit_cast(uint4, l);
    }
    // Yo[plane][r1][r2][o]
    uint4* gdst = reinterpret_cast<uint4*>(yo + grp * (int64_t)G::YO_GRP);
    for (int e = threadIdx.x; e < LL * LL; e += 256) {
        const int r1 = e / LL, r2 = e % LL;
        float v[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) v[o] = s[(o * LL + r1) * SPF + r2];
        bf16x8 h, l;
        split8(v, h, l);
        gdst[e] = __builtin_bit_cast(uint4, h);
        gdst[LL * LL + e] = __builtin_bit_cast(uint4, l);
    }
}

template <int LL> constexpr size_t lds_prep() { return sizeof(float) * 8 * LL * (LL + 1); }
template <int LL> constexpr size_t lds_pass1() { return sizeof(__bf16) * Geo<LL>::ST_YT; }
template <int LL> constexpr size_t lds_pass2() {
    return sizeof(float) * 4 * LL * Geo<LL>::BP + sizeof(__bf16) * Geo<LL>::ST;
}

}  // namespace b16w
}  // namespace srmra
