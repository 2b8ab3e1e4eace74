// BF16 split-precision single pass for L_low = 48 and K^2 <= 4 on
// v_mfma_f32_16x16x32_bf16: the 48 x 48 score map of an (observation,
// component) pair is exactly 3 x 3 tiles of 16 x 16, so no tile work is padding
// (the 32 x 32 tiling of srmra_bf16w_impl.h uses 56% of its work at L_low 48),
// and the posterior weights, the back-projection and the posterior mass follow
// the scores in the same workgroup (no second pass recomputing them).
//
// A workgroup is 4 waves, wave w the component w (all K^2 <= 4 components of
// its observations), and takes its chunk's observations in groups of 4.  For a
// group, wave w holds the 4 x 9 tiles S_o[t2][t1] of its component (t2 in tile
// row R, t1 in tile column C) in 144 accumulator registers per lane.
//
// Score tile (R, C), k over the pixels in runs of 8 r1: k-step s (0..71) gives
// lane group kg the run rho = 4 s + kg, i.e. column b2 = rho / 6 and rows
// r1 = 8 (rho % 6) + e, e = 0..7:
//   A[t2][k] = y_o[r1][(b2 + t2) % 48]         (16 bytes of the staged yT planes)
//   B[k][t1] = x_c[(r1 - t1) % 48][b2] / sigma^2  (prebuilt per step, split hi/lo)
// and the shift prior beta[c][t2][t1] is added once the tile is complete (the
// accumulators start from zero: started from beta, whose magnitude is that of
// ||x_c||^2 / 2 sigma^2, every FP32 accumulation would round at that scale), so
// a tile ends as the log-joint terms of its 256 shifts.
// Back-projection for each row a1, k = (two t2 rows, 4 observations):
//   Z[q2][t1] = sum_{t2, o} y_o[a1][(q2 + t2) % 48] * w_o[t1][t2]
// over k-steps (R, h): lane group kg holds t2 = 16 R + 4 kg + 2 h + (e >> 2) and
// o = e & 3 -- rows of its own score accumulators, so the weights are the B
// fragments as they stand -- and the A fragment is two 8-byte records of the
// staged 4-observation layout Yo4[plane][a1][col][4].  Z (3 x 3 tiles over
// (q2, t1)) is folded into b_c[(a1 - t1) % 48][q2] in the wave's own LDS
// accumulator, four consecutive q2 per 16-byte update.
// The posterior mass c_c[t1][t2] of the lane's 36 (t1, t2) slots is added into
// the chunk's partial in global memory group by group (nine 16-byte runs).
#pragma once
#include "srmra_bf16s_impl.h"

namespace srmra {
namespace b16n {

using b16::split8;
using b16s::floatx4;

constexpr int LL = 48;
constexpr int T = 3;                  // 16-wide tiles per axis
constexpr int NKS = LL * LL / 32;     // k-steps of 32 per score tile
constexpr int NOB = 4;                // observations per group
constexpr int NW = 4;                 // waves (component slots) per workgroup
constexpr int NT = 64 * NW;
constexpr int BP = LL + 4;            // b accumulator row pitch (floats)
constexpr int PL = LL * LL;           // Yo4 plane stride in 8-byte records

// The prepared layouts are those of the 2 x 2-tile form at L_low 48:
// yT [N][3 slices][plane][col][16 r1], Yo [ceil(N/8)][plane][r1][r2][8].
typedef b16w::Prep Prep;

// x of component c (less mu, times 1/sigma^2) as B fragments of tile column C:
// lane (t1 = 16 C + (lane & 15), kg = lane >> 4) of k-step s holds
// x_c[(8 (rho % 6) + e - t1) mod 48][rho / 6], rho = 4 s + kg, e = 0..7, split
// into hi and lo.  Layout [c][C][s][plane][lane] of 16-byte fragments.
__device__ __forceinline__ void pack_xb_body(const StepArgs& p, const float* __restrict__ x, int c, int C,
                                             int s, uint4* __restrict__ xb) {
    const int lane = threadIdx.x & 63;
    const int c1 = c / p.K, c2 = c % p.K;
    const int t1 = 16 * C + (lane & 15), kg = lane >> 4;
    const int rho = 4 * s + kg, b2 = rho / 6, r0 = 8 * (rho % 6);
    const float mu = centre_of(p.centre);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int r = r0 + e - t1;
        r = r < 0 ? r + LL : r;
        v[e] = (x[(int64_t)(c1 + r * p.K) * p.Lh + (c2 + b2 * p.K)] - mu) * p.inv_s2;
    }
    bf16x8 h, l;
    split8(v, h, l);
    uint4* dst = xb + ((int64_t)((c * T + C) * NKS + s) * 2) * 64;
    dst[lane] = __builtin_bit_cast(uint4, h);
    dst[64 + lane] = __builtin_bit_cast(uint4, l);
}

// staged yT: ys[o][plane][col][48 r1] with the six 8-r1 runs of a column
// stored at run ^ ((col >> 2) & 1), so that 16-byte reads of 8 consecutive
// columns at one run fall in distinct banks
__device__ __forceinline__ int run_slot(int col, int run) { return run ^ ((col >> 2) & 1); }

// yT planes of observations [o0, o0 + 4) into ys, zeros past N
__device__ __forceinline__ void stage_yT(const Prep& q, int64_t N, int64_t o0, __bf16* ys) {
    constexpr int CH = 3 * 2 * LL * 2;          // 16-byte chunks per observation
    for (int e = threadIdx.x; e < NOB * CH; e += NT) {
        const int o = e / CH, r = e % CH;       // r = ((jb * 2 + plane) * 48 + col) * 2 + half
        const int jb = r / (4 * LL), pc = (r >> 1) % (2 * LL), half = r & 1;
        const int plane = pc / LL, col = pc % LL;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (o0 + o < N) v = reinterpret_cast<const uint4*>(q.yT + (o0 + o) * (int64_t)(3 * 2 * LL * 16))[r];
        *reinterpret_cast<uint4*>(ys + ((o * 2 + plane) * LL + col) * LL + 8 * run_slot(col, 2 * jb + half)) = v;
    }
}

// Yo4 of observations [o0, o0 + 4) (o0 a multiple of 4): their half of the
// prepared 8-observation group, [plane][a1][col][4 obs] (8-byte records)
__device__ __forceinline__ void stage_yo4(const Prep& q, int64_t o0, __bf16* yo4) {
    constexpr int CH = 2 * LL * LL;
    const uint4* src = reinterpret_cast<const uint4*>(q.yo + (o0 / 8) * (int64_t)(2 * LL * LL * 8));
    const int half = (int)((o0 / 4) & 1);
    uint2* dst = reinterpret_cast<uint2*>(yo4);
    for (int e = threadIdx.x; e < CH; e += NT) {
        const uint4 v = src[e];
        dst[e] = half ? make_uint2(v.z, v.w) : make_uint2(v.x, v.y);
    }
}

template <int NP>
__device__ __forceinline__ void mfma3(const bf16x8& ah, const bf16x8& al, const bf16x8 (&bh)[T],
                                      const bf16x8 (&bl)[T], floatx4 (&acc)[T]) {
#pragma unroll
    for (int C = 0; C < T; ++C) acc[C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[C], acc[C], 0, 0, 0);
#pragma unroll
    for (int C = 0; C < T; ++C) acc[C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[C], acc[C], 0, 0, 0);
#pragma unroll
    for (int C = 0; C < T; ++C) acc[C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[C], acc[C], 0, 0, 0);
    if constexpr (NP == 4) {
#pragma unroll
        for (int C = 0; C < T; ++C) acc[C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl[C], acc[C], 0, 0, 0);
    }
}

template <int NP>
__device__ __forceinline__ void fused_body(const StepArgs& p, const Prep& q, int chunk_i, float* lds) {
    float* bacc = lds;                                                 // NW x 48 x BP
    __bf16* ys = reinterpret_cast<__bf16*>(bacc + NW * LL * BP);       // yT, then Yo4, of the group
    float2* red = reinterpret_cast<float2*>(ys + NOB * 2 * LL * LL);   // NW x NOB
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i16 = lane & 15, kg = lane >> 4;
    const bool cok = wave < p.KK;
    const int comp = cok ? wave : p.KK - 1;
    float* bw = bacc + wave * LL * BP;
    for (int e = lane; e < LL * BP; e += 64) bw[e] = 0.f;
    const int64_t chunk = chunk_i;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    const uint4* xbase = p.xb + (int64_t)comp * T * NKS * 128 + lane;
    const float* bet = p.betaT + (int64_t)comp * (LL * LL);
    for (int64_t o0 = c0; o0 < c1; o0 += NOB) {
        __syncthreads();
        stage_yT(q, p.N, o0, ys);
        __syncthreads();
        // lane holds t1 = 16 C + i16, t2 = 16 R + 4 kg + v of each tile
        floatx4 acc[NOB][T][T];
#pragma unroll
        for (int o = 0; o < NOB; ++o)
#pragma unroll
            for (int R = 0; R < T; ++R)
#pragma unroll
                for (int C = 0; C < T; ++C) acc[o][R][C] = floatx4{0.f, 0.f, 0.f, 0.f};
        // ---- scores
        bf16x8 bh[T], bl[T], nh[T], nl[T];
#pragma unroll
        for (int C = 0; C < T; ++C) {
            bh[C] = __builtin_bit_cast(bf16x8, xbase[(C * NKS) * 128]);
            bl[C] = __builtin_bit_cast(bf16x8, xbase[(C * NKS) * 128 + 64]);
        }
        for (int s = 0; s < NKS; ++s) {
            const int sn = s + 1 < NKS ? s + 1 : s;
#pragma unroll
            for (int C = 0; C < T; ++C) {
                nh[C] = __builtin_bit_cast(bf16x8, xbase[(C * NKS + sn) * 128]);
                nl[C] = __builtin_bit_cast(bf16x8, xbase[(C * NKS + sn) * 128 + 64]);
            }
            const int rho = 4 * s + kg, b2 = rho / 6, run = rho % 6;
#pragma unroll
            for (int R = 0; R < T; ++R) {
                int col = b2 + 16 * R + i16;
                col = col >= LL ? col - LL : col;
                col = col >= LL ? col - LL : col;
                const __bf16* a = ys + col * LL + 8 * run_slot(col, run);
#pragma unroll
                for (int o = 0; o < NOB; ++o) {
                    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(a + (o * 2) * LL * LL);
                    const bf16x8 al = *reinterpret_cast<const bf16x8*>(a + (o * 2 + 1) * LL * LL);
                    mfma3<NP>(ah, al, bh, bl, acc[o][R]);
                }
            }
#pragma unroll
            for (int C = 0; C < T; ++C) {
                bh[C] = nh[C];
                bl[C] = nl[C];
            }
        }
        // the shift prior (and the observations past N out of every sum: their
        // terms exp(-inf) = 0)
#pragma unroll
        for (int R = 0; R < T; ++R)
#pragma unroll
            for (int C = 0; C < T; ++C)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float b = bet[(16 * R + 4 * kg + v) * LL + 16 * C + i16];
#pragma unroll
                    for (int o = 0; o < NOB; ++o) acc[o][R][C][v] += b;
                }
        bool ook[NOB];
#pragma unroll
        for (int o = 0; o < NOB; ++o) {
            ook[o] = o0 + o < p.N;
            if (!ook[o]) {
#pragma unroll
                for (int R = 0; R < T; ++R)
#pragma unroll
                    for (int C = 0; C < T; ++C) acc[o][R][C] = floatx4{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
            }
        }
        // the wave's (max, sum exp) per observation, then the block's log-sum-exp
        float mw[NOB], sw[NOB];
#pragma unroll
        for (int o = 0; o < NOB; ++o) {
            float m = -INFINITY;
#pragma unroll
            for (int R = 0; R < T; ++R)
#pragma unroll
                for (int C = 0; C < T; ++C)
#pragma unroll
                    for (int v = 0; v < 4; ++v) m = fmaxf(m, acc[o][R][C][v]);
            for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
            mw[o] = m;
            const float mref = m > -INFINITY ? m : 0.f;
            float sum = 0.f;
#pragma unroll
            for (int R = 0; R < T; ++R)
#pragma unroll
                for (int C = 0; C < T; ++C)
#pragma unroll
                    for (int v = 0; v < 4; ++v) sum += fast_exp(acc[o][R][C][v] - mref);
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            sw[o] = sum;
        }
        float2 lse[NOB];
        b16::block_lse<NOB, NW>(p, mw, sw, wave, o0, p.N, wave == 0, [&](int k) { return k < p.KK; }, red, lse);
        // every wave is past its score: the buffer takes the group's Yo4
        stage_yo4(q, o0, ys);
        // posterior weights as B fragments of the back-projection (k-step (R, h):
        // element e = weight of t2 = 16 R + 4 kg + 2 h + (e >> 2), observation
        // e & 3), and the lane's posterior masses into the chunk's partial
        bf16x8 wh[T][T][2], wl[T][T][2];
        const bool first = o0 == c0;
#pragma unroll
        for (int C = 0; C < T; ++C) {
            float* cp = p.cpart + (chunk * p.KK + comp) * (LL * LL) + (16 * C + i16) * LL + 4 * kg;
#pragma unroll
            for (int R = 0; R < T; ++R) {
                float4 cm = (cok && !first) ? *reinterpret_cast<const float4*>(cp + 16 * R) : make_float4(0.f, 0.f, 0.f, 0.f);
                float wv[4][NOB];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float msum = 0.f;
#pragma unroll
                    for (int o = 0; o < NOB; ++o) {
                        // an observation past N has lse (0, 0) and only -inf terms
                        const float ww = fast_exp((acc[o][R][C][v] - lse[o].x) - lse[o].y);
                        wv[v][o] = ww;
                        msum += ww;
                    }
                    switch (v) {
                        case 0: cm.x += msum; break;
                        case 1: cm.y += msum; break;
                        case 2: cm.z += msum; break;
                        default: cm.w += msum; break;
                    }
                }
                if (cok) *reinterpret_cast<float4*>(cp + 16 * R) = cm;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    float w8[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) w8[e] = wv[2 * h + (e >> 2)][e & 3];
                    split8(w8, wh[C][R][h], wl[C][R][h]);
                }
            }
        }
        __syncthreads();   // Yo4 staged
        if (cok) {
            for (int a1 = 0; a1 < LL; ++a1) {
                const uint2* yrow = reinterpret_cast<const uint2*>(ys) + a1 * LL;
                floatx4 z[T][T];
#pragma unroll
                for (int M = 0; M < T; ++M)
#pragma unroll
                    for (int C = 0; C < T; ++C) z[M][C] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int R = 0; R < T; ++R)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int M = 0; M < T; ++M) {
                            // lane row q2 = 16 M + i16: columns (q2 + t2) % 48 and the next
                            int k0 = 16 * M + i16 + 16 * R + 4 * kg + 2 * h;
                            k0 = k0 >= LL ? k0 - LL : k0;
                            k0 = k0 >= LL ? k0 - LL : k0;
                            const int k1 = k0 + 1 >= LL ? k0 + 1 - LL : k0 + 1;
                            const uint2 h0 = yrow[k0], h1 = yrow[k1];
                            const uint2 l0 = yrow[PL + k0], l1 = yrow[PL + k1];
                            const bf16x8 ah = __builtin_bit_cast(bf16x8, make_uint4(h0.x, h0.y, h1.x, h1.y));
                            const bf16x8 al = __builtin_bit_cast(bf16x8, make_uint4(l0.x, l0.y, l1.x, l1.y));
                            bf16x8 bhh[T], bll[T];
#pragma unroll
                            for (int C = 0; C < T; ++C) {
                                bhh[C] = wh[C][R][h];
                                bll[C] = wl[C][R][h];
                            }
                            mfma3<NP>(ah, al, bhh, bll, z[M]);
                        }
                // lane holds Z[q2 = 16 M + 4 kg + v][t1 = 16 C + i16]:
                // b_c[(a1 - t1) % 48][q2 .. q2 + 3] += Z (the wave's own accumulator;
                // the 16 lanes of one update hit 16 different rows)
#pragma unroll
                for (int C = 0; C < T; ++C) {
                    int q1 = a1 - (16 * C + i16);
                    q1 = q1 < 0 ? q1 + LL : q1;
                    float* brow = bw + q1 * BP + 4 * kg;
#pragma unroll
                    for (int M = 0; M < T; ++M) {
                        float4* d = reinterpret_cast<float4*>(brow + 16 * M);
                        float4 t = *d;
                        t.x += z[M][C][0];
                        t.y += z[M][C][1];
                        t.z += z[M][C][2];
                        t.w += z[M][C][3];
                        *d = t;
                    }
                }
            }
        }
    }
    // ---- this block's partial of b for the wave's component
    __syncthreads();
    if (cok) {
        float* bo = p.bpart + (chunk * p.KK + comp) * (LL * LL);
        for (int e = lane; e < LL * LL; e += 64) bo[e] = bw[(e / LL) * BP + (e % LL)];
    }
}

constexpr size_t lds_fused() {
    return sizeof(float) * NW * LL * BP + sizeof(__bf16) * NOB * 2 * LL * LL + sizeof(float2) * NW * NOB;
}

}  // namespace b16n
}  // namespace srmra
