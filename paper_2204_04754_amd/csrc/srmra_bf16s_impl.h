// BF16 split-precision matrix-core form for L_low = 16: one 16x16 score tile
// per (observation, component) on v_mfma_f32_16x16x32_bf16 (no padding), the
// operand split and products of srmra_bf16_impl.h.
//
// 16x16x32 lane layout: A[i][k] from lane (i = l % 16, kg = l / 16) with
// k = 8 kg + e; B[k][j] from lane (j = l % 16, kg); D[i][j] in lane
// (j = l % 16, kg) as rows i = 4 kg + v, v = 0..3.
// Score tile (rows t2, cols t1), k-step ks = 0..7 over the pixels: lane group
// kg reads column b2 = 2 ks + (kg >> 1) and the run of 8 r1 starting at
// 8 (kg & 1):
//   A[t2][k] = y_i[r1][(b2 + t2) % 16]   (prepared yT planes, 16 bytes per lane)
//   B[k][t1] = x_c[(r1 - t1) % 16][b2]   (prebuilt per step, split hi/lo)
// Back-projection (row a1), k = (t2 = 4 kg + v, o = e) over 8 observations:
//   Z[q2][t1] = sum_v sum_{kg,e} y_e[a1][(q2 + 4 kg + v) % 16] * w_e[t1][4 kg + v],
// folded into b_c[(a1 - t1) % 16][q2].
//
// A wave owns 8 observations x 4 component slots; a block is 4 waves laid
// out as WO observation slots x WC component slots (WO * WC = 4), so it
// covers 8 WO observations and 4 WC components.  Pass 1 writes one (max, sum)
// partial per observation and group of 4 components (slot s covers
// components 4s..4s+3; the ceil(K^2 / 4) slots with a component are written,
// waves whose 4 slots are all past K^2 stay idle).
#pragma once
#include "srmra_bf16w_impl.h"

namespace srmra {
namespace b16s {

using b16::split8;
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int LL = 16;
constexpr int NK = 8;        // k-steps of 32 per score tile
constexpr int SP = 24;       // staged yT row pitch in bf16 (16 r1 + 8): conflict-free 16-byte reads
constexpr int BP = LL + 1;   // b accumulator pitch (floats)

// The prepared layouts are those of the 2 x 2-tile form at L_low 16 (one r1
// slice): yT [N][plane][col][16 r1], Yo [ceil(N/8)][plane][r1][col][8].
typedef b16w::Prep Prep;

template <int NP>
__device__ __forceinline__ floatx4 mfma_split(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                              const bf16x8& bl, floatx4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    if constexpr (NP == 4) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl, c, 0, 0, 0);
    return c;
}

// x of component c (less mu) as B fragments of every k-step: layout
// [c][ks][plane][lane] of 16-byte fragments; one wave per (c, ks).
__device__ __forceinline__ void pack_xb_body(const StepArgs& p, const float* __restrict__ x, int c, int ks,
                                             uint4* __restrict__ xb) {
    const int lane = threadIdx.x & 63;
    const int c1 = c / p.K, c2 = c % p.K;
    const int t1 = lane & 15, kg = lane >> 4;
    const int b2 = 2 * ks + (kg >> 1), r0 = 8 * (kg & 1);
    const float mu = centre_of(p.centre);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int r = (r0 + e - t1) & (LL - 1);
        v[e] = x[(int64_t)(c1 + r * p.K) * p.Lh + (c2 + b2 * p.K)] - mu;
    }
    bf16x8 h, l;
    split8(v, h, l);
    uint4* dst = xb + ((int64_t)(c * NK + ks) * 2) * 64;
    dst[lane] = __builtin_bit_cast(uint4, h);
    dst[64 + lane] = __builtin_bit_cast(uint4, l);
}

// block layout: WC component slots of 4 components per block (WC in {1, 2, 4};
// a block then covers 8 (4 / WC) observations and 4 WC components).  The
// default for K^2 components; the plan's tuning table may pick another, and
// the kernels read it from p.cpb = 4 WC.
__host__ __device__ inline int wc_of(int KK) { return KK <= 4 ? 1 : (KK <= 8 ? 2 : 4); }
__device__ __forceinline__ int wc_in(const StepArgs& p) { return p.cpb >> 2; }

// yT of the block's observations [o0, o0 + 8 WO) into LDS st[o][plane][col][SP]
__device__ __forceinline__ void stage_yT(const Prep& q, int64_t N, int64_t o0, int nob, __bf16* st) {
    constexpr int CH = 2 * LL * 2;                 // 16-byte chunks per observation
    for (int e = threadIdx.x; e < nob * CH; e += 256) {
        const int o = e / CH, r = e % CH;          // r = (plane * 16 + col) * 2 + half
        uint4 v = make_uint4(0, 0, 0, 0);
        if (o0 + o < N) v = reinterpret_cast<const uint4*>(q.yT + (o0 + o) * (int64_t)(2 * LL * LL))[r];
        *reinterpret_cast<uint4*>(st + (o * 2 * LL + (r >> 1)) * SP + (r & 1) * 8) = v;
    }
}

// Yo of the block's observation groups [o0 / 8, o0 / 8 + ngrp) into LDS
// (contiguous: 2 x 16 x 16 x 8 bf16 per group); groups past the last one of
// the N observations are zero-filled
__device__ __forceinline__ void stage_yo(const Prep& q, int64_t N, int64_t o0, int ngrp, __bf16* st) {
    constexpr int CH = 2 * LL * LL;                // 16-byte chunks per group
    const int64_t g0 = o0 / 8;
    const int64_t nvalid = min<int64_t>(ngrp, (N + 7) / 8 - g0);
    const uint4* src = reinterpret_cast<const uint4*>(q.yo + g0 * (int64_t)(2 * LL * LL * 8));
    uint4* dst = reinterpret_cast<uint4*>(st);
    for (int e = threadIdx.x; e < ngrp * CH; e += 256)
        dst[e] = e / CH < nvalid ? src[e] : make_uint4(0, 0, 0, 0);
}

// Scores of the wave's 8 observations (staged slots obase..obase+7) x 4
// components (global indices cg[0..3], clamped).  PF: request the next
// k-step's B fragments before this k-step's products (pass 1; in pass 2 the
// extra registers would spill).  Either way every accumulator sees the same
// products in the same order.
template <int NP, bool PF>
__device__ __forceinline__ void score(const StepArgs& p, const __bf16* st, int obase, const int (&cg)[4],
                                      floatx4 (&acc)[8][4]) {
    const int lane = threadIdx.x & 63;
    const int t2 = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[o][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const uint4* bsrc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bsrc[c] = p.xb + (int64_t)cg[c] * NK * 128 + lane;
    bf16x8 pbh[4], pbl[4];   // PF: the fragments of the coming k-step
    if constexpr (PF) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            pbh[c] = __builtin_bit_cast(bf16x8, bsrc[c][0]);
            pbl[c] = __builtin_bit_cast(bf16x8, bsrc[c][64]);
        }
    }
    for (int ks = 0; ks < NK; ++ks) {
        bf16x8 bh[4], bl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if constexpr (PF) {
                bh[c] = pbh[c];
                bl[c] = pbl[c];
                const int kn = ks + 1 < NK ? ks + 1 : ks;   // the last step re-reads its own
                pbh[c] = __builtin_bit_cast(bf16x8, bsrc[c][kn * 128]);
                pbl[c] = __builtin_bit_cast(bf16x8, bsrc[c][kn * 128 + 64]);
            } else {
                bh[c] = __builtin_bit_cast(bf16x8, bsrc[c][ks * 128]);
                bl[c] = __builtin_bit_cast(bf16x8, bsrc[c][ks * 128 + 64]);
            }
        }
        const int b2 = 2 * ks + (kg >> 1);
        const int col = (b2 + t2) & (LL - 1);
        const __bf16* arow = st + (obase * 2 * LL + col) * SP + 8 * (kg & 1);
        bf16x8 ah[8], al[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            ah[o] = *reinterpret_cast<const bf16x8*>(arow + (o * 2 * LL) * SP);
            al[o] = *reinterpret_cast<const bf16x8*>(arow + (o * 2 * LL + LL) * SP);
        }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // products in sweeps over the 32 independent accumulators
#pragma unroll
        for (int o = 0; o < 8; ++o)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[o][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[o], bh[c], acc[o][c], 0, 0, 0);
#pragma unroll
        for (int o = 0; o < 8; ++o)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[o][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[o], bl[c], acc[o][c], 0, 0, 0);
#pragma unroll
        for (int o = 0; o < 8; ++o)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[o][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[o], bh[c], acc[o][c], 0, 0, 0);
        if constexpr (NP == 4) {
#pragma unroll
            for (int o = 0; o < 8; ++o)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[o][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[o], bl[c], acc[o][c], 0, 0, 0);
        }
    }
}

// bias of a lane's slots: bet[c][v] at (t1 = lane % 16, t2 = 4 (lane / 16) + v); -inf for c >= KK
__device__ __forceinline__ void lane_bias(const StepArgs& p, const int (&cgl)[4], float (&bet)[4][4]) {
    const int lane = threadIdx.x & 63;
    const int t1 = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            bet[c][v] = cgl[c] < p.KK ? p.betaT[(int64_t)cgl[c] * (LL * LL) + (4 * kg + v) * LL + t1] : -INFINITY;
}

// ============================================================================
// Pass 1.  Item (chunk, component group g): components 4 WC g ..; wave (wo, wc)
// = observation slot wo, component slot wc.
__device__ __forceinline__ void wave_slots(const StepArgs& p, int cgroup, int& wo, int& wc, int (&cgl)[4],
                                           int (&cgc)[4], int& WO) {
    const int WC = wc_in(p);
    WO = 4 / WC;
    const int wave = threadIdx.x >> 6;
    wo = wave % WO;
    wc = wave / WO;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cgl[c] = (cgroup * WC + wc) * 4 + c;             // global component (may be >= KK)
        cgc[c] = cgl[c] < p.KK ? cgl[c] : p.KK - 1;      // clamped for loads
    }
}

template <int NP>
__device__ __forceinline__ void pass1_body(const StepArgs& p, const Prep& q, int chunk, int cgroup,
                                           float* lds) {
    __bf16* st = reinterpret_cast<__bf16*>(lds);
    const int lane = threadIdx.x & 63;
    int wo, wc, WO, cgl[4], cgc[4];
    wave_slots(p, cgroup, wo, wc, cgl, cgc, WO);
    const bool active = cgl[0] < p.KK;                    // wave-uniform
    float bet[4][4];
    lane_bias(p, cgl, bet);
    const int nob = 8 * WO;
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    const int slot = cgroup * wc_in(p) + wc;              // partial index of this wave's components
    for (int64_t o0 = c0; o0 < c1; o0 += nob) {
        __syncthreads();
        stage_yT(q, p.N, o0, nob, st);
        __syncthreads();
        if (!active) continue;
        floatx4 acc[8][4];
        score<NP, true>(p, st, 8 * wo, cgc, acc);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int64_t oi = o0 + 8 * wo + o;
            float mx = -INFINITY;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float a = acc[o][c][v] * p.inv_s2 + bet[c][v];
                    acc[o][c][v] = a;
                    mx = fmaxf(mx, a);
                }
            for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
            float s = 0.f;
            if (mx > -INFINITY) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (acc[o][c][v] > -INFINITY) s += fast_exp(acc[o][c][v] - mx);
            }
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (lane == 0 && oi < c1) p.part[(int64_t)slot * p.N + oi] = make_float2(mx, s);
        }
    }
}

// ============================================================================
// Pass 2: posterior weights, posterior mass and back-projection of the wave's
// 8 observations x 4 components; per-chunk partials of the block's components.
template <int NP>
__device__ __forceinline__ void pass2_body(const StepArgs& p, const Prep& q, int chunk, int cgroup,
                                           float* lds) {
    float* bacc = lds;                                                   // [4 waves][4 comps][16][BP]
    __bf16* st = reinterpret_cast<__bf16*>(bacc + 16 * LL * BP);         // staging (yT, then Yo)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, kg = lane >> 4;
    int wo, wc, WO, cgl[4], cgc[4];
    wave_slots(p, cgroup, wo, wc, cgl, cgc, WO);
    const bool active = cgl[0] < p.KK;
    float* bw = bacc + wave * 4 * LL * BP;
    for (int e = lane; e < 4 * LL * BP; e += 64) bw[e] = 0.f;
    float bet[4][4], cnt[4][4];
    lane_bias(p, cgl, bet);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) cnt[c][v] = 0.f;
    const int nob = 8 * WO;
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += nob) {
        __syncthreads();
        stage_yT(q, p.N, o0, nob, st);
        __syncthreads();
        bf16x8 wh[4][4], wl[4][4];   // [component][v]: B fragments over k = (t2, o)
        if (active) {
            floatx4 acc[8][4];
            score<NP, false>(p, st, 8 * wo, cgc, acc);
            float2 lse[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int64_t oi = o0 + 8 * wo + o;
                lse[o] = oi < c1 ? p.lse[oi] : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float w[8];
#pragma unroll
                    for (int o = 0; o < 8; ++o) {
                        float ww = 0.f;
                        if (o0 + 8 * wo + o < c1) {
                            const float a = acc[o][c][v] * p.inv_s2 + bet[c][v];
                            ww = a > -INFINITY ? fast_exp((a - lse[o].x) - lse[o].y) : 0.f;
                        }
                        w[o] = ww;
                        cnt[c][v] += ww;
                    }
                    split8(w, wh[c][v], wl[c][v]);
                }
        }
        __syncthreads();
        stage_yo(q, p.N, o0, WO, st);
        __syncthreads();
        if (!active) continue;
        const __bf16* yg = st + wo * (2 * LL * LL * 8);   // this wave's 8-observation group
        for (int a1 = 0; a1 < LL; ++a1) {
            const __bf16* yrow = yg + a1 * LL * 8;
            bf16x8 ah[4], al[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = (j + 4 * kg + v) & (LL - 1);
                ah[v] = *reinterpret_cast<const bf16x8*>(yrow + col * 8);
                al[v] = *reinterpret_cast<const bf16x8*>(yrow + LL * LL * 8 + col * 8);
            }
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            floatx4 z[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) z[c] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int c = 0; c < 4; ++c) z[c] = mfma_split<NP>(ah[v], al[v], wh[c][v], wl[c][v], z[c]);
            // lane holds Z_c[q2 = 4 kg + vv][t1 = j]; b_c[(a1 - t1) % 16][q2] += Z
            const int q1 = (a1 - j) & (LL - 1);
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) bw[(c * LL + q1) * BP + 4 * kg + vv] += z[c][vv];
        }
    }
    __syncthreads();
    // per-chunk partials: the WO waves of each component slot summed in order
    const int WC = wc_in(p);
    for (int e = threadIdx.x; e < WC * 4 * LL * LL; e += 256) {
        const int s = e / (4 * LL * LL), r = e % (4 * LL * LL);   // s = component slot wc
        const int c = r / (LL * LL), qq = r % (LL * LL);
        const int comp = (cgroup * WC + s) * 4 + c;
        if (comp >= p.KK) continue;
        float sum = 0.f;
        for (int w = 0; w < WO; ++w)
            sum += bacc[((s * WO + w) * 4 + c) * LL * BP + (qq / LL) * BP + (qq % LL)];
        p.bpart[((int64_t)chunk * p.KK + comp) * (LL * LL) + qq] = sum;
    }
    // posterior mass: lane holds c[t1 = j][t2 = 4 kg + v]; the WO waves of a
    // component slot go through LDS (reusing the b accumulators)
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) bw[(c * LL + j) * BP + 4 * kg + v] = cnt[c][v];
    __syncthreads();
    for (int e = threadIdx.x; e < WC * 4 * LL * LL; e += 256) {
        const int s = e / (4 * LL * LL), r = e % (4 * LL * LL);
        const int c = r / (LL * LL), tt = r % (LL * LL);
        const int comp = (cgroup * WC + s) * 4 + c;
        if (comp >= p.KK) continue;
        float sum = 0.f;
        for (int w = 0; w < WO; ++w)
            sum += bacc[((s * WO + w) * 4 + c) * LL * BP + (tt / LL) * BP + (tt % LL)];
        p.cpart[((int64_t)chunk * p.KK + comp) * (LL * LL) + tt] = sum;
    }
}

constexpr size_t lds_pass1() { return sizeof(__bf16) * 32 * 2 * LL * SP; }
constexpr size_t lds_pass2() {
    return sizeof(float) * 16 * LL * BP +
           sizeof(__bf16) * (32 * 2 * LL * SP > 4 * 2 * LL * LL * 8 ? 32 * 2 * LL * SP : 4 * 2 * LL * LL * 8);
}

}  // namespace b16s
}  // namespace srmra
