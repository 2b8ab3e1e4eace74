// BF16 split-precision matrix-core form at L_low 8 and 12: the Ll x Ll score
// maps of 8 observations and NCW components are packed into 32x32 tiles with
// no padding (v_mfma_f32_32x32x16_bf16; operands split as in srmra_bf16_impl.h).
//
// Score block of one wave: rows R = 8 t2 + o (its 8 observations at every
// offset t2), columns C = Ll c + t1 (its NCW components at every offset t1).
// Ll * 8 and Ll * NCW are multiples of 32, so every element of every tile is
// the score of one shift of one observation.  k = Ll b2 + r1 runs over the
// pixels, 16 per k-step (lane half g holds k = 16 s + 8 g + e, e = 0..7):
//   A[R][k] = y_o[r1][(b2 + t2) % Ll] = yT_o[(k + Ll t2) mod Ll^2]
//   B[k][C] = x_c[(r1 - t1) % Ll][b2] / sigma^2     (prebuilt per step)
// with yT_o the transpose of y_o flattened, so a lane's 8 values are one run of
// it (Ll 8) or two runs of 4 (Ll 12).  The shift prior is added once the tile
// is complete, as in the other BF16 forms.
// Accumulator element v of row tile rt in lane (j = lane & 31, g = lane >> 5)
// is row R = 32 rt + 8 (v >> 2) + 4 g + (v & 3): observation o = 4 g + (v & 3)
// at offset t2 = 4 rt + (v >> 2), column C = 32 ct + j.
// Back-projection (right-hand side of eq. x_EM), k = R over the score rows:
//   Z[(a1, q2)][C] = sum_R y_o[a1][(q2 + t2) % Ll] * w[R][C],
// 16 rows per k-step (rt, p): the B values of a lane are its own posterior
// weights v = 8 p + e (rows 32 rt + 16 p + 8 (e >> 2) + 4 g + (e & 3)), its A
// values are y_o[a1][(q2 + t2) % Ll] of the observations 4 g .. 4 g + 3 at
// t2 = 4 rt + 2 p and 4 rt + 2 p + 1: two 8-byte records of the
// observation-interleaved planes Yo[a1][col][8 obs].  Then
// b_c[(a1 - t1) % Ll][q2] += Z; the lanes of one update never meet on an
// element (a lane half has one (a1, q2), its lanes distinct (c, t1), and the
// halves are 4 rows, i.e. 4 different q2, apart).
//
// A workgroup is 4 waves: WO = 4 / WCB observation slots of 8 observations x
// WCB blocks of NCW components (p.cpb = WCB NCW).  Single pass (all K^2
// components in the workgroup): the waves of one observation slot exchange
// their (max, sum) through LDS.  Two passes (K^2 > 4 NCW): WCB = 4, pass 1
// writes one (max, sum) per (wave, observation), pass 2 reads the combined
// log-sum-exp.  At the end of a chunk the WO waves of a component block add
// their b and posterior-mass sums in slot order into the chunk's partial.
#pragma once
#include "srmra_bf16_impl.h"

namespace srmra {
namespace b16p {

using b16::split8;

template <int LL> struct Geo {
    static_assert(LL == 8 || LL == 12, "packed tiles: L_low 8 or 12");
    static constexpr int NO = 8;                        // observations per wave
    static constexpr int NCW = LL == 8 ? 4 : 8;         // components per wave
    static constexpr int NR = LL * NO / 32;             // score row tiles: 2, 3
    static constexpr int NCT = LL * NCW / 32;           // score column tiles: 1, 3
    static constexpr int NKS = LL * LL / 16;            // score k-steps: 4, 9
    static constexpr int NZT = (LL * LL + 31) / 32;     // back-projection row tiles: 2, 5
    static constexpr int PL = LL * LL;                  // one plane of one observation (bf16)
    static constexpr int YTS = 2 * PL + 8;              // staged yT per observation (bf16)
    static constexpr int YO = 2 * PL * NO;              // Yo per 8-observation group (bf16)
    static constexpr int BPL = LL + 1;                  // b accumulator row pitch (floats)
    static constexpr int MAXT = 32;                     // observations per block tile, at most
    // Ll 8: the x fragments (8 of them) stay in registers for the whole chunk,
    // and so does Z (2 tiles), folded once at the end of the chunk
    static constexpr bool XREG = LL == 8;
    static constexpr bool ZREG = LL == 8;
};

// components per wave (host side too)
__host__ __device__ constexpr int ncw_of(int LL) { return LL == 8 ? 4 : 8; }

// x as B fragments: global column tile gct (component block gct / NCT, tile
// gct % NCT), k-step s: lane (j, g) holds x_c[(r1 - t1) % Ll][b2] (less mu, over
// sigma^2) for column C = 32 (gct % NCT) + j = Ll (c - NCW block) + t1 and
// k = 16 s + 8 g + e = Ll b2 + r1; zeros for components past K^2.
// Layout [gct][s][plane][lane] of 16-byte fragments.
template <int LL>
__device__ __forceinline__ void pack_xb_body(const StepArgs& p, const float* __restrict__ x, int gct, int s,
                                             uint4* __restrict__ xb) {
    using G = Geo<LL>;
    const int lane = threadIdx.x & 63;
    const int j = lane & 31, g = lane >> 5;
    const int cb = gct / G::NCT, C = 32 * (gct % G::NCT) + j;
    const int c = cb * G::NCW + C / LL, t1 = C % LL;
    const float mu = centre_of(p.centre);
    float v[8];
    const int c1 = c / p.K, c2 = c % p.K;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 16 * s + 8 * g + e;
        const int b2 = k / LL, r1 = k % LL;
        int r = r1 - t1;
        r = r < 0 ? r + LL : r;
        v[e] = c < p.KK ? (x[(int64_t)(c1 + r * p.K) * p.Lh + (c2 + b2 * p.K)] - mu) * p.inv_s2 : 0.f;
    }
    bf16x8 h, l;
    split8(v, h, l);
    uint4* dst = xb + ((int64_t)(gct * G::NKS + s) * 2) * 64;
    dst[lane] = __builtin_bit_cast(uint4, h);
    dst[64 + lane] = __builtin_bit_cast(uint4, l);
}

// yT of observations [o0, o0 + nob) into LDS (YTS bf16 per observation), zeros past N
template <int LL>
__device__ __forceinline__ void stage_yT(const b16::Prep& q, int64_t N, int64_t o0, int nob, __bf16* ys) {
    using G = Geo<LL>;
    constexpr int CH = 2 * G::PL / 8;   // 16-byte chunks per observation
    for (int e = threadIdx.x; e < nob * CH; e += 256) {
        const int o = e / CH, r = e % CH;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (o0 + o < N) v = reinterpret_cast<const uint4*>(q.yT + (o0 + o) * (int64_t)(2 * G::PL))[r];
        *reinterpret_cast<uint4*>(ys + o * G::YTS + 8 * r) = v;
    }
}

// Yo of the 8-observation groups [o0 / 8, o0 / 8 + ngrp) into LDS, zeros past the last group
template <int LL>
__device__ __forceinline__ void stage_yo(const b16::Prep& q, int64_t N, int64_t o0, int ngrp, __bf16* yo) {
    using G = Geo<LL>;
    constexpr int CH = G::YO / 8;
    const int64_t g0 = o0 / 8;
    const int64_t nvalid = min<int64_t>(ngrp, (N + 7) / 8 - g0);
    const uint4* src = reinterpret_cast<const uint4*>(q.yo + g0 * (int64_t)G::YO);
    uint4* dst = reinterpret_cast<uint4*>(yo);
    for (int e = threadIdx.x; e < ngrp * CH; e += 256) dst[e] = e / CH < nvalid ? src[e] : make_uint4(0, 0, 0, 0);
}

template <int NP>
__device__ __forceinline__ void products(const bf16x8& ah, const bf16x8& al, const bf16x8& bh, const bf16x8& bl,
                                         floatx16& c, int which) {
    // which: 0 = hi hi, 1 = hi lo, 2 = lo hi, 3 = lo lo
    if (which == 0) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
    else if (which == 1) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
    else if (which == 2) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
    else c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bl, c, 0, 0, 0);
}

// Score tiles of a wave: its 8 observations (staged slots ob .. ob + 7) x the
// NCT column tiles starting at global tile gct0.  XREG: xh / xl hold the
// wave's fragments of every k-step.
template <int LL, int NP, int NCT>
__device__ __forceinline__ void score(const StepArgs& p, const __bf16* ys, int ob, int gct0,
                                      const bf16x8 (&xh)[Geo<LL>::XREG ? Geo<LL>::NKS : 1],
                                      const bf16x8 (&xl)[Geo<LL>::XREG ? Geo<LL>::NKS : 1],
                                      floatx16 (&acc)[Geo<LL>::NR][NCT]) {
    using G = Geo<LL>;
    constexpr int NR = G::NR;
    static_assert(!G::XREG || NCT == 1, "fragments in registers: one column tile");
    const int lane = threadIdx.x & 63;
    const int i = lane & 31, g = lane >> 5;
#pragma unroll
    for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = floatx16{0};
    // the lane's A row in each row tile: observation slot and Ll t2
    const __bf16* arow[NR];
    int aoff[NR];
#pragma unroll
    for (int rt = 0; rt < NR; ++rt) {
        const int R = 32 * rt + i;
        arow[rt] = ys + (ob + (R & 7)) * G::YTS;
        aoff[rt] = LL * (R >> 3) + 8 * g;
    }
    const uint4* bsrc = p.xb + (int64_t)gct0 * G::NKS * 128 + lane;
    bf16x8 bh[NCT], bl[NCT];
    if constexpr (!G::XREG) {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            bh[ct] = __builtin_bit_cast(bf16x8, bsrc[(ct * G::NKS) * 128]);
            bl[ct] = __builtin_bit_cast(bf16x8, bsrc[(ct * G::NKS) * 128 + 64]);
        }
    }
    auto step = [&](int s) {
        bf16x8 nh[NCT], nl[NCT];
        if constexpr (G::XREG) {
            bh[0] = xh[s];
            bl[0] = xl[s];
        } else {
            // the next k-step's fragments are requested before this step's products
            const int sn = s + 1 < G::NKS ? s + 1 : s;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                nh[ct] = __builtin_bit_cast(bf16x8, bsrc[(ct * G::NKS + sn) * 128]);
                nl[ct] = __builtin_bit_cast(bf16x8, bsrc[(ct * G::NKS + sn) * 128 + 64]);
            }
        }
        bf16x8 ah[NR], al[NR];
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) {
            int f = 16 * s + aoff[rt];
            f = f >= G::PL ? f - G::PL : f;
            if constexpr (LL == 8) {
                ah[rt] = *reinterpret_cast<const bf16x8*>(arow[rt] + f);
                al[rt] = *reinterpret_cast<const bf16x8*>(arow[rt] + G::PL + f);
            } else {
                const int f2 = f + 4 >= G::PL ? f + 4 - G::PL : f + 4;
                const uint2 h0 = *reinterpret_cast<const uint2*>(arow[rt] + f);
                const uint2 h1 = *reinterpret_cast<const uint2*>(arow[rt] + f2);
                const uint2 l0 = *reinterpret_cast<const uint2*>(arow[rt] + G::PL + f);
                const uint2 l1 = *reinterpret_cast<const uint2*>(arow[rt] + G::PL + f2);
                ah[rt] = __builtin_bit_cast(bf16x8, make_uint4(h0.x, h0.y, h1.x, h1.y));
                al[rt] = __builtin_bit_cast(bf16x8, make_uint4(l0.x, l0.y, l1.x, l1.y));
            }
        }
        // the split products in sweeps over the independent accumulators
#pragma unroll
        for (int w = 0; w < NP; ++w)
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) products<NP>(ah[rt], al[rt], bh[ct], bl[ct], acc[rt][ct], w);
        if constexpr (!G::XREG) {
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                bh[ct] = nh[ct];
                bl[ct] = nl[ct];
            }
        }
    };
    if constexpr (G::XREG) {
        // the register-held fragments are indexed by constants only
#pragma unroll
        for (int s = 0; s < G::NKS; ++s) step(s);
    } else {
#pragma unroll 1
        for (int s = 0; s < G::NKS; ++s) step(s);
    }
}

template <int LL> constexpr size_t lds_bytes() {
    using G = Geo<LL>;
    return sizeof(float2) * 4 * G::NO +                                // (max, sum) exchange
           sizeof(float) * 4 * G::NCW * LL * G::BPL +                  // b accumulators
           sizeof(__bf16) * (G::MAXT * G::YTS + (G::MAXT / 8) * G::YO);   // staged yT, Yo
}

// MODE 1: pass 1 (partials per wave); 2: pass 2 (weights from p.lse); 3: the
// single pass.  chunk_i: observation chunk; cg: component group (cpb components).
template <int LL, int NP, int MODE>
__device__ __forceinline__ void body(const StepArgs& p, const b16::Prep& q, int chunk_i, int cg, float* lds) {
    using G = Geo<LL>;
    constexpr int NR = G::NR, NCT = G::NCT, NCW = G::NCW;
    static_assert(sizeof(float) * 4 * NCW * G::PL <= sizeof(__bf16) * (G::MAXT * G::YTS + (G::MAXT / 8) * G::YO),
                  "the masses of the 4 waves fit over the staging area");
    float2* red = reinterpret_cast<float2*>(lds);                          // 4 waves x 8
    float* bacc = reinterpret_cast<float*>(red + 4 * G::NO);               // 4 x NCW x Ll x BPL
    __bf16* ys = reinterpret_cast<__bf16*>(bacc + 4 * NCW * LL * G::BPL);  // MAXT x YTS
    __bf16* yo = ys + G::MAXT * G::YTS;                                    // MAXT / 8 x YO
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 31, g = lane >> 5;
    const int wcb = p.cpb / NCW, wo = 4 / wcb;
    const int ws = wave / wcb, cs = wave % wcb;          // observation slot, component block slot
    const int gcb = cg * wcb + cs;                       // global component block of the wave
    const int comp0 = gcb * NCW;
    const bool wact = comp0 < p.KK;                      // the wave has a component
    const int ntile = wo * G::NO;
    float* bw = bacc + wave * NCW * LL * G::BPL;
    if constexpr (MODE != 1)
        for (int e = lane; e < NCW * LL * G::BPL; e += 64) bw[e] = 0.f;
    // the lane's columns: component (local) and offset t1 of each column tile
    int ccl[NCT], ct1[NCT];
    bool cok[NCT];
    const float* bet[NCT];   // the prior row of the column's component (clamped past K^2)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        const int C = 32 * ct + j;
        ccl[ct] = C / LL;
        ct1[ct] = C % LL;
        cok[ct] = comp0 + ccl[ct] < p.KK;
        bet[ct] = p.betaT + (int64_t)min(comp0 + ccl[ct], p.KK - 1) * G::PL + ct1[ct];
    }
    bf16x8 xh[G::XREG ? G::NKS : 1], xl[G::XREG ? G::NKS : 1];
    if constexpr (G::XREG) {
        const uint4* bsrc = p.xb + (int64_t)gcb * NCT * G::NKS * 128 + lane;
#pragma unroll
        for (int s = 0; s < G::NKS; ++s) {
            xh[s] = wact ? __builtin_bit_cast(bf16x8, bsrc[s * 128]) : bf16x8{};
            xl[s] = wact ? __builtin_bit_cast(bf16x8, bsrc[s * 128 + 64]) : bf16x8{};
        }
    }
    floatx16 zacc[G::ZREG ? G::NZT : 1][NCT];
    if constexpr (G::ZREG)
#pragma unroll
        for (int zt = 0; zt < G::NZT; ++zt)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) zacc[zt][ct] = floatx16{0};
    float mass[NR][NCT][4];
#pragma unroll
    for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int m = 0; m < 4; ++m) mass[rt][ct][m] = 0.f;
    const int64_t chunk = chunk_i;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t t0 = c0; t0 < c1; t0 += ntile) {
        __syncthreads();
        stage_yT<LL>(q, p.N, t0, ntile, ys);
        if constexpr (MODE != 1) stage_yo<LL>(q, p.N, t0, wo, yo);
        __syncthreads();
        // compiler-only barrier: the per-tile loads below (the prior, the
        // log-sum-exp) stay inside the loop instead of being held in registers
        // across it
        asm volatile("" ::: "memory");
        const int64_t obs0 = t0 + ws * G::NO;   // the wave's 8 observations
        bool ook[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ook[u] = obs0 + 4 * g + u < p.N;
        // the score tiles of one column tile at a time (with more than one,
        // they are computed twice: once for the log-sum-exp, once for the
        // weights): tile(ct) leaves the log-joint terms a = score + beta of
        // column tile ct in acc, -inf in masked slots
        floatx16 acc[NR][1];
        auto tile = [&](int ct) {
            if (wact) score<LL, NP, 1>(p, ys, ws * G::NO, gcb * NCT + ct, xh, xl, acc);
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float b = bet[ct][(4 * rt + m) * LL];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool ok = wact && cok[ct] && ook[u];
                        acc[rt][0][4 * m + u] = ok ? acc[rt][0][4 * m + u] + b : -INFINITY;
                    }
                }
        };
        // (max, sum exp) of the lane half's 4 observations over the wave's
        // columns: per lane over the column tiles (rescaled as the maximum
        // grows), then over the lanes of the half
        float mw[4], sw[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            mw[u] = -INFINITY;
            sw[u] = 0.f;
        }
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            tile(ct);
            float mc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) mc[u] = mw[u];
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int v = 0; v < 16; ++v) mc[v & 3] = fmaxf(mc[v & 3], acc[rt][0][v]);
            float ref[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ref[u] = mc[u] > -INFINITY ? mc[u] : 0.f;
                sw[u] *= fast_exp(mw[u] - ref[u]);
                mw[u] = mc[u];
            }
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int v = 0; v < 16; ++v) sw[v & 3] += fast_exp(acc[rt][0][v] - ref[v & 3]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float m = mw[u];
            for (int off = 1; off < 32; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
            const float ref = m > -INFINITY ? m : 0.f;
            float t = sw[u] * fast_exp(mw[u] - ref);
            for (int off = 1; off < 32; off <<= 1) t += __shfl_xor(t, off);
            mw[u] = m;
            sw[u] = t;
        }
        if constexpr (MODE == 1) {
            // one partial per (component block, observation)
            if (j == 0) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (ook[u]) p.part[(int64_t)gcb * p.N + obs0 + 4 * g + u] = make_float2(mw[u], sw[u]);
            }
            continue;
        }
        float2 lse[4];
        if constexpr (MODE == 3) {
            // the wcb waves of the observation slot combine their pairs: lane
            // 4 o + k (o < 8 observations, k < 4 block slots) takes wave k's pair
            // of observation o, the group of 4 lanes its maximum and its FP64 sum
            // (a fixed tree, the same in every lane), and lane 4 o the log
            if (j == 0) {
#pragma unroll
                for (int u = 0; u < 4; ++u) red[wave * G::NO + 4 * g + u] = make_float2(mw[u], sw[u]);
            }
            __syncthreads();
            const int o = (lane >> 2) & 7, k = lane & 3;
            const bool act = lane < 32 && k < wcb && (cg * wcb + k) * NCW < p.KK;
            const float2 e = act ? red[(ws * wcb + k) * G::NO + o] : make_float2(-INFINITY, 0.f);
            float m = e.x;
            m = fmaxf(m, __shfl_xor(m, 1));
            m = fmaxf(m, __shfl_xor(m, 2));
            double t = (act && e.x > -INFINITY) ? (double)e.y * exp((double)e.x - (double)m) : 0.0;
            t += __shfl_xor(t, 1);
            t += __shfl_xor(t, 2);
            const float sf = (float)t;
            const float lg = m > -INFINITY ? (float)log((double)sf) : 0.f;
            if (cs == 0 && lane < 32 && k == 0 && obs0 + o < p.N) p.part[obs0 + o] = make_float2(m, sf);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float mo = __shfl(m, 4 * (4 * g + u)), lo = __shfl(lg, 4 * (4 * g + u));
                lse[u] = mo > -INFINITY ? make_float2(mo, lo) : make_float2(0.f, 0.f);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                lse[u] = ook[u] ? p.lse[obs0 + 4 * g + u] : make_float2(0.f, 0.f);
        }
        if (!wact) continue;
        const __bf16* yw = yo + ws * G::YO;
        // one column tile at a time: its posterior weights, their mass per
        // (component, shift), the weights as B fragments, and the back-projection
        // of its columns over every row tile of Z
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            if (NCT > 1) tile(ct);
            bf16x8 wh[NR][2], wl[NR][2];
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int pp = 0; pp < 2; ++pp) {
                    float w[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int v = 8 * pp + e;
                        // a masked slot is -inf: exp(-inf) = 0
                        w[e] = fast_exp((acc[rt][0][v] - lse[v & 3].x) - lse[v & 3].y);
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        mass[rt][ct][2 * pp + h] += (w[4 * h] + w[4 * h + 1]) + (w[4 * h + 2] + w[4 * h + 3]);
                    split8(w, wh[rt][pp], wl[rt][pp]);
                }
            auto zrow = [&](int zt) {
                const int rz = 32 * zt + j;          // A row (a1, q2) of this lane
                const bool rok = rz < G::PL;
                const int a1 = rok ? rz / LL : 0, q2 = rok ? rz % LL : 0;
                // 16-byte records (a1, col) of 8 observations; this half's 4 are the g-th 8 bytes
                const uint2* yrow = reinterpret_cast<const uint2*>(yw) + a1 * LL * 2 + g;
                floatx16 z;
                if constexpr (G::ZREG) z = zacc[zt][ct];
                else z = floatx16{0};
#pragma unroll
                for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                    for (int pp = 0; pp < 2; ++pp) {
                        int col0 = q2 + 4 * rt + 2 * pp;
                        col0 = col0 >= LL ? col0 - LL : col0;
                        const int col1 = col0 + 1 >= LL ? col0 + 1 - LL : col0 + 1;
                        const uint2 h0 = yrow[2 * col0], h1 = yrow[2 * col1];
                        const uint2 l0 = yrow[2 * col0 + G::PL * 2], l1 = yrow[2 * col1 + G::PL * 2];
                        bf16x8 ah = __builtin_bit_cast(bf16x8, make_uint4(h0.x, h0.y, h1.x, h1.y));
                        bf16x8 al = __builtin_bit_cast(bf16x8, make_uint4(l0.x, l0.y, l1.x, l1.y));
                        if (!rok) {
                            ah = bf16x8{};
                            al = bf16x8{};
                        }
#pragma unroll
                        for (int w = 0; w < NP; ++w) products<NP>(ah, al, wh[rt][pp], wl[rt][pp], z, w);
                    }
                if constexpr (G::ZREG) {
                    zacc[zt][ct] = z;
                } else {
                    // b_c[(a1 - t1) % Ll][q2] += Z[(a1, q2)][(c, t1)]
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int r = 32 * zt + 8 * (v >> 2) + 4 * g + (v & 3);
                        if (r < G::PL) {
                            int q1 = r / LL - ct1[ct];
                            q1 = q1 < 0 ? q1 + LL : q1;
                            bw[(ccl[ct] * LL + q1) * G::BPL + r % LL] += z[v];
                        }
                    }
                }
            };
            if constexpr (G::ZREG) {
                // the register-held Z tiles are indexed by constants only
#pragma unroll
                for (int zt = 0; zt < G::NZT; ++zt) zrow(zt);
            } else {
#pragma unroll 1
                for (int zt = 0; zt < G::NZT; ++zt) zrow(zt);
            }
        }
    }
    if constexpr (MODE == 1) return;
    if constexpr (G::ZREG) {
        if (wact) {
#pragma unroll
            for (int zt = 0; zt < G::NZT; ++zt)
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int r = 32 * zt + 8 * (v >> 2) + 4 * g + (v & 3);
                        if (r < G::PL) {
                            int q1 = r / LL - ct1[ct];
                            q1 = q1 < 0 ? q1 + LL : q1;
                            bw[(ccl[ct] * LL + q1) * G::BPL + r % LL] += zacc[zt][ct][v];
                        }
                    }
        }
    }
    // the two lane halves hold the observations 0..3 and 4..7 of each mass slot
#pragma unroll
    for (int rt = 0; rt < NR; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int m = 0; m < 4; ++m) mass[rt][ct][m] += __shfl_xor(mass[rt][ct][m], 32);
    // the waves of different observation slots hold partial sums of the same
    // components: each wave's mass goes to LDS (over the staging area, free
    // once every wave is past its last tile) beside its b accumulators, and the
    // chunk's partial of a component is their sum in slot order
    __syncthreads();
    float* massw = reinterpret_cast<float*>(ys);   // 4 waves x NCW x Ll^2 (t1 Ll + t2)
    if (g == 0) {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int rt = 0; rt < NR; ++rt)
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    massw[(wave * NCW + ccl[ct]) * G::PL + ct1[ct] * LL + 4 * rt + m] = mass[rt][ct][m];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < wcb * NCW * G::PL; e += 256) {
        const int csl = e / (NCW * G::PL), rem = e % (NCW * G::PL);
        const int cl = rem / G::PL, idx = rem % G::PL;
        const int comp = (cg * wcb + csl) * NCW + cl;
        if (comp >= p.KK) continue;
        float bs = 0.f, ms = 0.f;
        for (int k = 0; k < wo; ++k) {
            const int wv = k * wcb + csl;
            bs += bacc[((wv * NCW + cl) * LL + idx / LL) * G::BPL + idx % LL];
            ms += massw[(wv * NCW + cl) * G::PL + idx];
        }
        p.bpart[(chunk * p.KK + comp) * G::PL + idx] = bs;
        p.cpart[(chunk * p.KK + comp) * G::PL + idx] = ms;
    }
}

}  // namespace b16p
}  // namespace srmra
