// BF16 split-precision matrix-core form of the two passes of the EM step
// (L_low in {24, 32}: one 32x32 MFMA tile per (observation, component)).
//
// Every FP32 operand v is split as v = hi + lo + O(2^-17 |v|) with
// hi = bf16_rne(v), lo = bf16_rne(v - hi); a product is formed as
// hi*hi + hi*lo + lo*hi (NP = 3) or with lo*lo as well (NP = 4) with
// v_mfma_f32_32x32x16_bf16 and FP32 accumulation.
//
// Score tile (rows t2, cols t1, k = (b2, r1) over the pixels, runs of 8 r1):
//   A[t2][k] = y_i[r1][(b2+t2) % Ll]   from prepared BF16 hi/lo planes of y
//              stored column-major per observation (yT[col][r1]), so a lane's 8
//              k-values are 16 contiguous bytes;
//   B[k][t1] = x_c[(r1-t1) % Ll][b2]   read as FP32 from LDS and split on the fly.
// Back-projection (component c, the wave's 8 observations), for each a1:
//   Z[q2][t1] = sum_{t2, o} y_o[a1][(q2+t2) % Ll] * w_{o,c}[t1][t2]
// with the posterior w taken straight from the score accumulators (a lane holds
// column t1 and the rows t2 of its accumulator for all 8 observations, which
// is exactly its B fragment over k = (t2, o)), and A from the prepared
// observation-interleaved planes Yo[a1][col][o].  Z is folded into
// b_c[(a1 - t1) % Ll][q2] in the wave's private LDS accumulator.
#pragma once
#include "srmra_common.h"

namespace srmra {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace b16 {

constexpr int R1P = 32;               // padded r1 range (zeros past Ll)
constexpr int PITCH = R1P + 8;        // yT row pitch in bf16 (80 bytes: conflict-free b128)
template <int LL> struct Geo {
    static constexpr int RL = R1P + LL;               // fp32 x row length in LDS
    static constexpr int YT_OBS = 2 * LL * PITCH;     // bf16 per observation (both planes)
    static constexpr int YO_GRP = 2 * LL * LL * 8;    // bf16 per 8-observation group
    static constexpr int BP = LL + 1;                 // b accumulator pitch (floats)
};

// global prepared layout: [ynorm N doubles][yT N x 2 x Ll x 32][Yo ceil(N/8) x 2 x Ll x Ll x 8]
struct Prep {
    const __bf16* yT;
    const __bf16* yo;
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// v = hi + lo with hi = bf16_rne(v), lo = bf16_rne(v - hi); two values per
// conversion instruction (v_cvt_pk_bf16_f32), and float(hi) recovered by
// placing the 16 bits in the upper half of an FP32 word.
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& h, bf16x8& l) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        const f32x2 a = {v[e], v[e + 1]};
        const bf16x2 hh = __builtin_convertvector(a, bf16x2);
        const unsigned bits = __builtin_bit_cast(unsigned, hh);
        const float h0 = __builtin_bit_cast(float, bits << 16);
        const float h1 = __builtin_bit_cast(float, bits & 0xffff0000u);
        const f32x2 r = {v[e] - h0, v[e + 1] - h1};
        const bf16x2 ll = __builtin_convertvector(r, bf16x2);
        h[e] = hh[0];
        h[e + 1] = hh[1];
        l[e] = ll[0];
        l[e + 1] = ll[1];
    }
}

template <int NP>
__device__ __forceinline__ floatx16 mfma_split(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                               const bf16x8& bl, floatx16 c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
    if constexpr (NP == 4) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bl, c, 0, 0, 0);
    return c;
}

// Number of k-steps (b2, 16-row block of r1) of one score tile.
template <int LL> constexpr int nk() { return LL * (R1P / 16); }

// x of component c (less the offset mu) over sigma^2 as the MFMA B operand of every k-step of
// the score tile (the tile then accumulates <y, R_t x_c> / sigma^2 directly):
// lane (t1 = lane & 31, g = lane >> 5) of k-step (b2, jb) holds the 8 values
// x_c[(16 jb + 8 g + e - t1) mod Ll][b2], e = 0..7, split into BF16 hi and lo.
// Layout [c][k-step][plane][lane] of 16-byte fragments (one 1 KiB coalesced
// load per wave and plane).  One block of 64 threads per (component, k-step).
template <int LL>
__device__ __forceinline__ void pack_xb_body(const StepArgs& p, const float* __restrict__ x, int c,
                                             int ks, uint4* __restrict__ xb) {
    const int lane = threadIdx.x & 63;
    const int c1 = c / p.K, c2 = c % p.K;
    const int b2 = ks / (R1P / 16), jb = ks % (R1P / 16);
    const int t1 = lane & 31, g = lane >> 5;
    const int t1e = t1 < LL ? t1 : t1 - LL;
    const float mu = centre_of(p.centre);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int r = 16 * jb + 8 * g + e - t1e;
        r = ((r % LL) + LL) % LL;
        v[e] = (x[(int64_t)(c1 + r * p.K) * p.Lh + (c2 + b2 * p.K)] - mu) * p.inv_s2;
    }
    bf16x8 h, l;
    split8(v, h, l);
    uint4* dst = xb + ((int64_t)(c * nk<LL>() + ks) * 2) * 64;
    dst[lane] = __builtin_bit_cast(uint4, h);
    dst[64 + lane] = __builtin_bit_cast(uint4, l);
}

// yT planes of observations [o0, o0 + NOB) into LDS (row pitch PITCH), zeros past N.
template <int LL, int NOB = 8, int NT = 256>
__device__ __forceinline__ void load_yT(const StepArgs& p, const Prep& q, int64_t o0, __bf16* ys) {
    constexpr int CH = 2 * LL * (R1P / 8);     // 16-byte chunks per observation
    for (int e = threadIdx.x; e < NOB * CH; e += NT) {
        const int o = e / CH, r = e % CH;
        const int row = r / (R1P / 8), part = r % (R1P / 8);   // row = plane*LL + col
        uint4 v = make_uint4(0, 0, 0, 0);
        if (o0 + o < p.N)
            v = reinterpret_cast<const uint4*>(q.yT + (o0 + o) * (int64_t)(2 * LL * R1P))[r];
        *reinterpret_cast<uint4*>(ys + (o * 2 * LL + row) * PITCH + part * 8) = v;
    }
}

// Yo group of observations [o0, o0 + 8) (o0 multiple of 8) into LDS.
template <int LL>
__device__ __forceinline__ void load_yo(const Prep& q, int64_t o0, __bf16* yo) {
    constexpr int CH = 2 * LL * LL;            // 16-byte chunks (8 obs x bf16) per group
    const uint4* src = reinterpret_cast<const uint4*>(q.yo + (o0 / 8) * (int64_t)(2 * LL * LL * 8));
    for (int e = threadIdx.x; e < CH; e += 256) reinterpret_cast<uint4*>(yo)[e] = src[e];
}

// Score tiles for NO observations (slots o_slot[k]) x NC components (LDS slots cs[k]).
template <int LL, int NO, int NC, int NP>
__device__ __forceinline__ void score(const StepArgs& p, const __bf16* ys, const int (&oslot)[NO],
                                      const int (&cgl)[NC], floatx16 (&acc)[NO][NC]) {
    constexpr int JS = R1P / 16;
    const int lane = threadIdx.x & 63;
    const int i = lane & 31, g = lane >> 5;
    const int t2e = i < LL ? i : i - LL;
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[o][c] = floatx16{0};
    // B fragments of this lane for every component: xb[c][ks][plane][lane].
    // Double-buffered in registers: the fragments of k-step ks + 1 are requested
    // before the MFMAs of k-step ks, so their L2 latency overlaps a whole k-step.
    const uint4* bsrc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) bsrc[c] = p.xb + (int64_t)cgl[c] * nk<LL>() * 128 + lane;
    bf16x8 bh[NC], bl[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        bh[c] = __builtin_bit_cast(bf16x8, bsrc[c][0]);
        bl[c] = __builtin_bit_cast(bf16x8, bsrc[c][64]);
    }
    if constexpr (NC == 2 && NO == 4) {
        // four observations, two components: observation by observation, the
        // six (eight) products of one observation alternate between its two
        // accumulators, and the A fragments of the next observation -- for the
        // last one, of the first observation of the next k-step -- are requested
        // before them, so an LDS round trip hides behind six products
        bf16x8 ah[2], al[2];
        auto arow_of = [&](int b2, int o) {
            int col = b2 + t2e;
            col = col >= LL ? col - LL : col;
            return ys + (oslot[o] * 2 * LL + col) * PITCH + 8 * g;
        };
        auto load = [&](int slot, int b2, int j, int o) {
            const __bf16* r = arow_of(b2, o);
            ah[slot] = *reinterpret_cast<const bf16x8*>(r + 16 * j);
            al[slot] = *reinterpret_cast<const bf16x8*>(r + LL * PITCH + 16 * j);
        };
        load(0, 0, 0, 0);
        for (int b2 = 0; b2 < LL; ++b2) {
#pragma unroll
            for (int j = 0; j < JS; ++j) {
                const int ks = b2 * JS + j;
                const int kn = ks + 1 < nk<LL>() ? ks + 1 : ks;   // the last step re-reads its own
                bf16x8 nh[NC], nl[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    nh[c] = __builtin_bit_cast(bf16x8, bsrc[c][kn * 128]);
                    nl[c] = __builtin_bit_cast(bf16x8, bsrc[c][kn * 128 + 64]);
                }
                // the next k-step's (b2, j)
                const int jn = j + 1 < JS ? j + 1 : 0;
                const int b2n = j + 1 < JS ? b2 : (b2 + 1 < LL ? b2 + 1 : b2);
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    const int cur = o & 1;
                    if (o + 1 < NO) load(cur ^ 1, b2, j, o + 1);
                    else load(cur ^ 1, b2n, jn, 0);
                    asm volatile("" ::: "memory");
                    __builtin_amdgcn_sched_barrier(0);
                    floatx16& a0 = acc[o][0];
                    floatx16& a1 = acc[o][1];
                    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[cur], bh[0], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[cur], bh[1], a1, 0, 0, 0);
                    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[cur], bl[0], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[cur], bl[1], a1, 0, 0, 0);
                    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[cur], bh[0], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[cur], bh[1], a1, 0, 0, 0);
                    if constexpr (NP == 4) {
                        a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[cur], bl[0], a0, 0, 0, 0);
                        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[cur], bl[1], a1, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    bh[c] = nh[c];
                    bl[c] = nl[c];
                }
            }
        }
        return;
    }
    for (int b2 = 0; b2 < LL; ++b2) {
        int col = b2 + t2e;
        col = col >= LL ? col - LL : col;
        const __bf16* arow[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) arow[o] = ys + (oslot[o] * 2 * LL + col) * PITCH + 8 * g;
#pragma unroll
        for (int j = 0; j < JS; ++j) {
            const int ks = b2 * JS + j;
            const int kn = ks + 1 < nk<LL>() ? ks + 1 : ks;   // the last step re-reads its own
            bf16x8 nh[NC], nl[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                nh[c] = __builtin_bit_cast(bf16x8, bsrc[c][kn * 128]);
                nl[c] = __builtin_bit_cast(bf16x8, bsrc[c][kn * 128 + 64]);
            }
            // compiler-only barrier: keeps the requests here instead of letting the
            // compiler re-issue them next to their use (no instruction, no wait)
            asm volatile("" ::: "memory");
            if constexpr (NC == 1 && NO == 8) {
                // eight observations, one component: the A fragments of two
                // observations are requested while the products of the previous
                // two run, and the two accumulators of a pair alternate so that
                // consecutive products never depend on each other
                bf16x8 ah[8], al[8];
                auto load = [&](int o) {
                    ah[o] = *reinterpret_cast<const bf16x8*>(arow[o] + 16 * j);
                    al[o] = *reinterpret_cast<const bf16x8*>(arow[o] + LL * PITCH + 16 * j);
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
                    floatx16& a0 = acc[o][0];
                    floatx16& a1 = acc[o + 1][0];
                    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o], bh[0], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o + 1], bh[0], a1, 0, 0, 0);
                    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o], bl[0], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o + 1], bl[0], a1, 0, 0, 0);
                    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], bh[0], a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o + 1], bh[0], a1, 0, 0, 0);
                    if constexpr (NP == 4) {
                        a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], bl[0], a0, 0, 0, 0);
                        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o + 1], bl[0], a1, 0, 0, 0);
                    }
                }
                bh[0] = nh[0];
                bl[0] = nl[0];
                continue;
            }
            bf16x8 ah[NO], al[NO];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                ah[o] = *reinterpret_cast<const bf16x8*>(arow[o] + 16 * j);
                al[o] = *reinterpret_cast<const bf16x8*>(arow[o] + LL * PITCH + 16 * j);
            }
            // the three split products in separate sweeps over the independent
            // accumulators, so consecutive MFMAs never depend on each other
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[o][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o], bh[c], acc[o][c], 0, 0, 0);
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[o][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[o], bl[c], acc[o][c], 0, 0, 0);
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[o][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], bh[c], acc[o][c], 0, 0, 0);
            if constexpr (NP == 4) {
#pragma unroll
                for (int o = 0; o < NO; ++o)
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        acc[o][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], bl[c], acc[o][c], 0, 0, 0);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bh[c] = nh[c];
                bl[c] = nl[c];
            }
        }
    }
}

__device__ __forceinline__ int acc_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// ============================================================================
// Pass 1.  Block = 8 observations x 4 components; wave w: observations 4*(w&1)..+4,
// components 2*(w>>1)..+2 of the block's group.  Partials per component pair.
template <int LL, int NP>
__device__ __forceinline__ void bf16_pass1_body(const StepArgs& p, const Prep& q, int chunk, int cg,
                                                float* lds) {
    using G = Geo<LL>;
    __bf16* ys = reinterpret_cast<__bf16*>(lds);                       // 8 x 2 x Ll x PITCH
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int og = wave & 1, cgw = wave >> 1;
    const int oslot[4] = {4 * og, 4 * og + 1, 4 * og + 2, 4 * og + 3};
    const int cslot[2] = {2 * cgw, 2 * cgw + 1};
    // global component indices of the wave's two components (clamped; masked later)
    const int cgl[2] = {min(cg * 4 + cslot[0], p.KK - 1), min(cg * 4 + cslot[1], p.KK - 1)};
    const int cpair = cg * 2 + cgw;                 // global component-pair index
    const int j = lane & 31;
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += 8) {
        __syncthreads();
        load_yT<LL>(p, q, o0, ys);
        __syncthreads();
        floatx16 acc[4][2];
        score<LL, 4, 2, NP>(p, ys, oslot, cgl, acc);
        float mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
        // the bias of a lane's (component, t1, t2) slots does not depend on the
        // observation: load it once per tile
        float bet[2][16];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int cc = cg * 4 + cslot[c];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int t2 = acc_row(v, lane);
                bet[c][v] = (cc < p.KK && t2 < LL && j < LL)
                                ? p.betaT[(int64_t)cc * (LL * LL) + t2 * LL + j] : -INFINITY;
            }
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const bool ook = o0 + oslot[o] < p.N;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float a = ook ? acc[o][c][v] + bet[c][v] : -INFINITY;
                    acc[o][c][v] = a;
                    mx[o] = fmaxf(mx[o], a);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            for (int off = 32; off > 0; off >>= 1) mx[o] = fmaxf(mx[o], __shfl_xor(mx[o], off));
            float s = 0.f;
            if (mx[o] > -INFINITY) {
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        if (acc[o][c][v] > -INFINITY) s += fast_exp(acc[o][c][v] - mx[o]);
            }
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            const int64_t og_ = o0 + oslot[o];
            if (lane == 0 && og_ < p.N && cpair * 2 < p.KK)
                p.part[(int64_t)cpair * p.N + og_] = make_float2(mx[o], s);
        }
    }
}

// Log-sum-exp of NOB observations over the components of a block from the
// waves' own (max, sum exp) pairs, exchanged through LDS (red: [NS waves][NOB]
// float2).  Every wave of the block calls it (two barriers); wave `slot` stores
// its pairs, and slots k with use(k) take part.  The combine runs on NOB groups
// of NS lanes (lane o NS + k holds observation o, slot k): the group's maximum,
// its terms s_k exp(m_k - m) in FP64 summed over the group in a fixed tree
// order, taken from the group's first lane.  The combined pair is also written as
// the observation's single partial (its log-likelihood term is formed from it
// later) by the `writer` wave, and lse[o] = (m, log sum) for every observation.
template <int NOB, int NS, typename Use>
__device__ __forceinline__ void block_lse(const StepArgs& p, const float (&mw)[NOB], const float (&sw)[NOB],
                                          int slot, int64_t obs0, int64_t c1, bool writer, Use use,
                                          float2* red, float2 (&lse)[NOB]) {
    static_assert(NOB * NS <= 64 && (NS & (NS - 1)) == 0, "one lane per (observation, slot)");
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int o = 0; o < NOB; ++o) red[slot * NOB + o] = make_float2(mw[o], sw[o]);
    }
    __syncthreads();
    const int og = lane / NS, k = lane % NS;
    const bool act = lane < NOB * NS && use(k);
    const float2 e = act ? red[k * NOB + og] : make_float2(-INFINITY, 0.f);
    float m = e.x;
#pragma unroll
    for (int off = 1; off < NS; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    double t = (act && e.x > -INFINITY) ? (double)e.y * exp((double)e.x - (double)m) : 0.0;
#pragma unroll
    for (int off = 1; off < NS; off <<= 1) t += __shfl_xor(t, off);
    t = __shfl(t, og * NS);              // the group's first lane's sum, in every lane of it
    const float sf = (float)t;
    const float lg = m > -INFINITY ? (float)log((double)sf) : 0.f;
    if (writer && k == 0 && lane < NOB * NS && obs0 + og < c1) p.part[obs0 + og] = make_float2(m, sf);
#pragma unroll
    for (int o = 0; o < NOB; ++o) {
        const float mo = __shfl(m, o * NS), lo = __shfl(lg, o * NS);
        lse[o] = mo > -INFINITY ? make_float2(mo, lo) : make_float2(0.f, 0.f);
    }
    __syncthreads();   // red is rewritten by the next group
}

// ============================================================================
// Pass 2.  Block = 8 observations x 4 components; wave w owns component
// cg*4 + w for all 8 observations.  FUSED (K^2 <= 4, one component group):
// the single pass -- LSE from the block's own scores instead of pass 1.
template <int LL, int NP, bool FUSED = false>
__device__ __forceinline__ void bf16_pass2_body(const StepArgs& p, const Prep& q, int chunk_i, int cg,
                                                float* lds) {
    using G = Geo<LL>;
    float* bacc = lds;                                                  // 4 x Ll x BP
    __bf16* ys = reinterpret_cast<__bf16*>(bacc + 4 * LL * G::BP);      // 8 x 2 x Ll x PITCH
    __bf16* yo = ys + 8 * 2 * LL * PITCH;                               // 2 x Ll x Ll x 8
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 31, g = lane >> 5;
    const int comp = cg * 4 + wave;
    const bool cok = comp < p.KK;
    float* bw = bacc + wave * LL * G::BP;
    for (int e = lane; e < LL * G::BP; e += 64) bw[e] = 0.f;
    float cnt[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) cnt[v] = 0.f;
    const int oslot[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    const int cgl[1] = {cok ? comp : p.KK - 1};
    const int q2e = j < LL ? j : j - LL;
    const int64_t c0 = (int64_t)chunk_i * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += 8) {
        __syncthreads();
        load_yT<LL>(p, q, o0, ys);
        load_yo<LL>(q, o0, yo);
        __syncthreads();
        floatx16 acc[8][1];
        score<LL, 8, 1, NP>(p, ys, oslot, cgl, acc);
        // posterior weights, posterior mass, BF16 hi/lo fragments over k = (t2, o)
        bf16x8 wh[16], wl[16];
        float2 lse[8];
        if constexpr (FUSED) {
            // this wave's (max, sum exp) per observation, then the 4 waves combined
            float mw[8], sw[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                mw[o] = -INFINITY;
                sw[o] = 0.f;
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int t2 = acc_row(v, lane);
                const bool sok = cok && t2 < LL && j < LL;
                const float bet = sok ? p.betaT[(int64_t)comp * (LL * LL) + t2 * LL + j] : 0.f;
#pragma unroll
                for (int o = 0; o < 8; ++o)
                    if (sok && o0 + o < p.N) mw[o] = fmaxf(mw[o], acc[o][0][v] + bet);
            }
#pragma unroll
            for (int o = 0; o < 8; ++o)
                for (int off = 32; off > 0; off >>= 1) mw[o] = fmaxf(mw[o], __shfl_xor(mw[o], off));
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int t2 = acc_row(v, lane);
                const bool sok = cok && t2 < LL && j < LL;
                const float bet = sok ? p.betaT[(int64_t)comp * (LL * LL) + t2 * LL + j] : 0.f;
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const float a = acc[o][0][v] + bet;
                    if (sok && o0 + o < p.N && a > -INFINITY) sw[o] += fast_exp(a - mw[o]);
                }
            }
#pragma unroll
            for (int o = 0; o < 8; ++o)
                for (int off = 32; off > 0; off >>= 1) sw[o] += __shfl_xor(sw[o], off);
            float2* red = reinterpret_cast<float2*>(yo + 2 * LL * LL * 8);
            block_lse<8, 4>(p, mw, sw, wave, o0, p.N, wave == 0,
                            [&](int k) { return k < p.KK; }, red, lse);
        } else {
#pragma unroll
            for (int o = 0; o < 8; ++o) lse[o] = (o0 + o < p.N) ? p.lse[o0 + o] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int t2 = acc_row(v, lane);
            const bool sok = cok && t2 < LL && j < LL;
            const float bet = sok ? p.betaT[(int64_t)comp * (LL * LL) + t2 * LL + j] : 0.f;
            float w[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                float ww = 0.f;
                if (sok && o0 + o < p.N) {
                    const float a = acc[o][0][v] + bet;
                    ww = a > -INFINITY ? fast_exp((a - lse[o].x) - lse[o].y) : 0.f;
                }
                w[o] = ww;
                cnt[v] += ww;
            }
            split8(w, wh[v], wl[v]);
        }
        // back-projection for each a1, folded into the wave's b accumulator;
        // accumulator rows v with t2 >= Ll (Ll = 24: v >= 12) carry no weight
        constexpr int NV = LL == 24 ? 12 : 16;
        constexpr int PF = 4;
        for (int a1 = 0; a1 < LL; ++a1) {
            const __bf16* yrow = yo + a1 * LL * 8;
            // A fragments requested PF rows v ahead of their products; two
            // partial sums alternate so that consecutive MFMAs are independent
            bf16x8 ah[NV], al[NV];
            auto load_a = [&](int v) {
                int col = q2e + acc_row(v, lane);
                col = col >= LL ? col - LL : col;
                ah[v] = *reinterpret_cast<const bf16x8*>(yrow + col * 8);
                al[v] = *reinterpret_cast<const bf16x8*>(yrow + LL * LL * 8 + col * 8);
            };
#pragma unroll
            for (int v = 0; v < PF; ++v) load_a(v);
            floatx16 zp[2] = {floatx16{0}, floatx16{0}};
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (v + PF < NV) load_a(v + PF);
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                zp[v & 1] = mfma_split<NP>(ah[v], al[v], wh[v], wl[v], zp[v & 1]);
            }
            floatx16 z;
#pragma unroll
            for (int e = 0; e < 16; ++e) z[e] = zp[0][e] + zp[1][e];
            // z lane holds Z[q2 = acc_row(v)][t1 = j]; b_c[(a1 - t1) % Ll][q2] += Z
            if (j < LL) {
                int q1 = a1 - j;
                q1 = q1 < 0 ? q1 + LL : q1;
                float* brow = bw + q1 * G::BP;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int q2 = acc_row(v, lane);
                    if (q2 < LL) brow[q2] += z[v];
                }
            }
        }
    }
    // ---- store this block's partials for component `comp`
    __syncthreads();
    const int64_t chunk = chunk_i;
    if (cok) {
        float* bo = p.bpart + (chunk * p.KK + comp) * (LL * LL);
        for (int e = lane; e < LL * LL; e += 64) bo[e] = bw[(e / LL) * G::BP + (e % LL)];
        // c: lane holds c[t1 = j][t2 = acc_row(v)]
        float* co = p.cpart + (chunk * p.KK + comp) * (LL * LL);
        if (j < LL) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int t2 = acc_row(v, lane);
                if (t2 < LL) co[j * LL + t2] = cnt[v];
            }
        }
    }
}

// ============================================================================
// Single pass for 4 < K^2 <= 16 (L_low 24, 32): a workgroup of 8 waves holds
// all K^2 components of groups of 4 observations.  Wave w scores the 4
// observations against components 2w, 2w + 1 (8 tiles, as a pass-1 wave), the
// eight waves' (max, sum exp) per observation are combined through LDS into
// the log-sum-exp, and each wave back-projects its components from its own
// accumulators.  The back-projection of component c for each a1,
//   Z[q2][t1] = sum_{t2, o} y_o[a1][(q2 + t2) % Ll] * w_{o,c}[t1][t2],
// runs over k = (t2, o) in k-steps of two t2 rows x 4 observations: the B
// fragment of k-step s (lane half g) is the weights of rows
// 8 (s >> 1) + 4 g + 2 (s & 1) + {0, 1} of the lane's accumulators for the
// 4 observations, the A fragment the matching values of the staged
// observations, stored [plane][a1][column][4 observations] (one 8-byte record
// per column: two records per fragment).  The posterior mass of a
// (component, shift) is owned by one lane of one wave for the whole chunk and
// summed into the chunk's partial in global memory group by group, as four
// 16-byte runs per lane and component (registers and LDS are both full).
constexpr int F16_NOB = 4;   // observations per group
constexpr int F16_NCW = 2;   // components per wave
constexpr int F16_NW = 8;    // waves per workgroup
constexpr int F16_NT = 64 * F16_NW;

// Yo4 for the 4 observations [o0, o0 + 4) (o0 a multiple of 4): their half
// of the prepared 8-observation group, both planes, [plane][a1][col][4 obs].
template <int LL>
__device__ __forceinline__ void load_yo4(const Prep& q, int64_t o0, __bf16* yo4) {
    constexpr int CH = 2 * LL * LL;            // 16-byte records (8 obs x bf16) per group
    const uint4* src = reinterpret_cast<const uint4*>(q.yo + (o0 / 8) * (int64_t)(2 * LL * LL * 8));
    const int half = (int)((o0 / 4) & 1);
    uint2* dst = reinterpret_cast<uint2*>(yo4);
    for (int e = threadIdx.x; e < CH; e += F16_NT) {
        const uint4 v = src[e];
        dst[e] = half ? make_uint2(v.z, v.w) : make_uint2(v.x, v.y);
    }
}

template <int LL, int NP>
__device__ __forceinline__ void bf16_fused16_body(const StepArgs& p, const Prep& q, int chunk_i,
                                                  float* lds) {
    using G = Geo<LL>;
    constexpr int NOB = F16_NOB, NCW = F16_NCW, NW = F16_NW;
    // b accumulator pitch: rows of 16-byte runs, so that a lane adds its four
    // consecutive q2 of a row in one read-modify-write (the 32 lanes of one
    // update hit 32 different rows; a pitch of Ll + 4 floats spreads them over the banks)
    constexpr int BPF = LL + 4;
    float* bacc = lds;                                                  // NW x NCW x Ll x BPF
    __bf16* ys = reinterpret_cast<__bf16*>(bacc + NW * NCW * LL * BPF);  // NOB x 2 x Ll x PITCH
    __bf16* yo4 = ys + NOB * 2 * LL * PITCH;                            // 2 x Ll x Ll x NOB
    float2* red = reinterpret_cast<float2*>(yo4 + 2 * LL * LL * NOB);   // NW x NOB
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 31, g = lane >> 5;
    int comp[NCW], cgl[NCW];
    bool cok[NCW];
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
        comp[c] = wave * NCW + c;
        cok[c] = comp[c] < p.KK;
        cgl[c] = cok[c] ? comp[c] : p.KK - 1;
    }
    float* bw = bacc + wave * NCW * LL * BPF;
    for (int e = lane; e < NCW * LL * BPF; e += 64) bw[e] = 0.f;
    const int oslot[NOB] = {0, 1, 2, 3};
    const int q2e = j < LL ? j : j - LL;
    const int64_t chunk = chunk_i;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += NOB) {
        __syncthreads();
        load_yT<LL, NOB, F16_NT>(p, q, o0, ys);
        load_yo4<LL>(q, o0, yo4);
        __syncthreads();
        // the B fragments carry x / sigma^2 and the shift prior is added once the
        // tiles are complete (accumulators started from beta, of the magnitude of
        // ||x_c||^2 / 2 sigma^2, would round every FP32 accumulation at that
        // scale), so the tiles end as the log-joint terms a = <y, R_t x_c> / sigma^2 + beta
        bool ook[NOB];
#pragma unroll
        for (int o = 0; o < NOB; ++o) ook[o] = o0 + o < p.N;
        // every slot a shift of this observation: L_low 32 (no rows / columns
        // past L_low), both components and all four observations present
        const bool full = LL == 32 && cok[0] && cok[1] && ook[NOB - 1];
        auto slot_ok = [&](int c, int v) { return cok[c] && acc_row(v, lane) < LL && j < LL; };
        floatx16 acc[NOB][NCW];
        score<LL, NOB, NCW, NP>(p, ys, oslot, cgl, acc);
#pragma unroll
        for (int c = 0; c < NCW; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float bet = slot_ok(c, v)
                    ? p.betaT[(int64_t)comp[c] * (LL * LL) + acc_row(v, lane) * LL + j] : 0.f;
#pragma unroll
                for (int o = 0; o < NOB; ++o) acc[o][c][v] += bet;
            }
        if (!full) {   // masked slots out of every sum below
#pragma unroll
            for (int c = 0; c < NCW; ++c)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const bool sok = slot_ok(c, v);
#pragma unroll
                    for (int o = 0; o < NOB; ++o)
                        if (!(sok && ook[o])) acc[o][c][v] = -INFINITY;
                }
        }
        // the wave's (max, sum exp) per observation (a term of -inf adds
        // exp(-inf) = 0)
        float mw[NOB], sw[NOB];
#pragma unroll
        for (int o = 0; o < NOB; ++o) {
            mw[o] = -INFINITY;
            sw[o] = 0.f;
        }
#pragma unroll
        for (int c = 0; c < NCW; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v)
#pragma unroll
                for (int o = 0; o < NOB; ++o) mw[o] = fmaxf(mw[o], acc[o][c][v]);
#pragma unroll
        for (int o = 0; o < NOB; ++o)
            for (int off = 32; off > 0; off >>= 1) mw[o] = fmaxf(mw[o], __shfl_xor(mw[o], off));
        float mref[NOB];
#pragma unroll
        for (int o = 0; o < NOB; ++o) mref[o] = mw[o] > -INFINITY ? mw[o] : 0.f;
#pragma unroll
        for (int c = 0; c < NCW; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v)
#pragma unroll
                for (int o = 0; o < NOB; ++o) sw[o] += fast_exp(acc[o][c][v] - mref[o]);
#pragma unroll
        for (int o = 0; o < NOB; ++o)
            for (int off = 32; off > 0; off >>= 1) sw[o] += __shfl_xor(sw[o], off);
        float2 lse[NOB];
        block_lse<NOB, NW>(p, mw, sw, wave, o0, p.N, wave == 0,
                           [&](int k) { return k * NCW < p.KK; }, red, lse);
        // posterior weights and mass of both components, the weights as B
        // fragments over k = (two t2 rows, 4 obs) (the accumulators are dead
        // after this), then the back-projection for each a1 (k-steps with t2
        // rows >= Ll carry no weight: at Ll = 24 the last two are skipped), one
        // A fragment per k-step serving both components, folded into the
        // wave's b accumulators
        bf16x8 wh[NCW][8], wl[NCW][8];
        // the lane's posterior masses c[t1 = j][t2 = 8 m + 4 g + 0..3] of a
        // component are four 16-byte runs of the chunk's partial
        constexpr int NM = LL == 24 ? 3 : 4;
        const bool first = o0 == c0;
#pragma unroll
        for (int c = 0; c < NCW; ++c) {
            float4* co = reinterpret_cast<float4*>(p.cpart + (chunk * p.KK + comp[c]) * (LL * LL) + j * LL + 4 * g);
            const bool own = cok[c] && j < LL;
            float4 cm[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
                cm[m] = (own && !first && m < NM) ? co[2 * m] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                float w[8];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int v = 2 * s8 + r;
                    float m = 0.f;
#pragma unroll
                    for (int o = 0; o < NOB; ++o) {
                        // an observation past N has lse (0, 0) and only -inf terms
                        const float ww = fast_exp((acc[o][c][v] - lse[o].x) - lse[o].y);
                        w[4 * r + o] = ww;
                        m += ww;
                    }
                    float4& q = cm[v >> 2];
                    switch (v & 3) {
                        case 0: q.x += m; break;
                        case 1: q.y += m; break;
                        case 2: q.z += m; break;
                        default: q.w += m; break;
                    }
                }
                split8(w, wh[c][s8], wl[c][s8]);
            }
            // the chunk's running sums, owned by this lane
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (own && m < NM) co[2 * m] = cm[m];
        }
        constexpr int NS = LL == 24 ? 6 : 8;
        constexpr int PF = 2;
        constexpr int PL = LL * LL;                          // plane stride in records
        for (int a1 = 0; a1 < LL; ++a1) {
            const uint2* yrow = reinterpret_cast<const uint2*>(yo4) + a1 * LL;
            bf16x8 ah[NS], al[NS];
            auto load_a = [&](int s8) {
                int k0 = q2e + 8 * (s8 >> 1) + 4 * g + 2 * (s8 & 1);
                k0 = k0 >= LL ? k0 - LL : k0;
                const int k1 = k0 + 1 >= LL ? k0 + 1 - LL : k0 + 1;
                const uint2 h0 = yrow[k0], h1 = yrow[k1];
                const uint2 l0 = yrow[PL + k0], l1 = yrow[PL + k1];
                ah[s8] = __builtin_bit_cast(bf16x8, make_uint4(h0.x, h0.y, h1.x, h1.y));
                al[s8] = __builtin_bit_cast(bf16x8, make_uint4(l0.x, l0.y, l1.x, l1.y));
            };
#pragma unroll
            for (int s8 = 0; s8 < PF; ++s8) load_a(s8);
            floatx16 z[NCW];
#pragma unroll
            for (int c = 0; c < NCW; ++c) z[c] = floatx16{0};
#pragma unroll
            for (int s8 = 0; s8 < NS; ++s8) {
                if (s8 + PF < NS) load_a(s8 + PF);
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < NCW; ++c)
                    z[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s8], wh[c][s8], z[c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < NCW; ++c)
                    z[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s8], wl[c][s8], z[c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < NCW; ++c)
                    z[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s8], wh[c][s8], z[c], 0, 0, 0);
                if constexpr (NP == 4) {
#pragma unroll
                    for (int c = 0; c < NCW; ++c)
                        z[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s8], wl[c][s8], z[c], 0, 0, 0);
                }
            }
            // lane holds Z[q2 = acc_row(v)][t1 = j] (rows 8 m + 4 g + 0..3 for
            // v = 4 m .. 4 m + 3); b_c[(a1 - t1) % Ll][q2] += Z, four q2 at a time
            if (j < LL) {
                int q1 = a1 - j;
                q1 = q1 < 0 ? q1 + LL : q1;
#pragma unroll
                for (int c = 0; c < NCW; ++c) {
                    float* brow = bw + (c * LL + q1) * BPF + 4 * g;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        if (8 * m + 4 * g < LL) {
                            float4* d = reinterpret_cast<float4*>(brow + 8 * m);
                            float4 t = *d;
                            t.x += z[c][4 * m];
                            t.y += z[c][4 * m + 1];
                            t.z += z[c][4 * m + 2];
                            t.w += z[c][4 * m + 3];
                            *d = t;
                        }
                    }
                }
            }
        }
    }
    // ---- this block's partials of b for the wave's components
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
        if (!cok[c]) continue;
        const float* bc = bw + c * LL * BPF;
        float* bo = p.bpart + (chunk * p.KK + comp[c]) * (LL * LL);
        for (int e = lane; e < LL * LL; e += 64) bo[e] = bc[(e / LL) * BPF + (e % LL)];
    }
}

// ---- per-job preparation: BF16 hi/lo planes of y - mu in both layouts, and
// the FP64 squared norms ||y_i - mu||^2.  One block per group of 8
// observations: the group is staged in LDS with coalesced 16-byte reads, then
// every 16-byte output run (8 BF16 values of one plane) is assembled in
// registers and stored whole.  PACKED (the packed-tile form at L_low 8 / 12):
// yT is the transpose flattened without padding, yT[o][plane][col * Ll + r1].
template <int LL, bool PACKED = false>
__global__ __launch_bounds__(256) void k_prep_bf16(const float* __restrict__ y, int64_t N,
                                                   const double* __restrict__ centre,
                                                   __bf16* __restrict__ yT, __bf16* __restrict__ yo,
                                                   double* __restrict__ ynorm) {
    constexpr int SP = LL + 1;                     // LDS row pitch (floats)
    __shared__ float s[8 * LL * SP];               // [o][r1][r2]
    const int64_t grp = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int P4 = LL * LL / 4;
    const float mu = centre_of(centre);
    for (int e = threadIdx.x; e < 8 * P4; e += 256) {
        const int o = e / P4, q = e % P4;
        const int64_t oi = grp * 8 + o;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (oi < N) {
            v = reinterpret_cast<const float4*>(y + oi * (int64_t)(LL * LL))[q];
            v.x -= mu; v.y -= mu; v.z -= mu; v.w -= mu;
        }
        const int r1 = (4 * q) / LL, r2 = (4 * q) % LL;
        float* d = s + (o * LL + r1) * SP + r2;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
    }
    __syncthreads();
    // squared norms, same order as obs_norms_body: wave w handles observations 2w, 2w+1
    for (int k = 0; k < 2; ++k) {
        const int o = 2 * wave + k;
        const int64_t oi = grp * 8 + o;
        double acc = 0.0;
        for (int p = lane; p < P4; p += 64) {
            const int r1 = (4 * p) / LL, r2 = (4 * p) % LL;
            const float* d = s + (o * LL + r1) * SP + r2;
#pragma unroll
            for (int e = 0; e < 4; ++e) acc += (double)d[e] * d[e];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0 && oi < N) ynorm[oi] = acc;
    }
    if constexpr (PACKED) {
        // yT[o][plane][f], f = col * Ll + r1: runs of 8 consecutive f
        constexpr int RUNS = LL * LL / 8;
        for (int e = threadIdx.x; e < 8 * RUNS; e += 256) {
            const int o = e / RUNS, r = e % RUNS;
            const int64_t oi = grp * 8 + o;
            if (oi >= N) continue;
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int f = 8 * r + k;
                v[k] = s[(o * LL + f % LL) * SP + f / LL];
            }
            bf16x8 h, l;
            split8(v, h, l);
            uint4* t = reinterpret_cast<uint4*>(yT + oi * (int64_t)(2 * LL * LL));
            t[r] = __builtin_bit_cast(uint4, h);
            t[RUNS + r] = __builtin_bit_cast(uint4, l);
        }
    }
    // yT[o][plane][r2][r1]: runs of 8 consecutive r1 (zeros past Ll)
    constexpr int JR = R1P / 8;
    for (int e = threadIdx.x; e < (PACKED ? 0 : 8 * LL * JR); e += 256) {
        const int o = e / (LL * JR), r = e % (LL * JR);
        const int r2 = r / JR, jb = r % JR;
        const int64_t oi = grp * 8 + o;
        if (oi >= N) continue;
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r1 = 8 * jb + k;
            v[k] = r1 < LL ? s[(o * LL + r1) * SP + r2] : 0.f;
        }
        bf16x8 h, l;
        split8(v, h, l);
        uint4* t = reinterpret_cast<uint4*>(yT + oi * (int64_t)(2 * LL * R1P));
        t[r2 * JR + jb] = __builtin_bit_cast(uint4, h);
        t[LL * JR + r2 * JR + jb] = __builtin_bit_cast(uint4, l);
    }
    // Yo[plane][r1][r2][o]: runs of the 8 observations (zeros past N)
    uint4* g = reinterpret_cast<uint4*>(yo + grp * (int64_t)(2 * LL * LL * 8));
    for (int e = threadIdx.x; e < LL * LL; e += 256) {
        const int r1 = e / LL, r2 = e % LL;
        float v[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) v[o] = s[(o * LL + r1) * SP + r2];
        bf16x8 h, l;
        split8(v, h, l);
        g[e] = __builtin_bit_cast(uint4, h);
        g[LL * LL + e] = __builtin_bit_cast(uint4, l);
    }
}

template <int LL> constexpr size_t lds_pass1() {
    return sizeof(__bf16) * 8 * 2 * LL * PITCH;
}
template <int LL> constexpr size_t lds_pass2() {
    using G = Geo<LL>;
    return sizeof(float) * (4 * LL * G::BP) +
           sizeof(__bf16) * (8 * 2 * LL * PITCH + 2 * LL * LL * 8);
}
// the single pass: pass 2's LDS plus the (max, sum) exchange
template <int LL> constexpr size_t lds_fused() { return lds_pass2<LL>() + sizeof(float2) * 4 * 8; }
// the single pass at 4 < K^2 <= 16
template <int LL> constexpr size_t lds_fused16() {
    using G = Geo<LL>;
    return sizeof(float) * (F16_NW * F16_NCW * LL * (LL + 4)) +   // b accumulators (pitch Ll + 4)
           sizeof(__bf16) * (F16_NOB * 2 * LL * PITCH + 2 * LL * LL * F16_NOB) +
           sizeof(float2) * F16_NW * F16_NOB;
}

}  // namespace b16
}  // namespace srmra
