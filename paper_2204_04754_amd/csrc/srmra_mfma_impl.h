// FP32 matrix-core (MFMA) form of the two passes of the EM step.
//
// Each (observation i, component c) pair has an Ll x Ll score map
// S_{i,c}[t1][t2] (all low-resolution offsets t of sub-image x_c).  It is one
// implicit GEMM with k = (b2, r1) running over the Ll^2 pixels:
//     A[t2][k] = y_i[r1][(b2 + t2) mod Ll]        (rows: offsets t2)
//     B[k][t1] = x_c[(r1 - t1) mod Ll][b2]         (cols: offsets t1)
// computed with v_mfma_f32_32x32x2_f32 from LDS-resident tiles.  Maps smaller than
// 32x32 pack several observations (rows) and components (cols) into one 32x32
// tile; 64x64 maps use 2x2 tiles.  The N x Lh^2 score matrix is never stored.
//
// Pass 1 reduces the tile to (max, sum exp) per observation and component group
// (the streaming log-sum-exp of eq. weights_EM).  Pass 2 recomputes the same
// tiles with the same instruction sequence, forms w = exp(a - lse_i), and runs
// the back-projection (eq. x_EM right-hand side) as a second implicit GEMM with
// k = (a1, t2, observation):
//     A[q2][k] = y_i[a1][(q2 + t2) mod Ll],  B[k][q1] = w_{i,c}[(a1 - q1) mod Ll][t2]
// accumulating b_c[q1][q2] over all observations of the block's chunk, together
// with the posterior mass c_(c,t) = sum_i w_{i,c}[t].
#pragma once
#include "srmra_common.h"

namespace srmra {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Row / column slot of the 32x32 score tile (rb, cb) for MFMA lane index i (or j).
template <int LL> struct Slots {
    using TL = Tile<LL>;
    // observation slot (within the wave) and offset t2 of A-row i in row tile rb
    __device__ static __forceinline__ void row(int rb, int i, int& oslot, int& t2) {
        if constexpr (TL::T <= 32) { oslot = rb * TL::G + i / TL::T; t2 = i % TL::T; }
        else { oslot = 0; t2 = rb * 32 + i; }
    }
    // component slot (within the block's group) and offset t1 of B-col j in col tile cb
    __device__ static __forceinline__ void col(int cb, int j, int& cslot, int& t1) {
        if constexpr (TL::T <= 32) { cslot = cb * TL::G + j / TL::T; t1 = j % TL::T; }
        else { cslot = 0; t1 = cb * 32 + j; }
    }
};

__device__ __forceinline__ int wrap_once(int v, int n) { return v >= n ? v - n : v; }

// Load the block's components (xt2 and betaT) into LDS.  Components past KK are
// clamped to the last one (their results are masked).
template <int LL>
__device__ __forceinline__ void load_x_group(const StepArgs& p, int cg, float* Xs) {
    using TL = Tile<LL>;
    for (int cs = 0; cs < TL::CPW; ++cs) {
        int c = cg * TL::CPW + cs;
        if (c >= p.KK) c = p.KK - 1;
        const float* src = p.xt2 + (int64_t)c * LL * 2 * LL;
        for (int e = threadIdx.x; e < LL * 2 * LL; e += 256) Xs[cs * TL::XS + e] = src[e];
    }
}

// Load observations [o0, o0 + nt), less the offset mu, into LDS rows of stride
// OS (zeros past N).
template <int LL>
__device__ __forceinline__ void load_y_tile(const StepArgs& p, int64_t o0, float* Ys,
                                            int nt = Tile<LL>::NT) {
    using TL = Tile<LL>;
    constexpr int P4 = LL * LL / 4;
    const float mu = centre_of(p.centre);
    for (int e = threadIdx.x; e < nt * P4; e += 256) {
        const int o = e / P4, q = e % P4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (o0 + o < p.N) {
            v = reinterpret_cast<const float4*>(p.y + (o0 + o) * (int64_t)(LL * LL))[q];
            v.x -= mu; v.y -= mu; v.z -= mu; v.w -= mu;
        }
        float* d = Ys + o * TL::OS + 4 * q;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
    }
}

// Score tiles of one wave: acc[rb][cb] for its OPW observations x CPW components.
template <int LL>
__device__ __forceinline__ void score_tiles(const float* Ys, const float* Xs, int wave_obs0,
                                            floatx16 (&acc)[2][2]) {
    using TL = Tile<LL>;
    using SL = Slots<LL>;
    const int lane = threadIdx.x & 63;
    const int i = lane & 31, g = lane >> 5;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = floatx16{0};
    int abase[2], t2e[2], bbase[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        int os, t2;
        SL::row(rb, i, os, t2);
        t2e[rb] = t2 < LL ? t2 : t2 - LL;
        abase[rb] = (wave_obs0 + os) * TL::OS + g * LL;
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        int cs, t1;
        SL::col(cb, i, cs, t1);
        const int t1e = t1 < LL ? t1 : t1 - LL;
        bbase[cb] = cs * TL::XS + LL - t1e + g;
    }
    for (int b2 = 0; b2 < LL; ++b2) {
        const float* ap[2];
        const float* bp[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) ap[rb] = Ys + abase[rb] + wrap_once(b2 + t2e[rb], LL);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) bp[cb] = Xs + bbase[cb] + b2 * 2 * LL;
#pragma unroll
        for (int jj = 0; jj < LL / 2; ++jj) {
            float a0 = ap[0][2 * jj * LL], a1 = ap[1][2 * jj * LL];
            float b0 = bp[0][2 * jj], b1 = bp[1][2 * jj];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
}

// Value a = S/sigma^2 + beta of accumulator element v of tile (rb, cb), or -inf
// when the slot is padding.  Also returns the observation slot.
template <int LL>
__device__ __forceinline__ float tile_logit(const StepArgs& p, int cg,
                                            int64_t wave_obs_g, int rb, int cb, int v, float s,
                                            int& oslot) {
    using SL = Slots<LL>;
    using TL = Tile<LL>;
    const int lane = threadIdx.x & 63;
    const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int colj = lane & 31;
    int t2, cs, t1;
    SL::row(rb, row, oslot, t2);
    SL::col(cb, colj, cs, t1);
    const bool ok = t1 < LL && t2 < LL && (cg * TL::CPW + cs) < p.KK && (wave_obs_g + oslot) < p.N;
    if (!ok) return -INFINITY;
    const int c = cg * TL::CPW + cs;
    return s * p.inv_s2 + p.betaT[(int64_t)c * (LL * LL) + t2 * LL + t1];
}

// ============================================================================
// Pass 1: streaming log-sum-exp partials.
// grid = (n_chunks, n_cg); block = 256 (4 waves).
template <int LL>
__device__ __forceinline__ void mfma_pass1_body(const StepArgs& p, int chunk, int cg, float* lds) {
    using TL = Tile<LL>;
    float* Xs = lds;
    float* Ys = Xs + TL::CPW * TL::XS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    load_x_group<LL>(p, cg, Xs);
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += TL::NT) {
        __syncthreads();
        load_y_tile<LL>(p, o0, Ys);
        __syncthreads();
        const int wobs = wave * TL::OPW;
        const int64_t wobs_g = o0 + wobs;
        floatx16 acc[2][2];
        score_tiles<LL>(Ys, Xs, wobs, acc);
        float mx[TL::OPW], sm[TL::OPW];
#pragma unroll
        for (int k = 0; k < TL::OPW; ++k) { mx[k] = -INFINITY; sm[k] = 0.f; }
        float av[2][2][16];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int os;
                    const float a = tile_logit<LL>(p, cg, wobs_g, rb, cb, v, acc[rb][cb][v], os);
                    av[rb][cb][v] = a;
                    mx[os] = fmaxf(mx[os], a);
                }
#pragma unroll
        for (int k = 0; k < TL::OPW; ++k)
            for (int off = 32; off > 0; off >>= 1) mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], off));
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int os, t2;
                    const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    Slots<LL>::row(rb, row, os, t2);
                    const float a = av[rb][cb][v];
                    if (a > -INFINITY) sm[os] += fast_exp(a - mx[os]);
                }
#pragma unroll
        for (int k = 0; k < TL::OPW; ++k) {
            for (int off = 32; off > 0; off >>= 1) sm[k] += __shfl_xor(sm[k], off);
            if (lane == 0 && wobs_g + k < p.N)
                p.part[(int64_t)cg * p.N + wobs_g + k] = make_float2(mx[k], sm[k]);
        }
    }
}

// ============================================================================
// Pass 2: posterior and back-projection.
// LDS: Xs, Ys as in pass 1, plus per wave W[OPW][Ll(t2)][Ll(t1)] for one
// component at a time, and the per-block c / b reduction scratch.
template <int LL> struct BP {
    using TL = Tile<LL>;
    // floats of W per wave (T = 8 stores the two components of a column pair)
    static constexpr int WS = TL::OPW * LL * LL * (TL::T == 8 ? 2 : 1);
    // number of back-projection accumulators (floats) per lane per component
    static constexpr int NACC = TL::T == 64 ? 64 : (TL::T == 32 ? 16 : 4);
    // c accumulators per lane per column tile
    static constexpr int NCNT = TL::T == 64 ? 32 : 16 / TL::G;
};

// Back-projection of one component for the wave's observations.
// bacc layout: T=32 -> one 32x32 tile (16 regs); T=64 -> 2x2 tiles; T<=16 ->
// one 16x16 tile (4 regs).  Ws holds w_{o}[t2][t1] for o < OPW (for T=8 the
// two components of a column pair are stored back to back).
template <int LL>
__device__ __forceinline__ void backproject(const float* Ys, const float* Ws, int wave_obs0,
                                            float* bacc) {
    using TL = Tile<LL>;
    const int lane = threadIdx.x & 63;
    if constexpr (TL::T == 32) {
        const int i = lane & 31, g = lane >> 5;
        const int q2e = i < LL ? i : i - LL;
        const int q1e = q2e;  // column j = lane & 31 as well
        floatx16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = bacc[v];
        const float* ya = Ys + (wave_obs0 + g) * TL::OS;
        const float* wb = Ws + g * LL * LL;
        int rsh = q1e == 0 ? 0 : LL - q1e;   // (a1 - q1) mod Ll at a1 = 0
        for (int a1 = 0; a1 < LL; ++a1) {
            const float* yrow = ya + a1 * LL;
            int col = q2e;
#pragma unroll
            for (int t2 = 0; t2 < LL; ++t2) {
                const float av = yrow[col];
                const float bv = wb[t2 * LL + rsh];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
                col = wrap_once(col + 1, LL);
            }
            rsh = wrap_once(rsh + 1, LL);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) bacc[v] = acc[v];
    } else if constexpr (TL::T == 64) {
        const int i = lane & 31, g = lane >> 5;
        floatx16 acc[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[rb][cb][v] = bacc[(rb * 2 + cb) * 16 + v];
        int q2e[2], q1e[2], rsh[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int q = b * 32 + i;
            q2e[b] = q < LL ? q : q - LL;
            q1e[b] = q2e[b];
            rsh[b] = q1e[b] == 0 ? 0 : LL - q1e[b];
        }
        const float* ya = Ys + wave_obs0 * TL::OS;
        for (int a1 = 0; a1 < LL; ++a1) {
            const float* yrow = ya + a1 * LL;
            int col[2] = {wrap_once(q2e[0] + g, LL), wrap_once(q2e[1] + g, LL)};
#pragma unroll 4
            for (int tt = 0; tt < LL / 2; ++tt) {
                const int t2 = 2 * tt + g;
                const float a0 = yrow[col[0]], a1v = yrow[col[1]];
                const float b0 = Ws[t2 * LL + rsh[0]], b1 = Ws[t2 * LL + rsh[1]];
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1v, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1v, b1, acc[1][1], 0, 0, 0);
                col[0] = wrap_once(col[0] + 2, LL);
                col[1] = wrap_once(col[1] + 2, LL);
            }
            rsh[0] = wrap_once(rsh[0] + 1, LL);
            rsh[1] = wrap_once(rsh[1] + 1, LL);
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) bacc[(rb * 2 + cb) * 16 + v] = acc[rb][cb][v];
    } else {
        // T = 16 or 8: v_mfma_f32_16x16x4_f32, rows q2 (lane & 15), cols q1 (T=16) or
        // (component pair member, q1) (T=8), k-group (lane >> 4) = observation.
        const int r = lane & 15, kg = lane >> 4;
        const int q2e = (r % TL::T) < LL ? (r % TL::T) : (r % TL::T) - LL;
        int q1e, pair;
        if constexpr (TL::T == 16) { q1e = q2e; pair = 0; }
        else { pair = r >> 3; const int q = r & 7; q1e = q < LL ? q : q - LL; }
        floatx4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = bacc[v];
        constexpr int OSTEPS = TL::OPW / 4;  // 1 (T=16) or 2 (T=8)
#pragma unroll
        for (int os = 0; os < OSTEPS; ++os) {
            const int o = os * 4 + kg;
            const float* ya = Ys + (wave_obs0 + o) * TL::OS;
            const float* wb = Ws + (o * (TL::T == 8 ? 2 : 1) + pair) * LL * LL;
            int rsh = q1e == 0 ? 0 : LL - q1e;
            for (int a1 = 0; a1 < LL; ++a1) {
                const float* yrow = ya + a1 * LL;
                int col = q2e;
#pragma unroll
                for (int t2 = 0; t2 < LL; ++t2) {
                    const float av = yrow[col];
                    const float bv = wb[t2 * LL + rsh];
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
                    col = wrap_once(col + 1, LL);
                }
                rsh = wrap_once(rsh + 1, LL);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) bacc[v] = acc[v];
    }
}

// Back-projection of the wave's posterior tiles (acc holds w for every
// (observation, component) slot of the wave; padding slots hold 0): w of one
// component (or component pair for T=8) at a time goes to the wave's LDS tile
// Ws, then into the running sums bacc[u].
template <int LL, int NU>
__device__ __forceinline__ void backproject_tiles(const float* Ys, float* Ws, int wobs,
                                                  floatx16 (&acc)[2][2],
                                                  float (&bacc)[NU][BP<LL>::NACC]) {
    using TL = Tile<LL>;
    const int lane = threadIdx.x & 63;
    const int j = lane & 31;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        // layout of Ws: [o][t2][t1] (T=8: [o][pair][t2][t1])
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    int os, t2, cs, t1;
                    Slots<LL>::row(rb, row, os, t2);
                    Slots<LL>::col(cb, j, cs, t1);
                    bool mine;
                    int dst;
                    if constexpr (TL::T == 64) {
                        mine = true;
                        dst = t2 * LL + t1;
                    } else if constexpr (TL::T == 8) {
                        mine = (cs >> 1) == u;
                        dst = ((os * 2 + (cs & 1)) * LL + t2) * LL + t1;
                    } else {
                        mine = cs == u;
                        dst = (os * LL + t2) * LL + t1;
                    }
                    if (mine && t1 < LL && t2 < LL) Ws[dst] = acc[rb][cb][v];
                }
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): W stores visible to the wave
        __builtin_amdgcn_wave_barrier();
        backproject<LL>(Ys, Ws, wobs, bacc[u]);
        __builtin_amdgcn_wave_barrier();
    }
}

// Posterior mass c of the wave's w tiles, accumulated per lane.
template <int LL>
__device__ __forceinline__ void count_tile(float (&cnt)[2][BP<LL>::NCNT], int rb, int cb, int v,
                                           float w) {
    using TL = Tile<LL>;
    if constexpr (TL::T == 64) cnt[cb][rb * 16 + v] += w;
    else cnt[cb][v % BP<LL>::NCNT] += w;
}

// Block reduction of c and b and one store per chunk.  The 4 waves form WO =
// 4 / WC observation groups x WC component groups (wave = wo * WC + g); group g
// of the block holds components (cg + g) * CPW + cs.  Sums over the WO waves of
// a group run in a fixed order (pairwise for WO = 4).
template <int LL, int NU>
__device__ __forceinline__ void store_chunk_partials(const StepArgs& p, int64_t chunk, int cg,
                                                     int WC, float* red,
                                                     const float (&cnt)[2][BP<LL>::NCNT],
                                                     const float (&bacc)[NU][BP<LL>::NACC]) {
    using TL = Tile<LL>;
    using B = BP<LL>;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int PER = TL::CPW * LL * LL;
    const int WO = 4 / WC;
    auto fold = [&](const float* r, int e) -> float {
        const int g = e / PER, k = e % PER;
        if (WO == 4)
            return (r[(0 * WC + g) * PER + k] + r[(1 * WC + g) * PER + k]) +
                   (r[(2 * WC + g) * PER + k] + r[(3 * WC + g) * PER + k]);
        if (WO == 2) return r[g * PER + k] + r[(WC + g) * PER + k];
        return r[g * PER + k];
    };
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * PER; e += 256) red[e] = 0.f;
    __syncthreads();
    {
        const int j = lane & 31;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int k = 0; k < B::NCNT; ++k) {
                int rb, v;
                if constexpr (TL::T == 64) { rb = k >> 4; v = k & 15; }
                else { rb = 0; v = k; }
                const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                int os, t2, cs, t1;
                Slots<LL>::row(rb, row, os, t2);
                Slots<LL>::col(cb, j, cs, t1);
                if (t1 < LL && t2 < LL) red[wave * PER + (cs * LL + t1) * LL + t2] += cnt[cb][k];
            }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < WC * PER; e += 256) {
        const int c = (cg + e / PER) * TL::CPW + (e % PER) / (LL * LL);
        const float s = fold(red, e);
        if (c < p.KK) p.cpart[(chunk * p.KK + c) * (LL * LL) + (e % (LL * LL))] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * PER; e += 256) red[e] = 0.f;
    __syncthreads();
    {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            if constexpr (TL::T == 32) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int q2 = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const int q1 = lane & 31;
                    if (q1 < LL && q2 < LL) red[wave * PER + (u * LL + q1) * LL + q2] += bacc[u][v];
                }
            } else if constexpr (TL::T == 64) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int v = 0; v < 16; ++v) {
                            const int q2 = rb * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                            const int q1 = cb * 32 + (lane & 31);
                            if (q1 < LL && q2 < LL)
                                red[wave * PER + (u * LL + q1) * LL + q2] += bacc[u][(rb * 2 + cb) * 16 + v];
                        }
            } else {
                // 16x16x4 output: lane holds D[4*(lane>>4)+v][lane&15]
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rrow = 4 * (lane >> 4) + v;
                    const int ccol = lane & 15;
                    int q2 = rrow % TL::T, q1, cs;
                    if constexpr (TL::T == 16) { q1 = ccol; cs = u; }
                    else { q1 = ccol & 7; cs = 2 * u + (ccol >> 3); }
                    // T=8: rows 8..15 duplicate rows 0..7; keep the lower half only
                    const bool dup = TL::T == 8 && rrow >= 8;
                    if (!dup && q1 < LL && q2 < LL) red[wave * PER + (cs * LL + q1) * LL + q2] += bacc[u][v];
                }
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < WC * PER; e += 256) {
        const int c = (cg + e / PER) * TL::CPW + (e % PER) / (LL * LL);
        const float s = fold(red, e);
        if (c < p.KK) p.bpart[(chunk * p.KK + c) * (LL * LL) + (e % (LL * LL))] = s;
    }
}

template <int LL>
__device__ __forceinline__ void mfma_pass2_body(const StepArgs& p, int chunk_i, int cg, float* lds) {
    using TL = Tile<LL>;
    using B = BP<LL>;
    float* Xs = lds;
    float* Ys = Xs + TL::CPW * TL::XS;
    float* Wall = Ys + TL::NT * TL::OS;
    const int wave = threadIdx.x >> 6;
    float* Ws = Wall + wave * B::WS;
    load_x_group<LL>(p, cg, Xs);
    // number of back-projection "units": components (T>=16) or component pairs (T=8)
    constexpr int NU = TL::T == 8 ? TL::CPW / 2 : TL::CPW;
    float bacc[NU][B::NACC];
    float cnt[2][B::NCNT];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int k = 0; k < B::NACC; ++k) bacc[u][k] = 0.f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int k = 0; k < B::NCNT; ++k) cnt[cb][k] = 0.f;

    const int64_t c0 = (int64_t)chunk_i * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += TL::NT) {
        __syncthreads();
        load_y_tile<LL>(p, o0, Ys);
        __syncthreads();
        const int wobs = wave * TL::OPW;
        const int64_t wobs_g = o0 + wobs;
        floatx16 acc[2][2];
        score_tiles<LL>(Ys, Xs, wobs, acc);
        float2 lse_o[TL::OPW];
#pragma unroll
        for (int k = 0; k < TL::OPW; ++k)
            lse_o[k] = (wobs_g + k < p.N) ? p.lse[wobs_g + k] : make_float2(0.f, 0.f);
        // w = exp(a - lse) in place; accumulate c
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int os;
                    const float a = tile_logit<LL>(p, cg, wobs_g, rb, cb, v, acc[rb][cb][v], os);
                    const float w = a > -INFINITY ? fast_exp((a - lse_o[os].x) - lse_o[os].y) : 0.f;
                    acc[rb][cb][v] = w;
                    count_tile<LL>(cnt, rb, cb, v, w);
                }
        backproject_tiles<LL, NU>(Ys, Ws, wobs, acc, bacc);
    }
    store_chunk_partials<LL, NU>(p, chunk_i, cg, 1, lds, cnt, bacc);
}

// ============================================================================
// Single pass (FP32 MFMA) for instances whose K^2 components fit in one block:
// the 4 waves form WO = 4 / WC observation groups x WC component groups of CPW
// components.  Every wave scores its observations against its group, reduces
// (max, sum exp) per observation, and the WC waves of an observation group
// combine these through LDS in a fixed order into the full log-sum-exp; the
// posterior w = exp(a - max_wave) * exp(max_wave - lse) then feeds the same
// back-projection as pass 2.  The score map is computed once per pair.  The
// combined (max, sum) per observation is stored (n_part = 1) for the
// log-likelihood reduction that follows.
// grid = (n_chunks); block = 256.
template <int LL>
__device__ __forceinline__ void mfma_fused_body(const StepArgs& p, int chunk_i, float* lds) {
    using TL = Tile<LL>;
    using B = BP<LL>;
    const int WC = p.fuse_wc, WO = 4 / WC;
    const int ntf = WO * TL::OPW;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wc = wave % WC, wo = wave / WC;
    float* Xs = lds;
    float* Ys = Xs + WC * TL::CPW * TL::XS;
    float* Wall = Ys + ntf * TL::OS;
    float* Ws = Wall + wave * B::WS;
    for (int g = 0; g < WC; ++g) load_x_group<LL>(p, g, Xs + g * TL::CPW * TL::XS);
    const float* Xw = Xs + wc * TL::CPW * TL::XS;
    const bool active = wc * TL::CPW < p.KK;   // a group past the last component only waits
    constexpr int NU = TL::T == 8 ? TL::CPW / 2 : TL::CPW;
    float bacc[NU][B::NACC];
    float cnt[2][B::NCNT];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int k = 0; k < B::NACC; ++k) bacc[u][k] = 0.f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int k = 0; k < B::NCNT; ++k) cnt[cb][k] = 0.f;

    const int64_t c0 = (int64_t)chunk_i * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += ntf) {
        __syncthreads();
        load_y_tile<LL>(p, o0, Ys, ntf);
        __syncthreads();
        const int wobs = wo * TL::OPW;
        const int64_t wobs_g = o0 + wobs;
        floatx16 acc[2][2];
        float mx[TL::OPW], sm[TL::OPW];
#pragma unroll
        for (int k = 0; k < TL::OPW; ++k) { mx[k] = -INFINITY; sm[k] = 0.f; }
        if (active) {
            score_tiles<LL>(Ys, Xw, wobs, acc);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        int os;
                        const float a = tile_logit<LL>(p, wc, wobs_g, rb, cb, v, acc[rb][cb][v], os);
                        acc[rb][cb][v] = a;
                        mx[os] = fmaxf(mx[os], a);
                    }
#pragma unroll
            for (int k = 0; k < TL::OPW; ++k)
                for (int off = 32; off > 0; off >>= 1) mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], off));
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        int os, t2;
                        const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        Slots<LL>::row(rb, row, os, t2);
                        const float a = acc[rb][cb][v];
                        const float e = a > -INFINITY ? fast_exp(a - mx[os]) : 0.f;
                        acc[rb][cb][v] = e;
                        sm[os] += e;
                    }
#pragma unroll
            for (int k = 0; k < TL::OPW; ++k)
                for (int off = 32; off > 0; off >>= 1) sm[k] += __shfl_xor(sm[k], off);
        }
        // exchange (max, sum) between the component groups through the first
        // 2*OPW floats of each wave's W tile (free until w is written below)
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < TL::OPW; ++k) { Ws[2 * k] = mx[k]; Ws[2 * k + 1] = sm[k]; }
        }
        __syncthreads();
        float scale[TL::OPW];
#pragma unroll
        for (int k = 0; k < TL::OPW; ++k) {
            float M = -INFINITY;
            for (int g = 0; g < WC; ++g) M = fmaxf(M, Wall[(wo * WC + g) * B::WS + 2 * k]);
            float S = 0.f;
            for (int g = 0; g < WC; ++g) {
                const float mg = Wall[(wo * WC + g) * B::WS + 2 * k];
                const float sg = Wall[(wo * WC + g) * B::WS + 2 * k + 1];
                if (mg > -INFINITY) S += sg * fast_exp(mg - M);
            }
            const bool valid = wobs_g + k < p.N && M > -INFINITY;
            scale[k] = valid && mx[k] > -INFINITY ? fast_exp((mx[k] - M) - __logf(S)) : 0.f;
            if (valid && wc == 0 && lane == 0) p.part[wobs_g + k] = make_float2(M, S);
        }
        __syncthreads();   // every wave has read the exchange before W is overwritten
        if (active) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        int os, t2;
                        const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        Slots<LL>::row(rb, row, os, t2);
                        const float w = acc[rb][cb][v] * scale[os];
                        acc[rb][cb][v] = w;
                        count_tile<LL>(cnt, rb, cb, v, w);
                    }
            backproject_tiles<LL, NU>(Ys, Ws, wobs, acc, bacc);
        }
    }
    store_chunk_partials<LL, NU>(p, chunk_i, 0, WC, lds, cnt, bacc);
}

template <int LL> constexpr size_t lds_score_mfma() {
    using TL = Tile<LL>;
    return sizeof(float) * (size_t)(TL::CPW * TL::XS + TL::NT * TL::OS);
}
// LDS of the single pass with WC component groups per block (0 if WC is not
// 1, 2 or 4)
template <int LL> constexpr size_t lds_fused_mfma(int WC) {
    using TL = Tile<LL>;
    if (WC != 1 && WC != 2 && WC != 4) return 0;
    size_t a = sizeof(float) * ((size_t)WC * TL::CPW * TL::XS + (size_t)(4 / WC) * TL::OPW * TL::OS +
                                4 * (size_t)BP<LL>::WS);
    size_t r = sizeof(float) * (size_t)(4 * TL::CPW * LL * LL);
    return a > r ? a : r;
}
template <int LL> constexpr size_t lds_backproject_mfma() {
    using TL = Tile<LL>;
    size_t a = lds_score_mfma<LL>() + sizeof(float) * (size_t)(4 * BP<LL>::WS);
    size_t r = sizeof(float) * (size_t)(4 * TL::CPW * LL * LL);
    return a > r ? a : r;
}

}  // namespace srmra
