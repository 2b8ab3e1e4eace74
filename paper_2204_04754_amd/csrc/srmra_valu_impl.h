// Plain FP32 (vector ALU, no matrix cores) form of the two passes of the EM step.
//
// Same decomposition as the matrix-core form: a block owns a chunk of
// observations and a group of components; the Ll x Ll score map of every
// (observation, component) pair is computed from LDS-resident tiles by direct
// FMAs, S_{i,c}[t1][t2] = sum_{r1,b2} y_i[r1][(b2+t2)%Ll] x_c[(r1-t1)%Ll][b2].
// A thread owns a 4x4 block (t1 in T1..T1+3, t2 in T2..T2+3) of one component
// for NOV observations; along b2 the y operand is a sliding window (one new LDS
// value per step and observation), the x operand four LDS values per step.
// The back-projection b_c[q1][q2] = sum_i sum_{t1,t2} w_i[t1][t2] y_i[(q1+t1)%Ll][(q2+t2)%Ll]
// uses the same 4x4 ownership over (q1, q2) with a sliding window along t2.
#pragma once
#include "srmra_common.h"

namespace srmra {

template <int LL>
__device__ __forceinline__ void load_x_group_valu(const StepArgs& p, int cg, float* Xs) {
    using V = Valu<LL>;
    for (int cs = 0; cs < p.cpb; ++cs) {
        int c = cg * p.cpb + cs;
        if (c >= p.KK) c = p.KK - 1;
        const float* src = p.xt2 + (int64_t)c * LL * 2 * LL;
        for (int e = threadIdx.x; e < LL * 2 * LL; e += 256) Xs[cs * V::XS + e] = src[e];
    }
}

// y tile (less the offset mu) with every row doubled: Ys[o][r1][a] = y_o[r1][a % Ll] - mu,
// a in [0, 2Ll)
template <int LL>
__device__ __forceinline__ void load_y_tile_valu(const StepArgs& p, int64_t o0, int nt, float* Ys) {
    using V = Valu<LL>;
    const float mu = centre_of(p.centre);
    for (int e = threadIdx.x; e < nt * LL * LL; e += 256) {
        const int o = e / (LL * LL), q = e % (LL * LL);
        const int r1 = q / LL, r2 = q % LL;
        const float v = (o0 + o < p.N) ? p.y[(o0 + o) * (int64_t)(LL * LL) + q] - mu : 0.f;
        float* d = Ys + o * V::YS + r1 * 2 * LL;
        d[r2] = v;
        d[r2 + LL] = v;
    }
}

// 4x4 x NOV score block of one unit.
template <int LL>
__device__ __forceinline__ void valu_score(const float* Ys, const float* Xs, int o_loc, int cs,
                                           int T1, int T2, float (&acc)[Valu<LL>::NOV][4][4]) {
    using V = Valu<LL>;
#pragma unroll
    for (int o = 0; o < V::NOV; ++o)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[o][u][v] = 0.f;
    const float* xb = Xs + cs * V::XS + LL - T1;       // + b2*2Ll + r1 - u
    for (int r1 = 0; r1 < LL; ++r1) {
        float win[V::NOV][4];
        const float* yr[V::NOV];
#pragma unroll
        for (int o = 0; o < V::NOV; ++o) {
            yr[o] = Ys + (o_loc + o) * V::YS + r1 * 2 * LL + T2;   // + b2 + v
#pragma unroll
            for (int v = 0; v < 4; ++v) win[o][v] = yr[o][v];
        }
        const float* xr = xb + r1;
#pragma unroll
        for (int b2 = 0; b2 < LL; ++b2) {
            float bx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) bx[u] = xr[b2 * 2 * LL - u];
#pragma unroll
            for (int o = 0; o < V::NOV; ++o)
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[o][u][v] = fmaf(win[o][v], bx[u], acc[o][u][v]);
            if (b2 + 1 < LL) {
#pragma unroll
                for (int o = 0; o < V::NOV; ++o) {
                    win[o][0] = win[o][1]; win[o][1] = win[o][2]; win[o][2] = win[o][3];
                    win[o][3] = yr[o][b2 + 4];
                }
            }
        }
    }
}

// Pass 1.  grid = (n_chunks, n_cg), block 256.  ntile observations per tile;
// units = (ntile/NOV) * cpb * (Ll/4)^2 <= 256.
template <int LL>
__device__ __forceinline__ void valu_pass1_body(const StepArgs& p, int chunk, int cg, float* lds) {
    using V = Valu<LL>;
    float* Xs = lds;
    float* Ys = Xs + p.cpb * V::XS;
    float2* Ps = reinterpret_cast<float2*>(Ys + p.ntile * V::YS);   // [256][NOV]
    load_x_group_valu<LL>(p, cg, Xs);
    const int units = (p.ntile / V::NOV) * p.cpb * V::BLK;
    const int u = threadIdx.x;
    int og = 0, cs = 0, t1b = 0, t2b = 0;
    if (u < units) {
        t2b = u % (LL / 4);
        t1b = (u / (LL / 4)) % (LL / 4);
        const int r = u / V::BLK;
        cs = r % p.cpb;
        og = r / p.cpb;
    }
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += p.ntile) {
        __syncthreads();
        load_y_tile_valu<LL>(p, o0, p.ntile, Ys);
        __syncthreads();
        if (u < units) {
            float acc[V::NOV][4][4];
            valu_score<LL>(Ys, Xs, og * V::NOV, cs, 4 * t1b, 4 * t2b, acc);
            const int c = cg * p.cpb + cs;
            const bool cok = c < p.KK;
#pragma unroll
            for (int o = 0; o < V::NOV; ++o) {
                const bool ook = cok && (o0 + og * V::NOV + o) < p.N;
                float mx = -INFINITY;
                float av[4][4];
#pragma unroll
                for (int uu = 0; uu < 4; ++uu)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int t1 = 4 * t1b + uu, t2 = 4 * t2b + v;
                        const float a = ook ? acc[o][uu][v] * p.inv_s2 +
                                                  p.betaT[(int64_t)c * (LL * LL) + t2 * LL + t1]
                                            : -INFINITY;
                        av[uu][v] = a;
                        mx = fmaxf(mx, a);
                    }
                float sm = 0.f;
                if (mx > -INFINITY) {
#pragma unroll
                    for (int uu = 0; uu < 4; ++uu)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (av[uu][v] > -INFINITY) sm += fast_exp(av[uu][v] - mx);
                }
                Ps[u * V::NOV + o] = make_float2(mx, sm);
            }
        }
        __syncthreads();
        // reduce per observation over all units that hold it (fixed order)
        for (int ol = threadIdx.x; ol < p.ntile; ol += 256) {
            const int oga = ol / V::NOV, o = ol % V::NOV;
            const int per = p.cpb * V::BLK;
            float m = -INFINITY;
            for (int k = 0; k < per; ++k) m = fmaxf(m, Ps[(oga * per + k) * V::NOV + o].x);
            float s = 0.f;
            if (m > -INFINITY)
                for (int k = 0; k < per; ++k) {
                    const float2 q = Ps[(oga * per + k) * V::NOV + o];
                    if (q.x > -INFINITY) s += q.y * fast_exp(q.x - m);
                }
            if (o0 + ol < p.N) p.part[(int64_t)cg * p.N + o0 + ol] = make_float2(m, s);
        }
    }
}

// Pass 2.  LDS: Xs, Ys (doubled rows), W[ntile][cpb][Ll][Ll] (t1-major), then
// reduction scratch.
template <int LL>
__device__ __forceinline__ void valu_pass2_body(const StepArgs& p, int chunk, int cg, float* lds) {
    using V = Valu<LL>;
    float* Xs = lds;
    float* Ys = Xs + p.cpb * V::XS;
    float* Ws = Ys + p.ntile * V::YS;
    load_x_group_valu<LL>(p, cg, Xs);
    const int units = (p.ntile / V::NOV) * p.cpb * V::BLK;
    const int u = threadIdx.x;
    int og = 0, cs = 0, t1b = 0, t2b = 0;
    if (u < units) {
        t2b = u % (LL / 4);
        t1b = (u / (LL / 4)) % (LL / 4);
        const int r = u / V::BLK;
        cs = r % p.cpb;
        og = r / p.cpb;
    }
    const int c = cg * p.cpb + cs;
    float cnt[4][4], bacc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) { cnt[a][b] = 0.f; bacc[a][b] = 0.f; }
    const int64_t c0 = (int64_t)chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o0 = c0; o0 < c1; o0 += p.ntile) {
        __syncthreads();
        load_y_tile_valu<LL>(p, o0, p.ntile, Ys);
        __syncthreads();
        if (u < units) {
            float acc[V::NOV][4][4];
            valu_score<LL>(Ys, Xs, og * V::NOV, cs, 4 * t1b, 4 * t2b, acc);
            const bool cok = c < p.KK;
#pragma unroll
            for (int o = 0; o < V::NOV; ++o) {
                const int64_t og_ = o0 + og * V::NOV + o;
                const bool ook = cok && og_ < p.N;
                const float2 l = ook ? p.lse[og_] : make_float2(0.f, 0.f);
                float* wdst = Ws + ((og * V::NOV + o) * p.cpb + cs) * (LL * LL);
#pragma unroll
                for (int uu = 0; uu < 4; ++uu)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int t1 = 4 * t1b + uu, t2 = 4 * t2b + v;
                        float w = 0.f;
                        if (ook) {
                            const float a = acc[o][uu][v] * p.inv_s2 +
                                            p.betaT[(int64_t)c * (LL * LL) + t2 * LL + t1];
                            w = a > -INFINITY ? fast_exp((a - l.x) - l.y) : 0.f;
                        }
                        cnt[uu][v] += w;
                        wdst[t1 * LL + t2] = w;
                    }
            }
        }
        __syncthreads();
        // back-projection: unit -> (og, cs, q1 block, q2 block); sums over its NOV obs
        if (u < units) {
            const int Q1 = 4 * t1b, Q2 = 4 * t2b;
#pragma unroll 1
            for (int o = 0; o < V::NOV; ++o) {
                const int ol = og * V::NOV + o;
                const float* yb = Ys + ol * V::YS;
                const float* wb = Ws + (ol * p.cpb + cs) * (LL * LL);
                for (int t1 = 0; t1 < LL; ++t1) {
                    const float* yr[4];
#pragma unroll
                    for (int uu = 0; uu < 4; ++uu) {
                        int r = Q1 + uu + t1;
                        r = r >= LL ? r - LL : r;
                        yr[uu] = yb + r * 2 * LL + Q2;   // + t2 + v
                    }
                    float win[4][4];
#pragma unroll
                    for (int uu = 0; uu < 4; ++uu)
#pragma unroll
                        for (int v = 0; v < 4; ++v) win[uu][v] = yr[uu][v];
                    const float* wr = wb + t1 * LL;
#pragma unroll
                    for (int t2 = 0; t2 < LL; ++t2) {
                        const float wv = wr[t2];
#pragma unroll
                        for (int uu = 0; uu < 4; ++uu)
#pragma unroll
                            for (int v = 0; v < 4; ++v) bacc[uu][v] = fmaf(wv, win[uu][v], bacc[uu][v]);
                        if (t2 + 1 < LL) {
#pragma unroll
                            for (int uu = 0; uu < 4; ++uu) {
                                win[uu][0] = win[uu][1]; win[uu][1] = win[uu][2]; win[uu][2] = win[uu][3];
                                win[uu][3] = yr[uu][t2 + 4];
                            }
                        }
                    }
                }
            }
        }
    }
    // ---- reduce over observation groups (fixed order) and store the chunk partials
    __syncthreads();
    float* red = lds;
    const int ngr = p.ntile / V::NOV;
    const int per = p.cpb * V::BLK;       // units per observation group
    // c
    if (u < units) {
#pragma unroll
        for (int uu = 0; uu < 4; ++uu)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[u * 16 + uu * 4 + v] = cnt[uu][v];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < per * 16; e += 256) {
        float s = 0.f;
        for (int g = 0; g < ngr; ++g) s += red[(g * per) * 16 + e];
        const int k = e / 16, uu = (e % 16) / 4, v = e % 4;
        const int csl = k / V::BLK, blk = k % V::BLK;
        const int tb2 = blk % (LL / 4), tb1 = blk / (LL / 4);
        const int cc = cg * p.cpb + csl;
        const int t1 = 4 * tb1 + uu, t2 = 4 * tb2 + v;
        if (cc < p.KK) p.cpart[(chunk * p.KK + cc) * (LL * LL) + t1 * LL + t2] = s;
    }
    __syncthreads();
    if (u < units) {
#pragma unroll
        for (int uu = 0; uu < 4; ++uu)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[u * 16 + uu * 4 + v] = bacc[uu][v];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < per * 16; e += 256) {
        float s = 0.f;
        for (int g = 0; g < ngr; ++g) s += red[(g * per) * 16 + e];
        const int k = e / 16, uu = (e % 16) / 4, v = e % 4;
        const int csl = k / V::BLK, blk = k % V::BLK;
        const int qb2 = blk % (LL / 4), qb1 = blk / (LL / 4);
        const int cc = cg * p.cpb + csl;
        const int q1 = 4 * qb1 + uu, q2 = 4 * qb2 + v;
        if (cc < p.KK) p.bpart[(chunk * p.KK + cc) * (LL * LL) + q1 * LL + q2] = s;
    }
}

}  // namespace srmra
