// FFT route of the EM step (SRMRA_FP32_FFT, L_low in {8, 12, 16, 24, 32, 48, 64}): the same
// step as the dense forms, with the contractions as products in the 2-D DFT
// domain of the L_low grid.  With (R_t v)[n] = v[n - t]:
//   score     S_{i,c}[t] = sum_n y_i[n] x_c[n - t]      = IDFT(Y_i . conj(X_c))[t]
//   back-proj b_c[q]     = sum_i sum_t w_{i,c}[t] y_i[q + t] = IDFT(sum_i Y_i . conj(W_{i,c}))[q]
//   mass      c_c[t]     = sum_i w_{i,c}[t]   (summed directly, no transform)
// Y_i (DFT of y_i - mu) is prepared once per job; X_c once per step.  Pass 1:
// team per observation, its (max, sum exp) over all components.  Pass 2: team
// per component (observations split over TPC teams), w = exp(a - LSE_i), its
// DFT, the frequency-domain sum of the back-projection and the spatial sum of
// w; per-chunk FP32 partials, summed in FP64, the former brought back by a
// separable FP64 inverse DFT.  One component per
// transform: packing two real signals into one complex transform would give a
// component of little posterior mass the rounding error of its heavier
// partner.  The transforms are the in-register team FFTs of srmra_fft_impl.h
// (O(L^2 log L) per pair instead of the dense 4 L^4).
#pragma once
#include "srmra_aux_impl.h"
#include "srmra_common.h"
#include "srmra_fft_impl.h"

namespace srmra {
namespace fft {

// L = 3 * 2^m: teams of L lanes over the whole 256-thread block (WIDE: they
// may span two waves, and their transposes wait on the block barrier), or
// 64 / L teams inside each wave (wave barriers; a quarter of the lanes idle at
// L 24 and 48)
__host__ __device__ constexpr bool row_wide(int L) { return L % 3 == 0; }
// teams of pass 2 per 256-thread block (pass 1's are its own): 2 L lanes each
// (L <= 32, and L 48: lane pairs), one team of four lanes per row (L 64), 256 / L
// teams of L lanes (L 12, 24)
__host__ __device__ inline int teams_of(int L) {
    if (L == 48) return 256 / (2 * L);
    if (L % 3 == 0) return row_wide(L) ? 256 / L : 4 * (64 / L);
    return L == 64 ? 1 : 256 / (2 * L);
}
// teams per component in pass 2 for KK components: TPC with CG = teams / TPC
// components per block over ceil(KK / CG) component groups, chosen for the
// largest share KK TPC / (groups x teams) of busy teams, then the fewest
// groups, then the fewest teams per component: at KK = 9 and 4 teams, one
// component per block on all 4 teams (every team busy) instead of 4
// components per block (the last group's block three quarters idle).  TPC
// is a power of 2 for the power-of-two L and any count for L = 3 * 2^m (10
// teams at L 24: 5 per component)
__host__ __device__ inline int tpc_of(int L, int KK) {
    const int teams = teams_of(L);
    int best = 1, best_busy = 0, best_all = 1, best_groups = 1 << 30;
    for (int tpc = 1; tpc <= teams; tpc = (L % 3 == 0) ? tpc + 1 : 2 * tpc) {
        const int cg = teams / tpc;
        const int groups = (KK + cg - 1) / cg;
        const int busy = KK * tpc, all = groups * teams;
        const long long lhs = (long long)busy * best_all, rhs = (long long)best_busy * all;
        if (lhs > rhs || (lhs == rhs && groups < best_groups)) {
            best = tpc;
            best_busy = busy;
            best_all = all;
            best_groups = groups;
        }
    }
    return best;
}

template <int L> struct Geo {
    static constexpr int TEAMS = 256 / L;
    static constexpr int BUF = L * (L + 1);   // float2 per team buffer
};

template <int L> constexpr size_t lds_bytes() {
    return sizeof(float2) * ((size_t)Geo<L>::TEAMS * Geo<L>::BUF + L / 2);
}

// ---- per job: Y_i = DFT(y_i - mu), [N][L][L] complex.  TRANSPOSED: stored in
// pairs along k2, Yp[i][k2 / 2][k1][k2 % 2] = Y_i[k1][k2], so that the thread
// of a team that holds row k1 of Y_i reads two elements per 16-byte load and
// the team's lanes read consecutive 16-byte words; otherwise natural order
// Y[i][k1][k2].
template <int L, bool TRANSPOSED>
__device__ __forceinline__ void prep_y_body(const float* __restrict__ y, int64_t N,
                                            const double* __restrict__ centre,
                                            float2* __restrict__ yhat) {
    extern __shared__ float2 sh[];
    float2* tw = sh + Geo<L>::TEAMS * Geo<L>::BUF;
    make_twiddles<L>(tw);
    __syncthreads();
    const int team = threadIdx.x / L, r = threadIdx.x % L;
    float2* buf = sh + team * Geo<L>::BUF;
    const float mu = centre_of(centre);
    const int64_t i = (int64_t)blockIdx.x * Geo<L>::TEAMS + team;
    if (i >= N) return;   // whole teams leave together (a team lies in one wave)
    float2 v[L];
    if constexpr (TRANSPOSED) {
        // thread r: column r of y_i in, row r of Y_i out (both coalesced over the team)
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = make_float2(y[(i * L + k) * L + r] - mu, 0.f);
        fft2_cols_then_rows<L, false>(v, buf, r, tw);
    } else {
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = make_float2(y[(i * L + r) * L + k] - mu, 0.f);
        fft2_rows_then_cols<L, false>(v, buf, r, tw);
    }
    if constexpr (TRANSPOSED) {   // v[k] = Y_i[r][k]
        float4* d = reinterpret_cast<float4*>(yhat) + i * (L / 2) * L + r;
#pragma unroll
        for (int k = 0; k < L; k += 2) d[(k / 2) * L] = make_float4(v[k].x, v[k].y, v[k + 1].x, v[k + 1].y);
    } else {                      // v[k] = Y_i[k][r]
#pragma unroll
        for (int k = 0; k < L; ++k) yhat[(i * L + k) * L + r] = v[k];
    }
}

// ---- per step: X_c = DFT(x_c - mu), stored in pairs along k2 like Y:
// Xp[c][k2 / 2][k1][k2 % 2] = X_c[k1][k2]; the first L threads of a block for
// component c, buf an L x (L + 1) transpose buffer, tw the full twiddle table
// (L entries, make_twiddles_n<L, L>, filled and synchronised by the caller)
template <int L>
__device__ __forceinline__ void pack_x_body(const float* __restrict__ x, int K, const double* __restrict__ centre,
                                            float2* __restrict__ xhat, int c, float2* buf, const float2* tw) {
    if (threadIdx.x >= L) return;
    const int c1 = c / K, c2 = c % K, Lh = K * L, r = threadIdx.x;
    const float mu = centre_of(centre);
    float2 v[L];
#pragma unroll
    for (int k = 0; k < L; ++k)   // column r of x_c: v[k] = x_c[k][r]
        v[k] = make_float2(x[(int64_t)(c1 + k * K) * Lh + (c2 + r * K)] - mu, 0.f);
    fft1any<L, false>(v, tw);
#pragma unroll
    for (int k = 0; k < L; ++k) buf[k * (L + 1) + r] = v[k];
    team_sync();
#pragma unroll
    for (int k = 0; k < L; ++k) v[k] = buf[r * (L + 1) + k];
    team_sync();
    fft1any<L, false>(v, tw);                                   // v[k] = X_c[r][k]
    float4* d = reinterpret_cast<float4*>(xhat) + (int64_t)c * (L / 2) * L + r;
#pragma unroll
    for (int k = 0; k < L; k += 2) d[(k / 2) * L] = make_float4(v[k].x, v[k].y, v[k + 1].x, v[k + 1].y);
}
template <int L> constexpr size_t pack_lds() { return sizeof(float2) * ((size_t)L * (L + 1) + L); }

// ---- the two passes at L <= 32: a team of 2L lanes (inside one wave) per
// image (lane pair (r, h): r the row or column, h which half of it), TEAMS
// teams per block
template <int L> struct GeoP {
    static constexpr int TEAMS = 256 / (2 * L);
    static constexpr int BUF = L * (L + 1);   // float2 per team buffer
};
// [team buffers TEAMS x BUF float2][twiddles L / 2][pair table L]
template <int L> constexpr size_t lds_pairs() {
    return sizeof(float2) * ((size_t)GeoP<L>::TEAMS * GeoP<L>::BUF + L / 2 + L);
}
// pass 2 with X_c staged: [X_c of each team's component, TEAMS x L x L float2,
// the paired layout] after the above
template <int L> constexpr size_t lds_pairs_xs() {
    return lds_pairs<L>() + sizeof(float2) * (size_t)GeoP<L>::TEAMS * L * L;
}

// Scores of (observation o, component c) for pair (r, h): s[k] = a at
// (t1 = (L/2) h + k, t2 = r).  Row r of Y_o conj(X_c) enters as its samples
// 2m + h, for which the team's lanes read consecutive words of the paired
// layouts.
template <int L>
__device__ __forceinline__ void score_pair(const StepArgs& p, const float2* __restrict__ yhat,
                                           const float2* xc, int64_t o, int c,
                                           float2* buf, int r, int h, const float2* tw, const float2* twh,
                                           float (&s)[L / 2]) {
    float2 v[L / 2];
    const float2* yr = yhat + ((int64_t)o * (L / 2) * L + r) * 2 + h;   // Y_o[r][2m + h] at yr[2 L m]
    const float2* xr = xc + r * 2 + h;                                   // X_c (xc: its L x L values)
#pragma unroll
    for (int m = 0; m < L / 2; ++m) v[m] = cmulc(yr[2 * L * m], xr[2 * L * m]);
    fft_pair_dit<L, true>(v, h, tw, twh);                  // v[k] = row r, n2 = (L/2) h + k
#pragma unroll
    for (int k = 0; k < L / 2; ++k) buf[r * (L + 1) + (L / 2) * h + k] = v[k];
    team_sync();
#pragma unroll
    for (int m = 0; m < L / 2; ++m) v[m] = buf[(2 * m + h) * (L + 1) + r];   // column r, rows 2m + h
    team_sync();
    fft_pair_dit<L, true>(v, h, tw, twh);                  // v[k] = S[(L/2) h + k][r]
    const float sc = p.inv_s2 / (float)(L * L);
    const float* bet = p.betaT + (int64_t)c * (L * L) + r * L + (L / 2) * h;   // betaT[c][t2 = r][t1]
#pragma unroll
    for (int k = 0; k < L / 2; ++k) s[k] = v[k].x * sc + bet[k];
}

__device__ __forceinline__ void lse_merge(float& m, float& s, float m2, float s2) {
    if (m2 == -INFINITY) return;
    if (m == -INFINITY) { m = m2; s = s2; return; }
    const float mn = fmaxf(m, m2);
    s = s * __expf(m - mn) + s2 * __expf(m2 - mn);
    m = mn;
}

// ---- pass 1: (max, sum exp) of every observation over all components.  Grid
// (chunks, component groups) like pass 2: the gridDim.y blocks of a chunk
// share its observations, so that pass 1 fills the device as pass 2 does.
template <int L>
__device__ __forceinline__ void pass1_pairs_body(const StepArgs& p, const float2* __restrict__ yhat,
                                                 const float2* __restrict__ xhat, int64_t chunk, int ysplit,
                                                 int nsplit, float2* sh) {
    float2* tw = sh + GeoP<L>::TEAMS * GeoP<L>::BUF;
    float2* twp = tw + L / 2;
    make_twiddles<L>(tw);
    make_pair_twiddles<L>(twp);
    __syncthreads();
    const int team = threadIdx.x / (2 * L), lt = threadIdx.x % (2 * L);
    const int r = lt >> 1, h = lt & 1;
    const float2* twh = twp + (L / 2) * h;
    float2* buf = sh + team * GeoP<L>::BUF;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o = c0 + team + (int64_t)GeoP<L>::TEAMS * ysplit; o < c1;
         o += (int64_t)GeoP<L>::TEAMS * nsplit) {
        float m = -INFINITY, sm = 0.f;
        for (int c = 0; c < p.KK; ++c) {
            float s[L / 2];
            score_pair<L>(p, yhat, xhat + (int64_t)c * L * L, o, c, buf, r, h, tw, twh, s);
            float mc = -INFINITY;
#pragma unroll
            for (int k = 0; k < L / 2; ++k) mc = fmaxf(mc, s[k]);
            float sc = 0.f;
            if (mc > -INFINITY) {
#pragma unroll
                for (int k = 0; k < L / 2; ++k) sc += s[k] > -INFINITY ? __expf(s[k] - mc) : 0.f;
            }
            lse_merge(m, sm, mc, sc);
        }
        // team reduction (the team is 2L consecutive lanes of one wave)
        for (int off = L; off > 0; off >>= 1) {
            const float m2 = __shfl_xor(m, off), s2 = __shfl_xor(sm, off);
            lse_merge(m, sm, m2, s2);
        }
        if (lt == 0) p.part[o] = make_float2(m, sm);
    }
}

// ---- pass 2: per component group, the sums over the chunk.  Component group
// g holds CG components, TPC = TEAMS / CG teams each (observations split over
// them); partials [chunk][c][k1][k2] of sum_i Y_i conj(W_i) (bpart, float2)
// and [chunk][c][t1][t2] of sum_i w_i (cpart, float).  XS: each team reads
// its component's X_c from a copy in LDS (lds_pairs_xs) instead of global
// memory (faster in the batched launches at L 32, whose items are short; the
// single-problem launch, LDS-bound on its transposes there, reads it from L2).
template <int L, bool XS = false>
__device__ __forceinline__ void pass2_pairs_body(const StepArgs& p, const float2* __restrict__ yhat,
                                                 const float2* __restrict__ xhat, int TPC,
                                                 float2* __restrict__ bpart, float* __restrict__ cpart,
                                                 int64_t chunk, int ysplit, float2* sh) {
    float2* tw = sh + GeoP<L>::TEAMS * GeoP<L>::BUF;
    float2* twp = tw + L / 2;
    make_twiddles<L>(tw);
    make_pair_twiddles<L>(twp);
    __syncthreads();
    const int team = threadIdx.x / (2 * L), lt = threadIdx.x % (2 * L);
    const int r = lt >> 1, h = lt & 1;
    const float2* twh = twp + (L / 2) * h;
    float2* buf = sh + team * GeoP<L>::BUF;
    float2* xs = twp + L + team * (L * L);   // the team's X_c (XS)
    const int CG = GeoP<L>::TEAMS / TPC;
    const int c = ysplit * CG + team / TPC, u = team % TPC;
    const bool active = c < p.KK;
    if (XS && active) {
        const float4* src = reinterpret_cast<const float4*>(xhat + (int64_t)c * L * L);
        float4* dst = reinterpret_cast<float4*>(xs);
        for (int e = lt; e < L * L / 2; e += 2 * L) dst[e] = src[e];
    }
    __syncthreads();
    const float2* xcs = XS ? xs : xhat + (int64_t)(active ? c : 0) * L * L;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    float2 ab[L / 2];   // sum of Y conj(W) at (k1 = r, k2 = (L/2) h + k)
    float acw[L / 2];   // posterior mass at (t1 = (L/2) h + k, t2 = r)
#pragma unroll
    for (int k = 0; k < L / 2; ++k) { ab[k] = make_float2(0.f, 0.f); acw[k] = 0.f; }
    if (active) {
        for (int64_t o = c0 + u; o < c1; o += TPC) {
            float s[L / 2];
            score_pair<L>(p, yhat, xcs, o, c, buf, r, h, tw, twh, s);
            const float2 lse = p.lse[o];
            float2 v[L / 2];
#pragma unroll
            for (int k = 0; k < L / 2; ++k) {
                const float w = s[k] > -INFINITY ? __expf((s[k] - lse.x) - lse.y) : 0.f;
                acw[k] += w;
                v[k] = make_float2(w, 0.f);
            }
            // column t2 = r (its half (L/2) h..), transformed along t1, then the rows
            fft_pair_dif<L, false>(v, h, tw, twh);               // v[k] = k1 = 2k + h, column r
#pragma unroll
            for (int k = 0; k < L / 2; ++k) buf[(2 * k + h) * (L + 1) + r] = v[k];
            team_sync();
#pragma unroll
            for (int m = 0; m < L / 2; ++m) v[m] = buf[r * (L + 1) + 2 * m + h];   // row k1 = r, n2 = 2m + h
            team_sync();
            fft_pair_dit<L, false>(v, h, tw, twh);               // v[k] = W[r][(L/2) h + k]
            // Y_o[r][(L/2) h + k], k and k + 1 in one 16-byte word of the paired layout
            const float4* yr = reinterpret_cast<const float4*>(yhat) + ((int64_t)o * (L / 2) + (L / 4) * h) * L + r;
#pragma unroll
            for (int k = 0; k < L / 2; k += 2) {
                const float4 a = yr[(k / 2) * L];
                const float2 t0 = cmulc(make_float2(a.x, a.y), v[k]);
                const float2 t1 = cmulc(make_float2(a.z, a.w), v[k + 1]);
                ab[k].x += t0.x; ab[k].y += t0.y;
                ab[k + 1].x += t1.x; ab[k + 1].y += t1.y;
            }
        }
    }
    // sum the TPC teams of each component in a fixed order, one plane at a time
    // (each lane keeps its own L/2 slots of the team buffer)
    for (int plane = 0; plane < 2; ++plane) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < L / 2; ++k)
            buf[lt * (L / 2) + k] = plane == 0 ? ab[k] : make_float2(acw[k], 0.f);
        __syncthreads();
        if (active && u == 0) {
            for (int k = 0; k < L / 2; ++k) {
                float2 t = make_float2(0.f, 0.f);
                for (int j = 0; j < TPC; ++j) {
                    const float2 e = sh[(team + j) * GeoP<L>::BUF + lt * (L / 2) + k];
                    t.x += e.x; t.y += e.y;
                }
                if (plane == 0) bpart[((chunk * p.KK + c) * L + r) * L + (L / 2) * h + k] = t;   // [k1][k2]
                else cpart[((chunk * p.KK + c) * L + (L / 2) * h + k) * L + r] = t.x;            // [t1][t2]
            }
        }
    }
}

// ---- L_low 64: one team per block, four lanes per row (lane 4r + q holds a
// quarter of row r, see fft_quad_dit / fft_quad_dif), so a lane keeps 16
// complex values of an image; the LDS transposes are ordered by the block
// barrier, and every thread of the block belongs to the one team.  Two
// transpose buffers alternate, so that a transpose needs one barrier (between
// its writes and its reads): the next write to a buffer comes after the other
// buffer's barrier, which every thread reaches only once done reading.
namespace quad {
constexpr int L = 64, NV = L / 4;
constexpr int BUF = L * (L + 1);
// pass 2: two transpose buffers, the twiddles (L / 2) and one (max, sum) slot per wave
constexpr size_t lds() { return sizeof(float2) * (2 * (size_t)BUF + L / 2 + 4); }
// pass 1: a score's transpose moves the real parts through one buffer of L (L + 1)
// floats and the imaginary parts through another (two barriers per transpose,
// half the LDS, twice the blocks per CU); then the twiddles and the slots
constexpr size_t lds1() { return sizeof(float) * 2 * (size_t)BUF + sizeof(float2) * (L / 2 + 4); }

// scores of (observation o, component c) for lane (r, q): s[k] = a at
// (t1 = 16 quad_block(q) + k, t2 = r)
__device__ __forceinline__ void score(const StepArgs& p, const float2* __restrict__ yhat,
                                      const float2* __restrict__ xhat, int64_t o, int c, float2* buf,
                                      int r, int q, int bq, const float2* tw, float (&s)[NV]) {
    float2 v[NV];
    // Y_o[r][4m + q] of the paired layout [k2 / 2][k1][k2 % 2] at yr[4 L m]
    const float2* yr = yhat + (((int64_t)o * (L / 2) + (q >> 1)) * L + r) * 2 + (q & 1);
    const float2* xr = xhat + (((int64_t)c * (L / 2) + (q >> 1)) * L + r) * 2 + (q & 1);
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = cmulc(yr[4 * L * m], xr[4 * L * m]);
    fft_quad_dit<L, true>(v, q, tw);                       // v[k] = row r, n2 = 16 bq + k
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[r * (L + 1) + 16 * bq + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = buf[(4 * m + q) * (L + 1) + r];   // column r, rows 4m + q
    fft_quad_dit<L, true>(v, q, tw);                       // v[k] = S[16 bq + k][r]
    const float sc = p.inv_s2 / (float)(L * L);
    const float* bet = p.betaT + (int64_t)c * (L * L) + r * L + 16 * bq;   // betaT[c][t2 = r][t1]
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = v[k].x * sc + bet[k];
}

// the same scores with the transpose by halves through the float buffers bre, bim
__device__ __forceinline__ void score_h(const StepArgs& p, const float2* __restrict__ yhat,
                                        const float2* __restrict__ xhat, int64_t o, int c, float* bre,
                                        float* bim, int r, int q, int bq, const float2* tw, float (&s)[NV]) {
    float2 v[NV];
    const float2* yr = yhat + (((int64_t)o * (L / 2) + (q >> 1)) * L + r) * 2 + (q & 1);
    const float2* xr = xhat + (((int64_t)c * (L / 2) + (q >> 1)) * L + r) * 2 + (q & 1);
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = cmulc(yr[4 * L * m], xr[4 * L * m]);
    fft_quad_dit<L, true>(v, q, tw);                       // v[k] = row r, n2 = 16 bq + k
    // a thread writes a buffer only after the barrier that follows every
    // thread's reads of it in the previous score
#pragma unroll
    for (int k = 0; k < NV; ++k) bre[r * (L + 1) + 16 * bq + k] = v[k].x;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m].x = bre[(4 * m + q) * (L + 1) + r];
#pragma unroll
    for (int k = 0; k < NV; ++k) bim[r * (L + 1) + 16 * bq + k] = v[k].y;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m].y = bim[(4 * m + q) * (L + 1) + r];   // column r, rows 4m + q
    fft_quad_dit<L, true>(v, q, tw);                       // v[k] = S[16 bq + k][r]
    const float sc = p.inv_s2 / (float)(L * L);
    const float* bet = p.betaT + (int64_t)c * (L * L) + r * L + 16 * bq;   // betaT[c][t2 = r][t1]
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = v[k].x * sc + bet[k];
}
}  // namespace quad

// pass 1 at L_low 64: block (chunk, y) takes the chunk's observations y,
// y + gridDim.y, ... (the same for all its threads)
__device__ __forceinline__ void pass1_quad_body(const StepArgs& p, const float2* __restrict__ yhat,
                                                const float2* __restrict__ xhat, int64_t chunk, int ysplit,
                                                int nsplit, float2* sh) {
    using namespace quad;
    float* bre = reinterpret_cast<float*>(sh);
    float* bim = bre + BUF;
    float2* tw = reinterpret_cast<float2*>(bim + BUF);
    float2* red = tw + L / 2;
    make_twiddles<L>(tw);
    __syncthreads();
    const int lt = threadIdx.x, r = lt >> 2, q = lt & 3, bq = quad_block(q);
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    for (int64_t o = c0 + ysplit; o < c1; o += nsplit) {
        float m = -INFINITY, sm = 0.f;
        for (int c = 0; c < p.KK; ++c) {
            float s[NV];
            score_h(p, yhat, xhat, o, c, bre, bim, r, q, bq, tw, s);
            float mc = -INFINITY;
#pragma unroll
            for (int k = 0; k < NV; ++k) mc = fmaxf(mc, s[k]);
            float sc = 0.f;
            if (mc > -INFINITY) {
#pragma unroll
                for (int k = 0; k < NV; ++k) sc += s[k] > -INFINITY ? __expf(s[k] - mc) : 0.f;
            }
            lse_merge(m, sm, mc, sc);
        }
        // the lanes of each wave by shuffles, then the four waves through LDS
        for (int off = 32; off > 0; off >>= 1) {
            const float m2 = __shfl_xor(m, off), s2 = __shfl_xor(sm, off);
            lse_merge(m, sm, m2, s2);
        }
        if ((lt & 63) == 0) red[lt >> 6] = make_float2(m, sm);
        __syncthreads();
        if (lt == 0) {
            for (int w = 1; w < 4; ++w) lse_merge(m, sm, red[w].x, red[w].y);
            p.part[o] = make_float2(m, sm);
        }
    }
}

// pass 2 at L_low 64: block (chunk, c), one component; partials written directly
__device__ __forceinline__ void pass2_quad_body(const StepArgs& p, const float2* __restrict__ yhat,
                                                const float2* __restrict__ xhat, float2* __restrict__ bpart,
                                                float* __restrict__ cpart, int64_t chunk, int ysplit,
                                                float2* sh) {
    using namespace quad;
    float2* tw = sh + 2 * BUF;
    float2* shw = sh + BUF;   // the weights' transpose buffer (the scores' is sh)
    make_twiddles<L>(tw);
    __syncthreads();
    const int lt = threadIdx.x, r = lt >> 2, q = lt & 3, bq = quad_block(q);
    const int c = ysplit;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    float2 ab[NV];   // sum of Y conj(W) at (k1 = r, k2 = 16 bq + k)
    float acw[NV];   // posterior mass at (t1 = 16 bq + k, t2 = r)
#pragma unroll
    for (int k = 0; k < NV; ++k) { ab[k] = make_float2(0.f, 0.f); acw[k] = 0.f; }
    for (int64_t o = c0; o < c1; ++o) {
        float s[NV];
        score(p, yhat, xhat, o, c, sh, r, q, bq, tw, s);
        const float2 lse = p.lse[o];
        float2 v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const float w = s[k] > -INFINITY ? __expf((s[k] - lse.x) - lse.y) : 0.f;
            acw[k] += w;
            v[k] = make_float2(w, 0.f);
        }
        // column t2 = r (its block 16 bq..), transformed along t1, then the rows
        fft_quad_dif<L, false>(v, q, tw);                  // v[k] = k1 = 4k + q, column r
#pragma unroll
        for (int k = 0; k < NV; ++k) shw[(4 * k + q) * (L + 1) + r] = v[k];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = shw[r * (L + 1) + 4 * m + q];   // row k1 = r, n2 = 4m + q
        fft_quad_dit<L, false>(v, q, tw);                  // v[k] = W[r][16 bq + k]
        // Y_o[r][16 bq + k], k and k + 1 in one 16-byte word of the paired layout
        const float4* yr = reinterpret_cast<const float4*>(yhat) + ((int64_t)o * (L / 2) + 8 * bq) * L + r;
#pragma unroll
        for (int k = 0; k < NV; k += 2) {
            const float4 a = yr[(k / 2) * L];
            const float2 t0 = cmulc(make_float2(a.x, a.y), v[k]);
            const float2 t1 = cmulc(make_float2(a.z, a.w), v[k + 1]);
            ab[k].x += t0.x; ab[k].y += t0.y;
            ab[k + 1].x += t1.x; ab[k + 1].y += t1.y;
        }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        bpart[((chunk * p.KK + c) * L + r) * L + 16 * bq + k] = ab[k];      // [k1][k2]
        cpart[((chunk * p.KK + c) * L + 16 * bq + k) * L + r] = acw[k];     // [t1][t2]
    }
}

// ---- L_low = 3 * 2^m (12, 24, 48): teams of L lanes, one row (then column) of
// an image per lane (256 / L teams over the block, see row_wide).  The layouts
// of Y and X, the partials and the meaning of every sum are those of the
// power-of-two passes.
namespace row {
template <int L> struct G {
    static constexpr bool WIDE = row_wide(L);
    static constexpr int TEAMS = WIDE ? 256 / L : 4 * (64 / L);   // teams per 256-thread block
    static constexpr int BUF = L * (L + 1);     // float2 per team transpose buffer
    // Pass 1 at L >= 24 transposes by halves (the real parts, then the
    // imaginary parts, through L (L + 1) floats per team: two barriers more per
    // transpose, half the LDS, so that more blocks share a CU: at L 48 two
    // instead of one, at L 24 four instead of three).
    static constexpr bool H1 = L >= 24;
    static constexpr int PB1 = H1 ? (L * (L + 1) + 1) / 2 : BUF;   // float2 per team buffer, pass 1
};
// a team's exchange through its transpose buffer
template <int L> __device__ __forceinline__ void sync() {
    if constexpr (G<L>::WIDE) __syncthreads();
    else team_sync();
}
// preparation, DFT and pass 2: [transpose buffers TEAMS x BUF float2][twiddles L float2]
template <int L> constexpr size_t lds() { return sizeof(float2) * ((size_t)G<L>::TEAMS * G<L>::BUF + L); }
// pass 1: [transpose buffers TEAMS x PB1 float2][twiddles L float2]
template <int L> constexpr size_t lds_pass1() { return sizeof(float2) * ((size_t)G<L>::TEAMS * G<L>::PB1 + L); }

// the team's L x L complex image, one row or column v per lane, written at
// wi(k) and read back at ri(m) of the team's buffer (every lane of the block
// reaches the barriers; lanes with !on touch nothing)
template <int L, bool H, typename WI, typename RI>
__device__ __forceinline__ void exchange(float2 (&v)[L], float2* buf, WI wi, RI ri, bool on) {
    if constexpr (H) {
        float* b = reinterpret_cast<float*>(buf);
        if (on) {
#pragma unroll
            for (int k = 0; k < L; ++k) b[wi(k)] = v[k].x;
        }
        sync<L>();
        if (on) {
#pragma unroll
            for (int m = 0; m < L; ++m) v[m].x = b[ri(m)];
        }
        sync<L>();
        if (on) {
#pragma unroll
            for (int k = 0; k < L; ++k) b[wi(k)] = v[k].y;
        }
        sync<L>();
        if (on) {
#pragma unroll
            for (int m = 0; m < L; ++m) v[m].y = b[ri(m)];
        }
        sync<L>();
    } else {
        if (on) {
#pragma unroll
            for (int k = 0; k < L; ++k) buf[wi(k)] = v[k];
        }
        sync<L>();
        if (on) {
#pragma unroll
            for (int m = 0; m < L; ++m) v[m] = buf[ri(m)];
        }
        sync<L>();
    }
}

// lane -> (team, row r); on: the lane belongs to a team (lanes that do not
// touch no team buffer but reach every barrier)
template <int L> __device__ __forceinline__ void team_of(int& team, int& r, bool& on) {
    if constexpr (G<L>::WIDE) {
        const int t = threadIdx.x;
        on = t < G<L>::TEAMS * L;
        team = on ? t / L : 0;
        r = t % L;
    } else {
        constexpr int TPW = 64 / L;
        const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
        on = ln < TPW * L;
        team = wave * TPW + (on ? ln / L : 0);
        r = ln % L;
    }
}

// scores of (observation o, component c) for lane r: s[k] = a at (t1 = k, t2 = r).
// Row r of Y_o conj(X_c) is inverse-transformed along k2, the team exchanges
// rows for columns, and column r is inverse-transformed along k1.
// Lanes with !on only reach the barriers (s = -inf).  H: transpose by halves.
template <int L, bool H>
__device__ __forceinline__ void score(const StepArgs& p, const float2* __restrict__ yhat,
                                      const float2* __restrict__ xhat, int64_t o, int c, float2* buf, int r,
                                      const float2* tw, float (&s)[L], bool on = true) {
    float2 v[L];
    if (on) {
        const float4* yr = reinterpret_cast<const float4*>(yhat) + (int64_t)o * (L / 2) * L + r;
        const float4* xr = reinterpret_cast<const float4*>(xhat) + (int64_t)c * (L / 2) * L + r;
#pragma unroll
        for (int m = 0; m < L / 2; ++m) {
            const float4 a = yr[m * L], b = xr[m * L];
            v[2 * m] = cmulc(make_float2(a.x, a.y), make_float2(b.x, b.y));
            v[2 * m + 1] = cmulc(make_float2(a.z, a.w), make_float2(b.z, b.w));
        }
        fft1m<L, true>(v, tw);                                  // v[n2]: row k1 = r
    }
    // row r out, column n2 = r in
    exchange<L, H>(v, buf, [&](int k) { return r * (L + 1) + k; }, [&](int m) { return m * (L + 1) + r; }, on);
    if (on) {
        fft1m<L, true>(v, tw);                                  // v[k] = S[k][r]
        const float sc = p.inv_s2 / (float)(L * L);
        const float* bet = p.betaT + (int64_t)c * (L * L) + r * L;   // betaT[c][t2 = r][t1]
#pragma unroll
        for (int k = 0; k < L; ++k) s[k] = v[k].x * sc + bet[k];
    } else {
#pragma unroll
        for (int k = 0; k < L; ++k) s[k] = -INFINITY;
    }
}

// pass 1: (max, sum exp) of every observation over all components; a team per
// observation, the chunk's observations split over the gridDim.y blocks of the chunk
template <int L>
__device__ __forceinline__ void pass1_body(const StepArgs& p, const float2* __restrict__ yhat,
                                           const float2* __restrict__ xhat, int64_t chunk, int ysplit,
                                           int nsplit, float2* sh) {
    float2* tw = sh + G<L>::TEAMS * G<L>::PB1;
    make_twiddles_n<L, L>(tw);
    __syncthreads();
    int team, r;
    bool on;
    team_of<L>(team, r, on);
    float2* buf = sh + team * G<L>::PB1;
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    // the same trip count in every lane of the block (the teams' barriers)
    for (int64_t base = c0 + (int64_t)G<L>::TEAMS * ysplit; base < c1; base += (int64_t)G<L>::TEAMS * nsplit) {
        const int64_t o = base + team;
        const bool act = on && o < c1;
        const int64_t oc = act ? o : c0;   // an observation to read for lanes past the chunk
        float m = -INFINITY, sm = 0.f;
        for (int c = 0; c < p.KK; ++c) {
            float s[L];
            score<L, G<L>::H1>(p, yhat, xhat, oc, c, buf, r, tw, s, on);
            float mc = -INFINITY;
#pragma unroll
            for (int k = 0; k < L; ++k) mc = fmaxf(mc, s[k]);
            float sc = 0.f;
            if (mc > -INFINITY) {
#pragma unroll
                for (int k = 0; k < L; ++k) sc += s[k] > -INFINITY ? __expf(s[k] - mc) : 0.f;
            }
            lse_merge(m, sm, mc, sc);
        }
        // the team's L lanes merged in lane order by its first lane
        if (on) buf[r] = make_float2(m, sm);
        sync<L>();
        if (act && r == 0) {
            for (int k = 1; k < L; ++k) lse_merge(m, sm, buf[k].x, buf[k].y);
            p.part[o] = make_float2(m, sm);
        }
        sync<L>();
    }
}

// pass 2: per component group, the sums over the chunk (TPC teams per
// component, observations split over them): partials of sum_i Y_i conj(W_i)
// [chunk][c][k1][k2] (complex) and of sum_i w_i [chunk][c][t1][t2]
template <int L>
__device__ __forceinline__ void pass2_body(const StepArgs& p, const float2* __restrict__ yhat,
                                           const float2* __restrict__ xhat, int TPC, float2* __restrict__ bpart,
                                           float* __restrict__ cpart, int64_t chunk, int ysplit, float2* sh) {
    float2* tw = sh + G<L>::TEAMS * G<L>::BUF;
    make_twiddles_n<L, L>(tw);
    int team, r;
    bool on;
    team_of<L>(team, r, on);
    float2* buf = sh + team * G<L>::BUF;
    const int CG = G<L>::TEAMS / TPC;
    const int c = ysplit * CG + team / TPC, u = team % TPC;
    const bool active = on && team < CG * TPC && c < p.KK;
    __syncthreads();
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    float2 ab[L];   // sum of Y conj(W) at (k1 = r, k2 = k)
    float acw[L];   // posterior mass at (t1 = k, t2 = r)
#pragma unroll
    for (int k = 0; k < L; ++k) {
        ab[k] = make_float2(0.f, 0.f);
        acw[k] = 0.f;
    }
    // the same trip count in every lane of the block (the teams' barriers);
    // inactive teams and observations past the chunk add nothing
    const int cc = active ? c : 0;
    for (int64_t base = c0; base < c1; base += TPC) {
        const int64_t o = base + u;
        const bool act = active && o < c1;
        const int64_t oc = act ? o : c0;
        float s[L];
        score<L, false>(p, yhat, xhat, oc, cc, buf, r, tw, s, on);
        const float2 lse = act ? p.lse[oc] : make_float2(0.f, 0.f);
        float2 v[L];
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const float w = (act && s[k] > -INFINITY) ? __expf((s[k] - lse.x) - lse.y) : 0.f;
            acw[k] += w;
            v[k] = make_float2(w, 0.f);
        }
        if (on) fft1m<L, false>(v, tw);                         // column t2 = r along t1: v[k1]
        // column t2 = r out, row k1 = r in
        exchange<L, false>(v, buf, [&](int k) { return k * (L + 1) + r; }, [&](int m) { return r * (L + 1) + m; }, on);
        if (act) {
            fft1m<L, false>(v, tw);                             // v[k] = W[r][k]
            const float4* yr = reinterpret_cast<const float4*>(yhat) + o * (L / 2) * L + r;
#pragma unroll
            for (int k = 0; k < L; k += 2) {
                const float4 a = yr[(k / 2) * L];
                const float2 t0 = cmulc(make_float2(a.x, a.y), v[k]);
                const float2 t1 = cmulc(make_float2(a.z, a.w), v[k + 1]);
                ab[k].x += t0.x; ab[k].y += t0.y;
                ab[k + 1].x += t1.x; ab[k + 1].y += t1.y;
            }
        }
    }
    // the TPC teams of each component summed in a fixed order: each team's
    // back-projection transform goes into its buffer ([k1][k2] at pitch L + 1),
    // then its masses ([t1][t2]), and the component's first team adds the
    // others' to its own, team by team
    const bool lead = active && u == 0;
    __syncthreads();
    if (on) {
#pragma unroll
        for (int k = 0; k < L; ++k) buf[r * (L + 1) + k] = ab[k];
    }
    __syncthreads();
    if (lead) {
        for (int j = 1; j < TPC; ++j) {
            const float2* o = sh + (team + j) * G<L>::BUF;
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const float2 e = o[r * (L + 1) + k];
                ab[k].x += e.x;
                ab[k].y += e.y;
            }
        }
    }
    __syncthreads();
    if (on) {
        float* bf = reinterpret_cast<float*>(buf);
#pragma unroll
        for (int k = 0; k < L; ++k) bf[k * L + r] = acw[k];
    }
    __syncthreads();
    if (lead) {
        for (int j = 1; j < TPC; ++j) {
            const float* o = reinterpret_cast<const float*>(sh + (team + j) * G<L>::BUF);
#pragma unroll
            for (int k = 0; k < L; ++k) acw[k] += o[k * L + r];
        }
#pragma unroll
        for (int k = 0; k < L; ++k) {
            bpart[((chunk * p.KK + c) * L + r) * L + k] = ab[k];      // [k1 = r][k2 = k]
            cpart[((chunk * p.KK + c) * L + k) * L + r] = acw[k];     // [t1 = k][t2 = r]
        }
    }
}

}  // namespace row

// ---- pass 2 at L_low 48 with lane-pair teams: lane pair (r, h) holds half of
// row (then column) r, as in the power-of-two pair teams, so a lane keeps 24
// complex values, 24 complex sums of Y conj(W) and 24 posterior masses instead
// of the row teams' 48 of each, and more waves fit a SIMD.  A team of 2 L = 96
// lanes spans waves (its transposes wait on the block barrier, every lane runs
// the same loop trips); two teams per 256-thread block, the last wave idles.
// Partials and sums as in the pair teams' pass 2.
namespace wpair {
template <int L> struct G {
    static constexpr int TEAMS = 256 / (2 * L);
    static constexpr int BUF = L * (L + 1);   // float2 per team transpose buffer
};
// [transpose buffers TEAMS x BUF float2][twiddles L float2][pair table L float2]
// [X_c of each team's component, TEAMS x L x L float2, the paired layout]
template <int L> constexpr size_t lds() {
    return sizeof(float2) * ((size_t)G<L>::TEAMS * G<L>::BUF + 2 * L + (size_t)G<L>::TEAMS * L * L);
}

template <int L>
__device__ __forceinline__ void pass2_body(const StepArgs& p, const float2* __restrict__ yhat,
                                           const float2* __restrict__ xhat, int TPC, float2* __restrict__ bpart,
                                           float* __restrict__ cpart, int64_t chunk, int ysplit, float2* sh) {
    float2* tw = sh + G<L>::TEAMS * G<L>::BUF;
    float2* twp = tw + L;
    make_twiddles_n<L, L>(tw);
    make_pair_twiddles<L>(twp);
    const int t = threadIdx.x;
    const bool on = t < G<L>::TEAMS * 2 * L;   // lanes of a team (pairs never straddle it)
    const int team = on ? t / (2 * L) : 0, lt = t % (2 * L);
    const int r = lt >> 1, h = lt & 1;
    const float2* twh = twp + (L / 2) * h;
    float2* buf = sh + team * G<L>::BUF;
    float2* xs = twp + L + team * (L * L);   // the team's X_c
    const int CG = G<L>::TEAMS / TPC;
    const int c = ysplit * CG + team / TPC, u = team % TPC;
    const bool active = on && team < CG * TPC && c < p.KK;
    const int cc = active ? c : 0;
    if (on) {
        const float4* src = reinterpret_cast<const float4*>(xhat + (int64_t)cc * L * L);
        float4* dst = reinterpret_cast<float4*>(xs);
        for (int e = lt; e < L * L / 2; e += 2 * L) dst[e] = src[e];
    }
    __syncthreads();
    const int64_t c0 = chunk * p.chunk_obs;
    const int64_t c1 = min<int64_t>(p.N, c0 + p.chunk_obs);
    float2 ab[L / 2];   // sum of Y conj(W) at (k1 = r, k2 = (L/2) h + k)
    float acw[L / 2];   // posterior mass at (t1 = (L/2) h + k, t2 = r)
#pragma unroll
    for (int k = 0; k < L / 2; ++k) {
        ab[k] = make_float2(0.f, 0.f);
        acw[k] = 0.f;
    }
    // the same trip count in every lane of the block (the teams' barriers);
    // inactive teams and observations past the chunk add nothing
    for (int64_t base = c0; base < c1; base += TPC) {
        const int64_t o = base + u;
        const bool act = active && o < c1;
        const int64_t oc = act ? o : c0;
        float2 v[L / 2];
        if (on) {
            // row r of Y_o conj(X_c) as its samples 2m + h, inverse-transformed
            const float2* yr = yhat + (oc * (L / 2) * L + r) * 2 + h;   // Y_o[r][2m + h] at yr[2 L m]
            const float2* xr = xs + r * 2 + h;
#pragma unroll
            for (int m = 0; m < L / 2; ++m) v[m] = cmulc(yr[2 * L * m], xr[2 * L * m]);
            fft_pair_dit<L, true>(v, h, tw, twh);                     // v[k] = row r, n2 = (L/2) h + k
#pragma unroll
            for (int k = 0; k < L / 2; ++k) buf[r * (L + 1) + (L / 2) * h + k] = v[k];
        }
        __syncthreads();
        if (on) {
#pragma unroll
            for (int m = 0; m < L / 2; ++m) v[m] = buf[(2 * m + h) * (L + 1) + r];   // column r, rows 2m + h
        }
        __syncthreads();
        if (on) {
            fft_pair_dit<L, true>(v, h, tw, twh);                     // v[k] = S[(L/2) h + k][r]
            const float sc = p.inv_s2 / (float)(L * L);
            const float* bet = p.betaT + (int64_t)cc * (L * L) + r * L + (L / 2) * h;   // betaT[c][t2 = r][t1]
            const float2 lse = act ? p.lse[oc] : make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < L / 2; ++k) {
                const float a = v[k].x * sc + bet[k];
                const float w = (act && a > -INFINITY) ? __expf((a - lse.x) - lse.y) : 0.f;
                acw[k] += w;
                v[k] = make_float2(w, 0.f);
            }
            // column t2 = r (its half (L/2) h..), transformed along t1, then the rows
            fft_pair_dif<L, false>(v, h, tw, twh);                    // v[k] = k1 = 2k + h, column r
#pragma unroll
            for (int k = 0; k < L / 2; ++k) buf[(2 * k + h) * (L + 1) + r] = v[k];
        }
        __syncthreads();
        if (on) {
#pragma unroll
            for (int m = 0; m < L / 2; ++m) v[m] = buf[r * (L + 1) + 2 * m + h];   // row k1 = r, n2 = 2m + h
        }
        __syncthreads();
        if (act) {
            fft_pair_dit<L, false>(v, h, tw, twh);                    // v[k] = W[r][(L/2) h + k]
            // Y_o[r][(L/2) h + k], k and k + 1 in one 16-byte word of the paired layout
            const float4* yr = reinterpret_cast<const float4*>(yhat) + (o * (L / 2) + (L / 4) * h) * L + r;
#pragma unroll
            for (int k = 0; k < L / 2; k += 2) {
                const float4 a = yr[(k / 2) * L];
                const float2 t0 = cmulc(make_float2(a.x, a.y), v[k]);
                const float2 t1 = cmulc(make_float2(a.z, a.w), v[k + 1]);
                ab[k].x += t0.x; ab[k].y += t0.y;
                ab[k + 1].x += t1.x; ab[k + 1].y += t1.y;
            }
        }
    }
    // sum the TPC teams of each component in a fixed order, one plane at a time
    // (each lane keeps its own L/2 slots of the team buffer)
    for (int plane = 0; plane < 2; ++plane) {
        __syncthreads();
        if (on) {
#pragma unroll
            for (int k = 0; k < L / 2; ++k)
                buf[lt * (L / 2) + k] = plane == 0 ? ab[k] : make_float2(acw[k], 0.f);
        }
        __syncthreads();
        if (active && u == 0) {
            for (int k = 0; k < L / 2; ++k) {
                float2 e = buf[lt * (L / 2) + k];
                for (int j = 1; j < TPC; ++j) {
                    const float2 f = sh[(team + j) * G<L>::BUF + lt * (L / 2) + k];
                    e.x += f.x; e.y += f.y;
                }
                if (plane == 0) bpart[((chunk * p.KK + c) * L + r) * L + (L / 2) * h + k] = e;   // [k1][k2]
                else cpart[((chunk * p.KK + c) * L + (L / 2) * h + k) * L + r] = e.x;            // [t1][t2]
            }
        }
    }
}
}  // namespace wpair

// ---- FP64 sums of the partials over chunks: the back-projection's transform
// [KK][L][L] complex, the posterior mass [KK][t1][t2] real (final)
// (block blk of the elements; red: 3 x 256 doubles of LDS)
__device__ __forceinline__ void reduce_body(const float2* __restrict__ bpart, const float* __restrict__ cpart,
                                            int n_chunks, int per, double2* __restrict__ bh,
                                            double* __restrict__ csum, int blk, double* red) {
    // the chunk slices of reduce_partials_body, for complex b
    const int le = threadIdx.x % kReduceElems, sl = threadIdx.x / kReduceElems;
    const int e = blk * kReduceElems + le;
    double2 sb = make_double2(0.0, 0.0);
    double sc = 0.0;
    if (e < per) {
        for (int k = sl; k < n_chunks; k += kReduceSlices) {
            const float2 b = bpart[(int64_t)k * per + e];
            sb.x += b.x; sb.y += b.y;
            sc += cpart[(int64_t)k * per + e];
        }
    }
    red[threadIdx.x] = sb.x;
    red[256 + threadIdx.x] = sb.y;
    red[512 + threadIdx.x] = sc;
    __syncthreads();
    if (sl == 0 && e < per) {
        double2 tb = make_double2(0.0, 0.0);
        double tc = 0.0;
        for (int s = 0; s < kReduceSlices; ++s) {
            tb.x += red[s * kReduceElems + le];
            tb.y += red[256 + s * kReduceElems + le];
            tc += red[512 + s * kReduceElems + le];
        }
        bh[e] = tb;
        csum[e] = tc;
    }
}

// ---- FP64 inverse DFT of the back-projection, one workgroup per component,
// separable: T[k1][q2] = sum_k2 B[k1][k2] w^(k2 q2) into LDS, then
// bsum[c][q1 L + q2] = Re sum_k1 T[k1][q2] w^(k1 q1) / L^2 (w = exp(2 pi i / L);
// the layout the finalize kernel reads).  Dynamic LDS: idft_lds<L>() bytes.
template <int L> constexpr size_t idft_lds() { return sizeof(double2) * L * L + 2 * sizeof(double) * L; }
template <int L>
__device__ __forceinline__ void idft_body(const double2* __restrict__ bh, double* __restrict__ bsum, int c,
                                          double2* T) {
    // T: [L][L] then the cosines and sines of 2 pi j / L
    double* cs = reinterpret_cast<double*>(T + L * L);   // [L]
    double* sn = cs + L;                                 // [L]
    if (threadIdx.x < L) sincospi(2.0 * (double)threadIdx.x / (double)L, &sn[threadIdx.x], &cs[threadIdx.x]);
    __syncthreads();
    const double2* B = bh + (int64_t)c * L * L;
    for (int e = threadIdx.x; e < L * L; e += 256) {
        const int k1 = e / L, q2 = e % L;
        double re = 0.0, im = 0.0;
        for (int k2 = 0; k2 < L; ++k2) {
            const int m = (k2 * q2) % L;
            const double2 b = B[k1 * L + k2];
            re += b.x * cs[m] - b.y * sn[m];
            im += b.x * sn[m] + b.y * cs[m];
        }
        T[e] = make_double2(re, im);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < L * L; e += 256) {
        const int q1 = e / L, q2 = e % L;
        double re = 0.0;
        for (int k1 = 0; k1 < L; ++k1) {
            const int m = (k1 * q1) % L;
            const double2 t = T[k1 * L + q2];
            re += t.x * cs[m] - t.y * sn[m];
        }
        bsum[(int64_t)c * L * L + e] = re * (1.0 / (double)(L * L));
    }
}

}  // namespace fft
}  // namespace srmra
