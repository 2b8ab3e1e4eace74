// Per-job and per-step helper kernels of the EM step: observation norms,
// packing of x into polyphase components with the log-prior bias, the
// cross-group log-sum-exp combine, and the FP64 M-step finalisation.
#pragma once
#include "srmra_common.h"

namespace srmra {

// ---------------------------------------------------------------- a0: ||y_i||^2
// One wave per observation; FP64 accumulation (the term -||y_i||^2/(2 sigma^2) of
// eq. likelihood_EM).
// Per-observation FP64 sums of y (for the offset mu): one wave per observation.
__device__ __forceinline__ void obs_sums_body(const float* __restrict__ y, int64_t N, int npix,
                                              double* __restrict__ ysum, int64_t blk) {
    const int lane = threadIdx.x & 63;
    const int64_t i = blk * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const float4* yi = reinterpret_cast<const float4*>(y + i * (int64_t)npix);
    double acc = 0.0;
#pragma unroll 4
    for (int p = lane; p < npix / 4; p += 64) {
        const float4 v = yi[p];
        acc += (double)v.x;
        acc += (double)v.y;
        acc += (double)v.z;
        acc += (double)v.w;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) ysum[i] = acc;
}

// mu = mean of all observation pixels (fixed-order FP64 reduction, one block of
// 1024 threads), rounded to FP32 (the value the kernels subtract); 0 when
// centring is off.  The model is invariant under y -> y - mu, x -> x - mu
// (x' shifts by mu; rho', w and the log-likelihood are unchanged).
__device__ __forceinline__ void centre_body(const double* __restrict__ ysum, int64_t N, int npix,
                                            int enable, double* __restrict__ centre, double* red) {
    double s = 0.0;
    if (enable)
        for (int64_t i = threadIdx.x; i < N; i += 1024) s += ysum[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *centre = enable ? (double)(float)(red[0] / ((double)N * npix)) : 0.0;
}

// ||y_i - mu||^2 in FP64 of the FP32 differences the kernels see: one wave per
// observation; lane l adds pixels 4(l + 64k) .. 4(l + 64k) + 3 in that order,
// then a fixed butterfly (the BF16 preparation kernel uses the same order, so
// every form sees the same norms).
__device__ __forceinline__ void obs_norms_body(const float* __restrict__ y, int64_t N, int npix,
                                               const double* __restrict__ centre,
                                               double* __restrict__ ynorm, int64_t blk) {
    const int lane = threadIdx.x & 63;
    const int64_t i = blk * 4 + (threadIdx.x >> 6);
    if (i >= N) return;
    const float mu = centre_of(centre);
    const float4* yi = reinterpret_cast<const float4*>(y + i * (int64_t)npix);
    double acc = 0.0;
#pragma unroll 4
    for (int p = lane; p < npix / 4; p += 64) {
        const float4 v = yi[p];
        const float d0 = v.x - mu, d1 = v.y - mu, d2 = v.z - mu, d3 = v.w - mu;
        acc += (double)d0 * d0;
        acc += (double)d1 * d1;
        acc += (double)d2 * d2;
        acc += (double)d3 * d3;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) ynorm[i] = acc;
}

// ---------------------------------------------------------------- a1: pack x
// One block per component c (x less the offset mu).  xt2[c][b2][a] =
// x_c[a mod Ll][b2] for a in [0, 2Ll); betaT[c][t2][t1] = log rho1[s1] +
// log rho2[s2] - ||x_c||^2 / (2 sigma^2), s = (t*K - c) mod Lh (eq. weights_EM
// with rho[s] = rho1[s1] rho2[s2]).
__device__ __forceinline__ void pack_x_body(const float* __restrict__ x,
                                            const float* __restrict__ log_rho, int K, int Ll,
                                            double inv_2s2, const double* __restrict__ centre,
                                            float* __restrict__ xt2,
                                            float* __restrict__ betaT, int c, double* red) {
    const int c1 = c / K, c2 = c % K;
    const int Lh = K * Ll;
    const float mu = centre_of(centre);
    double acc = 0.0;
    for (int e = threadIdx.x; e < Ll * Ll; e += 256) {
        const int l1 = e / Ll, l2 = e % Ll;
        const float v = x[(int64_t)(c1 + l1 * K) * Lh + (c2 + l2 * K)] - mu;
        acc += (double)v * (double)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double nx = red[0];
    float* xo = xt2 + (int64_t)c * Ll * 2 * Ll;
    for (int e = threadIdx.x; e < Ll * 2 * Ll; e += 256) {
        const int b2 = e / (2 * Ll), a = e % (2 * Ll);
        const int l1 = a % Ll;
        xo[e] = x[(int64_t)(c1 + l1 * K) * Lh + (c2 + b2 * K)] - mu;
    }
    float* bo = betaT + (int64_t)c * Ll * Ll;
    const float* lr1 = log_rho;
    const float* lr2 = log_rho + Lh;
    for (int e = threadIdx.x; e < Ll * Ll; e += 256) {
        const int t2 = e / Ll, t1 = e % Ll;
        const int s1 = ((t1 * K - c1) % Lh + Lh) % Lh;
        const int s2 = ((t2 * K - c2) % Lh + Lh) % Lh;
        bo[e] = (float)((double)lr1[s1] + (double)lr2[s2] - nx * inv_2s2);
    }
}

// ---------------------------------------------------------------- LSE combine
// lse[i] = log sum over component groups of sum * exp(max); also the FP64
// per-block sums of l_i = lse_i - ||y_i||^2/(2 sigma^2) (eq. likelihood_EM) and,
// optionally, l_i itself.
__device__ __forceinline__ void lse_combine_body(const float2* __restrict__ part, int n_cg,
                                                 int64_t N, const double* __restrict__ ynorm,
                                                 double inv_2s2, float2* __restrict__ lse,
                                                 double* __restrict__ llpart,
                                                 float* __restrict__ ll_obs, int64_t blk,
                                                 double* red) {
    const int64_t i = blk * 256 + threadIdx.x;
    double li = 0.0;
    if (i < N) {
        float m = -INFINITY;
        for (int g = 0; g < n_cg; ++g) m = fmaxf(m, part[(int64_t)g * N + i].x);
        double s = 0.0;
        if (m > -INFINITY) {
            for (int g = 0; g < n_cg; ++g) {
                const float2 p = part[(int64_t)g * N + i];
                if (p.x > -INFINITY) s += (double)p.y * exp((double)p.x - (double)m);
            }
        }
        const double L = (double)m + log(s);
        lse[i] = make_float2(m, (float)log(s));
        li = L - ynorm[i] * inv_2s2;
        if (ll_obs) ll_obs[i] = (float)li;
    }
    red[threadIdx.x] = li;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) llpart[blk] = red[0];
}

// ---------------------------------------------------------------- a5: finalize
// Stage 1: FP64 sums of the per-chunk partials, one thread per (component, index).
// FP64 reduction of per-chunk partials: elements per workgroup (its 256
// threads form 256 / kReduceElems slices, each summing every slice-th chunk)
constexpr int kReduceElems = 32;
constexpr int kReduceSlices = 256 / kReduceElems;

// Workgroup blk takes elements [kReduceElems blk, +kReduceElems); slice s of
// its threads sums the chunks s, s + kReduceSlices, ... in order, and the slice
// sums are added in slice order: a fixed order, independent of scheduling.
// red: 2 x 256 doubles of LDS.
__device__ __forceinline__ void reduce_partials_body(const float* __restrict__ bpart,
                                                     const float* __restrict__ cpart,
                                                     int n_chunks, int per_chunk,
                                                     double* __restrict__ bsum,
                                                     double* __restrict__ csum, int blk,
                                                     double* red) {
    const int le = threadIdx.x % kReduceElems, sl = threadIdx.x / kReduceElems;
    const int e = blk * kReduceElems + le;
    double sb = 0.0, sc = 0.0;
    if (e < per_chunk) {
        for (int k = sl; k < n_chunks; k += kReduceSlices) {
            sb += (double)bpart[(int64_t)k * per_chunk + e];
            sc += (double)cpart[(int64_t)k * per_chunk + e];
        }
    }
    red[threadIdx.x] = sb;
    red[256 + threadIdx.x] = sc;
    __syncthreads();
    if (sl == 0 && e < per_chunk) {
        double tb = 0.0, tc = 0.0;
        for (int s = 0; s < kReduceSlices; ++s) {
            tb += red[s * kReduceElems + le];
            tc += red[256 + s * kReduceElems + le];
        }
        bsum[e] = tb;
        csum[e] = tc;
    }
}

// Stage 2 (one block): A_c = sum_t c_(c,t); x_new[c1 + q1 K][c2 + q2 K] = b_c[q]/A_c + mu
// (eq. x_EM with P^{-1} = P^T: A is diagonal and constant on each component; b
// is the back-projection of y - mu); rho marginals (eq. rho_EM, product form);
// loglik = sum of block partials.  b_out (optional) is the back-projection of y
// itself, b + mu A_c.
// Ac: 256 doubles, red: blockDim doubles (blockDim = 1024)
__device__ __forceinline__ void finalize_body(const double* __restrict__ bsum,
                                              const double* __restrict__ csum, int K, int Ll,
                                              const float* __restrict__ x,
                                              const double* __restrict__ centre,
                                              const double* __restrict__ llpart, int n_ll,
                                              float* __restrict__ x_new,
                                              float* __restrict__ rho_new,
                                              float* __restrict__ log_rho_new,
                                              double* __restrict__ loglik,
                                              double* __restrict__ b_out,
                                              double* __restrict__ c_out, double* Ac, double* red) {
    const int Lh = K * Ll;
    const int KK = K * K;
    const int tid = threadIdx.x;
    // A_c: one pass per component, fixed-order tree
    for (int c = 0; c < KK; ++c) {
        double s = 0.0;
        for (int e = tid; e < Ll * Ll; e += 1024) s += csum[(int64_t)c * Ll * Ll + e];
        red[tid] = s;
        __syncthreads();
        for (int st = 512; st > 0; st >>= 1) {
            if (tid < st) red[tid] += red[tid + st];
            __syncthreads();
        }
        if (tid == 0) Ac[c] = red[0];
        __syncthreads();
    }
    double tot = 0.0;
    for (int c = 0; c < KK; ++c) tot += Ac[c];
    const double mu = (double)centre_of(centre);
    // x_new
    for (int e = tid; e < Lh * Lh; e += 1024) {
        const int m1 = e / Lh, m2 = e % Lh;
        const int c1 = m1 % K, c2 = m2 % K, q1 = m1 / K, q2 = m2 / K;
        const int c = c1 * K + c2;
        const double b = bsum[(int64_t)c * Ll * Ll + q1 * Ll + q2];
        const double a = Ac[c];
        x_new[e] = a > 0.0 ? (float)(b / a + mu) : x[e];
        if (b_out) b_out[e] = b + mu * a;
    }
    // rho marginals: c_s with s = (t*K - c) mod Lh
    for (int s1 = tid; s1 < Lh; s1 += 1024) {
        const int c1 = (K - s1 % K) % K;
        const int t1 = ((s1 + c1) / K) % Ll;
        double acc = 0.0;
        for (int c2 = 0; c2 < K; ++c2)
            for (int t2 = 0; t2 < Ll; ++t2) acc += csum[(int64_t)(c1 * K + c2) * Ll * Ll + t1 * Ll + t2];
        const double r = tot > 0.0 ? acc / tot : 0.0;
        rho_new[s1] = (float)r;
        if (log_rho_new) log_rho_new[s1] = (float)log(r);
    }
    for (int s2 = tid; s2 < Lh; s2 += 1024) {
        const int c2 = (K - s2 % K) % K;
        const int t2 = ((s2 + c2) / K) % Ll;
        double acc = 0.0;
        for (int c1 = 0; c1 < K; ++c1)
            for (int t1 = 0; t1 < Ll; ++t1) acc += csum[(int64_t)(c1 * K + c2) * Ll * Ll + t1 * Ll + t2];
        const double r = tot > 0.0 ? acc / tot : 0.0;
        rho_new[Lh + s2] = (float)r;
        if (log_rho_new) log_rho_new[Lh + s2] = (float)log(r);
    }
    if (c_out) {
        for (int e = tid; e < Lh * Lh; e += 1024) {
            const int s1 = e / Lh, s2 = e % Lh;
            const int c1 = (K - s1 % K) % K, c2 = (K - s2 % K) % K;
            const int t1 = ((s1 + c1) / K) % Ll, t2 = ((s2 + c2) / K) % Ll;
            c_out[e] = csum[(int64_t)(c1 * K + c2) * Ll * Ll + t1 * Ll + t2];
        }
    }
    // loglik
    double s = 0.0;
    for (int k = tid; k < n_ll; k += 1024) s += llpart[k];
    red[tid] = s;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) loglik[0] = red[0];
}

}  // namespace srmra
