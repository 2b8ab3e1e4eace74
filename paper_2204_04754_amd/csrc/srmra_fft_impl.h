// 2-D discrete Fourier transforms of L x L images (L in {8, 16, 32, 64}, and
// L = 3 * 2^m in {12, 24, 48}) by teams of L threads: a team's thread r holds
// row r (then column r) of the image as L complex values in registers and runs
// an iterative radix-2 decimation-in-time transform on it (for L = 3 M, one
// radix-3 step and three length-M transforms); rows and columns meet through the
// team's LDS buffer (pitch L + 1 complex, conflict-free for both).  A team
// sits inside one wave, so a wave barrier orders its LDS traffic.
// Forward: X[k] = sum_n x[n] exp(-2 pi i k.n / L); inverse: the conjugate
// twiddles, unscaled (callers apply 1 / L^2).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace srmra {
namespace fft {

template <int L> struct Log2;
template <> struct Log2<4> { static constexpr int v = 2; };
template <> struct Log2<8> { static constexpr int v = 3; };
template <> struct Log2<16> { static constexpr int v = 4; };
template <> struct Log2<32> { static constexpr int v = 5; };
template <> struct Log2<64> { static constexpr int v = 6; };

template <int L> __host__ __device__ constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 0; b < Log2<L>::v; ++b) r |= ((i >> b) & 1) << (Log2<L>::v - 1 - b);
    return r;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// twiddles tw[j] = exp(-2 pi i j / L), j < L/2, from double-precision sincospi
template <int L> __device__ __forceinline__ void make_twiddles(float2* tw) {
    for (int j = threadIdx.x; j < L / 2; j += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)j / (double)L, &s, &c);
        tw[j] = make_float2((float)c, (float)s);
    }
}

// in-register transform of v[0..L) (natural order in and out)
template <int L, bool INV>
__device__ __forceinline__ void fft1(float2 (&v)[L], const float2* __restrict__ tw) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int j = bitrev<L>(i);
        if (j > i) { const float2 t = v[i]; v[i] = v[j]; v[j] = t; }
    }
#pragma unroll
    for (int half = 1; half < L; half *= 2) {
        const int step = L / (2 * half);
#pragma unroll
        for (int j = 0; j < half; ++j) {
            float2 w = tw[j * step];
            if (INV) w.y = -w.y;
#pragma unroll
            for (int k = 0; k < L; k += 2 * half) {
                const float2 a = v[k + j];
                const float2 b = cmul(v[k + j + half], w);
                v[k + j] = make_float2(a.x + b.x, a.y + b.y);
                v[k + j + half] = make_float2(a.x - b.x, a.y - b.y);
            }
        }
    }
}

// in-register transform of v[0..N) (natural order in and out) with the
// twiddles of the length-N*TS table tw[j] = exp(-2 pi i j / (N TS)), j < N TS / 2
template <int N, bool INV, int TS>
__device__ __forceinline__ void fft1t(float2 (&v)[N], const float2* __restrict__ tw) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int j = bitrev<N>(i);
        if (j > i) { const float2 t = v[i]; v[i] = v[j]; v[j] = t; }
    }
#pragma unroll
    for (int half = 1; half < N; half *= 2) {
        const int step = N / (2 * half);
#pragma unroll
        for (int j = 0; j < half; ++j) {
            float2 w = tw[j * step * TS];
            if (INV) w.y = -w.y;
#pragma unroll
            for (int k = 0; k < N; k += 2 * half) {
                const float2 a = v[k + j];
                const float2 b = cmul(v[k + j + half], w);
                v[k + j] = make_float2(a.x + b.x, a.y + b.y);
                v[k + j + half] = make_float2(a.x - b.x, a.y - b.y);
            }
        }
    }
}

// twiddles tw[j] = exp(-2 pi i j / L), j < NTW, from double-precision sincospi
template <int L, int NTW> __device__ __forceinline__ void make_twiddles_n(float2* tw) {
    for (int j = threadIdx.x; j < NTW; j += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)j / (double)L, &s, &c);
        tw[j] = make_float2((float)c, (float)s);
    }
}

// In-register transform of v[0..L), L = 3 M with M a power of two (natural
// order in and out), the twiddle table tw[j] = exp(-2 pi i j / (S L)), j < S L
// (every S-th entry is used: S = 2 for the half transforms of a lane pair).
// With n = M n1 + n2 and k = k1 + 3 k2 (Cooley-Tukey with factors 3 and M):
//   X[k1 + 3 k2] = sum_{n2} W_M^{n2 k2} W_L^{n2 k1} sum_{n1} x[M n1 + n2] W_3^{n1 k1}:
// M three-point transforms, the twiddles W_L^{n2 k1}, then three length-M
// transforms (whose twiddles W_M^j = W_L^{3 j} are every third table entry).
// The three-point transform of (a, b, c): X0 = a + (b + c),
// X1,2 = a - (b + c) / 2 -/+ i (sqrt(3) / 2) (b - c) (signs swapped for the inverse).
template <int L, bool INV, int S = 1>
__device__ __forceinline__ void fft1m(float2 (&v)[L], const float2* __restrict__ tw) {
    constexpr int M = L / 3;
    constexpr float S3 = 0.866025403784438646763723f;   // sqrt(3) / 2
    float2 u[3][M];
#pragma unroll
    for (int n2 = 0; n2 < M; ++n2) {
        const float2 a = v[n2], b = v[M + n2], c = v[2 * M + n2];
        const float2 t1 = make_float2(b.x + c.x, b.y + c.y);
        const float2 t2 = make_float2(b.x - c.x, b.y - c.y);
        const float2 m = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
        // forward: -i S3 t2; inverse: +i S3 t2
        const float2 sr = INV ? make_float2(-S3 * t2.y, S3 * t2.x) : make_float2(S3 * t2.y, -S3 * t2.x);
        u[0][n2] = make_float2(a.x + t1.x, a.y + t1.y);
        float2 w1 = tw[S * n2], w2 = tw[S * 2 * n2];
        if (INV) { w1.y = -w1.y; w2.y = -w2.y; }
        u[1][n2] = n2 == 0 ? make_float2(m.x + sr.x, m.y + sr.y) : cmul(make_float2(m.x + sr.x, m.y + sr.y), w1);
        u[2][n2] = n2 == 0 ? make_float2(m.x - sr.x, m.y - sr.y) : cmul(make_float2(m.x - sr.x, m.y - sr.y), w2);
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) fft1t<M, INV, 3 * S>(u[k1], tw);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < M; ++k2) v[k1 + 3 * k2] = u[k1][k2];
}

// the transform of v[0..L) for any supported L (radix 2, or 3 x radix 2)
template <int L, bool INV>
__device__ __forceinline__ void fft1any(float2 (&v)[L], const float2* __restrict__ tw) {
    if constexpr (L % 3 == 0) fft1m<L, INV>(v, tw);
    else fft1<L, INV>(v, tw);
}

// the half-length transform of a lane pair's samples: radix 2, or 3 x radix 2
// (L / 2 = 24 at L 48), with every second entry of the length-L table
template <int N, bool INV>
__device__ __forceinline__ void fft_half(float2 (&v)[N], const float2* __restrict__ tw) {
    if constexpr (N % 3 == 0) fft1m<N, INV, 2>(v, tw);
    else fft1t<N, INV, 2>(v, tw);
}

__device__ __forceinline__ float2 shfl_pair(float2 a) {
    return make_float2(__shfl_xor(a.x, 1), __shfl_xor(a.y, 1));
}

// The pair table of a length-L transform: L / 2 ones, then W_L^k = exp(-2 pi i
// k / L), k < L / 2; lane h of a pair reads it from entry (L / 2) h, so that
// the butterflies below take no per-lane selects (lane 0 multiplies by one).
template <int L> __device__ __forceinline__ void make_pair_twiddles(float2* twp) {
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        if (j < L / 2) {
            twp[j] = make_float2(1.f, 0.f);
        } else {
            double s, c;
            sincospi(-2.0 * (double)(j - L / 2) / (double)L, &s, &c);
            twp[j] = make_float2((float)c, (float)s);
        }
    }
}

// A length-L transform held by the two lanes of a pair (h = lane & 1, L / 2
// values each), tw the length-L table (its first half for a power-of-two L),
// twh the lane's half of the pair table.
// Decimation in time: v holds the samples x[2m + h]; on return v[k] = X[(L/2) h + k]
// (X[k] = E[k] + W^k O[k], X[k + L/2] = E[k] - W^k O[k] from the two half
// transforms: lane 1 forms W^k O[k], and each lane adds its partner's value to,
// or subtracts its own from, the other's).
template <int L, bool INV>
__device__ __forceinline__ void fft_pair_dit(float2 (&v)[L / 2], int h, const float2* __restrict__ tw,
                                             const float2* __restrict__ twh) {
    fft_half<L / 2, INV>(v, tw);
    const float sg = h ? -1.f : 1.f;
#pragma unroll
    for (int k = 0; k < L / 2; ++k) {
        float2 w = twh[k];
        if (INV) w.y = -w.y;
        const float2 t = cmul(v[k], w);                  // lane 0: E[k]; lane 1: W^k O[k]
        const float2 q = shfl_pair(t);
        v[k] = make_float2(q.x + sg * t.x, q.y + sg * t.y);
    }
}
// Decimation in frequency: v holds the half x[(L/2) h + m]; on return v[k] = X[2k + h]
// (X[2k] from a + b, X[2k + 1] from (a - b) W^m, a and b the two halves).
template <int L, bool INV>
__device__ __forceinline__ void fft_pair_dif(float2 (&v)[L / 2], int h, const float2* __restrict__ tw,
                                             const float2* __restrict__ twh) {
    const float sg = h ? -1.f : 1.f;
#pragma unroll
    for (int k = 0; k < L / 2; ++k) {
        const float2 q = shfl_pair(v[k]);
        float2 w = twh[k];
        if (INV) w.y = -w.y;
        // lane 0: b + a; lane 1: (a - b) W^k
        v[k] = cmul(make_float2(q.x + sg * v[k].x, q.y + sg * v[k].y), w);
    }
    fft_half<L / 2, INV>(v, tw);
}

// ---- four lanes per row (L = 64): lane q of a row holds a quarter of it.
__device__ __forceinline__ float2 shfl_x(float2 a, int mask) {
    return make_float2(__shfl_xor(a.x, mask), __shfl_xor(a.y, mask));
}
// the block of L/4 outputs (decimation in time) or inputs (in frequency) of lane q:
// q with its two bits swapped
__device__ __forceinline__ int quad_block(int q) { return ((q & 1) << 1) | (q >> 1); }

// Decimation in time over the four lanes of a row: v holds x[4m + q]; on return
// v[j] = X[(L/4) quad_block(q) + j].  Each lane transforms its quarter, then
// two radix-2 stages across lanes: q with q ^ 2 form the length-L/2 transforms
// E_p of the samples 2n + p (p = q & 1; lane q < 2 keeps E_p[j], lane q >= 2
// E_p[j + L/4]), and q with q ^ 1 form X[k] = E_0[k] +- W_L^k E_1[k].
template <int L, bool INV>
__device__ __forceinline__ void fft_quad_dit(float2 (&v)[L / 4], int q, const float2* __restrict__ tw) {
    constexpr int N = L / 4;
    fft1t<N, INV, 4>(v, tw);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float2 o = shfl_x(v[j], 2);
        const float2 lo = q < 2 ? v[j] : o, hi = q < 2 ? o : v[j];
        float2 w = tw[2 * j];                     // W_{L/2}^j
        if (INV) w.y = -w.y;
        const float2 t = cmul(hi, w);
        v[j] = q < 2 ? make_float2(lo.x + t.x, lo.y + t.y) : make_float2(lo.x - t.x, lo.y - t.y);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float2 o = shfl_x(v[j], 1);
        const float2 e0 = (q & 1) ? o : v[j], e1 = (q & 1) ? v[j] : o;
        float2 w = tw[N * (q >> 1) + j];          // W_L^k, k = (L/4)(q >> 1) + j
        if (INV) w.y = -w.y;
        const float2 t = cmul(e1, w);
        v[j] = (q & 1) ? make_float2(e0.x - t.x, e0.y - t.y) : make_float2(e0.x + t.x, e0.y + t.y);
    }
}
// Decimation in frequency, the mirror: v holds x[(L/4) quad_block(q) + j]; on
// return v[j] = X[4j + q].  q with q ^ 1 split n and n + L/2 into the sums
// (even outputs) and the twiddled differences (odd outputs), q with q ^ 2 do
// the same within each length-L/2 sequence, then each lane transforms its quarter.
template <int L, bool INV>
__device__ __forceinline__ void fft_quad_dif(float2 (&v)[L / 4], int q, const float2* __restrict__ tw) {
    constexpr int N = L / 4;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float2 o = shfl_x(v[j], 1);
        const float2 a = (q & 1) ? o : v[j], b = (q & 1) ? v[j] : o;
        float2 w = tw[N * (q >> 1) + j];          // W_L^n, n = (L/4)(q >> 1) + j
        if (INV) w.y = -w.y;
        v[j] = (q & 1) ? cmul(make_float2(a.x - b.x, a.y - b.y), w) : make_float2(a.x + b.x, a.y + b.y);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float2 o = shfl_x(v[j], 2);
        const float2 a = (q >> 1) ? o : v[j], b = (q >> 1) ? v[j] : o;
        float2 w = tw[2 * j];                     // W_{L/2}^j
        if (INV) w.y = -w.y;
        v[j] = (q >> 1) ? cmul(make_float2(a.x - b.x, a.y - b.y), w) : make_float2(a.x + b.x, a.y + b.y);
    }
    fft1t<N, INV, 4>(v, tw);
}

__device__ __forceinline__ void team_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}


// Row transforms of v (this thread's row r), then column transforms through the
// team buffer buf [L][L + 1]; on return v holds column r of the 2-D transform
// (v[k] = X[k][r]).
template <int L, bool INV>
__device__ __forceinline__ void fft2_rows_then_cols(float2 (&v)[L], float2* buf, int r,
                                                    const float2* tw) {
    fft1<L, INV>(v, tw);
#pragma unroll
    for (int k = 0; k < L; ++k) buf[r * (L + 1) + k] = v[k];
    team_sync();
#pragma unroll
    for (int k = 0; k < L; ++k) v[k] = buf[k * (L + 1) + r];
    team_sync();
    fft1<L, INV>(v, tw);
}

// Column transforms of v (this thread's column c: v[k] = x[k][c]), then row
// transforms through buf; on return v holds row c of the 2-D transform.
template <int L, bool INV>
__device__ __forceinline__ void fft2_cols_then_rows(float2 (&v)[L], float2* buf, int c,
                                                    const float2* tw) {
    fft1<L, INV>(v, tw);
#pragma unroll
    for (int k = 0; k < L; ++k) buf[k * (L + 1) + c] = v[k];
    team_sync();
#pragma unroll
    for (int k = 0; k < L; ++k) v[k] = buf[c * (L + 1) + k];
    team_sync();
    fft1<L, INV>(v, tw);
}

}  // namespace fft
}  // namespace srmra
