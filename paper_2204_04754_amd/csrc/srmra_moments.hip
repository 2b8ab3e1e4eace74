// Empirical moments of eq. empiric_MOM: M1 = (1/N) sum_i y_i and
// M2 = (1/N) sum_i y_i y_i^T = (1/N) Y^T Y, Y the N x P stack of vectorised
// observations (P = Ll^2, pixel index n1 Ll + n2).  M2 is a symmetric rank-N
// product on FP32 matrix cores (v_mfma_f32_32x32x2_f32) in 128 x 128 tiles of
// the upper triangle; the observations are split into S chunks whose FP32
// partial tiles are summed in FP64 in a fixed order (deterministic), then
// mirrored.  M1: FP64 column sums per chunk, summed in the same way.
#include "srmra_moments.h"

namespace srmra {

typedef float floatx16m __attribute__((ext_vector_type(16)));

constexpr int kMT = 128;    // tile edge
constexpr int kMKB = 16;    // observations per LDS stage

__device__ __forceinline__ void pair_of(int q, int T, int& ti, int& tj) {
    // q enumerates the tile pairs (ti, tj), ti <= tj, row by row
    int t = 0;
    while (q >= T - t) {
        q -= T - t;
        ++t;
    }
    ti = t;
    tj = t + q;
}

// grid S x T (T + 1) / 2 blocks (chunks x tile pairs); block 256 = 4 waves,
// wave (rb, cb) owns rows rb*64.. and columns cb*64.. of the tile as 2 x 2
// MFMA tiles.  Blocks go round-robin to the 8 XCDs, so when S is a multiple of
// 8 every tile pair of chunk ch runs on XCD ch mod 8 and the chunk's rows are
// read into one L2.
__global__ __launch_bounds__(256, 2) void k_gram_tiles(const float* __restrict__ y, int64_t N, int P,
                                                      int T, int64_t chunk_obs, int S,
                                                      float* __restrict__ part) {
    __shared__ __align__(16) float As[kMKB][kMT];
    __shared__ __align__(16) float Bs[kMKB][kMT];
    const int npairs = T * (T + 1) / 2;
    int ch, q;
    if (S % 8 == 0) {
        const int xcd = blockIdx.x % 8, j = blockIdx.x / 8;
        ch = (j / npairs) * 8 + xcd;
        q = j % npairs;
    } else {
        ch = blockIdx.x / npairs;
        q = blockIdx.x % npairs;
    }
    int ti, tj;
    pair_of(q, T, ti, tj);
    const int i0 = ti * kMT, j0 = tj * kMT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rb = wave & 1, cb = wave >> 1, li = lane & 31, g = lane >> 5;
    floatx16m acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = floatx16m{0};
    const int64_t c0 = (int64_t)ch * chunk_obs;
    const int64_t c1 = min<int64_t>(N, c0 + chunk_obs);
    // each thread moves NE float4 of A and of B per stage; the next stage's are
    // requested before the current stage's MFMAs (register double buffer)
    constexpr int NE = kMKB * (kMT / 4) / 256;
    float4 ra[NE], rbuf[NE];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = threadIdx.x + u * 256;
            const int r = e / (kMT / 4), c4 = 4 * (e % (kMT / 4));
            const int64_t k = k0 + r;
            ra[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            rbuf[u] = ra[u];
            if (k < c1) {
                const float* row = y + k * (int64_t)P;
                if (i0 + c4 < P) ra[u] = *reinterpret_cast<const float4*>(row + i0 + c4);
                if (j0 + c4 < P) rbuf[u] = *reinterpret_cast<const float4*>(row + j0 + c4);
            }
        }
    };
    if (c0 < c1) fetch(c0);
    for (int64_t k0 = c0; k0 < c1; k0 += kMKB) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = threadIdx.x + u * 256;
            const int r = e / (kMT / 4), c4 = 4 * (e % (kMT / 4));
            *reinterpret_cast<float4*>(&As[r][c4]) = ra[u];
            *reinterpret_cast<float4*>(&Bs[r][c4]) = rbuf[u];
        }
        __syncthreads();
        if (k0 + kMKB < c1) fetch(k0 + kMKB);
#pragma unroll
        for (int kk = 0; kk < kMKB; kk += 2) {
            float a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = As[kk + g][rb * 64 + r * 32 + li];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = Bs[kk + g][cb * 64 + c * 32 + li];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[r], b[c], acc[r][c], 0, 0, 0);
        }
    }
    float* out = part + ((int64_t)ch * npairs + q) * (kMT * kMT);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = rb * 64 + r * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
                const int col = cb * 64 + c * 32 + li;
                out[row * kMT + col] = acc[r][c][v];
            }
}

// M2[p][q] = (1/N) sum over chunks of the partial tile holding (min, max) of
// (p, q) (the upper triangle), in FP64 in chunk order.
__global__ __launch_bounds__(256) void k_gram_reduce(const float* __restrict__ part, int S, int T,
                                                     int P, double inv_n, double* __restrict__ m2) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)P * P) return;
    int p = (int)(e / P), q = (int)(e % P);
    if (p > q) { const int t = p; p = q; q = t; }
    const int ti = p / kMT, tj = q / kMT;
    const int pair = ti * T - ti * (ti - 1) / 2 + (tj - ti);
    const int npairs = T * (T + 1) / 2;
    const int64_t off = (int64_t)pair * (kMT * kMT) + (p - ti * kMT) * kMT + (q - tj * kMT);
    double s = 0.0;
    for (int c = 0; c < S; ++c) s += (double)part[(int64_t)c * npairs * (kMT * kMT) + off];
    m2[e] = s * inv_n;
}

// per-chunk FP64 column sums: grid (S1, ceil(P / 256))
__global__ __launch_bounds__(256) void k_col_sums(const float* __restrict__ y, int64_t N, int P,
                                                  int64_t chunk_obs, double* __restrict__ part1) {
    const int p = blockIdx.y * 256 + threadIdx.x;
    if (p >= P) return;
    const int64_t c0 = (int64_t)blockIdx.x * chunk_obs;
    const int64_t c1 = min<int64_t>(N, c0 + chunk_obs);
    double s = 0.0;
    for (int64_t k = c0; k < c1; ++k) s += (double)y[k * (int64_t)P + p];
    part1[(int64_t)blockIdx.x * P + p] = s;
}

__global__ __launch_bounds__(256) void k_m1_reduce(const double* __restrict__ part1, int S1, int P,
                                                   double inv_n, double* __restrict__ m1) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int c = 0; c < S1; ++c) s += part1[(int64_t)c * P + p];
    m1[p] = s * inv_n;
}

// ---------------------------------------------------------------- host side
MomentsGeom moments_geom(int64_t N, int Ll, int cus) {
    MomentsGeom g;
    g.P = Ll * Ll;
    g.T = (g.P + kMT - 1) / kMT;
    g.npairs = g.T * (g.T + 1) / 2;
    // about four resident blocks per CU over all tile pairs
    int64_t S = (4LL * cus + g.npairs - 1) / g.npairs;
    if (S >= 8) S = (S + 7) / 8 * 8;                 // a multiple of 8: one XCD per chunk
    const int64_t smax = (N + kMKB - 1) / kMKB;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    int64_t chunk = (N + S - 1) / S;
    chunk = (chunk + kMKB - 1) / kMKB * kMKB;
    g.chunk = chunk;
    g.S = (int)S;                                    // the last chunks may be empty
    g.chunk1 = 256;
    g.S1 = (int)((N + g.chunk1 - 1) / g.chunk1);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    g.o_part = 0;
    g.o_part1 = al(sizeof(float) * (size_t)g.S * g.npairs * kMT * kMT);
    g.total = g.o_part1 + al(sizeof(double) * (size_t)g.S1 * g.P);
    return g;
}

hipError_t launch_moments(const float* y, int64_t N, int Ll, double* m1, double* m2, void* ws,
                          const MomentsGeom& g, hipStream_t s) {
    float* part = (float*)((char*)ws + g.o_part);
    double* part1 = (double*)((char*)ws + g.o_part1);
    const double inv_n = 1.0 / (double)N;
    hipLaunchKernelGGL(k_gram_tiles, dim3((unsigned)(g.S * g.npairs)), dim3(256), 0, s, y, N, g.P, g.T,
                       g.chunk, g.S, part);
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(((int64_t)g.P * g.P + 255) / 256)), dim3(256), 0, s,
                       (const float*)part, g.S, g.T, g.P, inv_n, m2);
    hipLaunchKernelGGL(k_col_sums, dim3(g.S1, (g.P + 255) / 256), dim3(256), 0, s, y, N, g.P, g.chunk1, part1);
    hipLaunchKernelGGL(k_m1_reduce, dim3((g.P + 255) / 256), dim3(256), 0, s, (const double*)part1, g.S1,
                       g.P, inv_n, m1);
    return hipGetLastError();
}

}  // namespace srmra
