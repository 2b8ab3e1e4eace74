// Kernels of the FFT route (bodies in srmra_fftp_impl.h) and their launches.
#include <atomic>

#include "srmra_fftp_impl.h"

namespace srmra {
namespace fft {

template <int L>
__global__ __launch_bounds__(256) void k_fft_prep_y(const float* __restrict__ y, int64_t N,
                                                    const double* __restrict__ centre,
                                                    float2* __restrict__ yhat) {
    prep_y_body<L, true>(y, N, centre, yhat);
}

// X_c for every component: block c, its first L threads
template <int L>
__global__ __launch_bounds__(256) void k_fft_pack_x(const float* __restrict__ x, int K,
                                                    const double* __restrict__ centre,
                                                    float2* __restrict__ xhat) {
    extern __shared__ float2 sh[];
    float2* tw = sh + L * (L + 1);
    make_twiddles_n<L, L>(tw);
    __syncthreads();
    pack_x_body<L>(x, K, centre, xhat, blockIdx.x, sh, tw);
}

// the two passes: grid (chunks, observation splits / component groups)
template <int L>
__global__ __launch_bounds__(256) void k_fft_pass1(StepArgs p, const float2* __restrict__ yhat,
                                                   const float2* __restrict__ xhat) {
    extern __shared__ float2 sh[];
    pass1_pairs_body<L>(p, yhat, xhat, blockIdx.x, blockIdx.y, gridDim.y, sh);
}
template <int L>
__global__ __launch_bounds__(256) void k_fft_pass2(StepArgs p, const float2* __restrict__ yhat,
                                                   const float2* __restrict__ xhat, int TPC,
                                                   float2* __restrict__ bpart, float* __restrict__ cpart) {
    extern __shared__ float2 sh[];
    pass2_pairs_body<L>(p, yhat, xhat, TPC, bpart, cpart, blockIdx.x, blockIdx.y, sh);
}
// four blocks per CU (at most 128 registers per lane; its LDS, 33 KB, allows them)
__global__ __launch_bounds__(256, 4) void k_fft_pass1_q(StepArgs p, const float2* __restrict__ yhat,
                                                     const float2* __restrict__ xhat) {
    extern __shared__ float2 sh[];
    pass1_quad_body(p, yhat, xhat, blockIdx.x, blockIdx.y, gridDim.y, sh);
}
__global__ __launch_bounds__(256) void k_fft_pass2_q(StepArgs p, const float2* __restrict__ yhat,
                                                     const float2* __restrict__ xhat, int /*TPC*/,
                                                     float2* __restrict__ bpart, float* __restrict__ cpart) {
    extern __shared__ float2 sh[];
    pass2_quad_body(p, yhat, xhat, bpart, cpart, blockIdx.x, blockIdx.y, sh);
}

namespace row {
template <int L>
__global__ __launch_bounds__(256) void k_prep_y(const float* __restrict__ y, int64_t N,
                                                const double* __restrict__ centre, float2* __restrict__ yhat) {
    extern __shared__ float2 sh[];
    float2* tw = sh + G<L>::TEAMS * G<L>::BUF;
    make_twiddles_n<L, L>(tw);
    __syncthreads();
    int team, r;
    bool on;
    team_of<L>(team, r, on);
    const int64_t i = (int64_t)blockIdx.x * G<L>::TEAMS + team;
    const bool act = on && i < N;   // every lane reaches the teams' barriers
    float2* buf = sh + team * G<L>::BUF;
    const float mu = centre_of(centre);
    float2 v[L];
    if (act) {
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = make_float2(y[(i * L + k) * L + r] - mu, 0.f);   // column r
        fft1m<L, false>(v, tw);
#pragma unroll
        for (int k = 0; k < L; ++k) buf[k * (L + 1) + r] = v[k];
    }
    row::sync<L>();
    if (act) {
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = buf[r * (L + 1) + k];   // row k1 = r
    }
    row::sync<L>();
    if (!act) return;
    fft1m<L, false>(v, tw);                                     // v[k] = Y_i[r][k]
    float4* d = reinterpret_cast<float4*>(yhat) + i * (L / 2) * L + r;
#pragma unroll
    for (int k = 0; k < L; k += 2) d[(k / 2) * L] = make_float4(v[k].x, v[k].y, v[k + 1].x, v[k + 1].y);
}

// two waves per SIMD (at most 256 registers per lane; pass 2 at L 48 runs
// lane-pair teams, half a row per lane, to fit)
template <int L>
__global__ __launch_bounds__(256, 2) void k_pass1(StepArgs p, const float2* __restrict__ yhat,
                                               const float2* __restrict__ xhat) {
    extern __shared__ float2 sh[];
    pass1_body<L>(p, yhat, xhat, blockIdx.x, blockIdx.y, gridDim.y, sh);
}
template <int L>
__global__ __launch_bounds__(256, 2) void k_pass2(StepArgs p, const float2* __restrict__ yhat,
                                               const float2* __restrict__ xhat, int TPC,
                                               float2* __restrict__ bpart, float* __restrict__ cpart) {
    extern __shared__ float2 sh[];
    if constexpr (L == 48) wpair::pass2_body<L>(p, yhat, xhat, TPC, bpart, cpart, blockIdx.x, blockIdx.y, sh);
    else pass2_body<L>(p, yhat, xhat, TPC, bpart, cpart, blockIdx.x, blockIdx.y, sh);
}
template <int L>
__global__ __launch_bounds__(256) void k_dft2(const float* __restrict__ in, int64_t count,
                                              float2* __restrict__ out) {
    extern __shared__ float2 sh[];
    float2* tw = sh + G<L>::TEAMS * G<L>::BUF;
    make_twiddles_n<L, L>(tw);
    __syncthreads();
    int team, r;
    bool on;
    team_of<L>(team, r, on);
    const int64_t i = (int64_t)blockIdx.x * G<L>::TEAMS + team;
    const bool act = on && i < count;   // every lane reaches the teams' barriers
    float2* buf = sh + team * G<L>::BUF;
    float2 v[L];
    if (act) {
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = make_float2(in[(i * L + r) * L + k], 0.f);   // row r
        fft1m<L, false>(v, tw);
#pragma unroll
        for (int k = 0; k < L; ++k) buf[r * (L + 1) + k] = v[k];
    }
    row::sync<L>();
    if (act) {
#pragma unroll
        for (int k = 0; k < L; ++k) v[k] = buf[k * (L + 1) + r];   // column r
    }
    row::sync<L>();
    if (!act) return;
    fft1m<L, false>(v, tw);                                     // v[k] = X[k][r]
#pragma unroll
    for (int k = 0; k < L; ++k) out[(i * L + k) * L + r] = v[k];
}
}  // namespace row

__global__ __launch_bounds__(256) void k_fft_reduce(const float2* __restrict__ bpart,
                                                    const float* __restrict__ cpart, int n_chunks,
                                                    int per, double2* __restrict__ bh,
                                                    double* __restrict__ csum) {
    __shared__ double red[3 * 256];
    reduce_body(bpart, cpart, n_chunks, per, bh, csum, blockIdx.x, red);
}

// one workgroup per component; dynamic LDS: idft_lds<L>() bytes
template <int L>
__global__ __launch_bounds__(256) void k_fft_idft(const double2* __restrict__ bh, double* __restrict__ bsum) {
    extern __shared__ double2 T[];
    idft_body<L>(bh, bsum, blockIdx.x, T);
}

// batched forward DFT of real images (utility): out[i][k1][k2]
template <int L>
__global__ __launch_bounds__(256) void k_dft2(const float* __restrict__ in, int64_t count,
                                              float2* __restrict__ out) {
    prep_y_body<L, false>(in, count, nullptr, out);
}

}  // namespace fft

// ---------------------------------------------------------------- host side
static bool mixed_ll(int LL) { return LL == 12 || LL == 24 || LL == 48; }
bool fft_supported(int LL) { return LL == 8 || LL == 16 || LL == 32 || LL == 64 || mixed_ll(LL); }

int fft_teams(int LL) { return fft::teams_of(LL); }
int fft_tpc(int LL, int KK) { return fft::tpc_of(LL, KK); }

size_t fft_lds(int LL, int pass) {   // dynamic LDS of pass 1 or 2
    switch (LL) {
        case 8: return fft::lds_pairs<8>();
        case 16: return fft::lds_pairs<16>();
        case 32: return fft::lds_pairs<32>();
        case 64: return pass == 1 ? fft::quad::lds1() : fft::quad::lds();
        case 12: return pass == 1 ? fft::row::lds_pass1<12>() : fft::row::lds<12>();
        case 24: return pass == 1 ? fft::row::lds_pass1<24>() : fft::row::lds<24>();
        case 48: return pass == 1 ? fft::row::lds_pass1<48>() : fft::wpair::lds<48>();
    }
    return 0;
}

// the same in the batched class launches (pass 2 at L 32 stages X_c in LDS)
size_t fft_lds_class(int LL, int pass) { return pass == 2 && LL == 32 ? fft::lds_pairs_xs<32>() : fft_lds(LL, pass); }

const void* fft_pass2_fn(int LL) {
    switch (LL) {
        case 8: return (const void*)fft::k_fft_pass2<8>;
        case 16: return (const void*)fft::k_fft_pass2<16>;
        case 32: return (const void*)fft::k_fft_pass2<32>;
        case 64: return (const void*)fft::k_fft_pass2_q;
        case 12: return (const void*)fft::row::k_pass2<12>;
        case 24: return (const void*)fft::row::k_pass2<24>;
        case 48: return (const void*)fft::row::k_pass2<48>;
    }
    return nullptr;
}

// Pass-1 blocks per chunk and component group: the chunks are sized for pass
// 2's blocks per CU, and pass 1 (one partial per observation) splits each
// chunk's observations over that many more blocks where more of its own fit a
// CU (cache: per kernel pair, filled on first use; 0 if the query fails).
static int pass1_split(const void* f1, size_t lds1, const void* f2, size_t lds2, std::atomic<int>& cache) {
    int sp = cache.load(std::memory_order_relaxed);
    if (sp == 0) {
        int b1 = 0, b2 = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, f1, 256, lds1) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, f2, 256, lds2) != hipSuccess)
            return 0;
        sp = (b1 > b2 && b2 > 0) ? (b1 + b2 - 1) / b2 : 1;
        cache.store(sp, std::memory_order_relaxed);
    }
    return sp;
}

// the passes at L_low = 3 * 2^m (what: 0 prepare Y, 1 X, 2 pass 1, 3 pass 2, 4 reduce)
template <int L>
static hipError_t fft_launch_row(int what, const StepArgs& p, const float* x, const float* y,
                                 void* yhat, void* xhat, void* bpart, void* cpart, hipStream_t s) {
    using G = fft::row::G<L>;
    const size_t lds = fft::row::lds<L>(), lp1 = fft::row::lds_pass1<L>();
    const size_t lp2 = L == 48 ? fft::wpair::lds<L>() : lds;
    auto attr = [&](const void* f, size_t bytes) {
        return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    };
    switch (what) {
        case 0:
            if (attr((const void*)fft::row::k_prep_y<L>, lds) != hipSuccess) return hipErrorInvalidValue;
            hipLaunchKernelGGL(fft::row::k_prep_y<L>, dim3((unsigned)((p.N + G::TEAMS - 1) / G::TEAMS)), dim3(256),
                               lds, s, y, p.N, p.centre, (float2*)yhat);
            break;
        case 1:
            if (hipFuncSetAttribute((const void*)fft::k_fft_pack_x<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)fft::pack_lds<L>()) != hipSuccess)
                return hipErrorInvalidValue;
            hipLaunchKernelGGL(fft::k_fft_pack_x<L>, dim3(p.KK), dim3(256), fft::pack_lds<L>(), s, x, p.K,
                               p.centre, (float2*)xhat);
            break;
        case 2:
        {
            if (attr((const void*)fft::row::k_pass1<L>, lp1) != hipSuccess) return hipErrorInvalidValue;
            static std::atomic<int> split{0};
            const int sp = pass1_split((const void*)fft::row::k_pass1<L>, lp1, (const void*)fft::row::k_pass2<L>,
                                       lp2, split);
            if (sp == 0) return hipErrorInvalidValue;
            hipLaunchKernelGGL(fft::row::k_pass1<L>, dim3(p.n_chunks, p.n_cg * sp), dim3(256), lp1, s, p,
                               (const float2*)yhat, (const float2*)xhat);
            break;
        }
        case 3:
            if (attr((const void*)fft::row::k_pass2<L>, lp2) != hipSuccess) return hipErrorInvalidValue;
            hipLaunchKernelGGL(fft::row::k_pass2<L>, dim3(p.n_chunks, p.n_cg), dim3(256), lp2, s, p,
                               (const float2*)yhat, (const float2*)xhat, fft_tpc(L, p.KK), (float2*)bpart,
                               (float*)cpart);
            break;
    }
    return hipGetLastError();
}

// the FP64 sums of the partials and the inverse DFT of the back-projection
template <int L>
static hipError_t fft_launch_reduce(const StepArgs& p, void* bpart, void* cpart, void* bh, double* bsum,
                                    double* csum, hipStream_t s) {
    const int per = p.KK * L * L;
    hipLaunchKernelGGL(fft::k_fft_reduce, dim3((per + kReduceElems - 1) / kReduceElems), dim3(256), 0, s,
                       (const float2*)bpart, (const float*)cpart, p.n_chunks, per, (double2*)bh, csum);
    (void)hipFuncSetAttribute((const void*)fft::k_fft_idft<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)fft::idft_lds<L>());
    hipLaunchKernelGGL(fft::k_fft_idft<L>, dim3(p.KK), dim3(256), fft::idft_lds<L>(), s, (const double2*)bh,
                       bsum);
    return hipGetLastError();
}

template <int L>
static hipError_t fft_launch_ll(int what, const StepArgs& p, const float* x, const float* y,
                                void* yhat, void* xhat, void* bpart, void* cpart, void* bh,
                                double* bsum, double* csum, hipStream_t s) {
    if (what == 4) return fft_launch_reduce<L>(p, bpart, cpart, bh, bsum, csum, s);
    if constexpr (L % 3 == 0) {
        return fft_launch_row<L>(what, p, x, y, yhat, xhat, bpart, cpart, s);
    } else {
        const size_t lds = fft::lds_bytes<L>();      // preparation and X: one lane per row
        const size_t lp = L == 64 ? fft::quad::lds() : fft::lds_pairs<L>();   // the passes
        const size_t lp1 = L == 64 ? fft::quad::lds1() : lp;                    // pass 1
        const int teams = 256 / L;
        switch (what) {
            case 0:   // prepare Y
                (void)hipFuncSetAttribute((const void*)fft::k_fft_prep_y<L>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(fft::k_fft_prep_y<L>, dim3((unsigned)((p.N + teams - 1) / teams)), dim3(256), lds, s,
                                   y, p.N, p.centre, (float2*)yhat);
                break;
            case 1:   // X
                (void)hipFuncSetAttribute((const void*)fft::k_fft_pack_x<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)fft::pack_lds<L>());
                hipLaunchKernelGGL(fft::k_fft_pack_x<L>, dim3(p.KK), dim3(256), fft::pack_lds<L>(), s, x, p.K,
                                   p.centre, (float2*)xhat);
                break;
            case 2: {
                auto f = L == 64 ? fft::k_fft_pass1_q : fft::k_fft_pass1<L == 64 ? 32 : L>;
                auto f2 = L == 64 ? fft::k_fft_pass2_q : fft::k_fft_pass2<L == 64 ? 32 : L>;
                (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lp1);
                static std::atomic<int> split{0};
                const int sp = pass1_split((const void*)f, lp1, (const void*)f2, lp, split);
                if (sp == 0) return hipErrorInvalidValue;
                hipLaunchKernelGGL(f, dim3(p.n_chunks, p.n_cg * sp), dim3(256), lp1, s, p, (const float2*)yhat,
                                   (const float2*)xhat);
                break;
            }
            case 3: {
                const int tpc = fft_tpc(L, p.KK);
                auto f = L == 64 ? fft::k_fft_pass2_q : fft::k_fft_pass2<L == 64 ? 32 : L>;
                (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lp);
                hipLaunchKernelGGL(f, dim3(p.n_chunks, p.n_cg), dim3(256), lp, s, p, (const float2*)yhat,
                                   (const float2*)xhat, tpc, (float2*)bpart, (float*)cpart);
                break;
            }
        }
        return hipGetLastError();
    }
}

hipError_t launch_fft(int LL, int what, const StepArgs& p, const float* x, const float* y,
                      void* yhat, void* xhat, void* bpart, void* cpart, void* bh,
                      double* bsum, double* csum, hipStream_t s) {
    switch (LL) {
        case 8: return fft_launch_ll<8>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
        case 16: return fft_launch_ll<16>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
        case 32: return fft_launch_ll<32>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
        case 64: return fft_launch_ll<64>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
        case 12: return fft_launch_ll<12>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
        case 24: return fft_launch_ll<24>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
        case 48: return fft_launch_ll<48>(what, p, x, y, yhat, xhat, bpart, cpart, bh, bsum, csum, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dft2(int L, const float* in, int64_t count, float2* out, hipStream_t s) {
    const int teams = 256 / L;
    const dim3 grid((unsigned)((count + teams - 1) / teams));
    size_t lds;
    switch (L) {
        case 8: lds = fft::lds_bytes<8>(); hipLaunchKernelGGL(fft::k_dft2<8>, grid, dim3(256), lds, s, in, count, out); break;
        case 16: lds = fft::lds_bytes<16>(); hipLaunchKernelGGL(fft::k_dft2<16>, grid, dim3(256), lds, s, in, count, out); break;
        case 32:
            lds = fft::lds_bytes<32>();
            (void)hipFuncSetAttribute((const void*)fft::k_dft2<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(fft::k_dft2<32>, grid, dim3(256), lds, s, in, count, out);
            break;
        case 64:
            lds = fft::lds_bytes<64>();
            (void)hipFuncSetAttribute((const void*)fft::k_dft2<64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(fft::k_dft2<64>, grid, dim3(256), lds, s, in, count, out);
            break;
        case 12: case 24: case 48: {
            const int tm = L == 12 ? fft::row::G<12>::TEAMS : (L == 24 ? fft::row::G<24>::TEAMS : fft::row::G<48>::TEAMS);
            const dim3 g((unsigned)((count + tm - 1) / tm));
            const void* f = L == 12 ? (const void*)fft::row::k_dft2<12>
                                    : (L == 24 ? (const void*)fft::row::k_dft2<24> : (const void*)fft::row::k_dft2<48>);
            lds = L == 12 ? fft::row::lds<12>() : (L == 24 ? fft::row::lds<24>() : fft::row::lds<48>());
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (L == 12) hipLaunchKernelGGL(fft::row::k_dft2<12>, g, dim3(256), lds, s, in, count, out);
            else if (L == 24) hipLaunchKernelGGL(fft::row::k_dft2<24>, g, dim3(256), lds, s, in, count, out);
            else hipLaunchKernelGGL(fft::row::k_dft2<48>, g, dim3(256), lds, s, in, count, out);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace srmra
