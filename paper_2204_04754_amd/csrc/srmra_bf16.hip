// BF16 split-precision kernels of the EM step (bodies in srmra_bf16_impl.h).
#include "srmra_bf16_impl.h"

namespace srmra {
namespace b16 {

// NP: 3 or 4 BF16 products per multiply-add
template <int LL, int NP>
__global__ __launch_bounds__(256, 2) void k_score_lse_bf16(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    bf16_pass1_body<LL, NP>(p, q, blockIdx.x, blockIdx.y, lds);
}

template <int LL, int NP>
__global__ __launch_bounds__(256) void k_backproject_bf16(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    bf16_pass2_body<LL, NP>(p, q, blockIdx.x, blockIdx.y, lds);
}

// x as MFMA B fragments: grid (KK, k-steps / 4), 256 threads (4 k-steps per block)
template <int LL>
__global__ __launch_bounds__(256) void k_pack_xb(StepArgs p, const float* __restrict__ x,
                                                 uint4* __restrict__ xb) {
    const int ks = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ks < nk<LL>()) pack_xb_body<LL>(p, x, blockIdx.x, ks, xb);
}

}  // namespace b16


// ---------------------------------------------------------------- host side
size_t bf16_xb_bytes(int LL, int KK) {
    if (LL != 24 && LL != 32) return 0;
    return (size_t)KK * LL * (b16::R1P / 16) * 128 * sizeof(uint4);
}

hipError_t launch_pack_xb(int LL, const StepArgs& p, const float* x, void* xb, hipStream_t s) {
    const int nks = LL * (b16::R1P / 16);
    const dim3 grid(p.KK, (nks + 3) / 4);
    if (LL == 24) hipLaunchKernelGGL(b16::k_pack_xb<24>, grid, dim3(256), 0, s, p, x, (uint4*)xb);
    else if (LL == 32) hipLaunchKernelGGL(b16::k_pack_xb<32>, grid, dim3(256), 0, s, p, x, (uint4*)xb);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t bf16_prepared_extra(int LL, int64_t N) {
    if (LL != 24 && LL != 32) return 0;
    const size_t yt = (size_t)N * 2 * LL * b16::R1P * 2;
    const size_t yo = (size_t)((N + 7) / 8) * 2 * LL * LL * 8 * 2;
    return ((yt + 255) / 256) * 256 + ((yo + 255) / 256) * 256;
}

static b16::Prep prep_ptrs(const void* prep_extra, int LL, int64_t N) {
    b16::Prep q;
    const char* b = (const char*)prep_extra;
    const size_t yt = (size_t)N * 2 * LL * b16::R1P * 2;
    q.yT = (const __bf16*)b;
    q.yo = (const __bf16*)(b + ((yt + 255) / 256) * 256);
    return q;
}

hipError_t launch_prep_bf16(int LL, const float* y, int64_t N, const double* centre, double* ynorm,
                            void* prep_extra, hipStream_t s) {
    b16::Prep q = prep_ptrs(prep_extra, LL, N);
    const dim3 grid((unsigned)((N + 7) / 8));
    if (LL == 24) hipLaunchKernelGGL(b16::k_prep_bf16<24>, grid, dim3(256), 0, s, y, N, centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    else if (LL == 32) hipLaunchKernelGGL(b16::k_prep_bf16<32>, grid, dim3(256), 0, s, y, N, centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int LL, int NP>
static hipError_t launch_bf16_ll(int pass, const StepArgs& p, const b16::Prep& q, hipStream_t s) {
    const dim3 grid(p.n_chunks, p.n_cg);
    if (pass == 1) {
        const size_t lds = b16::lds_pass1<LL>();
        (void)hipFuncSetAttribute((const void*)b16::k_score_lse_bf16<LL, NP>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((b16::k_score_lse_bf16<LL, NP>), grid, dim3(256), lds, s, p, q);
    } else {
        const size_t lds = b16::lds_pass2<LL>();
        (void)hipFuncSetAttribute((const void*)b16::k_backproject_bf16<LL, NP>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((b16::k_backproject_bf16<LL, NP>), grid, dim3(256), lds, s, p, q);
    }
    return hipGetLastError();
}

hipError_t launch_bf16(int LL, int np, int pass, const StepArgs& p, const void* prep_extra,
                       hipStream_t s) {
    const b16::Prep q = prep_ptrs(prep_extra, LL, p.N);
    if (LL == 24) return np == 4 ? launch_bf16_ll<24, 4>(pass, p, q, s) : launch_bf16_ll<24, 3>(pass, p, q, s);
    if (LL == 32) return np == 4 ? launch_bf16_ll<32, 4>(pass, p, q, s) : launch_bf16_ll<32, 3>(pass, p, q, s);
    return hipErrorInvalidValue;
}

template <int LL, int NP>
static void bf16_geom_ll(size_t& lds1, size_t& lds2, const void*& f1, const void*& f2) {
    lds1 = b16::lds_pass1<LL>();
    lds2 = b16::lds_pass2<LL>();
    f1 = (const void*)b16::k_score_lse_bf16<LL, NP>;
    f2 = (const void*)b16::k_backproject_bf16<LL, NP>;
}

bool bf16_geom(int LL, int np, int& cpb, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2) {
    cpb = 4;
    nt = 8;
    if (LL == 24) {
        if (np == 4) bf16_geom_ll<24, 4>(lds1, lds2, f1, f2);
        else bf16_geom_ll<24, 3>(lds1, lds2, f1, f2);
        return true;
    }
    if (LL == 32) {
        if (np == 4) bf16_geom_ll<32, 4>(lds1, lds2, f1, f2);
        else bf16_geom_ll<32, 3>(lds1, lds2, f1, f2);
        return true;
    }
    return false;
}

}  // namespace srmra
