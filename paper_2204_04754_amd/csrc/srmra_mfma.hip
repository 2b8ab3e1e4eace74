// FP32 matrix-core kernels of the EM step (bodies in srmra_mfma_impl.h).
#include "srmra_mfma_impl.h"

namespace srmra {

template <int LL>
__global__ __launch_bounds__(256) void k_score_lse_mfma(StepArgs p) {
    extern __shared__ float lds[];
    mfma_pass1_body<LL>(p, blockIdx.x, blockIdx.y, lds);
}

// two waves per SIMD where the body fits 256 registers without spilling and two
// blocks fit the LDS
template <int LL>
__global__ __launch_bounds__(256, (LL == 8 || LL >= 48) ? 1 : 2) void k_backproject_mfma(StepArgs p) {
    extern __shared__ float lds[];
    mfma_pass2_body<LL>(p, blockIdx.x, blockIdx.y, lds);
}

// single pass for instances whose components fit in one block
template <int LL>
__global__ __launch_bounds__(256, (LL == 8 || LL >= 48) ? 1 : 2) void k_fused_mfma(StepArgs p) {
    extern __shared__ float lds[];
    mfma_fused_body<LL>(p, blockIdx.x, lds);
}

#define SRMRA_INST_MFMA(LL)                                                     \
    template __global__ void k_score_lse_mfma<LL>(StepArgs);                    \
    template __global__ void k_backproject_mfma<LL>(StepArgs);                  \
    template __global__ void k_fused_mfma<LL>(StepArgs);

SRMRA_INST_MFMA(8)
SRMRA_INST_MFMA(12)
SRMRA_INST_MFMA(16)
SRMRA_INST_MFMA(24)
SRMRA_INST_MFMA(32)
SRMRA_INST_MFMA(48)
SRMRA_INST_MFMA(64)

}  // namespace srmra

// ---------------------------------------------------------------- launchers
namespace srmra {

template <int LL>
static hipError_t launch_mfma_ll(int pass, const StepArgs& p, hipStream_t s) {
    const dim3 grid(p.n_chunks, p.n_cg);
    if (pass == 3) {
        const size_t lds = lds_fused_mfma<LL>(p.fuse_wc);
        if (lds == 0 || p.n_cg != 1) return hipErrorInvalidValue;
        (void)hipFuncSetAttribute((const void*)k_fused_mfma<LL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_fused_mfma<LL>, dim3(p.n_chunks), dim3(256), lds, s, p);
    } else if (pass == 1) {
        const size_t lds = lds_score_mfma<LL>();
        (void)hipFuncSetAttribute((const void*)k_score_lse_mfma<LL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_score_lse_mfma<LL>, grid, dim3(256), lds, s, p);
    } else {
        const size_t lds = lds_backproject_mfma<LL>();
        (void)hipFuncSetAttribute((const void*)k_backproject_mfma<LL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_backproject_mfma<LL>, grid, dim3(256), lds, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_mfma(int LL, int pass, const StepArgs& p, hipStream_t s) {
    switch (LL) {
        case 8: return launch_mfma_ll<8>(pass, p, s);
        case 12: return launch_mfma_ll<12>(pass, p, s);
        case 16: return launch_mfma_ll<16>(pass, p, s);
        case 24: return launch_mfma_ll<24>(pass, p, s);
        case 32: return launch_mfma_ll<32>(pass, p, s);
        case 48: return launch_mfma_ll<48>(pass, p, s);
        case 64: return launch_mfma_ll<64>(pass, p, s);
    }
    return hipErrorInvalidValue;
}

template <int LL> static void mfma_geom_ll(int& cpw, int& nt, size_t& lds1, size_t& lds2,
                                           const void*& f1, const void*& f2) {
    cpw = Tile<LL>::CPW;
    nt = Tile<LL>::NT;
    lds1 = lds_score_mfma<LL>();
    lds2 = lds_backproject_mfma<LL>();
    f1 = (const void*)k_score_lse_mfma<LL>;
    f2 = (const void*)k_backproject_mfma<LL>;
}

// Single-pass geometry: WC component groups of CPW per block when ceil(KK / CPW)
// is at most 4 (3 rounds up to 4, the last group idles) and the LDS fits.
template <int LL> static bool mfma_fused_geom_ll(int KK, int& wc, int& nt, size_t& lds,
                                                 const void*& f) {
    using TL = Tile<LL>;
    const int ng = (KK + TL::CPW - 1) / TL::CPW;
    wc = ng == 1 ? 1 : (ng == 2 ? 2 : (ng <= 4 ? 4 : 0));
    if (wc == 0) return false;
    lds = lds_fused_mfma<LL>(wc);
    if (lds == 0 || lds > 160 * 1024) return false;
    nt = (4 / wc) * TL::OPW;
    f = (const void*)k_fused_mfma<LL>;
    return true;
}

bool mfma_fused_geom(int LL, int KK, int& wc, int& nt, size_t& lds, const void*& f) {
    switch (LL) {
        case 8: return mfma_fused_geom_ll<8>(KK, wc, nt, lds, f);
        case 12: return mfma_fused_geom_ll<12>(KK, wc, nt, lds, f);
        case 16: return mfma_fused_geom_ll<16>(KK, wc, nt, lds, f);
        case 24: return mfma_fused_geom_ll<24>(KK, wc, nt, lds, f);
        case 32: return mfma_fused_geom_ll<32>(KK, wc, nt, lds, f);
        case 48: return mfma_fused_geom_ll<48>(KK, wc, nt, lds, f);
        case 64: return mfma_fused_geom_ll<64>(KK, wc, nt, lds, f);
    }
    return false;
}

bool mfma_geom(int LL, int& cpw, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2) {
    switch (LL) {
        case 8: mfma_geom_ll<8>(cpw, nt, lds1, lds2, f1, f2); return true;
        case 12: mfma_geom_ll<12>(cpw, nt, lds1, lds2, f1, f2); return true;
        case 16: mfma_geom_ll<16>(cpw, nt, lds1, lds2, f1, f2); return true;
        case 24: mfma_geom_ll<24>(cpw, nt, lds1, lds2, f1, f2); return true;
        case 32: mfma_geom_ll<32>(cpw, nt, lds1, lds2, f1, f2); return true;
        case 48: mfma_geom_ll<48>(cpw, nt, lds1, lds2, f1, f2); return true;
        case 64: mfma_geom_ll<64>(cpw, nt, lds1, lds2, f1, f2); return true;
    }
    return false;
}

}  // namespace srmra
