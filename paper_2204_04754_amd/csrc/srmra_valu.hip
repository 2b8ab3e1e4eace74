// Plain FP32 (vector ALU) kernels of the EM step (bodies in srmra_valu_impl.h).
#include "srmra_valu_impl.h"

namespace srmra {

template <int LL>
__global__ __launch_bounds__(256) void k_score_lse_valu(StepArgs p) {
    extern __shared__ float lds[];
    valu_pass1_body<LL>(p, blockIdx.x, blockIdx.y, lds);
}

template <int LL>
__global__ __launch_bounds__(256) void k_backproject_valu(StepArgs p) {
    extern __shared__ float lds[];
    valu_pass2_body<LL>(p, blockIdx.x, blockIdx.y, lds);
}

#define SRMRA_INST_VALU(LL)                                                     \
    template __global__ void k_score_lse_valu<LL>(StepArgs);                    \
    template __global__ void k_backproject_valu<LL>(StepArgs);

SRMRA_INST_VALU(8)
SRMRA_INST_VALU(12)
SRMRA_INST_VALU(16)
SRMRA_INST_VALU(24)
SRMRA_INST_VALU(32)
SRMRA_INST_VALU(48)
SRMRA_INST_VALU(64)

}  // namespace srmra

// ---------------------------------------------------------------- launchers
namespace srmra {

template <int LL> static size_t lds_valu(int pass, int cpb, int nt) {
    using V = Valu<LL>;
    size_t f = (size_t)cpb * V::XS + (size_t)nt * V::YS;
    if (pass == 1) f += 2 * 256 * V::NOV;
    else f += (size_t)nt * cpb * LL * LL;
    f = f < 256 * 16 ? 256 * 16 : f;
    return f * sizeof(float);
}

template <int LL>
static hipError_t launch_valu_ll(int pass, const StepArgs& p, hipStream_t s) {
    const dim3 grid(p.n_chunks, p.n_cg);
    const size_t lds = lds_valu<LL>(pass, p.cpb, p.ntile);
    if (pass == 1) {
        (void)hipFuncSetAttribute((const void*)k_score_lse_valu<LL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_score_lse_valu<LL>, grid, dim3(256), lds, s, p);
    } else {
        (void)hipFuncSetAttribute((const void*)k_backproject_valu<LL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_backproject_valu<LL>, grid, dim3(256), lds, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_valu(int LL, int pass, const StepArgs& p, hipStream_t s) {
    switch (LL) {
        case 8: return launch_valu_ll<8>(pass, p, s);
        case 12: return launch_valu_ll<12>(pass, p, s);
        case 16: return launch_valu_ll<16>(pass, p, s);
        case 24: return launch_valu_ll<24>(pass, p, s);
        case 32: return launch_valu_ll<32>(pass, p, s);
        case 48: return launch_valu_ll<48>(pass, p, s);
        case 64: return launch_valu_ll<64>(pass, p, s);
    }
    return hipErrorInvalidValue;
}

template <int LL> static void valu_geom_ll(int KK, int& cpb, int& nt, size_t& lds1, size_t& lds2,
                                           const void*& f1, const void*& f2) {
    using V = Valu<LL>;
    cpb = 256 / V::BLK;
    if (cpb < 1) cpb = 1;
    if (cpb > KK) cpb = KK;
    int groups = 256 / (cpb * V::BLK);
    if (groups < 1) groups = 1;
    nt = groups * V::NOV;
    lds1 = lds_valu<LL>(1, cpb, nt);
    lds2 = lds_valu<LL>(2, cpb, nt);
    f1 = (const void*)k_score_lse_valu<LL>;
    f2 = (const void*)k_backproject_valu<LL>;
}

bool valu_geom(int LL, int KK, int& cpb, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2) {
    switch (LL) {
        case 8: valu_geom_ll<8>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
        case 12: valu_geom_ll<12>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
        case 16: valu_geom_ll<16>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
        case 24: valu_geom_ll<24>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
        case 32: valu_geom_ll<32>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
        case 48: valu_geom_ll<48>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
        case 64: valu_geom_ll<64>(KK, cpb, nt, lds1, lds2, f1, f2); return true;
    }
    return false;
}

}  // namespace srmra
