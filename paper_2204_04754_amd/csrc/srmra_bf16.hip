// BF16 split-precision kernels of the EM step (bodies in srmra_bf16_impl.h for
// L_low 24 and 32, srmra_bf16w_impl.h for L_low 48 and 64, srmra_bf16s_impl.h
// for L_low 16, srmra_bf16n_impl.h for the single pass at L_low 48, K^2 <= 4,
// srmra_bf16p_impl.h for L_low 8 and 12).
#include "../../include/srmra.h"
#include "srmra_bf16n_impl.h"
#include "srmra_bf16p_impl.h"

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

// single pass (K^2 <= 4): grid (chunks)
template <int LL, int NP>
__global__ __launch_bounds__(256) void k_fused_bf16(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    bf16_pass2_body<LL, NP, true>(p, q, blockIdx.x, 0, lds);
}

// single pass at 4 < K^2 <= 16: grid (chunks)
template <int LL, int NP>
__global__ __launch_bounds__(F16_NT, 1) void k_fused16_bf16(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    bf16_fused16_body<LL, NP>(p, q, blockIdx.x, lds);
}

// x as MFMA B fragments: grid (KK, k-steps / 4), 256 threads (4 k-steps per block)
template <int LL>
__global__ __launch_bounds__(256) void k_pack_xb(StepArgs p, const float* __restrict__ x,
                                                 uint4* __restrict__ xb) {
    const int ks = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ks < nk<LL>()) pack_xb_body<LL>(p, x, blockIdx.x, ks, xb);
}

}  // namespace b16

namespace b16w {

// Single-problem launches run a 1-D grid in which each XCD (blocks b with the
// same b mod 8) takes a contiguous range of (component, chunk) items,
// component-major, so the blocks resident on one XCD share one or two
// components' B fragments (K^2 MiB at Ll = 64) in that XCD's L2.
__device__ __forceinline__ bool xcd_item(const StepArgs& p, int per_xcd, int& chunk, int& comp) {
    const int b = blockIdx.x;
    const int idx = (b & 7) * per_xcd + (b >> 3);
    if (idx >= p.n_chunks * p.KK) return false;
    comp = idx / p.n_chunks;
    chunk = idx % p.n_chunks;
    return true;
}

template <int LL, int NP>
__global__ __launch_bounds__(256, 2) void k_score_lse(StepArgs p, Prep q, int per_xcd) {
    extern __shared__ float lds[];
    int chunk, comp;
    if (!xcd_item(p, per_xcd, chunk, comp)) return;
    pass1_body<LL, NP>(p, q, chunk, comp, lds);
}

template <int LL, int NP>
__global__ __launch_bounds__(256, 1) void k_backproject(StepArgs p, Prep q, int per_xcd) {
    extern __shared__ float lds[];
    int chunk, comp;
    if (!xcd_item(p, per_xcd, chunk, comp)) return;
    pass2_body<LL, NP>(p, q, chunk, comp, lds);
}

// grid (2 KK, k-steps / 4): block (c, tb1), 4 k-steps per block
template <int LL>
__global__ __launch_bounds__(256) void k_pack_xb(StepArgs p, const float* __restrict__ x,
                                                 uint4* __restrict__ xb) {
    const int ks = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ks < Geo<LL>::NK) pack_xb_body<LL>(p, x, blockIdx.x >> 1, blockIdx.x & 1, ks, xb);
}

}  // namespace b16w

namespace b16s {

template <int NP>
__global__ __launch_bounds__(256) void k_score_lse(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    b16s::pass1_body<NP>(p, q, blockIdx.x, blockIdx.y, lds);
}

template <int NP>
__global__ __launch_bounds__(256) void k_backproject(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    b16s::pass2_body<NP>(p, q, blockIdx.x, blockIdx.y, lds);
}


// grid (KK, 2): 4 k-steps per block
__global__ __launch_bounds__(256) void k_pack_xb(StepArgs p, const float* __restrict__ x,
                                                 uint4* __restrict__ xb) {
    const int ks = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ks < NK) pack_xb_body(p, x, blockIdx.x, ks, xb);
}

}  // namespace b16s

namespace b16n {

// single pass at L_low 48, K^2 <= 4: grid (chunks)
template <int NP>
__global__ __launch_bounds__(NT, 2) void k_fused(StepArgs p, Prep q) {
    extern __shared__ float lds[];
    fused_body<NP>(p, q, blockIdx.x, lds);
}

// grid (3 KK, k-steps / 4): block (c, tile column C), 4 k-steps per block
__global__ __launch_bounds__(256) void k_pack_xb(StepArgs p, const float* __restrict__ x,
                                                 uint4* __restrict__ xb) {
    const int s = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (s < NKS) pack_xb_body(p, x, blockIdx.x / T, blockIdx.x % T, s, xb);
}

}  // namespace b16n

namespace b16p {

template <int LL, int NP>
__global__ __launch_bounds__(256) void k_score_lse(StepArgs p, b16::Prep q) {
    extern __shared__ float lds[];
    body<LL, NP, 1>(p, q, blockIdx.x, blockIdx.y, lds);
}

template <int LL, int NP>
__global__ __launch_bounds__(256) void k_backproject(StepArgs p, b16::Prep q) {
    extern __shared__ float lds[];
    body<LL, NP, 2>(p, q, blockIdx.x, blockIdx.y, lds);
}

// single pass: grid (chunks)
template <int LL, int NP>
__global__ __launch_bounds__(256) void k_fused(StepArgs p, b16::Prep q) {
    extern __shared__ float lds[];
    body<LL, NP, 3>(p, q, blockIdx.x, 0, lds);
}

// grid (column tiles, k-steps / 4): one (column tile, k-step) per wave
template <int LL>
__global__ __launch_bounds__(256) void k_pack_xb(StepArgs p, const float* __restrict__ x, uint4* __restrict__ xb) {
    const int s = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (s < Geo<LL>::NKS) pack_xb_body<LL>(p, x, blockIdx.x, s, xb);
}

// component blocks of NCW components covering K^2, and the workgroup's block
// slots WCB of the single pass (0: two passes)
inline int n_blocks(int LL, int KK) { return (KK + ncw_of(LL) - 1) / ncw_of(LL); }
inline int fused_wcb(int LL, int KK) {
    const int nb = n_blocks(LL, KK);
    return nb <= 1 ? 1 : (nb <= 2 ? 2 : (nb <= 4 ? 4 : 0));
}

}  // namespace b16p


// ---------------------------------------------------------------- host side
static bool wide_ll(int LL) { return LL == 48 || LL == 64; }
// L_low 48 with all components in one workgroup (cpb 4): the 16 x 16-tile
// single pass (the two-pass form at L_low 48 takes one component per block)
static bool nine_tile(int LL, int cpb) { return LL == 48 && cpb == b16n::NW; }
static bool packed_ll(int LL) { return LL == 8 || LL == 12; }
bool bf16_supported(int LL) { return packed_ll(LL) || LL == 16 || LL == 24 || LL == 32 || wide_ll(LL); }

// pass-1 partials per observation: one per component pair (one-tile form), per
// (component, tile) (L_low 48 and 64) or per group of 4 components (L_low 16)
int bf16_parts(int LL, int KK) {
    if (LL == 16) return (KK + 3) / 4;
    if (packed_ll(LL)) return 4 * ((KK + 4 * b16p::ncw_of(LL) - 1) / (4 * b16p::ncw_of(LL)));   // one per wave
    return wide_ll(LL) ? 4 * KK : (KK + 1) / 2;
}

size_t bf16_xb_bytes(int LL, int KK) {
    if (LL == 16) return (size_t)KK * b16s::NK * 128 * sizeof(uint4);
    if (LL == 8) return (size_t)b16p::n_blocks(8, KK) * b16p::Geo<8>::NCT * b16p::Geo<8>::NKS * 128 * sizeof(uint4);
    if (LL == 12)
        return (size_t)b16p::n_blocks(12, KK) * b16p::Geo<12>::NCT * b16p::Geo<12>::NKS * 128 * sizeof(uint4);
    if (wide_ll(LL)) return (size_t)KK * 2 * LL * (LL / 16) * 128 * sizeof(uint4);
    if (LL != 24 && LL != 32) return 0;
    return (size_t)KK * LL * (b16::R1P / 16) * 128 * sizeof(uint4);
}

hipError_t launch_pack_xb(int LL, const StepArgs& p, const float* x, void* xb, hipStream_t s) {
    if (LL == 8) {
        using G = b16p::Geo<8>;
        hipLaunchKernelGGL(b16p::k_pack_xb<8>, dim3(b16p::n_blocks(8, p.KK) * G::NCT, (G::NKS + 3) / 4), dim3(256), 0,
                           s, p, x, (uint4*)xb);
        return hipGetLastError();
    }
    if (LL == 12) {
        using G = b16p::Geo<12>;
        hipLaunchKernelGGL(b16p::k_pack_xb<12>, dim3(b16p::n_blocks(12, p.KK) * G::NCT, (G::NKS + 3) / 4), dim3(256),
                           0, s, p, x, (uint4*)xb);
        return hipGetLastError();
    }
    if (LL == 16) {
        hipLaunchKernelGGL(b16s::k_pack_xb, dim3(p.KK, 2), dim3(256), 0, s, p, x, (uint4*)xb);
        return hipGetLastError();
    }
    if (nine_tile(LL, p.cpb)) {
        hipLaunchKernelGGL(b16n::k_pack_xb, dim3(b16n::T * p.KK, (b16n::NKS + 3) / 4), dim3(256), 0, s, p, x,
                           (uint4*)xb);
        return hipGetLastError();
    }
    if (wide_ll(LL)) {
        const int nks = LL * (LL / 16);
        const dim3 grid(2 * p.KK, (nks + 3) / 4);
        if (LL == 48) hipLaunchKernelGGL(b16w::k_pack_xb<48>, grid, dim3(256), 0, s, p, x, (uint4*)xb);
        else hipLaunchKernelGGL(b16w::k_pack_xb<64>, grid, dim3(256), 0, s, p, x, (uint4*)xb);
        return hipGetLastError();
    }
    const int nks = LL * (b16::R1P / 16);
    const dim3 grid(p.KK, (nks + 3) / 4);
    if (LL == 24) hipLaunchKernelGGL(b16::k_pack_xb<24>, grid, dim3(256), 0, s, p, x, (uint4*)xb);
    else if (LL == 32) hipLaunchKernelGGL(b16::k_pack_xb<32>, grid, dim3(256), 0, s, p, x, (uint4*)xb);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// bytes of the yT planes (the first prepared layout)
size_t bf16_yt_bytes(int LL, int64_t N) {
    return (size_t)N * 2 * LL * ((wide_ll(LL) || LL == 16 || packed_ll(LL)) ? LL : b16::R1P) * 2;
}

size_t bf16_prepared_extra(int LL, int64_t N) {
    if (!bf16_supported(LL)) return 0;
    const size_t yt = bf16_yt_bytes(LL, N);
    const size_t yo = (size_t)((N + 7) / 8) * 2 * LL * LL * 8 * 2;
    return ((yt + 255) / 256) * 256 + ((yo + 255) / 256) * 256;
}

static b16::Prep prep_ptrs(const void* prep_extra, int LL, int64_t N) {
    b16::Prep q;
    const char* b = (const char*)prep_extra;
    q.yT = (const __bf16*)b;
    q.yo = (const __bf16*)(b + ((bf16_yt_bytes(LL, N) + 255) / 256) * 256);
    return q;
}

template <int LL>
static hipError_t launch_prep_wide(const float* y, int64_t N, const double* centre, double* ynorm,
                                   const b16::Prep& q, hipStream_t s) {
    const size_t lds = b16w::lds_prep<LL>();
    if (hipFuncSetAttribute((const void*)b16w::k_prep<LL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(b16w::k_prep<LL>, dim3((unsigned)((N + 7) / 8)), dim3(256), lds, s, y, N,
                       centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    return hipGetLastError();
}

hipError_t launch_prep_bf16(int LL, const float* y, int64_t N, const double* centre, double* ynorm,
                            void* prep_extra, hipStream_t s) {
    b16::Prep q = prep_ptrs(prep_extra, LL, N);
    const dim3 grid((unsigned)((N + 7) / 8));
    if (LL == 16) return launch_prep_wide<16>(y, N, centre, ynorm, q, s);   // same layouts, one r1 slice
    if (LL == 48) return launch_prep_wide<48>(y, N, centre, ynorm, q, s);
    if (LL == 64) return launch_prep_wide<64>(y, N, centre, ynorm, q, s);
    if (LL == 8) hipLaunchKernelGGL((b16::k_prep_bf16<8, true>), grid, dim3(256), 0, s, y, N, centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    else if (LL == 12) hipLaunchKernelGGL((b16::k_prep_bf16<12, true>), grid, dim3(256), 0, s, y, N, centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    else if (LL == 24) hipLaunchKernelGGL(b16::k_prep_bf16<24>, grid, dim3(256), 0, s, y, N, centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    else if (LL == 32) hipLaunchKernelGGL(b16::k_prep_bf16<32>, grid, dim3(256), 0, s, y, N, centre, (__bf16*)q.yT, (__bf16*)q.yo, ynorm);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int LL, int NP>
static hipError_t launch_bf16_ll(int pass, const StepArgs& p, const b16::Prep& q, hipStream_t s) {
    if (pass == 3 && p.cpb == b16::F16_NCW * b16::F16_NW) {   // 16 component slots: 512 threads
        const size_t lds = b16::lds_fused16<LL>();
        if (hipFuncSetAttribute((const void*)b16::k_fused16_bf16<LL, NP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((b16::k_fused16_bf16<LL, NP>), dim3(p.n_chunks), dim3(b16::F16_NT), lds, s, p, q);
        return hipGetLastError();
    }
    if (pass == 3) {
        const size_t lds = b16::lds_fused<LL>();
        if (hipFuncSetAttribute((const void*)b16::k_fused_bf16<LL, NP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((b16::k_fused_bf16<LL, NP>), dim3(p.n_chunks), dim3(256), lds, s, p, q);
        return hipGetLastError();
    }
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

template <int LL, int NP>
static hipError_t launch_bf16w_ll(int pass, const StepArgs& p, const b16::Prep& q0, hipStream_t s) {
    b16w::Prep q;
    q.yT = q0.yT;
    q.yo = q0.yo;
    const int per_xcd = (p.n_chunks * p.KK + 7) / 8;
    const dim3 grid(8 * per_xcd);
    const void* f = pass == 1 ? (const void*)b16w::k_score_lse<LL, NP> : (const void*)b16w::k_backproject<LL, NP>;
    const size_t lds = pass == 1 ? b16w::lds_pass1<LL>() : b16w::lds_pass2<LL>();
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    if (pass == 1) hipLaunchKernelGGL((b16w::k_score_lse<LL, NP>), grid, dim3(256), lds, s, p, q, per_xcd);
    else hipLaunchKernelGGL((b16w::k_backproject<LL, NP>), grid, dim3(256), lds, s, p, q, per_xcd);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_bf16s(int pass, const StepArgs& p, const b16::Prep& q0, hipStream_t s) {
    b16s::Prep q;
    q.yT = q0.yT;
    q.yo = q0.yo;
    const dim3 grid(p.n_chunks, p.n_cg);
    const void* f = pass == 1 ? (const void*)b16s::k_score_lse<NP> : (const void*)b16s::k_backproject<NP>;
    const size_t lds = pass == 1 ? b16s::lds_pass1() : b16s::lds_pass2();
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    if (pass == 1) hipLaunchKernelGGL((b16s::k_score_lse<NP>), grid, dim3(256), lds, s, p, q);
    else hipLaunchKernelGGL((b16s::k_backproject<NP>), grid, dim3(256), lds, s, p, q);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_bf16n(const StepArgs& p, const b16::Prep& q0, hipStream_t s) {
    b16n::Prep q;
    q.yT = q0.yT;
    q.yo = q0.yo;
    const size_t lds = b16n::lds_fused();
    if (hipFuncSetAttribute((const void*)b16n::k_fused<NP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(b16n::k_fused<NP>, dim3(p.n_chunks), dim3(b16n::NT), lds, s, p, q);
    return hipGetLastError();
}

template <int LL, int NP>
static hipError_t launch_bf16p(int pass, const StepArgs& p, const b16::Prep& q, hipStream_t s) {
    const size_t lds = b16p::lds_bytes<LL>();
    const void* f = pass == 1 ? (const void*)b16p::k_score_lse<LL, NP>
                  : (pass == 2 ? (const void*)b16p::k_backproject<LL, NP> : (const void*)b16p::k_fused<LL, NP>);
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    if (pass == 1) hipLaunchKernelGGL((b16p::k_score_lse<LL, NP>), dim3(p.n_chunks, p.n_cg), dim3(256), lds, s, p, q);
    else if (pass == 2) hipLaunchKernelGGL((b16p::k_backproject<LL, NP>), dim3(p.n_chunks, p.n_cg), dim3(256), lds, s, p, q);
    else hipLaunchKernelGGL((b16p::k_fused<LL, NP>), dim3(p.n_chunks), dim3(256), lds, s, p, q);
    return hipGetLastError();
}

hipError_t launch_bf16(int LL, int np, int pass, const StepArgs& p, const void* prep_extra,
                       hipStream_t s) {
    const b16::Prep q = prep_ptrs(prep_extra, LL, p.N);
    if (LL == 8) return np == 4 ? launch_bf16p<8, 4>(pass, p, q, s) : launch_bf16p<8, 3>(pass, p, q, s);
    if (LL == 12) return np == 4 ? launch_bf16p<12, 4>(pass, p, q, s) : launch_bf16p<12, 3>(pass, p, q, s);
    if (pass == 3 && nine_tile(LL, p.cpb)) return np == 4 ? launch_bf16n<4>(p, q, s) : launch_bf16n<3>(p, q, s);
    if (LL == 16) return np == 4 ? launch_bf16s<4>(pass, p, q, s) : launch_bf16s<3>(pass, p, q, s);
    if (LL == 48) return np == 4 ? launch_bf16w_ll<48, 4>(pass, p, q, s) : launch_bf16w_ll<48, 3>(pass, p, q, s);
    if (LL == 64) return np == 4 ? launch_bf16w_ll<64, 4>(pass, p, q, s) : launch_bf16w_ll<64, 3>(pass, p, q, s);
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

template <int LL, int NP>
static void bf16w_geom_ll(size_t& lds1, size_t& lds2, const void*& f1, const void*& f2) {
    lds1 = b16w::lds_pass1<LL>();
    lds2 = b16w::lds_pass2<LL>();
    f1 = (const void*)b16w::k_score_lse<LL, NP>;
    f2 = (const void*)b16w::k_backproject<LL, NP>;
}

// The single pass when one workgroup holds all K^2 components of its
// observations: L_low 24 / 32 with K^2 <= 4 (8 observations x 4 components
// per workgroup) and with 4 < K^2 <= 16 (4 observations x 16 components;
// cpb and nt are set to that tile); L_low 48 with K^2 <= 4 (4 observations x
// 4 components on 16 x 16 tiles).  (At L_low 16 a single pass that
// keeps the scores of 8 observations x 4 components across the block's
// (max, sum) exchange spilled registers and measured no faster than the two
// passes, slower inside the batched form; L_low 16 keeps two passes.)
bool bf16_fused_geom(int LL, int KK, int np, int tile, int& cpb, int& nt, size_t& lds, const void*& f) {
    if (packed_ll(LL)) {
        // L_low 8 / 12: all components in one workgroup while they fit in 4 blocks
        const int wcb = b16p::fused_wcb(LL, KK);
        if (tile != 0 || wcb == 0) return false;
        cpb = wcb * b16p::ncw_of(LL);
        nt = 8 * (4 / wcb);
        if (LL == 8) {
            lds = b16p::lds_bytes<8>();
            f = np == 4 ? (const void*)b16p::k_fused<8, 4> : (const void*)b16p::k_fused<8, 3>;
        } else {
            lds = b16p::lds_bytes<12>();
            f = np == 4 ? (const void*)b16p::k_fused<12, 4> : (const void*)b16p::k_fused<12, 3>;
        }
        return true;
    }
    // the layout: the default for the shape, or the one the tile asks for
    const bool small = (LL == 24 || LL == 32) && KK <= 4;
    const bool wide = (LL == 24 || LL == 32) && KK <= b16::F16_NCW * b16::F16_NW;
    bool use_nine = false, use_small = false, use_wide = false;
    if (tile == 0) {
        use_nine = LL == 48 && KK <= b16n::NW;
        use_small = small;
        use_wide = wide && !small;
    } else {
        use_nine = tile == SRMRA_TILE_16X16 && LL == 48 && KK <= b16n::NW;
        use_small = tile == SRMRA_TILE_FUSED_8OBS && small;
        use_wide = tile == SRMRA_TILE_FUSED_4OBS && wide;
    }
    if (use_nine) {
        cpb = b16n::NW;
        nt = b16n::NOB;
        lds = b16n::lds_fused();
        f = np == 4 ? (const void*)b16n::k_fused<4> : (const void*)b16n::k_fused<3>;
        return true;
    }
    if (use_wide) {
        cpb = b16::F16_NCW * b16::F16_NW;
        nt = b16::F16_NOB;
        if (LL == 24) {
            lds = b16::lds_fused16<24>();
            f = np == 4 ? (const void*)b16::k_fused16_bf16<24, 4> : (const void*)b16::k_fused16_bf16<24, 3>;
        } else {
            lds = b16::lds_fused16<32>();
            f = np == 4 ? (const void*)b16::k_fused16_bf16<32, 4> : (const void*)b16::k_fused16_bf16<32, 3>;
        }
        return true;
    }
    if (use_small) {
        if (LL == 24) {
            lds = b16::lds_fused<24>();
            f = np == 4 ? (const void*)b16::k_fused_bf16<24, 4> : (const void*)b16::k_fused_bf16<24, 3>;
        } else {
            lds = b16::lds_fused<32>();
            f = np == 4 ? (const void*)b16::k_fused_bf16<32, 4> : (const void*)b16::k_fused_bf16<32, 3>;
        }
        return true;
    }
    (void)np;
    return false;
}

bool bf16_geom(int LL, int KK, int np, int tile, int& cpb, int& nt, size_t& lds1, size_t& lds2,
               const void*& f1, const void*& f2) {
    cpb = 4;
    nt = 8;
    // tile: the block layout where the form has a choice (L_low 16: component
    // slots WC in {1, 2, 4}; L_low 24 / 32 and 48: the single passes the shape
    // allows, or two passes); 0 = the default
    if (tile != 0) {
        bool valid = false;
        if (packed_ll(LL)) valid = tile == SRMRA_TILE_TWO_PASS;
        if (LL == 16) valid = tile == 1 || tile == 2 || tile == 4;
        if (LL == 24 || LL == 32)
            valid = tile == SRMRA_TILE_TWO_PASS || (tile == SRMRA_TILE_FUSED_8OBS && KK <= 4) ||
                    (tile == SRMRA_TILE_FUSED_4OBS && KK <= b16::F16_NCW * b16::F16_NW);
        if (LL == 48) valid = (tile == SRMRA_TILE_TWO_PASS || tile == SRMRA_TILE_16X16) && KK <= b16n::NW;
        if (!valid) return false;
    }
    if (packed_ll(LL)) {
        // two passes: 4 blocks of NCW components per workgroup, 8 observations
        cpb = 4 * b16p::ncw_of(LL);
        nt = 8;
        if (LL == 8) {
            lds1 = lds2 = b16p::lds_bytes<8>();
            f1 = np == 4 ? (const void*)b16p::k_score_lse<8, 4> : (const void*)b16p::k_score_lse<8, 3>;
            f2 = np == 4 ? (const void*)b16p::k_backproject<8, 4> : (const void*)b16p::k_backproject<8, 3>;
        } else {
            lds1 = lds2 = b16p::lds_bytes<12>();
            f1 = np == 4 ? (const void*)b16p::k_score_lse<12, 4> : (const void*)b16p::k_score_lse<12, 3>;
            f2 = np == 4 ? (const void*)b16p::k_backproject<12, 4> : (const void*)b16p::k_backproject<12, 3>;
        }
        return true;
    }
    if (LL == 16) {
        const int wc = tile ? tile : b16s::wc_of(KK);
        cpb = 4 * wc;
        nt = 8 * (4 / wc);
        lds1 = b16s::lds_pass1();
        lds2 = b16s::lds_pass2();
        f1 = np == 4 ? (const void*)b16s::k_score_lse<4> : (const void*)b16s::k_score_lse<3>;
        f2 = np == 4 ? (const void*)b16s::k_backproject<4> : (const void*)b16s::k_backproject<3>;
        return true;
    }
    if (wide_ll(LL)) {
        cpb = 1;   // one component per block, one tile per wave
        if (LL == 48) {
            if (np == 4) bf16w_geom_ll<48, 4>(lds1, lds2, f1, f2);
            else bf16w_geom_ll<48, 3>(lds1, lds2, f1, f2);
        } else {
            if (np == 4) bf16w_geom_ll<64, 4>(lds1, lds2, f1, f2);
            else bf16w_geom_ll<64, 3>(lds1, lds2, f1, f2);
        }
        return true;
    }
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
