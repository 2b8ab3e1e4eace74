// Batched form: one EM step of many independent instances (uneven L_low, K, N,
// sigma).  Work items (instance, observation chunk, component group) are
// grouped by (form, L_low) class and sorted by cost (largest first) on the
// host; each pass is one persistent launch per class, whose blocks take items
// through an atomic counter.  Each item runs exactly the device body of the
// single-instance kernels, so an instance's result does not depend on which
// other instances share the launch.  (One kernel per class keeps each body's
// own register allocation; a single kernel switching over all bodies spills.)
#include "srmra_aux_impl.h"
#include "srmra_batch.h"
#include "srmra_bf16n_impl.h"
#include "srmra_bf16p_impl.h"
#include "srmra_fftp_impl.h"
#include "srmra_mfma_impl.h"
#include "srmra_valu_impl.h"

namespace srmra {

__global__ void k_batch_reset(int* counters, int n) {
    if (threadIdx.x < n) counters[threadIdx.x] = 0;
}

// a1 for every (instance, component) item
__global__ __launch_bounds__(256) void k_batch_pack(const InstDesc* __restrict__ D,
                                                    const int2* __restrict__ items) {
    __shared__ double red[256];
    const int2 it = items[blockIdx.x];
    const InstDesc& d = D[it.x];
    pack_x_body(d.x, d.log_rho, d.p.K, d.LL, d.p.inv_2s2, d.p.centre, d.xt2_w, d.beta_w, it.y, red);
}

// the FFT form's X_c = DFT(x_c - mu) of component c (dynamic LDS: an L x (L + 1)
// transpose buffer and the twiddle table)
template <int L>
__device__ __forceinline__ void fft_pack_x(const InstDesc& d, int c, float2* sh) {
    float2* tw = sh + L * (L + 1);
    fft::make_twiddles_n<L, L>(tw);
    __syncthreads();
    fft::pack_x_body<L>(d.x, d.p.K, d.p.centre, d.xhat, c, sh, tw);
}

// BF16-form instances: x as MFMA B fragments, every k-step of one component;
// FFT-form instances: the DFT of one component
__global__ __launch_bounds__(256) void k_batch_pack_xb(const InstDesc* __restrict__ D,
                                                       const int2* __restrict__ items) {
    extern __shared__ float2 sh[];
    const int2 it = items[blockIdx.x];
    const InstDesc& d = D[it.x];
    if (d.form == FORM_FFT) {
        switch (d.LL) {
            case 8: fft_pack_x<8>(d, it.y, sh); break;
            case 12: fft_pack_x<12>(d, it.y, sh); break;
            case 16: fft_pack_x<16>(d, it.y, sh); break;
            case 24: fft_pack_x<24>(d, it.y, sh); break;
            case 32: fft_pack_x<32>(d, it.y, sh); break;
            case 48: fft_pack_x<48>(d, it.y, sh); break;
            case 64: fft_pack_x<64>(d, it.y, sh); break;
        }
        return;
    }
    if (d.form != FORM_BF16 && d.form != FORM_BF16X4 && d.form != FORM_BF16F && d.form != FORM_BF16X4F &&
        d.form != FORM_BF16W && d.form != FORM_BF16X4W)
        return;
    uint4* xb = const_cast<uint4*>(d.p.xb);
    if (d.LL == 8 || d.LL == 12) {
        // item component c packs component block c (its NCT column tiles), if there is one
        const int ncw = b16p::ncw_of(d.LL);
        if (it.y * ncw >= d.p.KK) return;
        if (d.LL == 8) {
            using G = b16p::Geo<8>;
            for (int e = threadIdx.x >> 6; e < G::NCT * G::NKS; e += 4)
                b16p::pack_xb_body<8>(d.p, d.x, it.y * G::NCT + e / G::NKS, e % G::NKS, xb);
        } else {
            using G = b16p::Geo<12>;
            for (int e = threadIdx.x >> 6; e < G::NCT * G::NKS; e += 4)
                b16p::pack_xb_body<12>(d.p, d.x, it.y * G::NCT + e / G::NKS, e % G::NKS, xb);
        }
    } else if (d.LL == 16) {
        for (int ks = threadIdx.x >> 6; ks < b16s::NK; ks += 4) b16s::pack_xb_body(d.p, d.x, it.y, ks, xb);
    } else if (d.LL == 48 && (d.form == FORM_BF16F || d.form == FORM_BF16X4F)) {
        for (int e = threadIdx.x >> 6; e < b16n::T * b16n::NKS; e += 4)
            b16n::pack_xb_body(d.p, d.x, it.y, e / b16n::NKS, e % b16n::NKS, xb);
    } else if (d.LL == 48 || d.LL == 64) {
        const int nk = d.LL * (d.LL / 16);
        for (int e = threadIdx.x >> 6; e < 2 * nk; e += 4) {
            if (d.LL == 48) b16w::pack_xb_body<48>(d.p, d.x, it.y, e / nk, e % nk, xb);
            else b16w::pack_xb_body<64>(d.p, d.x, it.y, e / nk, e % nk, xb);
        }
    } else if (d.LL == 24) {
        for (int ks = threadIdx.x >> 6; ks < b16::nk<24>(); ks += 4) b16::pack_xb_body<24>(d.p, d.x, it.y, ks, xb);
    } else {
        for (int ks = threadIdx.x >> 6; ks < b16::nk<32>(); ks += 4) b16::pack_xb_body<32>(d.p, d.x, it.y, ks, xb);
    }
}

__global__ __launch_bounds__(256) void k_batch_combine(const InstDesc* __restrict__ D,
                                                       const int2* __restrict__ items) {
    __shared__ double red[256];
    const int2 it = items[blockIdx.x];
    const InstDesc& d = D[it.x];
    lse_combine_body(d.p.part, d.n_part, d.p.N, d.p.ynorm, d.p.inv_2s2, d.p.lse, d.llpart,
                     nullptr, it.y, red);
}

__global__ __launch_bounds__(256) void k_batch_reduce(const InstDesc* __restrict__ D,
                                                      const int2* __restrict__ items) {
    __shared__ double red[512];
    const int2 it = items[blockIdx.x];
    const InstDesc& d = D[it.x];
    reduce_partials_body(d.p.bpart, d.p.cpart, d.p.n_chunks, d.p.KK * d.LL * d.LL, d.bsum, d.csum,
                         it.y, red);
}

// the FFT form: FP64 sums of the complex back-projection partials and of the
// posterior mass over chunks (items (instance, block)), then the FP64 inverse
// DFT of each component's back-projection (items (instance, component))
__global__ __launch_bounds__(256) void k_batch_fft_reduce(const InstDesc* __restrict__ D,
                                                          const int2* __restrict__ items) {
    __shared__ double red[3 * 256];
    const int2 it = items[blockIdx.x];
    const InstDesc& d = D[it.x];
    fft::reduce_body(reinterpret_cast<const float2*>(d.p.bpart), d.p.cpart, d.p.n_chunks,
                     d.p.KK * d.LL * d.LL, d.bh, d.csum, it.y, red);
}

__global__ __launch_bounds__(256) void k_batch_fft_idft(const InstDesc* __restrict__ D,
                                                        const int2* __restrict__ items) {
    extern __shared__ double2 T[];
    const int2 it = items[blockIdx.x];
    const InstDesc& d = D[it.x];
    switch (d.LL) {
        case 8: fft::idft_body<8>(d.bh, d.bsum, it.y, T); break;
        case 12: fft::idft_body<12>(d.bh, d.bsum, it.y, T); break;
        case 16: fft::idft_body<16>(d.bh, d.bsum, it.y, T); break;
        case 24: fft::idft_body<24>(d.bh, d.bsum, it.y, T); break;
        case 32: fft::idft_body<32>(d.bh, d.bsum, it.y, T); break;
        case 48: fft::idft_body<48>(d.bh, d.bsum, it.y, T); break;
        case 64: fft::idft_body<64>(d.bh, d.bsum, it.y, T); break;
    }
}

__global__ __launch_bounds__(1024) void k_batch_finalize(const InstDesc* __restrict__ D) {
    __shared__ double Ac[256];
    __shared__ double red[1024];
    const InstDesc& d = D[blockIdx.x];
    finalize_body(d.bsum, d.csum, d.p.K, d.LL, d.x, d.p.centre, d.llpart, d.n_ll, d.x_new,
                  d.rho_new, d.log_rho_new, d.loglik, nullptr, nullptr, Ac, red);
}

// Persistent pass kernel of one (form, L_low) class: every block takes items
// from the class's cost-sorted list through an atomic counter and leaves the
// loop once the counter passes the item count (every wave reaches the exit).
template <int PASS, int FORM, int LL>
__global__ __launch_bounds__(256, ((PASS == 1 && (FORM == FORM_BF16 || FORM == FORM_BF16X4) && LL != 16) ||
                                   (PASS == 2 && FORM == FORM_MFMA && LL >= 16 && LL <= 32) ||
                                   (PASS == 2 && FORM == FORM_FUSED && LL >= 16 && LL <= 24) ||
                                   ((FORM == FORM_BF16F || FORM == FORM_BF16X4F) && LL == 48) ||
                                   (FORM == FORM_FFT && (LL == 12 || LL == 24 || LL == 48))) ? 2 : 1)
void k_class_pass(const InstDesc* __restrict__ D,
                                                    const int4* __restrict__ items, int n_items,
                                                    int* __restrict__ counter) {
    // The work-item index is broadcast through the first word of the body's LDS
    // area: between the barrier that ends one item and the barrier after the
    // read, no body is using it.  (The largest body needs the full 160 KB.)
    extern __shared__ float lds[];
    int* next = reinterpret_cast<int*>(lds);
    for (;;) {
        if (threadIdx.x == 0) *next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = *next;
        __syncthreads();
        if (it >= n_items) break;
        const int4 w = items[it];
        const InstDesc& d = D[w.x];
        if constexpr (FORM == FORM_BF16 || FORM == FORM_BF16X4) {
            constexpr int NP = FORM == FORM_BF16X4 ? 4 : 3;
            b16::Prep q;
            q.yT = d.yT;
            q.yo = d.yo;
            if constexpr (LL == 8 || LL == 12) {
                b16p::body<LL, NP, PASS>(d.p, q, w.y, w.z, lds);
            } else if constexpr (LL == 16) {
                b16s::Prep qs;
                qs.yT = d.yT;
                qs.yo = d.yo;
                if constexpr (PASS == 1) b16s::pass1_body<NP>(d.p, qs, w.y, w.z, lds);
                else b16s::pass2_body<NP>(d.p, qs, w.y, w.z, lds);
            } else if constexpr (LL >= 48) {
                b16w::Prep qw;
                qw.yT = d.yT;
                qw.yo = d.yo;
                if constexpr (PASS == 1) b16w::pass1_body<LL, NP>(d.p, qw, w.y, w.z, lds);
                else b16w::pass2_body<LL, NP>(d.p, qw, w.y, w.z, lds);
            } else {
                if constexpr (PASS == 1) b16::bf16_pass1_body<LL, NP>(d.p, q, w.y, w.z, lds);
                else b16::bf16_pass2_body<LL, NP>(d.p, q, w.y, w.z, lds);
            }
        } else if constexpr (FORM == FORM_BF16F || FORM == FORM_BF16X4F) {
            constexpr int NP = FORM == FORM_BF16X4F ? 4 : 3;
            if constexpr (LL == 48) {
                b16n::Prep qn;
                qn.yT = d.yT;
                qn.yo = d.yo;
                b16n::fused_body<NP>(d.p, qn, w.y, lds);
            } else if constexpr (LL == 8 || LL == 12) {
                b16::Prep q;
                q.yT = d.yT;
                q.yo = d.yo;
                b16p::body<LL, NP, 3>(d.p, q, w.y, 0, lds);
            } else {
                b16::Prep q;
                q.yT = d.yT;
                q.yo = d.yo;
                b16::bf16_pass2_body<LL, NP, true>(d.p, q, w.y, 0, lds);
            }
        } else if constexpr (FORM == FORM_FFT) {
            float2* sh = reinterpret_cast<float2*>(lds);
            float2* bpart = reinterpret_cast<float2*>(d.p.bpart);
            if constexpr (LL == 64) {
                if constexpr (PASS == 1) fft::pass1_quad_body(d.p, d.yhat, d.xhat, w.y, w.z, d.p.n_cg, sh);
                else fft::pass2_quad_body(d.p, d.yhat, d.xhat, bpart, d.p.cpart, w.y, w.z, sh);
            } else if constexpr (LL % 3 == 0) {
                if constexpr (PASS == 1) fft::row::pass1_body<LL>(d.p, d.yhat, d.xhat, w.y, w.z, d.p.n_cg, sh);
                else if constexpr (LL == 48)
                    fft::wpair::pass2_body<LL>(d.p, d.yhat, d.xhat, fft::tpc_of(LL, d.p.KK), bpart, d.p.cpart,
                                               w.y, w.z, sh);
                else fft::row::pass2_body<LL>(d.p, d.yhat, d.xhat, fft::tpc_of(LL, d.p.KK), bpart, d.p.cpart,
                                              w.y, w.z, sh);
            } else {
                if constexpr (PASS == 1) fft::pass1_pairs_body<LL>(d.p, d.yhat, d.xhat, w.y, w.z, d.p.n_cg, sh);
                else fft::pass2_pairs_body<LL, LL == 32>(d.p, d.yhat, d.xhat, fft::tpc_of(LL, d.p.KK), bpart,
                                                          d.p.cpart, w.y, w.z, sh);
            }
        } else if constexpr (FORM == FORM_FUSED) {
            mfma_fused_body<LL>(d.p, w.y, lds);
        } else if constexpr (FORM == FORM_MFMA) {
            if constexpr (PASS == 1) mfma_pass1_body<LL>(d.p, w.y, w.z, lds);
            else mfma_pass2_body<LL>(d.p, w.y, w.z, lds);
        } else {
            if constexpr (PASS == 1) valu_pass1_body<LL>(d.p, w.y, w.z, lds);
            else valu_pass2_body<LL>(d.p, w.y, w.z, lds);
        }
        __syncthreads();
    }
}

// The BF16 single pass at 4 < K^2 <= 16 (512-thread workgroups), persistent
// over its class's items like k_class_pass.
template <int NP, int LL>
__global__ __launch_bounds__(b16::F16_NT, 1) void k_class_fused16(const InstDesc* __restrict__ D,
                                                                   const int4* __restrict__ items,
                                                                   int n_items, int* __restrict__ counter) {
    extern __shared__ float lds[];
    int* next = reinterpret_cast<int*>(lds);
    for (;;) {
        if (threadIdx.x == 0) *next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = *next;
        __syncthreads();
        if (it >= n_items) break;
        const int4 w = items[it];
        const InstDesc& d = D[w.x];
        b16::Prep q;
        q.yT = d.yT;
        q.yo = d.yo;
        b16::bf16_fused16_body<LL, NP>(d.p, q, w.y, lds);
        __syncthreads();
    }
}
template __global__ void k_class_fused16<3, 24>(const InstDesc*, const int4*, int, int*);
template __global__ void k_class_fused16<3, 32>(const InstDesc*, const int4*, int, int*);
template __global__ void k_class_fused16<4, 24>(const InstDesc*, const int4*, int, int*);
template __global__ void k_class_fused16<4, 32>(const InstDesc*, const int4*, int, int*);

#define SRMRA_CLASS(F, L)                                                                     \
    template __global__ void k_class_pass<1, F, L>(const InstDesc*, const int4*, int, int*);  \
    template __global__ void k_class_pass<2, F, L>(const InstDesc*, const int4*, int, int*);
SRMRA_CLASS(FORM_VALU, 8) SRMRA_CLASS(FORM_VALU, 12) SRMRA_CLASS(FORM_VALU, 16)
SRMRA_CLASS(FORM_VALU, 24) SRMRA_CLASS(FORM_VALU, 32) SRMRA_CLASS(FORM_VALU, 48)
SRMRA_CLASS(FORM_VALU, 64)
SRMRA_CLASS(FORM_MFMA, 8) SRMRA_CLASS(FORM_MFMA, 12) SRMRA_CLASS(FORM_MFMA, 16)
SRMRA_CLASS(FORM_MFMA, 24) SRMRA_CLASS(FORM_MFMA, 32) SRMRA_CLASS(FORM_MFMA, 48)
SRMRA_CLASS(FORM_MFMA, 64)
SRMRA_CLASS(FORM_BF16, 8) SRMRA_CLASS(FORM_BF16, 12)
SRMRA_CLASS(FORM_BF16, 16) SRMRA_CLASS(FORM_BF16, 24) SRMRA_CLASS(FORM_BF16, 32)
SRMRA_CLASS(FORM_BF16, 48) SRMRA_CLASS(FORM_BF16, 64)
SRMRA_CLASS(FORM_BF16X4, 8) SRMRA_CLASS(FORM_BF16X4, 12)
SRMRA_CLASS(FORM_BF16X4, 16) SRMRA_CLASS(FORM_BF16X4, 24) SRMRA_CLASS(FORM_BF16X4, 32)
SRMRA_CLASS(FORM_BF16X4, 48) SRMRA_CLASS(FORM_BF16X4, 64)
SRMRA_CLASS(FORM_FFT, 8) SRMRA_CLASS(FORM_FFT, 12) SRMRA_CLASS(FORM_FFT, 16) SRMRA_CLASS(FORM_FFT, 24)
SRMRA_CLASS(FORM_FFT, 32) SRMRA_CLASS(FORM_FFT, 48) SRMRA_CLASS(FORM_FFT, 64)
#undef SRMRA_CLASS
#define SRMRA_BF16F(F, L) template __global__ void k_class_pass<2, F, L>(const InstDesc*, const int4*, int, int*);
SRMRA_BF16F(FORM_BF16F, 8) SRMRA_BF16F(FORM_BF16F, 12)
SRMRA_BF16F(FORM_BF16F, 24) SRMRA_BF16F(FORM_BF16F, 32) SRMRA_BF16F(FORM_BF16F, 48)
SRMRA_BF16F(FORM_BF16X4F, 8) SRMRA_BF16F(FORM_BF16X4F, 12)
SRMRA_BF16F(FORM_BF16X4F, 24) SRMRA_BF16F(FORM_BF16X4F, 32) SRMRA_BF16F(FORM_BF16X4F, 48)
#undef SRMRA_BF16F
#define SRMRA_FUSED(L) template __global__ void k_class_pass<2, FORM_FUSED, L>(const InstDesc*, const int4*, int, int*);
SRMRA_FUSED(8) SRMRA_FUSED(12) SRMRA_FUSED(16) SRMRA_FUSED(24) SRMRA_FUSED(32) SRMRA_FUSED(48)
SRMRA_FUSED(64)
#undef SRMRA_FUSED

// ---------------------------------------------------------------- host side
const void* class_pass_fn(int pass, int form, int LL) {
#define SRMRA_PICK(F, L) \
    if (form == F && LL == L) return pass == 1 ? (const void*)k_class_pass<1, F, L> : (const void*)k_class_pass<2, F, L>;
    SRMRA_PICK(FORM_VALU, 8) SRMRA_PICK(FORM_VALU, 12) SRMRA_PICK(FORM_VALU, 16)
    SRMRA_PICK(FORM_VALU, 24) SRMRA_PICK(FORM_VALU, 32) SRMRA_PICK(FORM_VALU, 48)
    SRMRA_PICK(FORM_VALU, 64)
    SRMRA_PICK(FORM_MFMA, 8) SRMRA_PICK(FORM_MFMA, 12) SRMRA_PICK(FORM_MFMA, 16)
    SRMRA_PICK(FORM_MFMA, 24) SRMRA_PICK(FORM_MFMA, 32) SRMRA_PICK(FORM_MFMA, 48)
    SRMRA_PICK(FORM_MFMA, 64)
    SRMRA_PICK(FORM_BF16, 8) SRMRA_PICK(FORM_BF16, 12)
    SRMRA_PICK(FORM_BF16, 16) SRMRA_PICK(FORM_BF16, 24) SRMRA_PICK(FORM_BF16, 32)
    SRMRA_PICK(FORM_BF16, 48) SRMRA_PICK(FORM_BF16, 64)
    SRMRA_PICK(FORM_BF16X4, 8) SRMRA_PICK(FORM_BF16X4, 12)
    SRMRA_PICK(FORM_BF16X4, 16) SRMRA_PICK(FORM_BF16X4, 24) SRMRA_PICK(FORM_BF16X4, 32)
    SRMRA_PICK(FORM_BF16X4, 48) SRMRA_PICK(FORM_BF16X4, 64)
    SRMRA_PICK(FORM_FFT, 8) SRMRA_PICK(FORM_FFT, 12) SRMRA_PICK(FORM_FFT, 16) SRMRA_PICK(FORM_FFT, 24)
    SRMRA_PICK(FORM_FFT, 32) SRMRA_PICK(FORM_FFT, 48) SRMRA_PICK(FORM_FFT, 64)
#undef SRMRA_PICK
    // single pass: no pass-1 kernel
#define SRMRA_PICK(L) if (form == FORM_FUSED && LL == L) return pass == 2 ? (const void*)k_class_pass<2, FORM_FUSED, L> : nullptr;
    SRMRA_PICK(8) SRMRA_PICK(12) SRMRA_PICK(16) SRMRA_PICK(24) SRMRA_PICK(32) SRMRA_PICK(48) SRMRA_PICK(64)
#undef SRMRA_PICK
#define SRMRA_PICK(F, L) if (form == F && LL == L) return pass == 2 ? (const void*)k_class_pass<2, F, L> : nullptr;
    SRMRA_PICK(FORM_BF16F, 8) SRMRA_PICK(FORM_BF16F, 12)
    SRMRA_PICK(FORM_BF16F, 24) SRMRA_PICK(FORM_BF16F, 32) SRMRA_PICK(FORM_BF16F, 48)
    SRMRA_PICK(FORM_BF16X4F, 8) SRMRA_PICK(FORM_BF16X4F, 12)
    SRMRA_PICK(FORM_BF16X4F, 24) SRMRA_PICK(FORM_BF16X4F, 32) SRMRA_PICK(FORM_BF16X4F, 48)
#undef SRMRA_PICK
    if (pass == 2 && form == FORM_BF16W && LL == 24) return (const void*)k_class_fused16<3, 24>;
    if (pass == 2 && form == FORM_BF16W && LL == 32) return (const void*)k_class_fused16<3, 32>;
    if (pass == 2 && form == FORM_BF16X4W && LL == 24) return (const void*)k_class_fused16<4, 24>;
    if (pass == 2 && form == FORM_BF16X4W && LL == 32) return (const void*)k_class_fused16<4, 32>;
    return nullptr;
}

const void* batch_fft_idft_fn() { return (const void*)k_batch_fft_idft; }
size_t batch_pack_lds(int LL) { return sizeof(float2) * ((size_t)LL * (LL + 1) + LL); }
size_t batch_idft_lds(int LL) { return sizeof(double2) * (size_t)LL * LL + 2 * sizeof(double) * LL; }

hipError_t batch_enqueue(const BatchLaunch& L, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, L.counters, 2 * L.n_class);
    hipLaunchKernelGGL(k_batch_pack, dim3(L.n_pack), dim3(256), 0, s, L.desc, L.pack_items);
    hipLaunchKernelGGL(k_batch_pack_xb, dim3(L.n_pack), dim3(256), L.pack_lds, s, L.desc, L.pack_items);
    const bool par = L.aux[0] != nullptr && L.n_class > 1;
    for (int pass = 1; pass <= 2; ++pass) {
        // fork: the helper streams wait for everything enqueued so far
        if (par) {
            if (hipEventRecord(L.fork[pass - 1], s) != hipSuccess) return hipErrorUnknown;
            for (int a = 0; a < kAuxStreams; ++a)
                if (hipStreamWaitEvent(L.aux[a], L.fork[pass - 1], 0) != hipSuccess) return hipErrorUnknown;
        }
        // the single-pass classes (no pass-1 launch, no dependence on the
        // combine) run in the first phase, beside the pass-1 launches of the
        // others, so that the second phase holds only two-pass classes
        int slot = 0;
        for (int k = 0; k < L.n_class; ++k) {
            const ClassLaunch& c = L.cls[k];
            const bool single = c.form == FORM_FUSED || c.form == FORM_BF16F || c.form == FORM_BF16X4F ||
                                c.form == FORM_BF16W || c.form == FORM_BF16X4W;
            if (pass == 2 && single) continue;
            const int kp = single ? 2 : pass;   // which kernel of the class
            const void* f = class_pass_fn(kp, c.form, c.LL);
            if (!f) return hipErrorInvalidValue;
            const InstDesc* desc = L.desc;
            const int4* items = L.pass_items + c.item0;
            int n = c.n_items;
            int* counter = L.counters + 2 * k + (kp - 1);
            void* args[] = {(void*)&desc, (void*)&items, (void*)&n, (void*)&counter};
            const int lane = slot++ % (kAuxStreams + 1);
            hipStream_t sk = (par && lane > 0) ? L.aux[lane - 1] : s;
            const hipError_t e = hipLaunchKernel(f, dim3(kp == 1 ? c.blocks1 : c.blocks2),
                                                 dim3(class_threads(c.form)), args,
                                                 kp == 1 ? c.lds1 : c.lds2, sk);
            if (e != hipSuccess) return e;
        }
        // join: the caller's stream waits for every helper stream
        if (par) {
            for (int a = 0; a < kAuxStreams; ++a) {
                if (hipEventRecord(L.join[pass - 1][a], L.aux[a]) != hipSuccess) return hipErrorUnknown;
                if (hipStreamWaitEvent(s, L.join[pass - 1][a], 0) != hipSuccess) return hipErrorUnknown;
            }
        }
        if (pass == 1 && L.n_combine > 0)
            hipLaunchKernelGGL(k_batch_combine, dim3(L.n_combine), dim3(256), 0, s, L.desc, L.combine_items);
    }
    if (L.n_combine_late > 0)
        hipLaunchKernelGGL(k_batch_combine, dim3(L.n_combine_late), dim3(256), 0, s, L.desc,
                           L.combine_items + L.n_combine);
    if (L.n_reduce > 0)
        hipLaunchKernelGGL(k_batch_reduce, dim3(L.n_reduce), dim3(256), 0, s, L.desc, L.reduce_items);
    if (L.n_fft_reduce > 0) {
        hipLaunchKernelGGL(k_batch_fft_reduce, dim3(L.n_fft_reduce), dim3(256), 0, s, L.desc,
                           L.reduce_items + L.n_reduce);
        hipLaunchKernelGGL(k_batch_fft_idft, dim3(L.n_fft_idft), dim3(256), L.idft_lds, s, L.desc,
                           L.reduce_items + L.n_reduce + L.n_fft_reduce);
    }
    hipLaunchKernelGGL(k_batch_finalize, dim3(L.n_inst), dim3(1024), 0, s, L.desc);
    return hipGetLastError();
}

}  // namespace srmra
