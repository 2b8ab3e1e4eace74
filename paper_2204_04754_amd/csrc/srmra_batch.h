// Device descriptors of the batched form (shared by host and device code).
#pragma once
#include "srmra_common.h"

namespace srmra {

// FORM_FUSED: FP32 MFMA single pass (no pass-1 launch; the log-likelihood
// combine of these instances runs after pass 2)
// FORM_BF16F / FORM_BF16X4F: the BF16 split single pass (3 / 4 products)
// FORM_BF16W / FORM_BF16X4W: the BF16 split single pass at 4 < K^2 <= 16
// (512-thread workgroups)
// FORM_FFT: the FFT route (two passes, complex back-projection partials summed
// in FP64 and brought back by an FP64 inverse DFT per component)
enum { FORM_VALU = 0, FORM_MFMA = 1, FORM_BF16 = 2, FORM_FUSED = 3, FORM_BF16X4 = 4, FORM_BF16F = 5,
       FORM_BF16X4F = 6, FORM_BF16W = 7, FORM_BF16X4W = 8, FORM_FFT = 9 };

// threads per workgroup of a class's pass kernels
inline int class_threads(int form) { return (form == FORM_BF16W || form == FORM_BF16X4W) ? 512 : 256; }

struct InstDesc {
    StepArgs p;                  // per-instance step arguments (workspace pointers set)
    const __bf16* yT;            // BF16 prepared planes (BF16 forms only)
    const __bf16* yo;
    const float2* yhat;          // FFT form: prepared DFTs of the observations,
    float2* xhat;                // the DFTs of the components (per step)
    double2* bh;                 // and the FP64 sums of the back-projection's transform
    const float* x;              // iterate in (this parity)
    const float* log_rho;
    float* x_new;                // iterate out
    float* rho_new;
    float* log_rho_new;
    double* loglik;
    float* xt2_w;                // writable views of p.xt2 / p.betaT
    float* beta_w;
    double* llpart;
    double* bsum;
    double* csum;
    int LL, form, n_part, n_ll;
};

struct ClassLaunch {
    int form, LL, item0, n_items, blocks1, blocks2;
    size_t lds1, lds2;
};

constexpr int kMaxClasses = 16;
constexpr int kAuxStreams = 2;   // helper streams a plan runs classes on beside the caller's

struct BatchLaunch {
    const InstDesc* desc;        // device, n_inst entries
    const int4* pass_items;      // (instance, chunk, group, cost rank)
    const int2* pack_items;      // (instance, component)
    const int2* combine_items;   // (instance, block): two-pass instances, then single-pass ones
    const int2* reduce_items;    // (instance, block): real partials, then the FFT form's
                                 // complex ones (n_fft_reduce), then its inverse DFTs
                                 // (instance, component; n_fft_idft)
    int* counters;               // 2 per class
    int n_pack, n_combine, n_combine_late, n_reduce, n_inst, n_class;
    int n_fft_reduce, n_fft_idft;
    size_t pack_lds, idft_lds;   // dynamic LDS of the pack (FFT X) and inverse-DFT kernels
    ClassLaunch cls[kMaxClasses];
    // classes of one pass run concurrently: class k on the caller's stream when
    // k % (kAuxStreams + 1) == 0, else on aux[k % (kAuxStreams + 1) - 1], forked
    // from and joined back to the caller's stream through events (null: all on
    // the caller's stream)
    hipStream_t aux[kAuxStreams];
    hipEvent_t fork[2];
    hipEvent_t join[2][kAuxStreams];
};

hipError_t batch_enqueue(const BatchLaunch& L, hipStream_t s);
const void* class_pass_fn(int pass, int form, int LL);
const void* batch_fft_idft_fn();
size_t batch_pack_lds(int LL);    // dynamic LDS of the pack kernel for an FFT-form instance
size_t batch_idft_lds(int LL);

}  // namespace srmra
