// Per-job and per-step helper kernels of the EM step (bodies in srmra_aux_impl.h).
#include "srmra_aux_impl.h"

namespace srmra {

__global__ __launch_bounds__(256) void k_obs_sums(const float* __restrict__ y, int64_t N, int npix,
                                                  double* __restrict__ ysum) {
    obs_sums_body(y, N, npix, ysum, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_centre(const double* __restrict__ ysum, int64_t N, int npix,
                                                 int enable, double* __restrict__ centre) {
    __shared__ double red[1024];
    centre_body(ysum, N, npix, enable, centre, red);
}

__global__ __launch_bounds__(256) void k_obs_norms(const float* __restrict__ y, int64_t N, int npix,
                                                   const double* __restrict__ centre,
                                                   double* __restrict__ ynorm) {
    obs_norms_body(y, N, npix, centre, ynorm, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_pack_x(const float* __restrict__ x,
                                                const float* __restrict__ log_rho, int K, int Ll,
                                                double inv_2s2, const double* __restrict__ centre,
                                                float* __restrict__ xt2, float* __restrict__ betaT) {
    __shared__ double red[256];
    pack_x_body(x, log_rho, K, Ll, inv_2s2, centre, xt2, betaT, blockIdx.x, red);
}

__global__ __launch_bounds__(256) void k_lse_combine(const float2* __restrict__ part, int n_cg,
                                                     int64_t N, const double* __restrict__ ynorm,
                                                     double inv_2s2, float2* __restrict__ lse,
                                                     double* __restrict__ llpart,
                                                     float* __restrict__ ll_obs) {
    __shared__ double red[256];
    lse_combine_body(part, n_cg, N, ynorm, inv_2s2, lse, llpart, ll_obs, blockIdx.x, red);
}

__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ bpart,
                                                         const float* __restrict__ cpart,
                                                         int n_chunks, int per_chunk,
                                                         double* __restrict__ bsum,
                                                         double* __restrict__ csum) {
    __shared__ double red[512];
    reduce_partials_body(bpart, cpart, n_chunks, per_chunk, bsum, csum, blockIdx.x, red);
}

__global__ __launch_bounds__(1024) void k_finalize(const double* __restrict__ bsum,
                                                   const double* __restrict__ csum, int K, int Ll,
                                                   const float* __restrict__ x,
                                                   const double* __restrict__ centre,
                                                   const double* __restrict__ llpart, int n_ll,
                                                   float* __restrict__ x_new,
                                                   float* __restrict__ rho_new,
                                                   float* __restrict__ log_rho_new,
                                                   double* __restrict__ loglik,
                                                   double* __restrict__ b_out,
                                                   double* __restrict__ c_out) {
    __shared__ double Ac[256];
    __shared__ double red[1024];
    finalize_body(bsum, csum, K, Ll, x, centre, llpart, n_ll, x_new, rho_new, log_rho_new, loglik,
                  b_out, c_out, Ac, red);
}

}  // namespace srmra
