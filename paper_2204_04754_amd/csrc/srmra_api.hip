// C ABI of the SR-MRA EM step (see include/srmra.h): argument validation,
// workspace layout, launch geometry and the launch sequence of one step.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include <algorithm>

#include "../../include/srmra.h"
#include "srmra_aux_impl.h"
#include "srmra_batch.h"
#include "srmra_common.h"
#include "srmra_moments.h"

namespace srmra {
// aux kernels (srmra_aux.hip)
__global__ void k_obs_sums(const float*, int64_t, int, double*);
__global__ void k_centre(const double*, int64_t, int, int, double*);
__global__ void k_obs_norms(const float*, int64_t, int, const double*, double*);
__global__ void k_pack_x(const float*, const float*, int, int, double, const double*, float*, float*);
__global__ void k_lse_combine(const float2*, int, int64_t, const double*, double, float2*, double*,
                              float*);
__global__ void k_reduce_partials(const float*, const float*, int, int, double*, double*);
__global__ void k_finalize(const double*, const double*, int, int, const float*, const double*,
                           const double*, int, float*, float*, float*, double*, double*, double*);
// pass launchers (srmra_mfma.hip, srmra_valu.hip, srmra_bf16.hip)
hipError_t launch_mfma(int LL, int pass, const StepArgs& p, hipStream_t s);
hipError_t launch_valu(int LL, int pass, const StepArgs& p, hipStream_t s);
bool mfma_geom(int LL, int& cpw, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2);
bool mfma_fused_geom(int LL, int KK, int& wc, int& nt, size_t& lds, const void*& f);
bool valu_geom(int LL, int KK, int& cpb, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2);
bool bf16_geom(int LL, int KK, int np, int tile, int& cpb, int& nt, size_t& lds1, size_t& lds2,
               const void*& f1, const void*& f2);
bool bf16_fused_geom(int LL, int KK, int np, int tile, int& cpb, int& nt, size_t& lds, const void*& f);
hipError_t launch_bf16(int LL, int np, int pass, const StepArgs& p, const void* prep_extra,
                       hipStream_t s);
hipError_t launch_prep_bf16(int LL, const float* y, int64_t N, const double* centre, double* ynorm,
                            void* prep_extra, hipStream_t s);
size_t bf16_prepared_extra(int LL, int64_t N);
size_t bf16_xb_bytes(int LL, int KK);
size_t bf16_yt_bytes(int LL, int64_t N);
bool bf16_supported(int LL);
int bf16_parts(int LL, int KK);
hipError_t launch_pack_xb(int LL, const StepArgs& p, const float* x, void* xb, hipStream_t s);
// projection of Alg. 2 (srmra_project.hip)
size_t project_workspace_bytes(int Lh);
hipError_t launch_project(const float* x_in, float* x_out, int Lh, float* sigma_state, float decay,
                          void* workspace, hipStream_t s);
// FFT route (srmra_fft.hip)
bool fft_supported(int LL);
int fft_tpc(int LL, int KK);
int fft_teams(int LL);
size_t fft_lds(int LL, int pass);
size_t fft_lds_class(int LL, int pass);
const void* fft_pass2_fn(int LL);
hipError_t launch_fft(int LL, int what, const StepArgs& p, const float* x, const float* y,
                      void* yhat, void* xhat, void* bpart, void* cpart, void* bh,
                      double* bsum, double* csum, hipStream_t s);
hipError_t launch_dft2(int L, const float* in, int64_t count, float2* out, hipStream_t s);
// reconstruction error (srmra_quality.hip)
size_t shift_error_workspace_bytes(int Lh);
hipError_t launch_shift_error(const float* xh, const float* x, int Lh, double* err, int* best,
                              void* ws, hipStream_t s);
}  // namespace srmra

using namespace srmra;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool supported_ll(int LL) {
    return LL == 8 || LL == 12 || LL == 16 || LL == 24 || LL == 32 || LL == 48 || LL == 64;
}

bool valid_prec(int p) {
    return p == SRMRA_FP32_PLAIN || p == SRMRA_FP32_MFMA || p == SRMRA_BF16_SPLIT3 ||
           p == SRMRA_BF16_SPLIT4 || p == SRMRA_FP32_FFT;
}
bool is_bf16(int p) { return p == SRMRA_BF16_SPLIT3 || p == SRMRA_BF16_SPLIT4; }
int split_products(int p) { return p == SRMRA_BF16_SPLIT4 ? 4 : 3; }

// Device facts used by the launch geometry, cached per device id.
struct DeviceInfo {
    int cus = 0;
};
std::mutex g_dev_mu;
DeviceInfo g_dev[64];

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev[dev].cus == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        g_dev[dev].cus = n;
    }
    return g_dev[dev].cus;
}

int occupancy(const void* f, size_t lds, int threads = 256) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, threads, lds) != hipSuccess || n < 1) n = 1;
    return n;
}

// Launch geometry and workspace layout of one step.
struct Geom {
    int LL = 0, K = 0, Lh = 0, KK = 0, prec = 0;
    int64_t N = 0;
    int cpb = 0, n_cg = 0, n_part = 0, ntile = 0, n_chunks = 0, n_ll = 0;
    int fuse_wc = 0;   // FP32 MFMA single pass: component groups per block (0: two passes)
    int fuse_bf16 = 0; // BF16 split single pass (all components in one workgroup)
    // prepared buffer: [||y_i - mu||^2 N doubles][sum_i N doubles][mu][BF16 planes]
    size_t prep_bytes = 0, prep_sum_off = 0, prep_mu_off = 0, prep_extra_off = 0;
    int64_t chunk_obs = 0;
    size_t lds1 = 0, lds2 = 0;
    // workspace offsets
    size_t o_prep = 0, o_part = 0, o_lse = 0, o_xt2 = 0, o_beta = 0, o_bpart = 0, o_cpart = 0,
           o_llpart = 0, o_bsum = 0, o_csum = 0, o_xb = 0, o_xhat = 0, o_bh = 0, total = 0;
};

// the BF16 single pass with 16 component slots per workgroup (512 threads)
inline bool bf16_wide_block(const Geom& g) { return g.fuse_bf16 && g.cpb == 16 && (g.LL == 24 || g.LL == 32); }

int make_geom(int64_t N, int LL, int K, int prec, bool with_norms, Geom& g,
              int64_t chunk_override = 0, int tile = 0) {
    if (N < 1 || N > (int64_t)INT32_MAX || K < 1 || LL < 1) return SRMRA_EINVAL;
    if (!supported_ll(LL)) return SRMRA_EUNSUPPORTED;
    if ((int64_t)K * LL > 4096 || K * K > 256) return SRMRA_EUNSUPPORTED;
    if (!valid_prec(prec)) return SRMRA_EUNSUPPORTED;
    g.LL = LL; g.K = K; g.Lh = K * LL; g.KK = K * K; g.N = N; g.prec = prec;
    const void* f1 = nullptr;
    const void* f2 = nullptr;
    bool ok;
    // a block layout other than the default: only where the form offers it
    if (tile != 0 && prec != SRMRA_FP32_MFMA && !is_bf16(prec)) return SRMRA_EINVAL;
    if (prec == SRMRA_FP32_MFMA) {
        if (tile != 0 && tile != SRMRA_TILE_TWO_PASS) return SRMRA_EINVAL;
        ok = mfma_geom(LL, g.cpb, g.ntile, g.lds1, g.lds2, f1, f2);
        // one pass when all components of an observation fit in one block
        int wc = 0, nt = 0;
        size_t lds = 0;
        const void* ff = nullptr;
        const bool fused = ok && mfma_fused_geom(LL, g.KK, wc, nt, lds, ff);
        if (tile == SRMRA_TILE_TWO_PASS && !fused) return SRMRA_EINVAL;   // no choice to make
        if (fused && tile == 0) {
            g.fuse_wc = wc;
            g.cpb *= wc;
            g.ntile = nt;
            g.lds1 = 0;
            g.lds2 = lds;
            f1 = nullptr;
            f2 = ff;
        }
    } else if (is_bf16(prec)) {
        if (!bf16_supported(LL)) return SRMRA_EUNSUPPORTED;
        ok = bf16_geom(LL, g.KK, split_products(prec), tile, g.cpb, g.ntile, g.lds1, g.lds2, f1, f2);
        if (!ok) return SRMRA_EINVAL;   // a layout this shape does not offer
        size_t lds = 0;
        const void* ff = nullptr;
        if (bf16_fused_geom(LL, g.KK, split_products(prec), tile, g.cpb, g.ntile, lds, ff)) {
            g.fuse_bf16 = 1;
            g.lds1 = 0;
            g.lds2 = lds;
            f1 = nullptr;
            f2 = ff;
        }
    } else if (prec == SRMRA_FP32_FFT) {
        // pass 1: a team per observation over all components; pass 2: component
        // groups of CG = teams / tpc components
        ok = fft_supported(LL);
        if (ok) {
            const int teams = fft_teams(LL);
            g.cpb = teams / fft_tpc(LL, g.KK);   // components per pass-2 block
            g.ntile = teams;
            g.lds1 = fft_lds(LL, 1);
            g.lds2 = fft_lds(LL, 2);
            f2 = fft_pass2_fn(LL);
        }
    }
    else ok = valu_geom(LL, g.KK, g.cpb, g.ntile, g.lds1, g.lds2, f1, f2);
    if (!ok) return SRMRA_EUNSUPPORTED;
    g.n_cg = (g.KK + g.cpb - 1) / g.cpb;
    // pass-1 partials per observation: one per component group, or per component
    // pair for the BF16 form (two waves of a block hold different pairs)
    g.n_part = g.fuse_bf16 ? 1 : (is_bf16(prec) ? bf16_parts(LL, g.KK)
                                                : (prec == SRMRA_FP32_FFT ? 1 : g.n_cg));   // 1 for the single pass
    g.prep_sum_off = align_up(sizeof(double) * (size_t)N);
    g.prep_mu_off = g.prep_sum_off + align_up(sizeof(double) * (size_t)N);
    g.prep_extra_off = g.prep_mu_off + kAlign;
    g.prep_bytes = g.prep_extra_off + (is_bf16(prec) ? bf16_prepared_extra(LL, N) : 0) +
                   (prec == SRMRA_FP32_FFT ? sizeof(float2) * (size_t)N * LL * LL : 0);
    // one resident wave of blocks over the whole device for the heavier pass
    // (the BF16 single pass at K^2 > 4 runs 512-thread workgroups)
    const int occ = occupancy(f2, g.lds2, bf16_wide_block(g) ? 512 : 256);
    const int64_t target = (int64_t)device_cus() * occ;
    const int64_t tiles = (N + g.ntile - 1) / g.ntile;
    int64_t nch = target / g.n_cg;
    if (nch >= 16) nch -= nch % 8;               // same chunk -> same XCD for all groups
    if (nch < 1) nch = 1;
    if (nch > tiles) nch = tiles;
    int64_t tiles_per_chunk = (tiles + nch - 1) / nch;
    if (chunk_override > 0) tiles_per_chunk = std::min<int64_t>(tiles, (chunk_override + g.ntile - 1) / g.ntile);
    g.chunk_obs = tiles_per_chunk * g.ntile;
    g.n_chunks = (int)((N + g.chunk_obs - 1) / g.chunk_obs);
    g.n_ll = (int)((N + 255) / 256);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    g.o_prep = with_norms ? take(g.prep_bytes) : 0;
    g.o_part = take(sizeof(float2) * (size_t)g.n_part * (size_t)N);
    g.o_lse = take(sizeof(float2) * (size_t)N);
    g.o_xt2 = take(sizeof(float) * (size_t)g.KK * LL * 2 * LL);
    g.o_beta = take(sizeof(float) * (size_t)g.KK * LL * LL);
    const size_t pw = prec == SRMRA_FP32_FFT ? sizeof(float2) : sizeof(float);   // complex partials
    g.o_bpart = take(pw * (size_t)g.n_chunks * g.KK * LL * LL);
    g.o_cpart = take(pw * (size_t)g.n_chunks * g.KK * LL * LL);
    g.o_llpart = take(sizeof(double) * (size_t)g.n_ll);
    g.o_bsum = take(sizeof(double) * (size_t)g.KK * LL * LL);
    g.o_csum = take(sizeof(double) * (size_t)g.KK * LL * LL);
    g.o_xb = is_bf16(prec) ? take(bf16_xb_bytes(LL, g.KK)) : 0;
    if (prec == SRMRA_FP32_FFT) {
        g.o_xhat = take(sizeof(float2) * (size_t)g.KK * LL * LL);
        g.o_bh = take(2 * sizeof(double) * (size_t)g.KK * LL * LL);
    }
    g.total = off;
    return SRMRA_OK;
}

inline bool aligned(const void* p) { return ((uintptr_t)p % kAlign) == 0; }

int check_step_args(const float* y, int64_t N, int L_low, int K, const float* x,
                    const float* log_rho, float sigma, float* x_new, float* rho_new,
                    double* loglik) {
    if (!y || !x || !log_rho || !x_new || !rho_new || !loglik) return SRMRA_EINVAL;
    if ((uintptr_t)y % 16 != 0) return SRMRA_EINVAL;   // observations are read as float4
    if (!(sigma > 0.f) || !isfinite(sigma)) return SRMRA_EINVAL;
    if (N < 1 || L_low < 1 || K < 1) return SRMRA_EINVAL;
    const size_t Lh = (size_t)K * L_low;
    const char* xb = (const char*)x;
    const char* xn = (const char*)x_new;
    const size_t xbytes = Lh * Lh * sizeof(float);
    if (xn < xb + xbytes && xb < xn + xbytes) return SRMRA_EINVAL;   // x_new aliases x
    const char* rn = (const char*)rho_new;
    const char* lr = (const char*)log_rho;
    const size_t rbytes = 2 * Lh * sizeof(float);
    if (rn < lr + rbytes && lr < rn + rbytes) return SRMRA_EINVAL;
    return SRMRA_OK;
}

int run_step(const Geom& g, const float* y, const char* prep, const float* x,
             const float* log_rho, float sigma, float* x_new, float* rho_new,
             float* log_rho_new, double* loglik, float* ll_obs, double* b_out, double* c_out,
             char* ws, hipStream_t stream, hipEvent_t* ev = nullptr) {
    StepArgs p;
    memset(&p, 0, sizeof(p));
    const double* ynorm = (const double*)prep;
    const double* centre = (const double*)(prep + g.prep_mu_off);
    const void* prep_extra = prep + g.prep_extra_off;
    p.y = y;
    p.ynorm = ynorm;
    p.centre = centre;
    p.N = g.N;
    p.K = g.K;
    p.Lh = g.Lh;
    p.KK = g.KK;
    p.inv_s2 = (float)(1.0 / ((double)sigma * (double)sigma));
    p.inv_2s2 = 1.0 / (2.0 * (double)sigma * (double)sigma);
    p.xt2 = (const float*)(ws + g.o_xt2);
    p.betaT = (const float*)(ws + g.o_beta);
    p.xb = is_bf16(g.prec) ? (const uint4*)(ws + g.o_xb) : nullptr;
    p.part = (float2*)(ws + g.o_part);
    p.lse = (float2*)(ws + g.o_lse);
    p.bpart = (float*)(ws + g.o_bpart);
    p.cpart = (float*)(ws + g.o_cpart);
    p.n_chunks = g.n_chunks;
    p.n_cg = g.n_cg;
    p.cpb = g.cpb;
    p.ntile = g.ntile;
    p.chunk_obs = g.chunk_obs;
    p.fuse_wc = g.fuse_wc;
    const int LL = g.LL;
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], stream); };

    mark(0);
    hipLaunchKernelGGL(k_pack_x, dim3(g.KK), dim3(256), 0, stream, x, log_rho, g.K, LL, p.inv_2s2, centre,
                       (float*)(ws + g.o_xt2), (float*)(ws + g.o_beta));
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    if (is_bf16(g.prec) && launch_pack_xb(LL, p, x, ws + g.o_xb, stream) != hipSuccess)
        return SRMRA_EDEVICE;
    mark(1);
    if (g.prec == SRMRA_FP32_FFT) {
        void* yhat = (void*)((const char*)prep_extra);
        auto fft = [&](int what) {
            return launch_fft(LL, what, p, x, y, yhat, ws + g.o_xhat, ws + g.o_bpart, ws + g.o_cpart,
                              ws + g.o_bh, (double*)(ws + g.o_bsum),
                              (double*)(ws + g.o_csum), stream);
        };
        if (fft(1) != hipSuccess) return SRMRA_EDEVICE;
        mark(1);
        if (fft(2) != hipSuccess) return SRMRA_EDEVICE;
        mark(2);
        hipLaunchKernelGGL(k_lse_combine, dim3(g.n_ll), dim3(256), 0, stream, (const float2*)p.part,
                           g.n_part, g.N, ynorm, p.inv_2s2, p.lse, (double*)(ws + g.o_llpart), ll_obs);
        if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
        mark(3);
        if (fft(3) != hipSuccess) return SRMRA_EDEVICE;
        mark(4);
        if (fft(4) != hipSuccess) return SRMRA_EDEVICE;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, stream, (const double*)(ws + g.o_bsum),
                           (const double*)(ws + g.o_csum), g.K, LL, x, centre,
                           (const double*)(ws + g.o_llpart), g.n_ll, x_new, rho_new, log_rho_new, loglik,
                           b_out, c_out);
        if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
        mark(5);
        return SRMRA_OK;
    }
    auto pass = [&](int k) -> hipError_t {
        if (g.prec == SRMRA_FP32_MFMA) return launch_mfma(LL, k, p, stream);
        if (is_bf16(g.prec)) return launch_bf16(LL, split_products(g.prec), k, p, prep_extra, stream);
        return launch_valu(LL, k, p, stream);
    };
    auto combine = [&]() -> hipError_t {
        hipLaunchKernelGGL(k_lse_combine, dim3(g.n_ll), dim3(256), 0, stream, (const float2*)p.part,
                           g.n_part, g.N, ynorm, p.inv_2s2, p.lse, (double*)(ws + g.o_llpart), ll_obs);
        return hipGetLastError();
    };
    if (g.fuse_wc || g.fuse_bf16) {
        // single pass; its (max, sum) per observation feed the log-likelihood after it
        mark(2);
        mark(3);
        if ((g.fuse_wc ? launch_mfma(LL, 3, p, stream)
                       : launch_bf16(LL, split_products(g.prec), 3, p, prep_extra, stream)) != hipSuccess)
            return SRMRA_EDEVICE;
        mark(4);
        if (combine() != hipSuccess) return SRMRA_EDEVICE;
    } else {
        if (pass(1) != hipSuccess) return SRMRA_EDEVICE;
        mark(2);
        if (combine() != hipSuccess) return SRMRA_EDEVICE;
        mark(3);
        if (pass(2) != hipSuccess) return SRMRA_EDEVICE;
        mark(4);
    }
    const int per = g.KK * LL * LL;
    hipLaunchKernelGGL(k_reduce_partials, dim3((per + kReduceElems - 1) / kReduceElems), dim3(256), 0, stream,
                       (const float*)p.bpart, (const float*)p.cpart, g.n_chunks, per,
                       (double*)(ws + g.o_bsum), (double*)(ws + g.o_csum));
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, stream, (const double*)(ws + g.o_bsum),
                       (const double*)(ws + g.o_csum), g.K, LL, x, centre,
                       (const double*)(ws + g.o_llpart), g.n_ll, x_new, rho_new, log_rho_new, loglik,
                       b_out, c_out);
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    mark(5);
    return SRMRA_OK;
}

}  // namespace

extern "C" {

const char* srmra_status_string(int status) {
    switch (status) {
        case SRMRA_OK: return "ok";
        case SRMRA_EINVAL: return "invalid argument";
        case SRMRA_EUNSUPPORTED: return "unsupported shape or precision";
        case SRMRA_EWORKSPACE: return "workspace or prepared buffer too small or misaligned";
        case SRMRA_EDEVICE: return "device launch error";
        case SRMRA_ESCRATCH: return "shape needs more workspace than the library's scratch array";
    }
    return "unknown status";
}

const char* srmra_version(void) { return "srmra 0.1 gfx950"; }

size_t srmra_em_step_workspace_bytes(int64_t N, int L_low, int K, int precision) {
    Geom g;
    if (make_geom(N, L_low, K, precision, true, g) != SRMRA_OK) return 0;
    return g.total;
}

int srmra_em_step_passes(int64_t N, int L_low, int K, int precision) {
    Geom g;
    const int st = make_geom(N, L_low, K, precision, false, g);
    if (st != SRMRA_OK) return st;
    return (g.fuse_wc || g.fuse_bf16) ? 1 : 2;   // the FFT route makes two passes
}

size_t srmra_prepared_bytes(int64_t N, int L_low, int K, int precision) {
    Geom g;
    if (make_geom(N, L_low, K, precision, false, g) != SRMRA_OK) return 0;
    return g.prep_bytes;
}

// a0: squared norms (and for the BF16 form its operand planes, in the same
// read of y)
static int enqueue_prepare(const Geom& g, const float* y, char* prep, int centre_on,
                           hipStream_t stream) {
    double* ynorm = (double*)prep;
    double* ysum = (double*)(prep + g.prep_sum_off);
    double* centre = (double*)(prep + g.prep_mu_off);
    const unsigned blocks = (unsigned)((g.N + 3) / 4);
    hipLaunchKernelGGL(k_obs_sums, dim3(blocks), dim3(256), 0, stream, y, g.N, g.LL * g.LL, ysum);
    hipLaunchKernelGGL(k_centre, dim3(1), dim3(1024), 0, stream, (const double*)ysum, g.N, g.LL * g.LL,
                       centre_on, centre);
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    if (is_bf16(g.prec))
        return launch_prep_bf16(g.LL, y, g.N, centre, ynorm, prep + g.prep_extra_off, stream) == hipSuccess
                   ? SRMRA_OK : SRMRA_EDEVICE;
    hipLaunchKernelGGL(k_obs_norms, dim3(blocks), dim3(256), 0, stream, y, g.N, g.LL * g.LL,
                       (const double*)centre, ynorm);
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    if (g.prec == SRMRA_FP32_FFT) {   // the DFT of every centred observation
        StepArgs p;
        memset(&p, 0, sizeof(p));
        p.N = g.N;
        p.centre = centre;
        if (launch_fft(g.LL, 0, p, nullptr, y, prep + g.prep_extra_off, nullptr, nullptr, nullptr,
                       nullptr, nullptr, nullptr, stream) != hipSuccess)
            return SRMRA_EDEVICE;
    }
    return SRMRA_OK;
}

int srmra_prepare_observations_ex(const float* y, int64_t N, int L_low, int K, int precision,
                                  int centre, void* prep, size_t prep_bytes, hipStream_t stream) {
    if (!y || !prep || (uintptr_t)y % 16 != 0) return SRMRA_EINVAL;
    if (centre != 0 && centre != 1) return SRMRA_EINVAL;
    Geom g;
    const int st = make_geom(N, L_low, K, precision, false, g);
    if (st != SRMRA_OK) return st;
    if (!aligned(prep) || prep_bytes < g.prep_bytes) return SRMRA_EWORKSPACE;
    return enqueue_prepare(g, y, (char*)prep, centre, stream);
}

int srmra_prepare_observations(const float* y, int64_t N, int L_low, int K, int precision,
                               void* prep, size_t prep_bytes, hipStream_t stream) {
    return srmra_prepare_observations_ex(y, N, L_low, K, precision, 1, prep, prep_bytes, stream);
}

int srmra_em_step_debug(const float* y, const void* prep, size_t prep_bytes, int64_t N, int L_low,
                        int K, const float* x, const float* log_rho, float sigma, float* x_new,
                        float* rho_new, float* log_rho_new, double* loglik, float* ll_obs,
                        double* b_out, double* c_out, int precision, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
    int st = check_step_args(y, N, L_low, K, x, log_rho, sigma, x_new, rho_new, loglik);
    if (st != SRMRA_OK) return st;
    Geom g;
    st = make_geom(N, L_low, K, precision, prep == nullptr, g);
    if (st != SRMRA_OK) return st;
    if (!workspace || !aligned(workspace) || workspace_bytes < g.total) return SRMRA_EWORKSPACE;
    char* ws = (char*)workspace;
    const char* pp;
    if (prep) {
        if (!aligned(prep) || prep_bytes < g.prep_bytes) return SRMRA_EWORKSPACE;
        pp = (const char*)prep;
    } else {
        st = enqueue_prepare(g, y, ws + g.o_prep, 1, stream);
        if (st != SRMRA_OK) return st;
        pp = ws + g.o_prep;
    }
    return run_step(g, y, pp, x, log_rho, sigma, x_new, rho_new, log_rho_new, loglik, ll_obs,
                    b_out, c_out, ws, stream);
}

int srmra_em_step_prepared(const float* y, const void* prep, size_t prep_bytes, int64_t N,
                           int L_low, int K, const float* x, const float* log_rho, float sigma,
                           float* x_new, float* rho_new, float* log_rho_new, double* loglik,
                           int precision, void* workspace, size_t workspace_bytes,
                           hipStream_t stream) {
    if (!prep) return SRMRA_EINVAL;
    return srmra_em_step_debug(y, prep, prep_bytes, N, L_low, K, x, log_rho, sigma, x_new, rho_new,
                               log_rho_new, loglik, nullptr, nullptr, nullptr, precision, workspace,
                               workspace_bytes, stream);
}

int srmra_em_step_profiled(const float* y, const void* prep, size_t prep_bytes, int64_t N,
                           int L_low, int K, const float* x, const float* log_rho, float sigma,
                           float* x_new, float* rho_new, float* log_rho_new, double* loglik,
                           int precision, void* workspace, size_t workspace_bytes,
                           hipStream_t stream, hipEvent_t* events) {
    if (!prep || !events) return SRMRA_EINVAL;
    for (int k = 0; k < 6; ++k)
        if (!events[k]) return SRMRA_EINVAL;
    int st = check_step_args(y, N, L_low, K, x, log_rho, sigma, x_new, rho_new, loglik);
    if (st != SRMRA_OK) return st;
    Geom g;
    st = make_geom(N, L_low, K, precision, false, g);
    if (st != SRMRA_OK) return st;
    if (!workspace || !aligned(workspace) || workspace_bytes < g.total) return SRMRA_EWORKSPACE;
    if (!aligned(prep) || prep_bytes < g.prep_bytes) return SRMRA_EWORKSPACE;
    return run_step(g, y, (const char*)prep, x, log_rho, sigma, x_new, rho_new, log_rho_new,
                    loglik, nullptr, nullptr, nullptr, (char*)workspace, stream, events);
}

int srmra_em_step(const float* y, int64_t N, int L_low, int K, const float* x,
                  const float* log_rho, float sigma, float* x_new, float* rho_new, double* loglik,
                  int precision, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    return srmra_em_step_debug(y, nullptr, 0, N, L_low, K, x, log_rho, sigma, x_new, rho_new,
                               nullptr, loglik, nullptr, nullptr, nullptr, precision, workspace,
                               workspace_bytes, stream);
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free step
namespace {
// The workspace of srmra_em_step_noalloc: one fixed array per device.  Host
// code never names it directly (its host-side name is not a device address);
// it uses the per-device address resolved below.
static __device__ __align__(256) unsigned char scratch[SRMRA_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch[64] = {};

// This device's address of `scratch`, resolved once per device with that
// device current; nullptr if the runtime cannot resolve it.
void* scratch_address() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}
}  // namespace

extern "C" {

int srmra_em_step_noalloc(const float* y, int64_t N, int L_low, int K, const float* x,
                          const float* log_rho, float sigma, float* x_new, float* rho_new,
                          double* loglik, int precision, hipStream_t stream) {
    int st = check_step_args(y, N, L_low, K, x, log_rho, sigma, x_new, rho_new, loglik);
    if (st != SRMRA_OK) return st;
    Geom g;
    st = make_geom(N, L_low, K, precision, true, g);
    if (st != SRMRA_OK) return st;
    if (g.total > SRMRA_SCRATCH_BYTES) return SRMRA_ESCRATCH;
    void* ws = scratch_address();
    if (!ws) return SRMRA_EDEVICE;
    return srmra_em_step(y, N, L_low, K, x, log_rho, sigma, x_new, rho_new, loglik, precision, ws,
                         SRMRA_SCRATCH_BYTES, stream);
}

// ---------------------------------------------------------------- batched form
struct srmra_plan {
    int precision = 0;
    std::vector<srmra_problem> probs;
    std::vector<Geom> geoms;
    std::vector<int> form;
    std::vector<size_t> inst_off;
    std::vector<int4> pass_items;
    std::vector<int2> pack_items, combine_items, reduce_items;
    int n_combine_early = 0;   // combine items of two-pass instances (the rest run after pass 2)
    // reduce_items: n_reduce_plain real-partial items, then n_fft_reduce complex ones
    // and n_fft_idft inverse DFTs of the FFT-form instances
    int n_reduce_plain = 0, n_fft_reduce = 0, n_fft_idft = 0;
    size_t pack_lds = 0, idft_lds = 0;
    size_t o_desc = 0, o_pass = 0, o_pack = 0, o_comb = 0, o_red = 0, o_cnt = 0, total = 0;
    std::vector<ClassLaunch> classes;
    int parity = 0;
    bool uploaded = false;
    const void* uploaded_ws = nullptr;
    // helper streams (default priority) and events on which the classes of one
    // pass run concurrently; created with the plan on the current device
    hipStream_t aux[kAuxStreams] = {};
    hipEvent_t fork[2] = {};
    hipEvent_t join[2][kAuxStreams] = {};
    bool concurrent = false;
    // pinned host staging of the descriptors and work lists, read by the
    // asynchronous copies of the last upload until `staged` completes
    void* staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    ~srmra_plan() {
        if (staged_pending) (void)hipEventSynchronize(staged);
        if (staging) (void)hipHostFree(staging);
        if (staged) (void)hipEventDestroy(staged);
        for (int a = 0; a < kAuxStreams; ++a)
            if (aux[a]) (void)hipStreamDestroy(aux[a]);
        for (int q = 0; q < 2; ++q) {
            if (fork[q]) (void)hipEventDestroy(fork[q]);
            for (int a = 0; a < kAuxStreams; ++a)
                if (join[q][a]) (void)hipEventDestroy(join[q][a]);
        }
    }
};

namespace {

int form_of(int precision, int LL) {
    if (precision == SRMRA_FP32_FFT) return fft_supported(LL) ? FORM_FFT : -1;
    if (is_bf16(precision)) {
        if (!bf16_supported(LL)) return FORM_MFMA;
        return precision == SRMRA_BF16_SPLIT4 ? FORM_BF16X4 : FORM_BF16;   // (single pass: below)
    }
    return precision == SRMRA_FP32_MFMA ? FORM_MFMA : FORM_VALU;
}

// the precision a batched form runs in
int prec_of_form(int f) {
    switch (f) {
        case FORM_BF16: case FORM_BF16F: case FORM_BF16W: return SRMRA_BF16_SPLIT3;
        case FORM_BF16X4: case FORM_BF16X4F: case FORM_BF16X4W: return SRMRA_BF16_SPLIT4;
        case FORM_VALU: return SRMRA_FP32_PLAIN;
        case FORM_FFT: return SRMRA_FP32_FFT;
    }
    return SRMRA_FP32_MFMA;
}
bool is_bf16_form(int f) {
    return f == FORM_BF16 || f == FORM_BF16X4 || f == FORM_BF16F || f == FORM_BF16X4F || f == FORM_BF16W ||
           f == FORM_BF16X4W;
}
// forms with no pass-1 launch (their log-likelihood combine runs after pass 2)
bool single_pass_form(int f) {
    return f == FORM_FUSED || f == FORM_BF16F || f == FORM_BF16X4F || f == FORM_BF16W || f == FORM_BF16X4W;
}

// observations per work item: about 2^28 multiply-adds (or FFT flop), but no fewer than 128
// chunks per instance while an item keeps 2^24 or more (at small L_low 2^28
// is thousands of observations, and a class of a few instances would have
// fewer items than the device has CUs).  Shape-only, so an instance's
// partition does not depend on the rest of the batch.
int64_t default_chunk(const Geom& g) {
    // work per observation and item: L_low^4 multiply-adds per component for the
    // dense forms, about 40 L_low^2 log2 L_low flop for the FFT route's transforms
    const double per_obs = (double)g.cpb * (g.prec == SRMRA_FP32_FFT ? 40.0 * g.LL * g.LL * log2((double)g.LL)
                                                                      : (double)g.LL * g.LL * g.LL * g.LL);
    int64_t c = (int64_t)(268435456.0 / per_obs);
    const int64_t spread = (g.N + 127) / 128;
    if (spread < c) c = std::max<int64_t>(spread, (int64_t)(16777216.0 / per_obs));
    // one-component items (BF16 at L_low 48 and 64): about 4 items per CU over
    // the instance, so that the per-chunk partials (chunks x K^2 x L_low^2)
    // stay small
    if (g.cpb == 1 && is_bf16(g.prec)) c = std::max<int64_t>(c, (g.N * g.KK + 1023) / 1024);
    if (c < g.ntile) c = g.ntile;
    return c;
}

void fill_desc(srmra_plan* P, int i, int par, InstDesc& d, char* ws) {
    const Geom& g = P->geoms[i];
    const srmra_problem& pr = P->probs[i];
    char* w = ws + P->inst_off[i];
    memset(&d, 0, sizeof(d));
    StepArgs& p = d.p;
    p.y = pr.y;
    p.ynorm = (const double*)pr.prep;
    p.centre = (const double*)((const char*)pr.prep + g.prep_mu_off);
    p.N = g.N; p.K = g.K; p.Lh = g.Lh; p.KK = g.KK;
    p.inv_s2 = (float)(1.0 / ((double)pr.sigma * (double)pr.sigma));
    p.inv_2s2 = 1.0 / (2.0 * (double)pr.sigma * (double)pr.sigma);
    p.xt2 = (const float*)(w + g.o_xt2);
    p.betaT = (const float*)(w + g.o_beta);
    p.xb = is_bf16_form(P->form[i]) ? (const uint4*)(w + g.o_xb) : nullptr;
    if (P->form[i] == FORM_FFT) {
        d.yhat = (const float2*)((const char*)pr.prep + g.prep_extra_off);
        d.xhat = (float2*)(w + g.o_xhat);
        d.bh = (double2*)(w + g.o_bh);
    }
    p.part = (float2*)(w + g.o_part);
    p.lse = (float2*)(w + g.o_lse);
    p.bpart = (float*)(w + g.o_bpart);
    p.cpart = (float*)(w + g.o_cpart);
    p.n_chunks = g.n_chunks; p.n_cg = g.n_cg; p.cpb = g.cpb; p.ntile = g.ntile;
    p.chunk_obs = g.chunk_obs;
    p.fuse_wc = g.fuse_wc;
    if (is_bf16_form(P->form[i])) {
        const char* e = (const char*)pr.prep + g.prep_extra_off;
        d.yT = (const __bf16*)e;
        d.yo = (const __bf16*)(e + align_up(bf16_yt_bytes(g.LL, g.N)));
    }
    const bool flip = par == 1;
    d.x = flip ? pr.x_new : pr.x;
    d.log_rho = flip ? pr.log_rho_new : pr.log_rho;
    d.x_new = flip ? (float*)pr.x : pr.x_new;
    d.log_rho_new = flip ? (float*)pr.log_rho : pr.log_rho_new;
    d.rho_new = pr.rho_new;
    d.loglik = pr.loglik;
    d.xt2_w = (float*)(w + g.o_xt2);
    d.beta_w = (float*)(w + g.o_beta);
    d.llpart = (double*)(w + g.o_llpart);
    d.bsum = (double*)(w + g.o_bsum);
    d.csum = (double*)(w + g.o_csum);
    d.LL = g.LL; d.form = P->form[i]; d.n_part = g.n_part; d.n_ll = g.n_ll;
}

}  // namespace

int srmra_plan_form(int precision, int L_low) {
    if (!supported_ll(L_low)) return -1;
    if (!valid_prec(precision) || precision == SRMRA_FP32_FFT) return -1;
    return prec_of_form(form_of(precision, L_low));
}

int64_t srmra_plan_default_item_obs(int64_t N, int L_low, int K, int form_precision) {
    Geom g;
    const int st = make_geom(N, L_low, K, form_precision, false, g);
    if (st != SRMRA_OK) return st;
    return default_chunk(g);
}

int srmra_plan_create(const srmra_problem* probs, int count, int precision, srmra_plan** plan,
                      size_t* workspace_bytes) {
    return srmra_plan_create_tuned(probs, count, precision, nullptr, 0, plan, workspace_bytes);
}

int srmra_plan_create_tuned(const srmra_problem* probs, int count, int precision,
                            const srmra_tuning* table, int n_table, srmra_plan** plan,
                            size_t* workspace_bytes) {
    if (!plan || !workspace_bytes || !probs || count < 1 || count > 65535) return SRMRA_EINVAL;
    if (n_table < 0 || (n_table > 0 && !table)) return SRMRA_EINVAL;
    *plan = nullptr;
    *workspace_bytes = 0;
    if (!valid_prec(precision) || precision == SRMRA_FP32_FFT) return SRMRA_EUNSUPPORTED;
    // a table entry may keep the plan's precision, pick FP32 MFMA in a BF16
    // plan (more accurate), or pick the FFT route (FP32 transforms, FP64 sums)
    // where it covers the L_low; the BF16 form needs an L_low it is built for
    for (int k = 0; k < n_table; ++k) {
        const srmra_tuning& t = table[k];
        if (t.item_obs < 0) return SRMRA_EINVAL;
        if (t.precision != precision) continue;
        // a block layout only where the entry's form and shape offer it
        if (t.tile != 0) {
            Geom gt;
            const int st = make_geom(1024, t.L_low, t.K, t.form, false, gt, 0, t.tile);
            if (st != SRMRA_OK) return st == SRMRA_EUNSUPPORTED ? st : SRMRA_EINVAL;
        }
        const bool ok = t.form == precision || (is_bf16(precision) && t.form == SRMRA_FP32_MFMA) ||
                        t.form == SRMRA_FP32_FFT;
        if (!ok) return SRMRA_EINVAL;
        if (t.form == SRMRA_FP32_FFT && !fft_supported(t.L_low)) return SRMRA_EUNSUPPORTED;
        if (is_bf16(t.form) && !is_bf16_form(form_of(t.form, t.L_low))) return SRMRA_EUNSUPPORTED;
    }
    srmra_plan* P = new (std::nothrow) srmra_plan;
    if (!P) return SRMRA_EINVAL;
    P->precision = precision;
    P->probs.assign(probs, probs + count);
    struct Cost { int cls; double c; int4 it; };
    std::vector<Cost> costs;
    std::vector<int2> combine_late, fft_reduce, fft_idft;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    for (int i = 0; i < count; ++i) {
        const srmra_problem& pr = probs[i];
        int st = check_step_args(pr.y, pr.N, pr.L_low, pr.K, pr.x, pr.log_rho, pr.sigma, pr.x_new,
                                 pr.rho_new, pr.loglik);
        if (st == SRMRA_OK && (!pr.prep || !pr.log_rho_new || !aligned(pr.prep))) st = SRMRA_EINVAL;
        if (st != SRMRA_OK) { delete P; return st; }
        int f = form_of(precision, pr.L_low);
        int64_t item_obs = 0;
        int tile = 0;
        for (int k = 0; k < n_table; ++k) {   // first matching entry wins
            const srmra_tuning& t = table[k];
            if (t.precision == precision && t.L_low == pr.L_low && t.K == pr.K) {
                f = form_of(t.form, pr.L_low);
                item_obs = t.item_obs;
                tile = t.tile;
                break;
            }
        }
        const int fprec = prec_of_form(f);
        Geom g0;
        st = make_geom(pr.N, pr.L_low, pr.K, fprec, false, g0, 0, tile);
        if (st != SRMRA_OK) { delete P; return st; }
        Geom g;
        make_geom(pr.N, pr.L_low, pr.K, fprec, false, g, item_obs > 0 ? item_obs : default_chunk(g0), tile);
        if (pr.prep_bytes < g.prep_bytes) { delete P; return SRMRA_EWORKSPACE; }
        if (f == FORM_MFMA && g.fuse_wc) f = FORM_FUSED;
        if (bf16_wide_block(g)) f = f == FORM_BF16X4 ? FORM_BF16X4W : FORM_BF16W;
        else if (g.fuse_bf16) f = f == FORM_BF16X4 ? FORM_BF16X4F : FORM_BF16F;
        P->geoms.push_back(g);
        P->form.push_back(f);
        int cls = -1;
        for (size_t k = 0; k < P->classes.size(); ++k)
            if (P->classes[k].form == f && P->classes[k].LL == pr.L_low) cls = (int)k;
        if (cls < 0) {
            if ((int)P->classes.size() >= kMaxClasses) { delete P; return SRMRA_EUNSUPPORTED; }
            ClassLaunch c;
            memset(&c, 0, sizeof(c));
            c.form = f;
            c.LL = pr.L_low;
            P->classes.push_back(c);
            cls = (int)P->classes.size() - 1;
        }
        ClassLaunch& C = P->classes[cls];
        C.lds1 = std::max(C.lds1, g.lds1);
        C.lds2 = std::max(C.lds2, f == FORM_FFT ? fft_lds_class(pr.L_low, 2) : g.lds2);
        // one-component items are listed component-major, so that the blocks
        // running at one time share few components' B fragments in L2
        const bool comp_major = g.cpb == 1 && is_bf16_form(f);
        for (int a = 0; a < (comp_major ? g.n_cg : g.n_chunks); ++a) {
            for (int b = 0; b < (comp_major ? g.n_chunks : g.n_cg); ++b) {
                const int ch = comp_major ? b : a, cg = comp_major ? a : b;
                const int64_t nobs = std::min<int64_t>(g.chunk_obs, g.N - (int64_t)ch * g.chunk_obs);
                // relative cost (orders the classes, heaviest first, and the items in a class)
                const double dense = (double)g.LL * g.LL * g.LL * g.LL;
                const double fftc = 40.0 * g.LL * g.LL * log2((double)g.LL);   // transforms per pair
                const double cst = (double)nobs * g.cpb *
                                   (f == FORM_FFT ? fftc : dense *
                                   (f == FORM_VALU ? 2.0 : (f == FORM_BF16 ? 0.5 : (f == FORM_BF16X4 ? 0.67 :
                                    ((f == FORM_BF16F || f == FORM_BF16W) ? 0.35
                                     : ((f == FORM_BF16X4F || f == FORM_BF16X4W) ? 0.45 : 1.0))))));
                costs.push_back({cls, cst, make_int4(i, ch, cg, 0)});
            }
        }
        for (int c = 0; c < g.KK; ++c) P->pack_items.push_back(make_int2(i, c));
        for (int k = 0; k < g.n_ll; ++k)
            (single_pass_form(f) ? combine_late : P->combine_items).push_back(make_int2(i, k));
        const int per = g.KK * g.LL * g.LL;
        for (int k = 0; k < (per + kReduceElems - 1) / kReduceElems; ++k)
            (f == FORM_FFT ? fft_reduce : P->reduce_items).push_back(make_int2(i, k));
        if (f == FORM_FFT) {
            for (int c = 0; c < g.KK; ++c) fft_idft.push_back(make_int2(i, c));
            P->pack_lds = std::max(P->pack_lds, batch_pack_lds(g.LL));
            P->idft_lds = std::max(P->idft_lds, batch_idft_lds(g.LL));
        }
    }
    P->n_reduce_plain = (int)P->reduce_items.size();
    P->n_fft_reduce = (int)fft_reduce.size();
    P->n_fft_idft = (int)fft_idft.size();
    P->reduce_items.insert(P->reduce_items.end(), fft_reduce.begin(), fft_reduce.end());
    P->reduce_items.insert(P->reduce_items.end(), fft_idft.begin(), fft_idft.end());
    P->n_combine_early = (int)P->combine_items.size();
    P->combine_items.insert(P->combine_items.end(), combine_late.begin(), combine_late.end());
    // items grouped by class (heaviest class first), largest items first within a class
    std::vector<double> class_cost(P->classes.size(), 0.0);
    for (auto& c : costs) class_cost[c.cls] += c.c;
    std::vector<int> order(P->classes.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return class_cost[a] > class_cost[b]; });
    std::vector<int> rank(order.size());
    for (size_t k = 0; k < order.size(); ++k) rank[order[k]] = (int)k;
    std::stable_sort(costs.begin(), costs.end(), [&](const Cost& a, const Cost& b) {
        if (a.cls != b.cls) return rank[a.cls] < rank[b.cls];
        return a.c > b.c;
    });
    std::vector<ClassLaunch> sorted;
    for (int k : order) sorted.push_back(P->classes[k]);
    P->classes = sorted;
    for (size_t k = 0; k < costs.size(); ++k) {
        ClassLaunch& C = P->classes[rank[costs[k].cls]];
        if (C.n_items == 0) C.item0 = (int)k;
        C.n_items++;
        P->pass_items.push_back(costs[k].it);
    }
    P->o_desc = take(2 * sizeof(InstDesc) * (size_t)count);
    P->o_pass = take(sizeof(int4) * P->pass_items.size());
    P->o_pack = take(sizeof(int2) * P->pack_items.size());
    P->o_comb = take(sizeof(int2) * P->combine_items.size());
    P->o_red = take(sizeof(int2) * P->reduce_items.size());
    P->o_cnt = take(sizeof(int) * 2 * kMaxClasses);
    for (int i = 0; i < count; ++i) P->inst_off.push_back(take(P->geoms[i].total));
    P->total = off;
    const int cus = device_cus();
    for (auto& C : P->classes) {
        const void* f1 = class_pass_fn(1, C.form, C.LL);
        C.blocks1 = f1 ? cus * occupancy(f1, C.lds1) : 0;
        C.blocks2 = cus * occupancy(class_pass_fn(2, C.form, C.LL), C.lds2, class_threads(C.form));
    }
    // helper streams for concurrent classes (without them the classes run one
    // after another on the caller's stream)
    if (P->classes.size() > 1) {
        bool ok = true;
        for (int a = 0; a < kAuxStreams && ok; ++a)
            ok = hipStreamCreateWithFlags(&P->aux[a], hipStreamNonBlocking) == hipSuccess;
        for (int q = 0; q < 2 && ok; ++q) {
            ok = hipEventCreateWithFlags(&P->fork[q], hipEventDisableTiming) == hipSuccess;
            for (int a = 0; a < kAuxStreams && ok; ++a)
                ok = hipEventCreateWithFlags(&P->join[q][a], hipEventDisableTiming) == hipSuccess;
        }
        P->concurrent = ok;
        if (!ok) (void)hipGetLastError();
    }
    *plan = P;
    *workspace_bytes = P->total;
    return SRMRA_OK;
}

int srmra_plan_set_iterate(srmra_plan* plan, int index, const float* x, const float* log_rho,
                           float* x_new, float* rho_new, float* log_rho_new) {
    if (!plan || index < 0 || index >= (int)plan->probs.size()) return SRMRA_EINVAL;
    if (!x || !log_rho || !x_new || !rho_new || !log_rho_new || x == x_new) return SRMRA_EINVAL;
    srmra_problem& pr = plan->probs[index];
    pr.x = x; pr.log_rho = log_rho; pr.x_new = x_new; pr.rho_new = rho_new;
    pr.log_rho_new = log_rho_new;
    plan->uploaded = false;
    plan->parity = 0;
    return SRMRA_OK;
}

int srmra_plan_upload(srmra_plan* plan, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!plan || !workspace || !aligned(workspace)) return SRMRA_EINVAL;
    if (workspace_bytes < plan->total) return SRMRA_EWORKSPACE;
    char* ws = (char*)workspace;
    const int n = (int)plan->probs.size();
    // the descriptors and work lists go through a pinned staging copy owned by
    // the plan, so the copies are asynchronous; a previous upload's copies
    // must have left the staging buffer before it is rewritten
    const size_t b_desc = sizeof(InstDesc) * 2 * (size_t)n;
    const size_t b_pass = sizeof(int4) * plan->pass_items.size();
    const size_t b_pack = sizeof(int2) * plan->pack_items.size();
    const size_t b_comb = sizeof(int2) * plan->combine_items.size();
    const size_t b_red = sizeof(int2) * plan->reduce_items.size();
    const size_t need = b_desc + b_pass + b_pack + b_comb + b_red;
    if (plan->staged_pending && hipEventSynchronize(plan->staged) != hipSuccess) return SRMRA_EDEVICE;
    plan->staged_pending = false;
    if (!plan->staged && hipEventCreateWithFlags(&plan->staged, hipEventDisableTiming) != hipSuccess)
        return SRMRA_EDEVICE;
    if (plan->staging_bytes < need) {
        if (plan->staging) (void)hipHostFree(plan->staging);
        plan->staging = nullptr;
        plan->staging_bytes = 0;
        if (hipHostMalloc(&plan->staging, need, hipHostMallocDefault) != hipSuccess) return SRMRA_EDEVICE;
        plan->staging_bytes = need;
    }
    char* h = (char*)plan->staging;
    InstDesc* desc = (InstDesc*)h;
    for (int par = 0; par < 2; ++par)
        for (int i = 0; i < n; ++i) {
            desc[(size_t)par * n + i] = InstDesc{};
            fill_desc(plan, i, par, desc[(size_t)par * n + i], ws);
        }
    size_t off = b_desc;
    auto stage = [&](const void* src, size_t bytes) {
        memcpy(h + off, src, bytes);
        const char* p = h + off;
        off += bytes;
        return p;
    };
    const char* s_pass = stage(plan->pass_items.data(), b_pass);
    const char* s_pack = stage(plan->pack_items.data(), b_pack);
    const char* s_comb = stage(plan->combine_items.data(), b_comb);
    const char* s_red = stage(plan->reduce_items.data(), b_red);
    hipError_t e = hipMemcpyAsync(ws + plan->o_desc, h, b_desc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + plan->o_pass, s_pass, b_pass, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + plan->o_pack, s_pack, b_pack, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + plan->o_comb, s_comb, b_comb, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + plan->o_red, s_red, b_red, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(plan->staged, stream);
    if (e != hipSuccess) return SRMRA_EDEVICE;
    plan->staged_pending = true;
    if (plan->n_fft_idft > 0 &&
        hipFuncSetAttribute(batch_fft_idft_fn(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan->idft_lds) !=
            hipSuccess)
        return SRMRA_EDEVICE;
    for (auto& C : plan->classes) {
        for (int pass = 1; pass <= 2; ++pass) {
            const void* f = class_pass_fn(pass, C.form, C.LL);   // null: single-pass class, pass 1
            if (f && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(pass == 1 ? C.lds1 : C.lds2)) != hipSuccess)
                return SRMRA_EDEVICE;
        }
    }
    plan->uploaded = true;
    plan->uploaded_ws = workspace;
    plan->parity = 0;
    return SRMRA_OK;
}

int srmra_plan_execute(srmra_plan* plan, void* workspace, size_t workspace_bytes,
                       hipStream_t stream) {
    if (!plan || !workspace) return SRMRA_EINVAL;
    if (workspace_bytes < plan->total) return SRMRA_EWORKSPACE;
    if (!plan->uploaded || plan->uploaded_ws != workspace) {
        const int st = srmra_plan_upload(plan, workspace, workspace_bytes, stream);
        if (st != SRMRA_OK) return st;
    }
    char* ws = (char*)workspace;
    const int n = (int)plan->probs.size();
    BatchLaunch L;
    L.desc = (const InstDesc*)(ws + plan->o_desc) + (size_t)plan->parity * n;
    L.pass_items = (const int4*)(ws + plan->o_pass);
    L.pack_items = (const int2*)(ws + plan->o_pack);
    L.combine_items = (const int2*)(ws + plan->o_comb);
    L.reduce_items = (const int2*)(ws + plan->o_red);
    L.counters = (int*)(ws + plan->o_cnt);
    L.n_pack = (int)plan->pack_items.size();
    L.n_combine = plan->n_combine_early;
    L.n_combine_late = (int)plan->combine_items.size() - plan->n_combine_early;
    L.n_reduce = plan->n_reduce_plain;
    L.n_fft_reduce = plan->n_fft_reduce;
    L.n_fft_idft = plan->n_fft_idft;
    L.pack_lds = plan->pack_lds;
    L.idft_lds = plan->idft_lds;
    L.n_inst = n;
    L.n_class = (int)plan->classes.size();
    for (int k = 0; k < L.n_class; ++k) L.cls[k] = plan->classes[k];
    for (int a = 0; a < kAuxStreams; ++a) L.aux[a] = plan->concurrent ? plan->aux[a] : nullptr;
    for (int q = 0; q < 2; ++q) {
        L.fork[q] = plan->fork[q];
        for (int a = 0; a < kAuxStreams; ++a) L.join[q][a] = plan->join[q][a];
    }
    if (batch_enqueue(L, stream) != hipSuccess) return SRMRA_EDEVICE;
    plan->parity ^= 1;
    return SRMRA_OK;
}

int srmra_plan_parity(const srmra_plan* plan) { return plan ? plan->parity : -1; }

void srmra_plan_destroy(srmra_plan* plan) { delete plan; }

size_t srmra_project_workspace_bytes(int L_high) {
    if (L_high < 1 || L_high > 4096) return 0;
    return project_workspace_bytes(L_high);
}

int srmra_dft2(const float* in, int64_t count, int L, void* out, hipStream_t stream) {
    if (!in || !out || count < 1 || count > (int64_t)INT32_MAX * 8LL || !fft_supported(L))
        return SRMRA_EINVAL;
    return launch_dft2(L, in, count, (float2*)out, stream) == hipSuccess ? SRMRA_OK : SRMRA_EDEVICE;
}

size_t srmra_moments_workspace_bytes(int64_t N, int L_low) {
    if (N < 1 || L_low < 2 || L_low > 64 || L_low % 2) return 0;
    return moments_geom(N, L_low, device_cus()).total;
}

int srmra_moments(const float* y, int64_t N, int L_low, double* m1, double* m2, void* workspace,
                  size_t workspace_bytes, hipStream_t stream) {
    if (!y || !m1 || !m2 || (uintptr_t)y % 16 != 0) return SRMRA_EINVAL;
    if (N < 1 || N > (int64_t)INT32_MAX || L_low < 2 || L_low > 64 || L_low % 2) return SRMRA_EINVAL;
    const MomentsGeom g = moments_geom(N, L_low, device_cus());
    if (!workspace || !aligned(workspace) || workspace_bytes < g.total) return SRMRA_EWORKSPACE;
    return launch_moments(y, N, L_low, m1, m2, workspace, g, stream) == hipSuccess ? SRMRA_OK
                                                                                  : SRMRA_EDEVICE;
}

size_t srmra_shift_error_workspace_bytes(int L_high) {
    if (L_high < 1 || L_high > 512) return 0;
    return shift_error_workspace_bytes(L_high);
}

int srmra_shift_error(const float* x_hat, const float* x_ref, int L_high, double* err,
                      int* best_shift, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!x_hat || !x_ref || !err || L_high < 1 || L_high > 512) return SRMRA_EINVAL;
    if (!workspace || !aligned(workspace) || workspace_bytes < shift_error_workspace_bytes(L_high))
        return SRMRA_EWORKSPACE;
    return launch_shift_error(x_hat, x_ref, L_high, err, best_shift, workspace, stream) == hipSuccess
               ? SRMRA_OK : SRMRA_EDEVICE;
}

int srmra_project_gaussian(const float* x_in, float* x_out, int L_high, float* sigma_state,
                           float decay, void* workspace, size_t workspace_bytes,
                           hipStream_t stream) {
    if (!x_in || !x_out || !sigma_state || L_high < 1 || L_high > 4096) return SRMRA_EINVAL;
    if (!(decay > 0.f) || !isfinite(decay)) return SRMRA_EINVAL;
    if (!workspace || !aligned(workspace) || workspace_bytes < project_workspace_bytes(L_high))
        return SRMRA_EWORKSPACE;
    return launch_project(x_in, x_out, L_high, sigma_state, decay, workspace, stream) == hipSuccess
               ? SRMRA_OK : SRMRA_EDEVICE;
}

}  // extern "C"
