// C ABI of the SR-MRA EM step (see include/srmra.h): argument validation,
// workspace layout, launch geometry and the launch sequence of one step.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/srmra.h"
#include "srmra_common.h"

namespace srmra {
// aux kernels (srmra_aux.hip)
__global__ void k_obs_norms(const float*, int64_t, int, double*);
__global__ void k_pack_x(const float*, const float*, int, int, double, float*, float*);
__global__ void k_lse_combine(const float2*, int, int64_t, const double*, double, float*, double*,
                              float*);
__global__ void k_reduce_partials(const float*, const float*, int, int, double*, double*);
__global__ void k_finalize(const double*, const double*, int, int, const float*, const double*, int,
                           float*, float*, float*, double*, double*, double*);
// pass launchers (srmra_mfma.hip, srmra_valu.hip, srmra_bf16.hip)
hipError_t launch_mfma(int LL, int pass, const StepArgs& p, hipStream_t s);
hipError_t launch_valu(int LL, int pass, const StepArgs& p, hipStream_t s);
bool mfma_geom(int LL, int& cpw, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2);
bool valu_geom(int LL, int KK, int& cpb, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2);
bool bf16_geom(int LL, int& cpb, int& nt, size_t& lds1, size_t& lds2, const void*& f1,
               const void*& f2);
hipError_t launch_bf16(int LL, int pass, const StepArgs& p, const void* prep_extra, hipStream_t s);
hipError_t launch_prep_bf16(int LL, const float* y, int64_t N, void* prep_extra, hipStream_t s);
size_t bf16_prepared_extra(int LL, int64_t N);
}  // namespace srmra

using namespace srmra;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool supported_ll(int LL) {
    return LL == 8 || LL == 12 || LL == 16 || LL == 24 || LL == 32 || LL == 48 || LL == 64;
}

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

int occupancy(const void* f, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 256, lds) != hipSuccess || n < 1) n = 1;
    return n;
}

// Launch geometry and workspace layout of one step.
struct Geom {
    int LL = 0, K = 0, Lh = 0, KK = 0, prec = 0;
    int64_t N = 0;
    int cpb = 0, n_cg = 0, n_part = 0, ntile = 0, n_chunks = 0, n_ll = 0;
    size_t prep_bytes = 0, prep_extra_off = 0;
    int64_t chunk_obs = 0;
    size_t lds1 = 0, lds2 = 0;
    // workspace offsets
    size_t o_prep = 0, o_part = 0, o_lse = 0, o_xt2 = 0, o_beta = 0, o_bpart = 0, o_cpart = 0,
           o_llpart = 0, o_bsum = 0, o_csum = 0, total = 0;
};

int make_geom(int64_t N, int LL, int K, int prec, bool with_norms, Geom& g) {
    if (N < 1 || N > (int64_t)INT32_MAX || K < 1 || LL < 1) return SRMRA_EINVAL;
    if (!supported_ll(LL)) return SRMRA_EUNSUPPORTED;
    if ((int64_t)K * LL > 4096 || K * K > 256) return SRMRA_EUNSUPPORTED;
    if (prec != SRMRA_FP32_PLAIN && prec != SRMRA_FP32_MFMA && prec != SRMRA_BF16_SPLIT3)
        return SRMRA_EUNSUPPORTED;
    g.LL = LL; g.K = K; g.Lh = K * LL; g.KK = K * K; g.N = N; g.prec = prec;
    const void* f1 = nullptr;
    const void* f2 = nullptr;
    bool ok;
    if (prec == SRMRA_FP32_MFMA) ok = mfma_geom(LL, g.cpb, g.ntile, g.lds1, g.lds2, f1, f2);
    else if (prec == SRMRA_BF16_SPLIT3) ok = bf16_geom(LL, g.cpb, g.ntile, g.lds1, g.lds2, f1, f2);
    else ok = valu_geom(LL, g.KK, g.cpb, g.ntile, g.lds1, g.lds2, f1, f2);
    if (!ok) return SRMRA_EUNSUPPORTED;
    g.n_cg = (g.KK + g.cpb - 1) / g.cpb;
    // pass-1 partials per observation: one per component group, or per component
    // pair for the BF16 form (two waves of a block hold different pairs)
    g.n_part = prec == SRMRA_BF16_SPLIT3 ? (g.KK + 1) / 2 : g.n_cg;
    g.prep_extra_off = align_up(sizeof(double) * (size_t)N);
    g.prep_bytes = g.prep_extra_off + (prec == SRMRA_BF16_SPLIT3 ? bf16_prepared_extra(LL, N) : 0);
    // one resident wave of blocks over the whole device for the heavier pass
    const int occ = occupancy(f2, g.lds2);
    const int64_t target = (int64_t)device_cus() * occ;
    const int64_t tiles = (N + g.ntile - 1) / g.ntile;
    int64_t nch = target / g.n_cg;
    if (nch >= 16) nch -= nch % 8;               // same chunk -> same XCD for all groups
    if (nch < 1) nch = 1;
    if (nch > tiles) nch = tiles;
    const int64_t tiles_per_chunk = (tiles + nch - 1) / nch;
    g.chunk_obs = tiles_per_chunk * g.ntile;
    g.n_chunks = (int)((N + g.chunk_obs - 1) / g.chunk_obs);
    g.n_ll = (int)((N + 255) / 256);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    g.o_prep = with_norms ? take(g.prep_bytes) : 0;
    g.o_part = take(sizeof(float2) * (size_t)g.n_part * (size_t)N);
    g.o_lse = take(sizeof(float) * (size_t)N);
    g.o_xt2 = take(sizeof(float) * (size_t)g.KK * LL * 2 * LL);
    g.o_beta = take(sizeof(float) * (size_t)g.KK * LL * LL);
    g.o_bpart = take(sizeof(float) * (size_t)g.n_chunks * g.KK * LL * LL);
    g.o_cpart = take(sizeof(float) * (size_t)g.n_chunks * g.KK * LL * LL);
    g.o_llpart = take(sizeof(double) * (size_t)g.n_ll);
    g.o_bsum = take(sizeof(double) * (size_t)g.KK * LL * LL);
    g.o_csum = take(sizeof(double) * (size_t)g.KK * LL * LL);
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
    const void* prep_extra = prep + g.prep_extra_off;
    p.y = y;
    p.ynorm = ynorm;
    p.N = g.N;
    p.K = g.K;
    p.Lh = g.Lh;
    p.KK = g.KK;
    p.inv_s2 = (float)(1.0 / ((double)sigma * (double)sigma));
    p.inv_2s2 = 1.0 / (2.0 * (double)sigma * (double)sigma);
    p.xt2 = (const float*)(ws + g.o_xt2);
    p.betaT = (const float*)(ws + g.o_beta);
    p.part = (float2*)(ws + g.o_part);
    p.lse = (float*)(ws + g.o_lse);
    p.bpart = (float*)(ws + g.o_bpart);
    p.cpart = (float*)(ws + g.o_cpart);
    p.n_chunks = g.n_chunks;
    p.n_cg = g.n_cg;
    p.cpb = g.cpb;
    p.ntile = g.ntile;
    p.chunk_obs = g.chunk_obs;
    const int LL = g.LL;
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], stream); };

    mark(0);
    hipLaunchKernelGGL(k_pack_x, dim3(g.KK), dim3(256), 0, stream, x, log_rho, g.K, LL, p.inv_2s2,
                       (float*)(ws + g.o_xt2), (float*)(ws + g.o_beta));
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    mark(1);
    auto pass = [&](int k) -> hipError_t {
        if (g.prec == SRMRA_FP32_MFMA) return launch_mfma(LL, k, p, stream);
        if (g.prec == SRMRA_BF16_SPLIT3) return launch_bf16(LL, k, p, prep_extra, stream);
        return launch_valu(LL, k, p, stream);
    };
    hipError_t e = pass(1);
    if (e != hipSuccess) return SRMRA_EDEVICE;
    mark(2);
    hipLaunchKernelGGL(k_lse_combine, dim3(g.n_ll), dim3(256), 0, stream, (const float2*)p.part,
                       g.n_part, g.N, ynorm, p.inv_2s2, p.lse, (double*)(ws + g.o_llpart), ll_obs);
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    mark(3);
    e = pass(2);
    if (e != hipSuccess) return SRMRA_EDEVICE;
    mark(4);
    const int per = g.KK * LL * LL;
    hipLaunchKernelGGL(k_reduce_partials, dim3((per + 255) / 256), dim3(256), 0, stream,
                       (const float*)p.bpart, (const float*)p.cpart, g.n_chunks, per,
                       (double*)(ws + g.o_bsum), (double*)(ws + g.o_csum));
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, stream, (const double*)(ws + g.o_bsum),
                       (const double*)(ws + g.o_csum), g.K, LL, x, (const double*)(ws + g.o_llpart),
                       g.n_ll, x_new, rho_new, log_rho_new, loglik, b_out, c_out);
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
    }
    return "unknown status";
}

const char* srmra_version(void) { return "srmra 0.1 gfx950"; }

size_t srmra_em_step_workspace_bytes(int64_t N, int L_low, int K, int precision) {
    Geom g;
    if (make_geom(N, L_low, K, precision, true, g) != SRMRA_OK) return 0;
    return g.total;
}

size_t srmra_prepared_bytes(int64_t N, int L_low, int K, int precision) {
    Geom g;
    if (make_geom(N, L_low, K, precision, false, g) != SRMRA_OK) return 0;
    return g.prep_bytes;
}

static int enqueue_prepare(const Geom& g, const float* y, char* prep, hipStream_t stream) {
    hipLaunchKernelGGL(k_obs_norms, dim3((unsigned)((g.N + 3) / 4)), dim3(256), 0, stream, y, g.N,
                       g.LL * g.LL, (double*)prep);
    if (hipGetLastError() != hipSuccess) return SRMRA_EDEVICE;
    if (g.prec == SRMRA_BF16_SPLIT3 &&
        launch_prep_bf16(g.LL, y, g.N, prep + g.prep_extra_off, stream) != hipSuccess)
        return SRMRA_EDEVICE;
    return SRMRA_OK;
}

int srmra_prepare_observations(const float* y, int64_t N, int L_low, int K, int precision,
                               void* prep, size_t prep_bytes, hipStream_t stream) {
    if (!y || !prep || (uintptr_t)y % 16 != 0) return SRMRA_EINVAL;
    Geom g;
    const int st = make_geom(N, L_low, K, precision, false, g);
    if (st != SRMRA_OK) return st;
    if (!aligned(prep) || prep_bytes < g.prep_bytes) return SRMRA_EWORKSPACE;
    return enqueue_prepare(g, y, (char*)prep, stream);
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
        st = enqueue_prepare(g, y, ws + g.o_prep, stream);
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

// ---------------------------------------------------------------- batched form
struct srmra_plan {
    int precision = 0;
    std::vector<srmra_problem> probs;
};

int srmra_plan_create(const srmra_problem* probs, int count, int precision, srmra_plan** plan,
                      size_t* workspace_bytes) {
    (void)probs; (void)count; (void)precision;
    if (plan) *plan = nullptr;
    if (workspace_bytes) *workspace_bytes = 0;
    return SRMRA_EUNSUPPORTED;
}

int srmra_plan_set_iterate(srmra_plan* plan, int index, const float* x, const float* log_rho,
                           float* x_new, float* rho_new, float* log_rho_new) {
    (void)plan; (void)index; (void)x; (void)log_rho; (void)x_new; (void)rho_new; (void)log_rho_new;
    return SRMRA_EUNSUPPORTED;
}

int srmra_plan_upload(srmra_plan* plan, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    (void)plan; (void)workspace; (void)workspace_bytes; (void)stream;
    return SRMRA_EUNSUPPORTED;
}

int srmra_plan_execute(srmra_plan* plan, void* workspace, size_t workspace_bytes,
                       hipStream_t stream) {
    (void)plan; (void)workspace; (void)workspace_bytes; (void)stream;
    return SRMRA_EUNSUPPORTED;
}

void srmra_plan_destroy(srmra_plan* plan) { delete plan; }

}  // extern "C"
