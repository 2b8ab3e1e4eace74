// The paper's reconstruction error, error(x_hat) = min over circular 2-D
// translations s of ||R_s x_hat - x||_F / ||x||_F with (R_s v)[m] = v[m - s]
// (Sec. 5, the error measure).  Every distance is summed directly in FP64 (no
// ||a||^2 + ||b||^2 - 2<a, b> cancellation, so an exact recovery reads 0).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace srmra {

// One block per translation s = (s1, s2): d[s] = sum_m (x_hat[m - s] - x[m])^2.
__global__ __launch_bounds__(256) void k_shift_dist(const float* __restrict__ xh,
                                                    const float* __restrict__ x, int Lh,
                                                    double* __restrict__ d) {
    __shared__ double red[256];
    const int s1 = blockIdx.x / Lh, s2 = blockIdx.x % Lh;
    double acc = 0.0;
    for (int e = threadIdx.x; e < Lh * Lh; e += 256) {
        const int m1 = e / Lh, m2 = e % Lh;
        int a = m1 - s1, b = m2 - s2;
        a += a < 0 ? Lh : 0;
        b += b < 0 ? Lh : 0;
        const double v = (double)xh[a * Lh + b] - (double)x[e];
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) d[blockIdx.x] = red[0];
}

// One block of 1024: the smallest distance (lowest s1 * Lh + s2 on ties),
// ||x||^2 in FP64, the relative error and the minimising translation.
__global__ __launch_bounds__(1024) void k_shift_min(const double* __restrict__ d,
                                                   const float* __restrict__ x, int Lh,
                                                   double* __restrict__ err,
                                                   int* __restrict__ best) {
    __shared__ double bd[1024];
    __shared__ int bi[1024];
    __shared__ double nn[1024];
    const int n = Lh * Lh;
    double m = INFINITY, q = 0.0;
    int mi = n;
    for (int k = threadIdx.x; k < n; k += 1024) {
        if (d[k] < m) { m = d[k]; mi = k; }
        q += (double)x[k] * (double)x[k];
    }
    bd[threadIdx.x] = m;
    bi[threadIdx.x] = mi;
    nn[threadIdx.x] = q;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double o = bd[threadIdx.x + st];
            const int oi = bi[threadIdx.x + st];
            if (o < bd[threadIdx.x] || (o == bd[threadIdx.x] && oi < bi[threadIdx.x])) {
                bd[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
            nn[threadIdx.x] += nn[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *err = sqrt(bd[0]) / sqrt(nn[0]);
        if (best) {
            best[0] = bi[0] / Lh;
            best[1] = bi[0] % Lh;
        }
    }
}

size_t shift_error_workspace_bytes(int Lh) { return sizeof(double) * (size_t)Lh * Lh; }

hipError_t launch_shift_error(const float* xh, const float* x, int Lh, double* err, int* best,
                              void* ws, hipStream_t s) {
    hipLaunchKernelGGL(k_shift_dist, dim3((unsigned)(Lh * Lh)), dim3(256), 0, s, xh, x, Lh, (double*)ws);
    hipLaunchKernelGGL(k_shift_min, dim3(1), dim3(1024), 0, s, (const double*)ws, x, Lh, err, best);
    return hipGetLastError();
}

}  // namespace srmra
