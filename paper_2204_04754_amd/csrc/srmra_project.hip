// Projection step of the projected EM (Alg. 2) with a Gaussian-smoothing
// stand-in for the denoiser: x <- D(x, s), then s <- decay * s
// (eq. decaying_function with decay = 2^(-1/10)).  D(x, s) is a circular
// Gaussian blur of standard deviation s pixels of the L_high grid: taps
// k in [-R, R], R = min(floor(4 s + 1/2), L_high) (R = 0, the identity, when s
// is below 1/8, not positive or not finite), weights exp(-k^2 / 2 s^2)
// normalised to sum 1, along rows and then along columns, circular boundary.
// The noise level s is a device scalar, so a sequence of EM steps and
// projections needs no host work and can be captured as one graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace srmra {

// Workspace: [R (int), pad][weights 2 L_high + 1 floats][tmp L_high^2 floats]
constexpr int kTapsOff = 64;   // floats

__device__ __forceinline__ int taps_radius(float s, int Lh) {
    if (!(s > 0.f) || !isfinite(s)) return 0;
    const double r = floor(4.0 * (double)s + 0.5);
    return r >= (double)Lh ? Lh : (int)r;
}

// One block of 256 threads: the taps of the current s (FP64, normalised by a
// fixed-order sum), then the decayed s for the next projection.
__global__ __launch_bounds__(256) void k_project_taps(float* __restrict__ sigma_state, float decay,
                                                      int Lh, float* __restrict__ ws) {
    __shared__ double red[256];
    const float s = *sigma_state;
    const int R = taps_radius(s, Lh);
    const double inv = R > 0 ? 1.0 / (2.0 * (double)s * (double)s) : 0.0;
    double acc = 0.0;
    for (int k = threadIdx.x; k <= 2 * R; k += 256) {
        const double d = (double)(k - R);
        acc += exp(-d * d * inv);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double norm = red[0];
    float* w = ws + kTapsOff;
    for (int k = threadIdx.x; k <= 2 * R; k += 256) {
        const double d = (double)(k - R);
        w[k] = (float)(exp(-d * d * inv) / norm);
    }
    if (threadIdx.x == 0) {
        reinterpret_cast<int*>(ws)[0] = R;
        *sigma_state = s * decay;
    }
}

// axis 0 (rows index m1): out[m1][m2] = sum_k w[k] in[(m1 - k) mod Lh][m2]
__global__ __launch_bounds__(256) void k_blur_axis0(const float* __restrict__ in, float* __restrict__ out,
                                                    int Lh, const float* __restrict__ ws) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)Lh * Lh) return;
    const int R = reinterpret_cast<const int*>(ws)[0];
    const float* w = ws + kTapsOff;
    const int m1 = (int)(e / Lh), m2 = (int)(e % Lh);
    float acc = 0.f;
    for (int k = -R; k <= R; ++k) {
        int r = (m1 - k) % Lh;
        r += r < 0 ? Lh : 0;
        acc += w[k + R] * in[(int64_t)r * Lh + m2];
    }
    out[e] = acc;
}

// axis 1 (columns index m2)
__global__ __launch_bounds__(256) void k_blur_axis1(const float* __restrict__ in, float* __restrict__ out,
                                                    int Lh, const float* __restrict__ ws) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)Lh * Lh) return;
    const int R = reinterpret_cast<const int*>(ws)[0];
    const float* w = ws + kTapsOff;
    const int m1 = (int)(e / Lh), m2 = (int)(e % Lh);
    const float* row = in + (int64_t)m1 * Lh;
    float acc = 0.f;
    for (int k = -R; k <= R; ++k) {
        int c = (m2 - k) % Lh;
        c += c < 0 ? Lh : 0;
        acc += w[k + R] * row[c];
    }
    out[e] = acc;
}

size_t project_workspace_bytes(int Lh) {
    const size_t taps = sizeof(float) * ((size_t)kTapsOff + 2 * (size_t)Lh + 1);
    const size_t off = (taps + 255) / 256 * 256;
    return off + sizeof(float) * (size_t)Lh * Lh;
}

hipError_t launch_project(const float* x_in, float* x_out, int Lh, float* sigma_state, float decay,
                          void* workspace, hipStream_t s) {
    float* ws = (float*)workspace;
    const size_t taps = sizeof(float) * ((size_t)kTapsOff + 2 * (size_t)Lh + 1);
    float* tmp = (float*)((char*)workspace + (taps + 255) / 256 * 256);
    const unsigned blocks = (unsigned)(((int64_t)Lh * Lh + 255) / 256);
    hipLaunchKernelGGL(k_project_taps, dim3(1), dim3(256), 0, s, sigma_state, decay, Lh, ws);
    hipLaunchKernelGGL(k_blur_axis0, dim3(blocks), dim3(256), 0, s, x_in, tmp, Lh, (const float*)ws);
    hipLaunchKernelGGL(k_blur_axis1, dim3(blocks), dim3(256), 0, s, (const float*)tmp, x_out, Lh,
                       (const float*)ws);
    return hipGetLastError();
}

}  // namespace srmra
