// Shared definitions for the SR-MRA EM-step kernels (gfx950 / CDNA4).
//
// Index conventions (Sec. 1 eq. model_1 and the proof of Thm. 1):
//   polyphase component c = (c1, c2) in {0..K-1}^2, comp index c = c1*K + c2,
//   x_c[l1][l2] = x[c1 + l1*K][c2 + l2*K];
//   a shift s = (s1, s2) in Z_Lh^2 corresponds to (c, t) with
//   c = (-s) mod K, t = ceil(s / K) mod Ll, and s = (t*K - c) mod Lh;
//   then P R_s x = R^low_t x_c, i.e. y[n] = x_c[n - t].
// Score  S_{i,c}[t1][t2] = <y_i, R_t x_c> = sum_{r1,b2} y_i[r1][(b2+t2)%Ll] * x_c[(r1-t1)%Ll][b2].
// Back-projection (right-hand side of eq. x_EM, component c):
//   b_c[q1][q2] = sum_i sum_{a1,t2} w_{i,c}[(a1-q1)%Ll][t2] * y_i[a1][(q2+t2)%Ll].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srmra {

// ---------------------------------------------------------------- geometry
// Tile side of the per-(observation, component) Ll x Ll score map.
template <int LL> struct Tile {
    static constexpr int T = LL <= 8 ? 8 : (LL <= 16 ? 16 : (LL <= 32 ? 32 : 64));
    static constexpr int G = T <= 32 ? 32 / T : 1;      // obs per row tile, comps per col tile
    static constexpr int RB = 2, CB = 2;                 // register blocking of 32x32 tiles
    static constexpr int OPW = T <= 32 ? RB * G : 1;     // observations per wave
    static constexpr int CPW = T <= 32 ? CB * G : 1;     // components per wave (= per block)
    static constexpr int WAVES = 4;
    static constexpr int NT = WAVES * OPW;               // observations per block tile
    // LDS strides (floats) chosen so that the observations / components that share
    // one 32-lane half of an MFMA operand land in different banks.
    static constexpr int OS = ((LL * LL + 31) / 32) * 32 + (T < 32 ? T : 0);
    static constexpr int XS = ((LL * 2 * LL + 31) / 32) * 32 + (T < 32 ? T : 0);
    static constexpr int BS = ((LL * LL + 31) / 32) * 32 + (T < 32 ? T : 0);
};

// Vector-ALU form: each thread owns a 4x4 block of one component's score map for
// NOV observations.
template <int LL> struct Valu {
    static constexpr int NOV = 2;
    static constexpr int BLK = (LL / 4) * (LL / 4);       // 4x4 blocks per component
    static constexpr int YS = LL * 2 * LL + 4;            // doubled-row y stride (floats)
    static constexpr int XS = LL * 2 * LL + 4;
};

struct StepArgs {
    const float* y;          // [N][Ll][Ll]
    const double* ynorm;     // [N]  ||y_i - mu||^2
    const double* centre;    // device scalar mu: intensity offset taken off y and x (0: none)
    int64_t N;
    int K, Lh, KK;           // K, K*Ll, K*K
    float inv_s2;            // 1 / sigma^2
    double inv_2s2;          // 1 / (2 sigma^2)
    // per-step packed x
    const float* xt2;        // [KK][Ll][2Ll]  xt2[c][b2][a] = x_c[a % Ll][b2]
    const float* betaT;      // [KK][Ll(t2)][Ll(t1)]
    const uint4* xb;         // BF16 form: x as MFMA B fragments [KK][k-step][plane][lane]
    // pass-1 output / pass-2 input
    float2* part;            // [n_cg][N]  (max, sum) of exp over the group's shifts
    float2* lse;             // [N] (m_i, l_i): LSE_i = m_i + l_i with m_i the largest
                             // log-joint term (an FP32 value of the step's own
                             // arithmetic) and l_i = log sum_s exp(a_is - m_i), so a
                             // weight exp((a - m_i) - l_i) loses nothing to the
                             // rounding of a large LSE_i
    // pass-2 outputs
    float* bpart;            // [n_chunks][KK][Ll*Ll]   (q1*Ll + q2)
    float* cpart;            // [n_chunks][KK][Ll*Ll]   (t1*Ll + t2)
    int n_chunks, n_cg;      // grid: observation chunks x component groups
    int cpb;                 // components per block (component group size)
    int ntile;               // observations per block tile
    int64_t chunk_obs;       // observations per chunk (multiple of ntile)
    int fuse_wc;             // FP32 MFMA single pass: component groups per block (0: two passes)
};

__device__ __forceinline__ float fast_exp(float v) { return __expf(v); }

// The offset mu as the FP32 value every kernel subtracts (0 without centring).
__device__ __forceinline__ float centre_of(const double* centre) {
    return centre ? (float)*centre : 0.f;
}

}  // namespace srmra
