// Kernels of the Fourier-neural-operator surrogate (include/spfc_fno.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fno {

constexpr int C = 32;                 // channels of the Fourier layers
constexpr int MX = 16, MY = 16;       // retained kx, retained |ky| per sign
constexpr int NMODE = MX * 2 * MY;    // 512
constexpr int H = 64;                 // projection hidden width
constexpr int LAYERS = 4;
constexpr int TPB = 256;              // threads per workgroup of every kernel
constexpr int GRED = 512;             // workgroups of the 256-thread weight-gradient kernels
constexpr int GRED64 = 2048;          // workgroups of the 64-thread weight-gradient kernels

// ---------------------------------------------------------------- parameter layout
constexpr int64_t P_LW = 0, P_LB = 2 * C, P_L0 = P_LB + C;
constexpr int64_t W_SIZE = (int64_t)NMODE * C * C;
constexpr int64_t LAYER_SIZE = 2 * W_SIZE + C * C + C;
__host__ __device__ constexpr int64_t p_wr(int l) { return P_L0 + l * LAYER_SIZE; }
__host__ __device__ constexpr int64_t p_wi(int l) { return p_wr(l) + W_SIZE; }
__host__ __device__ constexpr int64_t p_pw(int l) { return p_wi(l) + W_SIZE; }
__host__ __device__ constexpr int64_t p_pb(int l) { return p_pw(l) + C * C; }
constexpr int64_t P_Q1 = P_L0 + LAYERS * LAYER_SIZE, P_QB1 = P_Q1 + H * C, P_Q2 = P_QB1 + H, P_QB2 = P_Q2 + H;
constexpr int64_t P_TOTAL = P_QB2 + 1;

// sizes of the per-workgroup weight-gradient partials
constexpr int PART_PW = C * C + C;          // Pw, Pb of one layer
constexpr int PART_PROJ = H * C + H + H + 1;  // Q1, q1, Q2, q2
constexpr int PART_LIFT = 2 * C + C;        // Lw, Lb
constexpr int PART_MAX = PART_PROJ;

// ---------------------------------------------------------------- bfloat16 storage
// float -> bf16 bits, round to nearest even (the hardware conversion of the target)
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
__host__ __device__ inline float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

template <typename T>
__device__ inline float ldf(const T* p, size_t i);
template <>
__device__ inline float ldf<float>(const float* p, size_t i) { return p[i]; }
template <>
__device__ inline float ldf<uint16_t>(const uint16_t* p, size_t i) { return bf2f(p[i]); }

// erf by Abramowitz and Stegun, Handbook of Mathematical Functions, formula 7.1.26:
// erf(a) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^{-a^2}, t = 1 / (1 + p a), a >= 0,
// absolute error <= 1.5e-7 (plus FP32 rounding) -- far below the bf16 resolution of the
// activations it feeds; branch free (the library erf takes two divergent paths).
__device__ inline float erf_as(float x) {
    const float a = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-a * a * 1.4426950408889634f);
    return copysignf(fmaf(-q * t, e, 1.0f), x);
}

// gelu(z) = z Phi(z), Phi the standard normal distribution function; and its derivative
__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f)); }
__device__ inline float gelu_d(float z) {
    return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * z * z);
}

// ---------------------------------------------------------------- kernel declarations
// (definitions in fno_kernels.hip; launch helpers for the host below)

// out [NMODE][planes]; scale s0 for kx = 0, s1 otherwise (generic plane transforms, used by
// the backward pass)
hipError_t launch_analysis_f32(int n, int planes, const float* in, float s0, float s1, float2* out, const float2* tw,
                               hipStream_t st);
hipError_t launch_synthesis(int n, int planes, const float2* in, float s0, float s1, float* out, int accumulate,
                            const float2* tw, hipStream_t st);
enum { MIX_FWD = 0, MIX_BWD_DATA = 1, MIX_BWD_WEIGHT = 2 };
// FWD: out = mix(a) with packed weights wpk [NMODE][64][64] bf16.
// BWD_DATA: out = gradient with respect to the mixing input, from a = gradient of its output.
// BWD_WEIGHT: gWr/gWi = weight gradients from a = mixing input, g = gradient of its output.
hipError_t launch_mix(int mode, int batch, const float2* a, const float2* g, const uint16_t* wpk, float2* out,
                      float* gwr, float* gwi, hipStream_t st);
hipError_t launch_pack_weights(const float* wr, const float* wi, uint16_t* wpk, hipStream_t st);

// Row/column form of the forward pass (see fno_kernels.hip).  Activations are
// channel-blocked: row (b, y) is one block [C / 8][n][8] of bf16.
// x-basis tables bx [2][n][32] and bxt [2][32][n] (bf16 hi, lo).
hipError_t launch_basis(int n, uint16_t* bx, uint16_t* bxt, hipStream_t st);
enum { RK_LIFT = 0, RK_LAYER = 1, RK_LAST = 2 };
struct RowIn {
    const float* phi;    // LIFT: fields [b][n][n]
    const float* eps;    // LIFT: [b]
    const float* prm;
    int layer;           // LAYER (0 .. LAYERS - 2), LAST (LAYERS - 1)
    const float* Z;      // LAYER, LAST: y half of the synthesis [32][n][b C]
    const uint16_t* v;   // LAYER, LAST: activations in
    uint16_t* vout;      // activations out (LAST: v4, optional)
    uint16_t* uout;      // LAYER: pre-activations (optional)
    float* xout;         // LIFT, LAYER: x half of the analysis [32][n][b C]; LAST: of the output [32][n][b]
    const uint16_t* bx;
    const uint16_t* bxt;
    const float2* tw;
};
hipError_t launch_row(int n, int batch, int kind, const RowIn& in, hipStream_t st);
// trig tables of the column kernels: ta, ts [2][2][32][n] bf16 each
hipError_t launch_trig(int n, uint16_t* ta, uint16_t* ts, hipStream_t st);
hipError_t launch_col_anal(int n, int planes, const float* xp, float s, float2* out, const uint16_t* ta,
                           hipStream_t st);
hipError_t launch_col_synth(int n, int planes, const float2* in, float s0, float s1, bool drop0, float* zout,
                            const uint16_t* ts, hipStream_t st);
hipError_t launch_finish(int n, int batch, const float* phi, const float* zo, const float2* tw, const float* target,
                         float* pred, float* gpred, float* lpart, float* gpart, hipStream_t st);
hipError_t launch_center(int n, int batch, const float* gpred, const float* gpart, float* gout, hipStream_t st);
hipError_t launch_project_bwd(int n, int batch, const uint16_t* v4, const float* prm, const float* gout, float* gv,
                              float* partials, hipStream_t st);
hipError_t launch_pointwise_bwd(int n, int batch, bool act, const float* gout, const uint16_t* u, const uint16_t* v,
                                const float* pw, float* gu, float* gv, float* partials, hipStream_t st);
hipError_t launch_lift_bwd(int n, int batch, const float* gv0, const float* phi, const float* eps, float* partials,
                           hipStream_t st);
hipError_t launch_reduce(const float* partials, int nrows, int cnt, float scale, float* dst, hipStream_t st);
hipError_t launch_adam(int64_t count, float* prm, const float* grad, float* m, float* v, float lr, float c1,
                       float c2, hipStream_t st);

}  // namespace fno
