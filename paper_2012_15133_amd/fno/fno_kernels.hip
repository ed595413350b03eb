// Kernels of the Fourier-neural-operator surrogate.  Every launch helper checks
// nothing about sizes: the host driver (fno.cpp) validates shapes before calling.
#include "fno_kernels.hpp"

namespace fno {

namespace {

__device__ inline float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// fixed-order workgroup sum, result in thread 0 (all threads must call)
__device__ inline float block_sum_f(float v, float* red /* >= TPB/64 floats of LDS */) {
    v = wave_sum_f(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0)
        for (int w = 0; w < TPB / 64; ++w) s += red[w];
    return s;
}

}  // namespace

// ---------------------------------------------------------------- truncated transforms

// One workgroup per plane.  out[m][plane] = s_kx sum_{y,x} in[y][x] e^{-2 pi i (kx x + ky y)/N}:
// rows in chunks of 16 (thread = (row, kx)) give X[y][kx], then the y sums (thread =
// (kx, two j)).
template <int N, typename TIn>
__global__ void __launch_bounds__(TPB) k_analysis(int planes, const TIn* in, float s0, float s1, float2* out,
                                                  const float2* twg) {
    __shared__ float2 tw[N];
    __shared__ float chunk[16 * N];
    __shared__ __align__(16) float2 X[N * MX];
    const int t = threadIdx.x, p = blockIdx.x;
    const TIn* src = in + (size_t)p * N * N;
    for (int i = t; i < N; i += TPB) tw[i] = twg[i];
    const int r = t >> 4, kx = t & 15;
    for (int y0 = 0; y0 < N; y0 += 16) {
        __syncthreads();
        for (int i = t; i < 16 * N; i += TPB) chunk[i] = ldf(src, (size_t)y0 * N + i);
        __syncthreads();
        float re = 0.f, im = 0.f;
        const float* row = chunk + r * N;
#pragma unroll 8
        for (int x = 0; x < N; ++x) {
            const float v = row[x];
            const float2 w = tw[(kx * x) & (N - 1)];
            re += v * w.x;
            im -= v * w.y;
        }
        X[(y0 + r) * MX + kx] = make_float2(re, im);
    }
    __syncthreads();
    const float s = kx == 0 ? s0 : s1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = (t >> 4) + 16 * h;
        const int ky = j < MY ? j : N - 2 * MY + j;
        float re = 0.f, im = 0.f;
#pragma unroll 8
        for (int y = 0; y < N; ++y) {
            const float2 a = X[y * MX + kx];
            const float2 w = tw[(ky * y) & (N - 1)];
            re += a.x * w.x + a.y * w.y;
            im += a.y * w.x - a.x * w.y;
        }
        out[(size_t)(kx * 2 * MY + j) * planes + p] = make_float2(re * s, im * s);
    }
}

// One workgroup per plane.  out[y][x] (+)= sum_m s_kx Re(in[m] e^{+2 pi i (kx x + ky y)/N}):
// Z[y][kx] = sum_j U[kx][j] e^{+i ky y}, then the x sums.
template <int N>
__global__ void __launch_bounds__(TPB) k_synthesis(int planes, const float2* in, float s0, float s1, float* out,
                                                   int accumulate, const float2* twg) {
    __shared__ float2 tw[N];
    __shared__ float2 U[NMODE];
    __shared__ float2 Z[N * MX];
    const int t = threadIdx.x, p = blockIdx.x;
    for (int i = t; i < N; i += TPB) tw[i] = twg[i];
    for (int m = t; m < NMODE; m += TPB) {
        const float s = (m >> 5) == 0 ? s0 : s1;
        const float2 u = in[(size_t)m * planes + p];
        U[m] = make_float2(u.x * s, u.y * s);
    }
    __syncthreads();
    const int kx = t & 15;
    for (int y = t >> 4; y < N; y += 16) {
        float re = 0.f, im = 0.f;
#pragma unroll 8
        for (int j = 0; j < 2 * MY; ++j) {
            const int ky = j < MY ? j : N - 2 * MY + j;
            const float2 w = tw[(ky * y) & (N - 1)];
            const float2 u = U[kx * 2 * MY + j];
            re += u.x * w.x - u.y * w.y;
            im += u.x * w.y + u.y * w.x;
        }
        Z[y * MX + kx] = make_float2(re, im);
    }
    __syncthreads();
    float* dst = out + (size_t)p * N * N;
    for (int i = t; i < N * N; i += TPB) {
        const int y = i / N, x = i - y * N;
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < MX; ++k) {
            const float2 z = Z[y * MX + k];
            const float2 w = tw[(k * x) & (N - 1)];
            acc += z.x * w.x - z.y * w.y;
        }
        dst[i] = accumulate ? dst[i] + acc : acc;
    }
}

// ---------------------------------------------------------------- complex mode mixing (MFMA)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// D (16 x 16, f32) += A (16 x 32) B (32 x 16) on one wave, bf16 operands from LDS:
// A(i, k) = As[i * ars + k * acs], B(k, n) = Bs[k * brs + n * bcs] (uint16 bf16 bits).
// Operand layout of v_mfma_f32_16x16x32_bf16: lane l holds A(l % 16, 8 (l / 16) + j) and
// B(8 (l / 16) + j, l % 16), j < 8; the result D(4 (l / 16) + j, l % 16), j < 4.
__device__ inline f32x4 mma16x16x32(f32x4 acc, const uint16_t* As, int ars, int acs, const uint16_t* Bs, int brs,
                                    int bcs) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kb = 8 * (lane >> 4);
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = __builtin_bit_cast(__bf16, As[r * ars + (kb + j) * acs]);
        b[j] = __builtin_bit_cast(__bf16, Bs[(kb + j) * brs + r * bcs]);
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// One workgroup (4 waves) per mode m.  Real form of the complex product with the
// 64 x 64 block matrix Wm = [[Wr, Wi], [-Wi, Wr]] of the mode:
//   FWD:        [Re U | Im U](b)  = [Re V | Im V](b) Wm
//   BWD_DATA:   [Re gV | Im gV](b) = [Re gU | Im gU](b) Wm^T
//   BWD_WEIGHT: gWm = sum_b [Re V | Im V](b)^T [Re gU | Im gU](b), folded into
//               gWr = gWm[0:32, 0:32] + gWm[32:64, 32:64], gWi = gWm[0:32, 32:64] - gWm[32:64, 0:32].
// Rows (samples) are padded to 32 with zeros.
template <int MODE>
__global__ void __launch_bounds__(TPB) k_mix(int batch, const float2* a, const float2* g, const uint16_t* wpk,
                                             float2* out, float* gwr, float* gwi) {
    constexpr int BMAX = 128;
    __shared__ uint16_t As[BMAX * 64];
    __shared__ uint16_t Gs[MODE == MIX_BWD_WEIGHT ? BMAX * 64 : 1];
    __shared__ uint16_t Ws[MODE == MIX_BWD_WEIGHT ? 1 : 64 * 64];
    __shared__ float Gw[MODE == MIX_BWD_WEIGHT ? 64 * 64 : 1];
    const int m = blockIdx.x, t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int bp = (batch + 31) & ~31;
    const int planes = batch * C;
    // samples x 64 real columns: column c < 32 is Re of channel c, c >= 32 Im of c - 32
    for (int i = t; i < bp * C; i += TPB) {
        const int b = i / C, c = i - b * C;
        float2 v = make_float2(0.f, 0.f);
        if (b < batch) v = a[(size_t)m * planes + b * C + c];
        As[b * 64 + c] = f2bf(v.x);
        As[b * 64 + C + c] = f2bf(v.y);
        if constexpr (MODE == MIX_BWD_WEIGHT) {
            float2 q = make_float2(0.f, 0.f);
            if (b < batch) q = g[(size_t)m * planes + b * C + c];
            Gs[b * 64 + c] = f2bf(q.x);
            Gs[b * 64 + C + c] = f2bf(q.y);
        }
    }
    if constexpr (MODE != MIX_BWD_WEIGHT) {
        const uint16_t* w = wpk + (size_t)m * 64 * 64;
        for (int i = t; i < 64 * 64; i += TPB) Ws[i] = w[i];
    }
    __syncthreads();
    const int col = lane & 15, rb = 4 * (lane >> 4);
    if constexpr (MODE == MIX_BWD_WEIGHT) {
        // rows k (64) = 4 waves x 16, columns n (64) = 4 tiles, reduction over samples
        f32x4 acc[4] = {};
        const int k0 = wave * 16;
        for (int b0 = 0; b0 < bp; b0 += 32)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = mma16x16x32(acc[nt], As + b0 * 64 + k0, 1, 64, Gs + b0 * 64 + nt * 16, 64, 1);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) Gw[(k0 + rb + j) * 64 + nt * 16 + col] = acc[nt][j];
        __syncthreads();
        for (int i = t; i < C * C; i += TPB) {
            const int ii = i / C, o = i - ii * C;
            gwr[(size_t)m * C * C + i] = Gw[ii * 64 + o] + Gw[(C + ii) * 64 + C + o];
            gwi[(size_t)m * C * C + i] = Gw[ii * 64 + C + o] - Gw[(C + ii) * 64 + o];
        }
    } else {
        for (int s0 = wave * 16; s0 < bp; s0 += 4 * 16) {
            f32x4 acc[4] = {};
#pragma unroll
            for (int k0 = 0; k0 < 64; k0 += 32)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    if constexpr (MODE == MIX_FWD)
                        acc[nt] = mma16x16x32(acc[nt], As + s0 * 64 + k0, 64, 1, Ws + k0 * 64 + nt * 16, 64, 1);
                    else  // B(k, n) = Wm(n, k)
                        acc[nt] = mma16x16x32(acc[nt], As + s0 * 64 + k0, 64, 1, Ws + nt * 16 * 64 + k0, 1, 64);
                }
            // D(b, n): n < 32 real part of channel n, n >= 32 imaginary part of n - 32
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int b = s0 + rb + j;
                    if (b < batch) out[(size_t)m * planes + b * C + nt * 16 + col] = make_float2(acc[nt][j], acc[nt + 2][j]);
                }
        }
    }
}

// ---------------------------------------------------------------- row / column form of the forward pass
//
// Activations (bf16) are stored channel-blocked: row (b, y) is one block of C N values
// [c / 8][x][c % 8], so that the 8 channels a matrix-core operand takes at one point are
// 16 contiguous bytes.
//
// X'[n][y][p], the x half of the analysis of plane p = b C + c, is planar in n (n < 16
// holds Re, n >= 16 Im of kx = n % 16) and plane-fastest:  X'[n][y][p] = sum_x v[p][y][x]
// Bx[x][n] with Bx[x][n] = cos(2 pi n x / N) (n < 16) and -sin(2 pi (n - 16) x / N)
// (n >= 16).  Z[n][y][p], the y half of the synthesis (kx weights included), likewise.

typedef short i16x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mfma32(const bf16x8& a, const bf16x8& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// v_mfma_f32_16x16x16_bf16: lane l holds A(l % 16, 4 (l / 16) + j), B(4 (l / 16) + j, l % 16)
// and D(4 (l / 16) + j, l % 16), j < 4 -- a result tile is itself a B operand.
__device__ inline f32x4 mfma16(const i16x4& a, const i16x4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline bf16x8 ld_bf8(const uint16_t* p) { return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p)); }
__device__ inline i16x4 ld_bf4(const uint16_t* p) { return __builtin_bit_cast(i16x4, *reinterpret_cast<const uint2*>(p)); }
__device__ inline uint32_t pack_pair(float a, float b) {
    typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
    const bf2_t h = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
    return __builtin_bit_cast(uint32_t, h);
}
__device__ inline float lo_of(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ inline float hi_of(uint32_t w) { return __builtin_bit_cast(float, w & 0xFFFF0000u); }
// f = hi + lo + O(2^-16 |f|), hi and lo bf16 (pairs converted together)
__device__ inline void split8(const float* f, bf16x8& hi, bf16x8& lo) {
    uint4 h, l;
    uint32_t* hp = &h.x;
    uint32_t* lp = &l.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        hp[j] = pack_pair(f[2 * j], f[2 * j + 1]);
        lp[j] = pack_pair(f[2 * j] - lo_of(hp[j]), f[2 * j + 1] - hi_of(hp[j]));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}
__device__ inline void split4(const float* f, i16x4& hi, i16x4& lo) {
    uint2 h, l;
    h.x = pack_pair(f[0], f[1]);
    h.y = pack_pair(f[2], f[3]);
    l.x = pack_pair(f[0] - lo_of(h.x), f[1] - hi_of(h.x));
    l.y = pack_pair(f[2] - lo_of(h.y), f[3] - hi_of(h.y));
    hi = __builtin_bit_cast(i16x4, h);
    lo = __builtin_bit_cast(i16x4, l);
}
// offset of (channel c, column x) inside a channel-blocked row of length N
__device__ inline int act_in_row(int N, int c, int x) { return ((c >> 3) * N + x) * 8 + (c & 7); }
// store 4 channels c .. c + 3 (c % 4 == 0) at one column from an f32 tile column
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pack_bf2(float a, float b) {
    const bf16x2 h = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
    return __builtin_bit_cast(uint32_t, h);
}
__device__ inline i16x4 pack_op4(float a, float b, float c, float d) {
    uint2 w;
    w.x = pack_bf2(a, b);
    w.y = pack_bf2(c, d);
    return __builtin_bit_cast(i16x4, w);
}
__device__ inline void store4(uint16_t* dst, const f32x4& v) {
    uint2 w;
    w.x = pack_bf2(v[0], v[1]);
    w.y = pack_bf2(v[2], v[3]);
    *reinterpret_cast<uint2*>(dst) = w;
}

// x-basis tables, bf16 hi + lo so that hi + lo carries FP32 accuracy:
// bx[part][x][n] = Bx[x][n], bxt[part][n][x] = Bx[x][n] (part 0: hi, 1: lo).
__global__ void __launch_bounds__(TPB) k_basis(int n, uint16_t* bx, uint16_t* bxt) {
    for (int e = blockIdx.x * TPB + threadIdx.x; e < n * 2 * MX; e += gridDim.x * TPB) {
        const int x = e / (2 * MX), c = e - x * 2 * MX;
        const int k = c & 15;
        const double a = 6.283185307179586476925286766559 * (double)((k * x) % n) / (double)n;
        const float v = c < MX ? (float)cos(a) : -(float)sin(a);
        const uint16_t h = f2bf(v), l = f2bf(v - bf2f(h));
        bx[e] = h;
        bx[n * 2 * MX + e] = l;
        bxt[c * n + x] = h;
        bxt[2 * MX * n + c * n + x] = l;
    }
}

constexpr int RROWS = 4;     // rows per workgroup of the row kernel
constexpr int XPITCH = 36;   // floats per channel in the LDS partials of the x-analysis

// Row kernel: one workgroup takes RROWS rows (b, y) in turn; wave w owns the x-tiles
// w N / 64 .. (w + 1) N / 64 - 1 of 16 points.
//   LIFT:  v0[c][x] = Lw[c][0] phi + Lw[c][1] eps + Lb[c]; X' of v0.
//   LAYER: u^T = Bx Z^T + v^T Pw^T + Pb (matrix cores, 16 x 16 tiles: rows x, columns
//          channels; Z and Bx as bf16 hi + lo, hi hi + lo hi + hi lo, and Pw as hi + lo:
//          FP32 accuracy); v' = gelu(u); X' of v' from the tiles directly (a result tile
//          is the B operand of the 16x16x16 product with BxT); v' and u stored
//          channel-blocked after a product with the identity transposes the tile.
//   LAST:  u as LAYER without the activation, v4 = bf16(u) (stored when vout is set);
//          the projection out = Q2 gelu(Q1 v4 + q1) + q2 on matrix cores (the transposed
//          v4 tile is the B operand); then the x half of the analysis of out into
//          xout[b][y][32].
struct RowParams {
    const float* phi;
    const float* eps;
    const float* prm;
    int layer;
    const float* Z;
    const uint16_t* v;
    uint16_t* vout;
    uint16_t* uout;
    float* xout;
    const uint16_t* bx;
    const uint16_t* bxt;
    const float2* tw;
};

template <int N, int KIND>
__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2))) k_rowmm(RowParams a) {
    constexpr int XPW = N / 64;
    // LAST: the projected row [N], analysis partials [8][32], twiddles [N] (float2),
    // q1 and Q2 [2][H]; otherwise two buffers of per-wave analysis partials
    constexpr int LDS_F = KIND == RK_LAST ? (N + 8 * 32 + 2 * N + 2 * H) : (2 * 4 * C * XPITCH);
    constexpr int ZP = 36;   // floats per (row, channel) of the staged Z rows
    __shared__ __align__(16) float lds[LDS_F];
    __shared__ __align__(16) float zs[KIND == RK_LIFT ? 4 : RROWS * C * ZP];   // Z[r][o][k]
    // LIFT: the input rows, double buffered; the next row is loaded (one value per thread)
    // while the current one is lifted
    __shared__ __align__(16) float phis[KIND == RK_LIFT ? 2 * N : 4];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, col = lane & 15, g = lane >> 4;
    const int b = blockIdx.y;
    const int planes = gridDim.y * C;   // plane stride of Z and X' (LAST's output analysis: gridDim.y)
    const float* prm = a.prm;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

    i16x4 ident;   // B(k = 4 g + j, n = col) = (4 g + j == col), bf16 1.0 = 0x3F80
#pragma unroll
    for (int j = 0; j < 4; ++j) ident[j] = (4 * g + j == col) ? (short)0x3F80 : (short)0;

    // constant operands
    bf16x8 bxh[XPW], bxl[XPW];        // A(x = x0 + col, k = 8 g + j) = Bx[x][k]
    i16x4 bth[XPW][2], btl[XPW][2];   // A(n = 16 nt + col, x = x0 + 4 g + j) = Bx[x][n]
    bf16x8 ph[2], pl[2];              // B(i = 8 g + j, o = 16 ot + col) = Pw[o][i]
    float pbv[2] = {0.f, 0.f};
#pragma unroll
    for (int xt = 0; xt < XPW; ++xt) {
        const int x0 = (wave * XPW + xt) * 16;
        if constexpr (KIND == RK_LAYER) {   // LAST reloads them per tile (register budget)
            bxh[xt] = ld_bf8(a.bx + (x0 + col) * 32 + 8 * g);
            bxl[xt] = ld_bf8(a.bx + N * 32 + (x0 + col) * 32 + 8 * g);
        }
        if constexpr (KIND != RK_LAST) {
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                bth[xt][nt] = ld_bf4(a.bxt + (16 * nt + col) * N + x0 + 4 * g);
                btl[xt][nt] = ld_bf4(a.bxt + 32 * N + (16 * nt + col) * N + x0 + 4 * g);
            }
        }
    }
    if constexpr (KIND != RK_LIFT) {
        const float* pw = prm + p_pw(a.layer);
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            const int o = 16 * ot + col;
            float f[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) f[j] = pw[o * C + 8 * g + j];
            split8(f, ph[ot], pl[ot]);
            pbv[ot] = pw[C * C + o];
        }
    }
    // lifting weights of channel 16 ct + col (x-analysis operand) and of channels
    // 16 ct + 4 g + j (stored values)
    float lw[2][3], ls[2][4][3];
    if constexpr (KIND == RK_LIFT) {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int c = 16 * ct + col;
            lw[ct][0] = prm[P_LW + 2 * c];
            lw[ct][1] = prm[P_LW + 2 * c + 1];
            lw[ct][2] = prm[P_LB + c];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c2 = 16 * ct + 4 * g + j;
                ls[ct][j][0] = prm[P_LW + 2 * c2];
                ls[ct][j][1] = prm[P_LW + 2 * c2 + 1];
                ls[ct][j][2] = prm[P_LB + c2];
            }
        }
    }
    // projection (LAST): A(k = 16 kt + col, c = 16 ot + 4 g + j) = Q1[k][c] in registers;
    // q1, Q2 in LDS
    i16x4 qh[KIND == RK_LAST ? 4 : 1][2], ql[KIND == RK_LAST ? 4 : 1][2];
    float q2c = 0.f;
    float* q1s = lds + N + 8 * 32 + 2 * N;
    float* q2s = q1s + H;
    if constexpr (KIND == RK_LAST) {
        const float* q = prm + P_Q1;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int ot = 0; ot < 2; ++ot) {
                float f[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) f[j] = q[(16 * kt + col) * C + 16 * ot + 4 * g + j];
                split4(f, qh[kt][ot], ql[kt][ot]);
            }
        q2c = q[H * C + 2 * H];
        float2* tws = reinterpret_cast<float2*>(lds + N + 8 * 32);
        for (int i = t; i < N; i += TPB) tws[i] = a.tw[i];
        if (t < H) {
            q1s[t] = q[H * C + t];
            q2s[t] = q[H * C + H + t];
        }
        __syncthreads();
    }

    // the Z rows of the workgroup's rows, staged in LDS as zs[r][o][k] (coalesced over the
    // planes of this sample); activations loaded one row ahead
    if constexpr (KIND != RK_LIFT) {
#pragma unroll
        for (int q = 0; q < RROWS * C * 32 / 4 / TPB; ++q) {
            const int f = t + TPB * q;
            const int o4 = f & 7, r = (f >> 3) % RROWS, n = f / (8 * RROWS);
            const float4 z = *reinterpret_cast<const float4*>(
                a.Z + ((size_t)n * N + blockIdx.x * RROWS + r) * planes + b * C + 4 * o4);
            float* d = zs + (r * C + 4 * o4) * ZP + n;
            d[0] = z.x;
            d[ZP] = z.y;
            d[2 * ZP] = z.z;
            d[3 * ZP] = z.w;
        }
        __syncthreads();
    }
    uint4 vq[XPW];
    auto load_row = [&](int yy) {
        const size_t ro = ((size_t)b * N + yy) * (size_t)(C * N);
        if constexpr (KIND == RK_LAYER)   // LAST loads them per tile (register budget)
#pragma unroll
            for (int xt = 0; xt < XPW; ++xt)
                vq[xt] = *reinterpret_cast<const uint4*>(a.v + ro + act_in_row(N, 8 * g, (wave * XPW + xt) * 16 + col));
    };
    if constexpr (KIND != RK_LIFT) load_row(blockIdx.x * RROWS);
    float phi_next = 0.f;
    if constexpr (KIND == RK_LIFT) {
        if (t < N) phis[t] = a.phi[((size_t)b * N + blockIdx.x * RROWS) * N + t];
        __syncthreads();
    }
    // LAST: the operands of one x-tile (basis rows hi / lo, activations), loaded one tile
    // ahead (the next row's first tile after a row's last) so that their loads overlap
    // the current tile's products; the last prefetch of the workgroup re-reads its own row
    struct TileOps {
        bf16x8 bh, bl, vt;
    };
    auto load_tile = [&](int yy, int xt) {
        const int x0 = (wave * XPW + xt) * 16;
        const size_t ro = ((size_t)b * N + yy) * (size_t)(C * N);
        TileOps o;
        o.bh = ld_bf8(a.bx + (x0 + col) * 32 + 8 * g);
        o.bl = ld_bf8(a.bx + N * 32 + (x0 + col) * 32 + 8 * g);
        o.vt = ld_bf8(a.v + ro + act_in_row(N, 8 * g, x0 + col));
        return o;
    };
    TileOps ahead{};
    if constexpr (KIND == RK_LAST) ahead = load_tile(blockIdx.x * RROWS, 0);

    for (int r = 0; r < RROWS; ++r) {
        const int y = blockIdx.x * RROWS + r;
        const size_t rowo = ((size_t)b * N + y) * (size_t)(C * N);
        f32x4 xa[2][2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) xa[ct][nt] = zero4;

        if constexpr (KIND == RK_LIFT) {
            const float e = a.eps[b];
            if (r + 1 < RROWS && t < N) phi_next = a.phi[((size_t)b * N + y + 1) * N + t];
            const float* frow = phis + (r & 1) * N;
#pragma unroll
            for (int xt = 0; xt < XPW; ++xt) {
                const int x0 = (wave * XPW + xt) * 16;
                const float4 f4 = *reinterpret_cast<const float4*>(frow + x0 + 4 * g);
                const float fc = frow[x0 + col];
                const float fv[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    float l4[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) l4[j] = lw[ct][0] * fv[j] + lw[ct][1] * e + lw[ct][2];
                    const i16x4 vb = pack_op4(l4[0], l4[1], l4[2], l4[3]);
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) {
                        xa[ct][nt] = mfma16(bth[xt][nt], vb, xa[ct][nt]);
                        xa[ct][nt] = mfma16(btl[xt][nt], vb, xa[ct][nt]);
                    }
                    f32x4 sv;
#pragma unroll
                    for (int j = 0; j < 4; ++j) sv[j] = ls[ct][j][0] * fc + ls[ct][j][1] * e + ls[ct][j][2];
                    store4(a.vout + rowo + act_in_row(N, 16 * ct + 4 * g, x0 + col), sv);
                }
            }
        } else {
            bf16x8 zh[2], zl[2];   // B(k = 8 g + j, o = 16 ot + col) = Z[o][k]
#pragma unroll
            for (int ot = 0; ot < 2; ++ot) {
                const float* zr = zs + (r * C + 16 * ot + col) * ZP + 8 * g;
                const float4 z0 = *reinterpret_cast<const float4*>(zr);
                const float4 z1 = *reinterpret_cast<const float4*>(zr + 4);
                const float f[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
                split8(f, zh[ot], zl[ot]);
            }
            bf16x8 vx[XPW];
            if constexpr (KIND == RK_LAYER)
#pragma unroll
                for (int xt = 0; xt < XPW; ++xt) vx[xt] = __builtin_bit_cast(bf16x8, vq[xt]);
            if (r + 1 < RROWS) load_row(y + 1);
            float* orow = lds;   // LAST: the projection of the row
            auto tile = [&](int xt) {
                const int x0 = (wave * XPW + xt) * 16;
                i16x4 rb[2];
                bf16x8 bh, bl, vt;
                if constexpr (KIND == RK_LAYER) {
                    bh = bxh[xt];
                    bl = bxl[xt];
                    vt = vx[xt];
                } else {
                    bh = ahead.bh;
                    bl = ahead.bl;
                    vt = ahead.vt;
                    const bool row_end = xt + 1 == XPW;
                    ahead = load_tile(row_end ? (r + 1 < RROWS ? y + 1 : y) : y, row_end ? 0 : xt + 1);
                }
#pragma unroll
                for (int ot = 0; ot < 2; ++ot) {
                    f32x4 acc = zero4;
                    acc = mfma32(bh, zh[ot], acc);
                    acc = mfma32(bh, zl[ot], acc);
                    acc = mfma32(bl, zh[ot], acc);
                    acc = mfma32(vt, ph[ot], acc);
                    acc = mfma32(vt, pl[ot], acc);
                    // acc[j] = u[o = 16 ot + col] at x = x0 + 4 g + j
                    float u[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) u[j] = acc[j] + pbv[ot];
                    const i16x4 ub = pack_op4(u[0], u[1], u[2], u[3]);
                    const i16x4 vb = KIND == RK_LAYER ? pack_op4(gelu(u[0]), gelu(u[1]), gelu(u[2]), gelu(u[3])) : ub;
                    // tv[j] = value at channel 16 ot + 4 g + j, x = x0 + col
                    const f32x4 tv = mfma16(vb, ident, zero4);
                    if constexpr (KIND == RK_LAYER) {
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) {
                            xa[ot][nt] = mfma16(bth[xt][nt], vb, xa[ot][nt]);
                            xa[ot][nt] = mfma16(btl[xt][nt], vb, xa[ot][nt]);
                        }
                        store4(a.vout + rowo + act_in_row(N, 16 * ot + 4 * g, x0 + col), tv);
                        if (a.uout)
                            store4(a.uout + rowo + act_in_row(N, 16 * ot + 4 * g, x0 + col),
                                   mfma16(ub, ident, zero4));
                    } else {
                        if (a.vout) store4(a.vout + rowo + act_in_row(N, 16 * ot + 4 * g, x0 + col), tv);
                        rb[ot] = pack_op4(tv[0], tv[1], tv[2], tv[3]);
                    }
                }
                if constexpr (KIND == RK_LAST) {
                    float s = 0.f;
#pragma unroll
                    for (int kt = 0; kt < 4; ++kt) {
                        f32x4 h = zero4;
#pragma unroll
                        for (int ot = 0; ot < 2; ++ot) {
                            h = mfma16(qh[kt][ot], rb[ot], h);
                            h = mfma16(ql[kt][ot], rb[ot], h);
                        }
                        // h[j]: hidden unit 16 kt + 4 g + j at x = x0 + col
                        const float4 q1 = *reinterpret_cast<const float4*>(q1s + 16 * kt + 4 * g);
                        const float4 q2 = *reinterpret_cast<const float4*>(q2s + 16 * kt + 4 * g);
                        s += q2.x * gelu(h[0] + q1.x);
                        s += q2.y * gelu(h[1] + q1.y);
                        s += q2.z * gelu(h[2] + q1.z);
                        s += q2.w * gelu(h[3] + q1.w);
                    }
                    s += __shfl_xor(s, 16, 64);
                    s += __shfl_xor(s, 32, 64);
                    if (g == 0) orow[x0 + col] = s + q2c;
                }
            };
            if constexpr (KIND == RK_LAYER) {
#pragma unroll
                for (int xt = 0; xt < XPW; ++xt) tile(xt);
            } else {   // one tile at a time (register budget)
#pragma unroll 1
                for (int xt = 0; xt < XPW; ++xt) tile(xt);
            }
        }

        if constexpr (KIND != RK_LAST) {
            // X' of the row: partial sums of each wave's x-tiles, added in wave order
            float* xp = lds + (r & 1) * (4 * C * XPITCH);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        xp[(wave * C + 16 * ct + col) * XPITCH + 16 * nt + 4 * g + j] = xa[ct][nt][j];
            // LIFT: the next input row into the other buffer (its last readers, the tiles of
            // row r - 1, are behind the previous barrier); read after the barrier below
            if constexpr (KIND == RK_LIFT)
                if (r + 1 < RROWS && t < N) phis[((r + 1) & 1) * N + t] = phi_next;
            __syncthreads();
            const int c = t & 31, n0 = (t >> 5) * 4;
            float4 sum = *reinterpret_cast<const float4*>(xp + c * XPITCH + n0);
#pragma unroll
            for (int w = 1; w < 4; ++w) {
                const float4 q = *reinterpret_cast<const float4*>(xp + (w * C + c) * XPITCH + n0);
                sum.x += q.x;
                sum.y += q.y;
                sum.z += q.z;
                sum.w += q.w;
            }
            float* dst = a.xout + ((size_t)n0 * N + y) * planes + b * C + c;
            const size_t ns = (size_t)N * planes;
            dst[0] = sum.x;
            dst[ns] = sum.y;
            dst[2 * ns] = sum.z;
            dst[3 * ns] = sum.w;
        } else {
            // x half of the analysis of the projected row: 8 parts of N / 8 points each
            __syncthreads();
            const float* orow = lds;
            float* pp = lds + N;
            const float2* tws = reinterpret_cast<const float2*>(lds + N + 8 * 32);
            const int n = t & 31, part = t >> 5, k = n & 15;
            float acc = 0.f;
            for (int x = part * (N / 8); x < (part + 1) * (N / 8); ++x) {
                const float2 w = tws[(k * x) & (N - 1)];
                acc += orow[x] * (n < 16 ? w.x : -w.y);
            }
            pp[part * 32 + n] = acc;
            __syncthreads();
            if (t < 32) {
                float sum = 0.f;
#pragma unroll
                for (int q = 0; q < 8; ++q) sum += pp[q * 32 + t];
                a.xout[((size_t)t * N + y) * gridDim.y + b] = sum;
            }
        }
    }
}

// Column kernels on matrix cores.  m = kx * 32 + j is the mode index, ky_j = j (j < 16) or
// N - 32 + j, phi = 2 pi ky_j y / N; spectra are [m][p] (plane fastest).
//   ANAL:  V[m][p] = s sum_y X'[y][p] e^{-i phi}:  Re = C X're + S X'im, Im = C X'im - S X're
//   SYNTH: Z[y][p] = sum_j w U[m][p] e^{+i phi}:   Re = C Ure - S Uim,   Im = S Ure + C Uim
// with C = cos phi, S = sin phi from bf16 hi + lo tables (and the data split likewise:
// hi hi + lo hi + hi lo per product, FP32 accuracy), w = s0 (kx = 0) or s1, and the mode
// kx = ky = 0 left out of SYNTH if drop0.  One wave per (kx, 16 planes).
__device__ inline int ky_of(int N, int j) { return j < MY ? j : N - 2 * MY + j; }

// trig tables: ta[part][cs][j][y] (ANAL, y fastest), ts[part][cs][y][j] (SYNTH, j fastest);
// part 0/1 = hi/lo, cs 0/1 = cos/sin
__global__ void __launch_bounds__(TPB) k_trig(int n, uint16_t* ta, uint16_t* ts) {
    const int total = 2 * MY * n;
    for (int e = blockIdx.x * TPB + threadIdx.x; e < total; e += gridDim.x * TPB) {
        const int j = e / n, y = e - j * n;
        const double a = 6.283185307179586476925286766559 * (double)(((long long)ky_of(n, j) * y) % n) / (double)n;
#pragma unroll
        for (int cs = 0; cs < 2; ++cs) {
            const float v = cs == 0 ? (float)cos(a) : (float)sin(a);
            const uint16_t h = f2bf(v), l = f2bf(v - bf2f(h));
            ta[(size_t)(0 * 2 + cs) * total + j * n + y] = h;
            ta[(size_t)(1 * 2 + cs) * total + j * n + y] = l;
            ts[(size_t)(0 * 2 + cs) * total + y * 2 * MY + j] = h;
            ts[(size_t)(1 * 2 + cs) * total + y * 2 * MY + j] = l;
        }
    }
}

template <int N, int PT>
__global__ void __launch_bounds__(TPB) k_col_anal(int planes, const float* xp, float s, float2* out,
                                                  const uint16_t* ta) {
    // A workgroup takes PT units (kx, 16 planes), consecutive in the planes.
    // PT = 4 (many planes): one wave per unit walks all rows y, loading each 16-row step
    // inside the loop.  PT = 1 (few planes: more workgroups): the four waves split the
    // rows of one unit, issue all of their loads before their products, and their
    // partial sums are added in wave order through LDS.
    constexpr int YS = 4 / PT, IT = N / 16 / YS;   // row ranges per unit, 16-row steps per wave
    __shared__ f32x4 part[YS > 1 ? YS - 1 : 1][6][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int tile = wave % PT, ys = wave / PT;
    const int ptiles = (planes + 15) / 16;
    const int unit = blockIdx.x * PT + tile;
    const bool live = unit < MX * ptiles;
    if (YS == 1 && !live) return;
    const int un = live ? unit : 0;
    const int kx = un / ptiles, p = (un - kx * ptiles) * 16 + col;
    const bool pin = live && p < planes;
    const size_t tsz = (size_t)2 * MY * N;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    f32x4 are[2], aim[2], asr[2];   // [jt]: C X're + S X'im, C X'im, S X're
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) are[jt] = aim[jt] = asr[jt] = zero4;
    auto step = [&](const float (&fr)[4], const float (&fi)[4], int y0) {
        i16x4 rh, rl, ih, il;
        split4(fr, rh, rl);
        split4(fi, ih, il);
#pragma unroll
        for (int jt = 0; jt < 2; ++jt) {
            const int o = (16 * jt + col) * N + y0 + 4 * g;
            const i16x4 ch = ld_bf4(ta + o), sh = ld_bf4(ta + tsz + o);
            const i16x4 cl = ld_bf4(ta + 2 * tsz + o), sl = ld_bf4(ta + 3 * tsz + o);
            are[jt] = mfma16(ch, rh, are[jt]);
            are[jt] = mfma16(cl, rh, are[jt]);
            are[jt] = mfma16(ch, rl, are[jt]);
            are[jt] = mfma16(sh, ih, are[jt]);
            are[jt] = mfma16(sl, ih, are[jt]);
            are[jt] = mfma16(sh, il, are[jt]);
            aim[jt] = mfma16(ch, ih, aim[jt]);
            aim[jt] = mfma16(cl, ih, aim[jt]);
            aim[jt] = mfma16(ch, il, aim[jt]);
            asr[jt] = mfma16(sh, rh, asr[jt]);
            asr[jt] = mfma16(sl, rh, asr[jt]);
            asr[jt] = mfma16(sh, rl, asr[jt]);
        }
    };
    if constexpr (YS == 1) {
        for (int y0 = 0; y0 < N; y0 += 16) {
            float fr[4], fi[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + 4 * g + i;
                fr[i] = pin ? xp[((size_t)kx * N + y) * planes + p] : 0.f;
                fi[i] = pin ? xp[((size_t)(16 + kx) * N + y) * planes + p] : 0.f;
            }
            step(fr, fi, y0);
        }
    } else {
        // lanes past the last plane read plane 0 and add zeros
        const int pc = p < planes ? p : 0;
        float xr[IT][4], xi[IT][4];
#pragma unroll
        for (int it = 0; it < IT; ++it)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = ys * (N / YS) + 16 * it + 4 * g + i;
                xr[it][i] = xp[((size_t)kx * N + y) * planes + pc];
                xi[it][i] = xp[((size_t)(16 + kx) * N + y) * planes + pc];
            }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            float fr[4], fi[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                fr[i] = pin ? xr[it][i] : 0.f;
                fi[i] = pin ? xi[it][i] : 0.f;
            }
            step(fr, fi, ys * (N / YS) + 16 * it);
        }
        if (ys > 0) {
            f32x4* d = &part[ys - 1][0][lane];
            d[0] = are[0];
            d[64] = are[1];
            d[128] = aim[0];
            d[192] = aim[1];
            d[256] = asr[0];
            d[320] = asr[1];
        }
        __syncthreads();
        if (ys != 0) return;
#pragma unroll
        for (int w = 0; w < YS - 1; ++w) {
            const f32x4* q = &part[w][0][lane];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                are[0][i] += q[0][i];
                are[1][i] += q[64][i];
                aim[0][i] += q[128][i];
                aim[1][i] += q[192][i];
                asr[0][i] += q[256][i];
                asr[1][i] += q[320][i];
            }
        }
    }
    if (!pin) return;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 16 * jt + 4 * g + i;
            out[(size_t)(kx * 2 * MY + j) * planes + p] = make_float2(are[jt][i] * s, (aim[jt][i] - asr[jt][i]) * s);
        }
}

template <int N>
__global__ void __launch_bounds__(TPB) k_col_synth(int planes, const float2* in, float s0, float s1, int drop0,
                                                   float* zout, const uint16_t* ts) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int ptiles = (planes + 15) / 16;
    const int unit = blockIdx.x * 4 + wave;
    if (unit >= MX * ptiles) return;
    const int kx = unit / ptiles, p = (unit - kx * ptiles) * 16 + col;
    const bool pin = p < planes;
    const size_t tsz = (size_t)2 * MY * N;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    // B(j = 8 g + i, p = col) = w U[kx * 32 + j][p]
    bf16x8 urh, url, uih, uil;
    {
        const float w = kx == 0 ? s0 : s1;
        float ur[8], ui[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = 8 * g + i;
            const float2 u = pin ? in[(size_t)(kx * 2 * MY + j) * planes + p] : make_float2(0.f, 0.f);
            const float f = (drop0 && kx == 0 && j == 0) ? 0.f : w;
            ur[i] = u.x * f;
            ui[i] = u.y * f;
        }
        split8(ur, urh, url);
        split8(ui, uih, uil);
    }
    for (int y0 = 0; y0 < N; y0 += 16) {
        // A(y = y0 + col, j = 8 g + i)
        const int o = (y0 + col) * 2 * MY + 8 * g;
        const bf16x8 ch = ld_bf8(ts + o), sh = ld_bf8(ts + tsz + o);
        const bf16x8 cl = ld_bf8(ts + 2 * tsz + o), sl = ld_bf8(ts + 3 * tsz + o);
        f32x4 cr = zero4, si = zero4, zi = zero4;
        cr = mfma32(ch, urh, cr);
        cr = mfma32(cl, urh, cr);
        cr = mfma32(ch, url, cr);
        si = mfma32(sh, uih, si);
        si = mfma32(sl, uih, si);
        si = mfma32(sh, uil, si);
        zi = mfma32(sh, urh, zi);
        zi = mfma32(sl, urh, zi);
        zi = mfma32(sh, url, zi);
        zi = mfma32(ch, uih, zi);
        zi = mfma32(cl, uih, zi);
        zi = mfma32(ch, uil, zi);
        if (pin) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + 4 * g + i;
                zout[((size_t)kx * N + y) * planes + p] = cr[i] - si[i];
                zout[((size_t)(16 + kx) * N + y) * planes + p] = zi[i];
            }
        }
    }
}

// Wm of every mode from the FP32 weights, as bf16: Wm[i][o] = Wr, Wm[i][32+o] = Wi,
// Wm[32+i][o] = -Wi, Wm[32+i][32+o] = Wr.
__global__ void __launch_bounds__(TPB) k_pack(const float* wr, const float* wi, uint16_t* wpk) {
    const int m = blockIdx.x;
    for (int e = threadIdx.x; e < 64 * 64; e += TPB) {
        const int k = e >> 6, n = e & 63;
        const int i = k & 31, o = n & 31;
        const float r = wr[(size_t)m * C * C + i * C + o], q = wi[(size_t)m * C * C + i * C + o];
        float v;
        if (k < C) v = n < C ? r : q;
        else v = n < C ? -q : r;
        wpk[(size_t)m * 64 * 64 + e] = f2bf(v);
    }
}

// ---------------------------------------------------------------- projection and loss

// pred = phi + the filtered increment without its mean: x half of the synthesis of
// zo[n][y][b] (planar, kx weights and the dropped k = 0 mode applied by the column
// kernel).  With a target: lpart = sum (pred - target)^2 per workgroup, gpred =
// 2 (pred - target) / (batch npts), gpart = its per-workgroup sums.
template <int N>
__global__ void __launch_bounds__(TPB) k_finish(int batch, const float* phi, const float* zo, const float2* twg,
                                                const float* target, float* pred, float* gpred, float* lpart,
                                                float* gpart) {
    constexpr int R = TPB / N;
    __shared__ float2 tw[N];
    __shared__ float zr[R * 32];
    __shared__ float red[TPB / 64];
    const int t = threadIdx.x, b = blockIdx.y, r = t / N, x = t - r * N;
    const int y = blockIdx.x * R + r;
    for (int i = t; i < N; i += TPB) tw[i] = twg[i];
    if (t < R * 32) zr[t] = zo[((size_t)(t & 31) * N + blockIdx.x * R + (t >> 5)) * batch + b];
    __syncthreads();
    float inc = 0.f;
#pragma unroll
    for (int kx = 0; kx < MX; ++kx) {
        const float2 w = tw[(kx * x) & (N - 1)];
        inc += zr[r * 32 + kx] * w.x - zr[r * 32 + 16 + kx] * w.y;
    }
    const size_t i = ((size_t)b * N + y) * N + x;
    const float yv = phi[i] + inc;
    if (pred) pred[i] = yv;
    if (target) {
        const float d = yv - target[i];
        const float gd = 2.f * d / ((float)batch * (float)(N * N));
        gpred[i] = gd;
        const int nwg = gridDim.x;
        const float l = block_sum_f(d * d, red);
        if (t == 0) lpart[(size_t)b * nwg + blockIdx.x] = l;
        const float gs = block_sum_f(gd, red);
        if (t == 0) gpart[(size_t)b * nwg + blockIdx.x] = gs;
    }
}

// ---------------------------------------------------------------- backward, weight-gradient partials

// the C channels of point p = y n + x of sample b from channel-blocked activations
__device__ inline void load_act(const uint16_t* a, int n, int b, int p, float* out) {
    const int y = p / n, x = p - y * n;
    const uint16_t* row = a + ((size_t)b * n + y) * (size_t)(C * n) + (size_t)x * 8;
#pragma unroll
    for (int cg = 0; cg < C / 8; ++cg) {
        const uint4 q = *reinterpret_cast<const uint4*>(row + (size_t)cg * n * 8);
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            out[cg * 8 + 2 * j] = bf2f((uint16_t)(w[j] & 0xFFFFu));
            out[cg * 8 + 2 * j + 1] = bf2f((uint16_t)(w[j] >> 16));
        }
    }
}

// The weight-gradient kernels run GRED workgroups that each take chunks of TPB points
// (chunk id = blockIdx.x, + GRED, ...; a chunk lies inside one sample), and write one
// row of partial sums; launch_reduce adds the rows in a fixed order.

// gout[b][p] = gpred[b][p] - mean_p(gpred[b]) (the adjoint of restoring the mean), the
// mean from the per-workgroup sums gpart of the finish pass
__global__ void __launch_bounds__(TPB) k_center(int npts, const float* gpred, const float* gpart, float* gout) {
    __shared__ float mean_s;
    const int b = blockIdx.y, nwg = gridDim.x;
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < nwg; ++w) s += gpart[(size_t)b * nwg + w];
        mean_s = s / (float)npts;
    }
    __syncthreads();
    const size_t i = (size_t)b * npts + blockIdx.x * TPB + threadIdx.x;
    gout[i] = gpred[i] - mean_s;
}

// projection (workgroups of 64 threads, one point each per chunk of 64 points): given
// g_out (the gradient of the projection output), recompute pre/h; gv4[c] = sum_k Q1[k][c] g_pre[k];
// partials: Q1 (g_pre v4), q1 (g_pre), Q2 (g_out h), q2 (g_out).  Thread t owns row k = t
// of Q1 and q1[t], Q2[t]; thread 0 also q2.
__global__ void __launch_bounds__(64) k_project_bwd(int n, int batch, const uint16_t* v4, const float* prm,
                                                    const float* gouts, float* gv, float* partials) {
    constexpr int Q = 64;
    const int npts = n * n;
    __shared__ float gp_s[H * Q];
    __shared__ float h_s[H * Q];
    __shared__ float x_s[C * Q];
    __shared__ float go_s[Q];
    const int t = threadIdx.x;
    const float* q = prm + P_Q1;   // uniform: scalar loads
    const int per = npts / Q, chunks = batch * per;
    float aQ1[C];
#pragma unroll
    for (int c = 0; c < C; ++c) aQ1[c] = 0.f;
    float aq1 = 0.f, aQ2 = 0.f, aq2 = 0.f;
    __syncthreads();
    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int b = ch / per;
        const int p = (ch - b * per) * Q + t;
        const float go = gouts[(size_t)b * npts + p];
        const size_t base = (size_t)b * C * npts + p;
        float x[C], gx[C];
        load_act(v4, n, b, p, x);
#pragma unroll
        for (int c = 0; c < C; ++c) gx[c] = 0.f;
        __syncthreads();   // the previous chunk's LDS is consumed
        for (int k = 0; k < H; ++k) {
            float pre = q[H * C + k];
#pragma unroll
            for (int c = 0; c < C; ++c) pre += q[k * C + c] * x[c];
            const float gpk = q[H * C + H + k] * go * gelu_d(pre);
            gp_s[k * Q + t] = gpk;
            h_s[k * Q + t] = gelu(pre);
#pragma unroll
            for (int c = 0; c < C; ++c) gx[c] += q[k * C + c] * gpk;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            gv[base + (size_t)c * npts] = gx[c];
            x_s[c * Q + t] = x[c];
        }
        go_s[t] = go;
        __syncthreads();
        for (int pt = 0; pt < Q; ++pt) {
            const float g = gp_s[t * Q + pt];
#pragma unroll
            for (int c = 0; c < C; ++c) aQ1[c] += g * x_s[c * Q + pt];
            aq1 += g;
            aQ2 += go_s[pt] * h_s[t * Q + pt];
            aq2 += go_s[pt];
        }
    }
    float* row = partials + (size_t)blockIdx.x * PART_PROJ;
#pragma unroll
    for (int c = 0; c < C; ++c) row[t * C + c] = aQ1[c];
    row[H * C + t] = aq1;
    row[H * C + H + t] = aQ2;
    if (t == 0) row[H * C + H + H] = aq2;
}

// pointwise layer (workgroups of 64 threads, one point each per chunk of 64 points):
// gu[o] = gout[o] gelu'(u[o]) (act) or gout[o]; gv[i] = sum_o Pw[o][i] gu[o];
// partials: Pw (gu v), Pb (gu).  Thread t owns Pw[o][i0..i0+15] with o = t / 2,
// i0 = 16 (t % 2), and Pb[o] if t is even.
__global__ void __launch_bounds__(64) k_pointwise_bwd(int n, int batch, int act, const float* gout,
                                                      const uint16_t* u, const uint16_t* v, const float* pw,
                                                      float* gu, float* gv, float* partials) {
    constexpr int Q = 64;
    const int npts = n * n;
    __shared__ float sw[C * C];
    __shared__ float g_s[C * Q];
    __shared__ float x_s[C * Q];
    const int t = threadIdx.x;
    for (int i = t; i < C * C; i += Q) sw[i] = pw[i];
    const int per = npts / Q, chunks = batch * per;
    const int o = t >> 1, i0 = (t & 1) * 16;
    float aw[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) aw[j] = 0.f;
    float ab = 0.f;
    __syncthreads();
    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int b = ch / per;
        const int p = (ch - b * per) * Q + t;
        const size_t base = (size_t)b * C * npts + p;
        __syncthreads();   // the previous chunk's LDS is consumed
        float g[C], uu[C], vv[C];
        if (act) load_act(u, n, b, p, uu);
        load_act(v, n, b, p, vv);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const size_t i = base + (size_t)c * npts;
            const float go = gout[i];
            g[c] = act ? go * gelu_d(uu[c]) : go;
            gu[i] = g[c];
            g_s[c * Q + t] = g[c];
            x_s[c * Q + t] = vv[c];
        }
        for (int i = 0; i < C; ++i) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c) s += sw[c * C + i] * g[c];
            gv[base + (size_t)i * npts] = s;
        }
        __syncthreads();
        for (int pt = 0; pt < Q; ++pt) {
            const float gg = g_s[o * Q + pt];
#pragma unroll
            for (int j = 0; j < 16; ++j) aw[j] += gg * x_s[(i0 + j) * Q + pt];
            ab += gg;
        }
    }
    float* row = partials + (size_t)blockIdx.x * PART_PW;
#pragma unroll
    for (int j = 0; j < 16; ++j) row[o * C + i0 + j] = aw[j];
    if ((t & 1) == 0) row[C * C + o] = ab;
}

// lifting: partials Lw[c][0] (g phi), Lw[c][1] (g eps), Lb[c] (g).  Each thread sums its
// points; the workgroup then adds the 256 thread sums of each value in order.
__global__ void __launch_bounds__(TPB) k_lift_bwd(int npts, int batch, const float* gv0, const float* phi,
                                                  const float* eps, float* partials) {
    __shared__ float red[TPB * (C + 1)];
    const int t = threadIdx.x;
    const int nwg = npts / TPB, chunks = batch * nwg;
    float a0[C], a1[C], a2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) a0[c] = a1[c] = a2[c] = 0.f;
    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int b = ch / nwg;
        const int p = (ch - b * nwg) * TPB + t;
        const size_t base = (size_t)b * C * npts + p;
        const float f = phi[(size_t)b * npts + p], e = eps[b];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float g = gv0[base + (size_t)c * npts];
            a0[c] += g * f;
            a1[c] += g * e;
            a2[c] += g;
        }
    }
    float* row = partials + (size_t)blockIdx.x * PART_LIFT;
    for (int kind = 0; kind < 3; ++kind) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c) red[t * (C + 1) + c] = kind == 0 ? a0[c] : (kind == 1 ? a1[c] : a2[c]);
        __syncthreads();
        if (t < C) {
            float sum = 0.f;
            for (int i = 0; i < TPB; ++i) sum += red[i * (C + 1) + t];
            if (kind < 2) row[2 * t + kind] = sum;
            else row[2 * C + t] = sum;
        }
    }
}

// dst[j] = scale * sum_r partials[r][j]: 64 columns per workgroup, four row slices
// (coalesced over the columns), the slices added in order.
__global__ void __launch_bounds__(TPB) k_reduce(const float* partials, int nrows, int cnt, float scale, float* dst) {
    __shared__ float part[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int r0 = (int)((long long)nrows * g / 4), r1 = (int)((long long)nrows * (g + 1) / 4);
    float s = 0.f;
    if (j < cnt)
        for (int r = r0; r < r1; ++r) s += partials[(size_t)r * cnt + j];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && j < cnt) dst[j] = scale * (((part[0][c] + part[1][c]) + part[2][c]) + part[3][c]);
}

// Adam with bias correction: c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void __launch_bounds__(TPB) k_adam(int64_t count, float* prm, const float* grad, float* m, float* v,
                                              float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= count) return;
    const float g = grad[i];
    const float mm = 0.9f * m[i] + 0.1f * g;
    const float vv = 0.999f * v[i] + 0.001f * g * g;
    m[i] = mm;
    v[i] = vv;
    prm[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

// ---------------------------------------------------------------- launch helpers

#define FNO_LAUNCH_N(KERNEL, ...)                                                                     \
    switch (n) {                                                                                       \
        case 64: hipLaunchKernelGGL((KERNEL<64>), __VA_ARGS__); break;                                 \
        case 128: hipLaunchKernelGGL((KERNEL<128>), __VA_ARGS__); break;                               \
        case 256: hipLaunchKernelGGL((KERNEL<256>), __VA_ARGS__); break;                               \
        default: return hipErrorInvalidValue;                                                          \
    }

template <typename TIn>
static hipError_t analysis_n(int n, int planes, const TIn* in, float s0, float s1, float2* out, const float2* tw,
                             hipStream_t st) {
    switch (n) {
        case 64: hipLaunchKernelGGL((k_analysis<64, TIn>), dim3(planes), dim3(TPB), 0, st, planes, in, s0, s1, out, tw); break;
        case 128: hipLaunchKernelGGL((k_analysis<128, TIn>), dim3(planes), dim3(TPB), 0, st, planes, in, s0, s1, out, tw); break;
        case 256: hipLaunchKernelGGL((k_analysis<256, TIn>), dim3(planes), dim3(TPB), 0, st, planes, in, s0, s1, out, tw); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_analysis_f32(int n, int planes, const float* in, float s0, float s1, float2* out, const float2* tw,
                               hipStream_t st) {
    return analysis_n<float>(n, planes, in, s0, s1, out, tw, st);
}

hipError_t launch_synthesis(int n, int planes, const float2* in, float s0, float s1, float* out, int accumulate,
                            const float2* tw, hipStream_t st) {
    FNO_LAUNCH_N(k_synthesis, dim3(planes), dim3(TPB), 0, st, planes, in, s0, s1, out, accumulate, tw)
    return hipGetLastError();
}

hipError_t launch_mix(int mode, int batch, const float2* a, const float2* g, const uint16_t* wpk, float2* out,
                      float* gwr, float* gwi, hipStream_t st) {
    if (mode == MIX_FWD)
        hipLaunchKernelGGL(k_mix<MIX_FWD>, dim3(NMODE), dim3(TPB), 0, st, batch, a, g, wpk, out, gwr, gwi);
    else if (mode == MIX_BWD_DATA)
        hipLaunchKernelGGL(k_mix<MIX_BWD_DATA>, dim3(NMODE), dim3(TPB), 0, st, batch, a, g, wpk, out, gwr, gwi);
    else
        hipLaunchKernelGGL(k_mix<MIX_BWD_WEIGHT>, dim3(NMODE), dim3(TPB), 0, st, batch, a, g, wpk, out, gwr, gwi);
    return hipGetLastError();
}

hipError_t launch_basis(int n, uint16_t* bx, uint16_t* bxt, hipStream_t st) {
    hipLaunchKernelGGL(k_basis, dim3((n * 2 * MX + TPB - 1) / TPB), dim3(TPB), 0, st, n, bx, bxt);
    return hipGetLastError();
}

hipError_t launch_row(int n, int batch, int kind, const RowIn& in, hipStream_t st) {
    RowParams a{in.phi, in.eps, in.prm, in.layer, in.Z, in.v, in.vout, in.uout, in.xout, in.bx, in.bxt, in.tw};
    const dim3 g(n / RROWS, batch), b(TPB);
#define FNO_ROW(NN)                                                                                  \
    if (kind == RK_LIFT) hipLaunchKernelGGL((k_rowmm<NN, RK_LIFT>), g, b, 0, st, a);               \
    else if (kind == RK_LAYER) hipLaunchKernelGGL((k_rowmm<NN, RK_LAYER>), g, b, 0, st, a);        \
    else hipLaunchKernelGGL((k_rowmm<NN, RK_LAST>), g, b, 0, st, a);
    switch (n) {
        case 64: FNO_ROW(64) break;
        case 128: FNO_ROW(128) break;
        case 256: FNO_ROW(256) break;
        default: return hipErrorInvalidValue;
    }
#undef FNO_ROW
    return hipGetLastError();
}

hipError_t launch_trig(int n, uint16_t* ta, uint16_t* ts, hipStream_t st) {
    hipLaunchKernelGGL(k_trig, dim3((2 * MY * n + TPB - 1) / TPB), dim3(TPB), 0, st, n, ta, ts);
    return hipGetLastError();
}

hipError_t launch_col_anal(int n, int planes, const float* xp, float s, float2* out, const uint16_t* ta,
                           hipStream_t st) {
    // four units per workgroup when that still gives two or more workgroups per CU, else
    // one (few planes: the rows of a unit split over four waves); measured at batch 64
    // (2048 and 64 planes) on 256^2
    const int units = MX * ((planes + 15) / 16);
    if (units >= 2048) {
        switch (n) {
            case 64: hipLaunchKernelGGL((k_col_anal<64, 4>), dim3((units + 3) / 4), dim3(TPB), 0, st, planes, xp, s, out, ta); break;
            case 128: hipLaunchKernelGGL((k_col_anal<128, 4>), dim3((units + 3) / 4), dim3(TPB), 0, st, planes, xp, s, out, ta); break;
            case 256: hipLaunchKernelGGL((k_col_anal<256, 4>), dim3((units + 3) / 4), dim3(TPB), 0, st, planes, xp, s, out, ta); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (n) {
            case 64: hipLaunchKernelGGL((k_col_anal<64, 1>), dim3(units), dim3(TPB), 0, st, planes, xp, s, out, ta); break;
            case 128: hipLaunchKernelGGL((k_col_anal<128, 1>), dim3(units), dim3(TPB), 0, st, planes, xp, s, out, ta); break;
            case 256: hipLaunchKernelGGL((k_col_anal<256, 1>), dim3(units), dim3(TPB), 0, st, planes, xp, s, out, ta); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_col_synth(int n, int planes, const float2* in, float s0, float s1, bool drop0, float* zout,
                            const uint16_t* ts, hipStream_t st) {
    const int units = MX * ((planes + 15) / 16);
    FNO_LAUNCH_N(k_col_synth, dim3((units + 3) / 4), dim3(TPB), 0, st, planes, in, s0, s1, drop0 ? 1 : 0, zout, ts)
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* wr, const float* wi, uint16_t* wpk, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(NMODE), dim3(TPB), 0, st, wr, wi, wpk);
    return hipGetLastError();
}

hipError_t launch_finish(int n, int batch, const float* phi, const float* zo, const float2* tw, const float* target,
                         float* pred, float* gpred, float* lpart, float* gpart, hipStream_t st) {
    FNO_LAUNCH_N(k_finish, dim3(n * n / TPB, batch), dim3(TPB), 0, st, batch, phi, zo, tw, target, pred, gpred, lpart,
                 gpart)
    return hipGetLastError();
}

hipError_t launch_center(int n, int batch, const float* gpred, const float* gpart, float* gout, hipStream_t st) {
    hipLaunchKernelGGL(k_center, dim3(n * n / TPB, batch), dim3(TPB), 0, st, n * n, gpred, gpart, gout);
    return hipGetLastError();
}

hipError_t launch_project_bwd(int n, int batch, const uint16_t* v4, const float* prm, const float* gout, float* gv,
                              float* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_project_bwd, dim3(GRED64), dim3(64), 0, st, n, batch, v4, prm, gout, gv, partials);
    return hipGetLastError();
}

hipError_t launch_pointwise_bwd(int n, int batch, bool act, const float* gout, const uint16_t* u, const uint16_t* v,
                                const float* pw, float* gu, float* gv, float* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_pointwise_bwd, dim3(GRED64), dim3(64), 0, st, n, batch, act ? 1 : 0, gout, u, v, pw, gu,
                       gv, partials);
    return hipGetLastError();
}

hipError_t launch_lift_bwd(int n, int batch, const float* gv0, const float* phi, const float* eps, float* partials,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_lift_bwd, dim3(GRED), dim3(TPB), 0, st, n * n, batch, gv0, phi, eps, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const float* partials, int nrows, int cnt, float scale, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3((cnt + 63) / 64), dim3(TPB), 0, st, partials, nrows, cnt, scale, dst);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* prm, const float* grad, float* m, float* v, float lr, float c1,
                       float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + TPB - 1) / TPB)), dim3(TPB), 0, st, count, prm, grad, m, v, lr,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace fno
