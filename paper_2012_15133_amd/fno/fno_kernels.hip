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

// ---------------------------------------------------------------- lifting

// v0[b][c][p] = Lw[c][0] phi[b][p] + Lw[c][1] eps[b] + Lb[c]
__global__ void __launch_bounds__(TPB) k_lift(int npts, const float* phi, const float* eps, const float* prm,
                                              uint16_t* v0) {
    const int b = blockIdx.y;
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= npts) return;
    const float f = phi[(size_t)b * npts + p], e = eps[b];
#pragma unroll
    for (int c = 0; c < C; ++c)
        v0[((size_t)b * C + c) * npts + p] = f2bf(prm[P_LW + 2 * c] * f + prm[P_LW + 2 * c + 1] * e + prm[P_LB + c]);
}

// ---------------------------------------------------------------- truncated transforms

// One workgroup per plane.  out[m][plane] = s_kx sum_{y,x} in[y][x] e^{-2 pi i (kx x + ky y)/N}:
// rows in chunks of 16 (thread = (row, kx)) give X[y][kx], then the y sums (thread =
// (kx, two j)).
template <int N, typename TIn>
__global__ void __launch_bounds__(TPB) k_analysis(int planes, const TIn* in, float s0, float s1, float2* out,
                                                  const float2* twg) {
    __shared__ float2 tw[N];
    __shared__ float chunk[16 * N];
    __shared__ float2 X[N * MX];
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

// X'[b][c][y][kx] = sum_x v[b][c][y][x] e^{-2 pi i kx x / N} (the x half of the analysis),
// Z[b][o][y][kx] = sum_j s_kx U[kx][j] e^{+2 pi i ky y / N} (the y half of the synthesis).
// Rows: one workgroup takes R = 256 / N rows (r, y) of one sample, thread = (r, x).

// bf16 DFT basis for the x half of the analysis, split in two parts so that hi + lo
// carries FP32 accuracy: B[x][n] = cos(2 pi n x / N) (n < 16), -sin(2 pi (n-16) x / N).
__global__ void __launch_bounds__(TPB) k_basis(int n, uint16_t* hi, uint16_t* lo) {
    for (int e = blockIdx.x * TPB + threadIdx.x; e < n * 2 * MX; e += gridDim.x * TPB) {
        const int x = e / (2 * MX), c = e - x * 2 * MX;
        const int k = c & 15;
        const double a = 6.283185307179586476925286766559 * (double)((k * x) % n) / (double)n;
        const float v = c < MX ? (float)cos(a) : -(float)sin(a);
        const uint16_t h = f2bf(v);
        hi[e] = h;
        lo[e] = f2bf(v - bf2f(h));
    }
}

// Row kernel.  LIFT: v = Lw phi + Lw eps + Lb.  LAYER: u = synth_x(Z) + Pw v + Pb,
// v' = gelu(u) (act) or u, as one matrix-core product per row:
//   u[o][x] = sum_k A[o][k] B[k][x],  A = [Re Z | Im Z | Pw] (32 x 64),
//   B = [cos(kx x) ; -sin(kx x) ; v] (64 x N),
// with A and the basis split into bf16 hi + lo parts (hi hi + lo hi + hi lo: FP32
// accuracy; v is stored as bf16 already).  Stores v' (bf16), u (bf16, if uout) and, if
// xout, X' = analysis_x(v') (bf16 v' times the hi + lo basis, FP32 sums).
template <int N, bool LIFT>
__global__ void __launch_bounds__(TPB) k_row(const float* phi, const float* eps, const float* prm, int layer,
                                             const float2* Z, const uint16_t* v, uint16_t* vout, uint16_t* uout,
                                             float2* xout, const uint16_t* bhi, const uint16_t* blo,
                                             const float2* twg) {
    constexpr int R = TPB / N;            // rows per workgroup
    __shared__ uint16_t Zh[R * C * 2 * MX], Zl[R * C * 2 * MX];   // [r][o][k < 32]
    __shared__ uint16_t Ph[C * C], Pl[C * C];                     // [o][i]
    __shared__ float pb[C];
    __shared__ uint16_t Vin[R * C * N];   // v of the rows [r][i][x]; later u
    __shared__ uint16_t Vs[R * C * N];    // v' of the rows, [r][c][x]
    const int t = threadIdx.x, r = t / N, x = t - r * N;
    const int b = blockIdx.y, y0 = blockIdx.x * R, y = y0 + r;
    const int npts = N * N;
    const size_t base = (size_t)b * C * npts + (size_t)y * N + x;   // + c * npts
    const int wave = t >> 6, lane = t & 63;
    const int col = lane & 15, rb = 4 * (lane >> 4);
    if constexpr (LIFT) {
        const float f = phi[(size_t)b * npts + (size_t)y * N + x], e = eps[b];
#pragma unroll
        for (int c = 0; c < C; ++c)
            Vs[(r * C + c) * N + x] = f2bf(prm[P_LW + 2 * c] * f + prm[P_LW + 2 * c + 1] * e + prm[P_LB + c]);
    } else {
        const float* pw = prm + p_pw(layer);
        for (int i = t; i < C * C; i += TPB) {
            const float w = pw[i];
            const uint16_t h = f2bf(w);
            Ph[i] = h;
            Pl[i] = f2bf(w - bf2f(h));
        }
        if (t < C) pb[t] = pw[C * C + t];
        for (int i = t; i < R * C * MX; i += TPB) {
            const int rr = i / (C * MX), rest = i - rr * C * MX, o = rest / MX, k = rest - o * MX;
            const float2 z = Z[(((size_t)b * C + o) * N + y0 + rr) * MX + k];
            const int a = (rr * C + o) * 2 * MX + k;
            const uint16_t hr = f2bf(z.x), hi = f2bf(z.y);
            Zh[a] = hr;
            Zl[a] = f2bf(z.x - bf2f(hr));
            Zh[a + MX] = hi;
            Zl[a + MX] = f2bf(z.y - bf2f(hi));
        }
#pragma unroll
        for (int i = 0; i < C; ++i) Vin[(r * C + i) * N + x] = v[base + (size_t)i * npts];
        __syncthreads();
        // tiles: per row 2 (o) x N/16 (x); R rows -> 32 tiles, 8 per wave
        f32x4 acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int tile = wave * 8 + q;
            const int rr = tile / (2 * N / 16), rest = tile - rr * (2 * N / 16);
            const int mt = rest / (N / 16), x0 = (rest - mt * (N / 16)) * 16;
            const uint16_t* zh = Zh + (rr * C + mt * 16) * 2 * MX;
            const uint16_t* zl = Zl + (rr * C + mt * 16) * 2 * MX;
            f32x4 a = {0.f, 0.f, 0.f, 0.f};
            // k < 32: the x-synthesis of the row's coefficients
            a = mma16x16x32(a, zh, 2 * MX, 1, bhi + x0 * 2 * MX, 1, 2 * MX);
            a = mma16x16x32(a, zl, 2 * MX, 1, bhi + x0 * 2 * MX, 1, 2 * MX);
            a = mma16x16x32(a, zh, 2 * MX, 1, blo + x0 * 2 * MX, 1, 2 * MX);
            // k >= 32: the pointwise layer Pw v
            const uint16_t* vb = Vin + rr * C * N + x0;
            a = mma16x16x32(a, Ph + mt * 16 * C, C, 1, vb, N, 1);
            a = mma16x16x32(a, Pl + mt * 16 * C, C, 1, vb, N, 1);
            acc[q] = a;
        }
        __syncthreads();   // Vin is read by every wave above; it now takes u
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int tile = wave * 8 + q;
            const int rr = tile / (2 * N / 16), rest = tile - rr * (2 * N / 16);
            const int mt = rest / (N / 16), x0 = (rest - mt * (N / 16)) * 16;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = mt * 16 + rb + j;
                const float u = acc[q][j] + pb[o];
                const int a = (rr * C + o) * N + x0 + col;
                Vin[a] = f2bf(u);
                Vs[a] = f2bf(layer < LAYERS - 1 ? gelu(u) : u);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        vout[base + (size_t)c * npts] = Vs[(r * C + c) * N + x];
        if constexpr (!LIFT)
            if (uout) uout[base + (size_t)c * npts] = Vin[(r * C + c) * N + x];
    }
    if (!xout) return;
    // X'[(r, c)][n] = sum_x Vs[(r, c)][x] B[x][n]: M = R * 32 rows, 32 columns, K = N
    constexpr int MT = R * C / 16, TILES = MT * 2;
    for (int tile = wave; tile < TILES; tile += TPB / 64) {
        const int mt = tile >> 1, nt = tile & 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < N; k0 += 32) {
            acc = mma16x16x32(acc, Vs + mt * 16 * N + k0, N, 1, bhi + k0 * 2 * MX + nt * 16, 2 * MX, 1);
            acc = mma16x16x32(acc, Vs + mt * 16 * N + k0, N, 1, blo + k0 * 2 * MX + nt * 16, 2 * MX, 1);
        }
        // D(row, col): row = (r, c), col n: n < 16 real part of kx = n, else imaginary of n - 16
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = mt * 16 + rb + j, rr = row / C, c = row - rr * C;
            float* dst = reinterpret_cast<float*>(xout + (((size_t)b * C + c) * N + y0 + rr) * MX + col);
            dst[nt] = acc[j];   // nt = 0: .x (real), 1: .y (imaginary)
        }
    }
}

// Column kernels, one workgroup per plane (b, c).  ANAL: V[m][plane] = s sum_y X'[y][kx] e^{-i ky y}.
// SYNTH: Z[plane][y][kx] = sum_j s_kx U[m][plane] e^{+i ky y}.
template <int N>
__global__ void __launch_bounds__(TPB) k_col_anal(int planes, const float2* xp, float s, float2* out,
                                                  const float2* twg) {
    __shared__ float2 tw[N];
    __shared__ float2 X[N * MX];
    const int t = threadIdx.x, p = blockIdx.x;
    for (int i = t; i < N; i += TPB) tw[i] = twg[i];
    for (int i = t; i < N * MX; i += TPB) X[i] = xp[(size_t)p * N * MX + i];
    __syncthreads();
    const int kx = t & 15;
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

template <int N>
__global__ void __launch_bounds__(TPB) k_col_synth(int planes, const float2* in, float s0, float s1, float2* zout,
                                                   const float2* twg) {
    constexpr int UP = 2 * MY + 1;   // padded row: the 16 kx of a wave fall in different banks
    __shared__ float2 tw[N];
    __shared__ float2 U[MX * UP];
    const int t = threadIdx.x, p = blockIdx.x;
    for (int i = t; i < N; i += TPB) tw[i] = twg[i];
    for (int m = t; m < NMODE; m += TPB) {
        const float sc = (m >> 5) == 0 ? s0 : s1;
        const float2 u = in[(size_t)m * planes + p];
        U[(m >> 5) * UP + (m & 31)] = make_float2(u.x * sc, u.y * sc);
    }
    __syncthreads();
    const int kx = t & 15;
    for (int y = t >> 4; y < N; y += 16) {
        float re = 0.f, im = 0.f;
#pragma unroll 8
        for (int j = 0; j < 2 * MY; ++j) {
            const int ky = j < MY ? j : N - 2 * MY + j;
            const float2 w = tw[(ky * y) & (N - 1)];
            const float2 u = U[kx * UP + j];
            re += u.x * w.x - u.y * w.y;
            im += u.x * w.y + u.y * w.x;
        }
        zout[((size_t)p * N + y) * MX + kx] = make_float2(re, im);
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

// ---------------------------------------------------------------- pointwise layer

// u[o] = w[o] + sum_i Pw[o][i] v[i] + Pb[o]; vout = gelu(u) (act) or u; uout = u (if set)
__global__ void __launch_bounds__(TPB) k_pointwise(int npts, int act, const float* w, const uint16_t* v,
                                                   const float* pw, const float* pb, uint16_t* vout, uint16_t* uout) {
    __shared__ float sw[C * C + C];
    for (int i = threadIdx.x; i < C * C; i += TPB) sw[i] = pw[i];
    if (threadIdx.x < C) sw[C * C + threadIdx.x] = pb[threadIdx.x];
    __syncthreads();
    const int b = blockIdx.y;
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= npts) return;
    const size_t base = (size_t)b * C * npts + p;
    float x[C];
#pragma unroll
    for (int i = 0; i < C; ++i) x[i] = bf2f(v[base + (size_t)i * npts]);
#pragma unroll 4
    for (int o = 0; o < C; ++o) {
        float u = w[base + (size_t)o * npts] + sw[C * C + o];
#pragma unroll
        for (int i = 0; i < C; ++i) u += sw[o * C + i] * x[i];
        if (uout) uout[base + (size_t)o * npts] = f2bf(u);
        vout[base + (size_t)o * npts] = f2bf(act ? gelu(u) : u);
    }
}

// ---------------------------------------------------------------- projection and loss

// out_raw[b][p] = sum_k Q2[k] gelu(sum_c Q1[k][c] v4[c] + q1[k]) + q2; part[b][wg] = sum over the workgroup
__global__ void __launch_bounds__(TPB) k_project(int npts, const uint16_t* v4, const float* prm, float* out_raw,
                                                 float* part) {
    __shared__ float red[TPB / 64];
    const float* q = prm + P_Q1;   // uniform: scalar loads
    const int b = blockIdx.y;
    const int p = blockIdx.x * TPB + threadIdx.x;
    float o = 0.f;
    if (p < npts) {
        const size_t base = (size_t)b * C * npts + p;
        float x[C];
#pragma unroll
        for (int c = 0; c < C; ++c) x[c] = bf2f(v4[base + (size_t)c * npts]);
        o = q[H * C + H + H];
#pragma unroll 2
        for (int k = 0; k < H; ++k) {
            float pre = q[H * C + k];
#pragma unroll
            for (int c = 0; c < C; ++c) pre += q[k * C + c] * x[c];
            o += q[H * C + H + k] * gelu(pre);
        }
        out_raw[(size_t)b * npts + p] = o;
    }
    const float s = block_sum_f(o, red);
    if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
}

// pred = phi + out - mean(out); with a target: lpart = sum (pred - target)^2 per workgroup,
// gpred = 2 (pred - target) / (batch npts), gpart = its per-workgroup sums.
__global__ void __launch_bounds__(TPB) k_finish(int npts, int batch, const float* phi, const float* out_raw,
                                                const float* part, const float* target, float* pred, float* gpred,
                                                float* lpart, float* gpart) {
    __shared__ float red[TPB / 64];
    __shared__ float mean_s;
    const int b = blockIdx.y, nwg = gridDim.x;
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < nwg; ++w) s += part[(size_t)b * nwg + w];
        mean_s = s / (float)npts;
    }
    __syncthreads();
    const int p = blockIdx.x * TPB + threadIdx.x;
    float d = 0.f, gd = 0.f;
    if (p < npts) {
        const size_t i = (size_t)b * npts + p;
        const float y = phi[i] + out_raw[i] - mean_s;
        if (pred) pred[i] = y;
        if (target) {
            d = y - target[i];
            gd = 2.f * d / ((float)batch * (float)npts);
            gpred[i] = gd;
        }
    }
    if (target) {
        const float l = block_sum_f(d * d, red);
        if (threadIdx.x == 0) lpart[(size_t)b * nwg + blockIdx.x] = l;
        const float gs = block_sum_f(gd, red);
        if (threadIdx.x == 0) gpart[(size_t)b * nwg + blockIdx.x] = gs;
    }
}

// ---------------------------------------------------------------- backward, weight-gradient partials

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
__global__ void __launch_bounds__(64) k_project_bwd(int npts, int batch, const uint16_t* v4, const float* prm,
                                                    const float* gouts, float* gv, float* partials) {
    constexpr int Q = 64;
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
#pragma unroll
        for (int c = 0; c < C; ++c) {
            x[c] = bf2f(v4[base + (size_t)c * npts]);
            gx[c] = 0.f;
        }
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
__global__ void __launch_bounds__(64) k_pointwise_bwd(int npts, int batch, int act, const float* gout,
                                                      const uint16_t* u, const uint16_t* v, const float* pw,
                                                      float* gu, float* gv, float* partials) {
    constexpr int Q = 64;
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
        float g[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const size_t i = base + (size_t)c * npts;
            const float go = gout[i];
            g[c] = act ? go * gelu_d(bf2f(u[i])) : go;
            gu[i] = g[c];
            g_s[c * Q + t] = g[c];
            x_s[c * Q + t] = bf2f(v[i]);
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

hipError_t launch_lift(int n, int batch, const float* phi, const float* eps, const float* prm, uint16_t* v0,
                       hipStream_t st) {
    const int npts = n * n;
    hipLaunchKernelGGL(k_lift, dim3((npts + TPB - 1) / TPB, batch), dim3(TPB), 0, st, npts, phi, eps, prm, v0);
    return hipGetLastError();
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

hipError_t launch_analysis_bf16(int n, int planes, const uint16_t* in, float s0, float s1, float2* out,
                                const float2* tw, hipStream_t st) {
    return analysis_n<uint16_t>(n, planes, in, s0, s1, out, tw, st);
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

hipError_t launch_basis(int n, uint16_t* hi, uint16_t* lo, hipStream_t st) {
    hipLaunchKernelGGL(k_basis, dim3((n * 2 * MX + TPB - 1) / TPB), dim3(TPB), 0, st, n, hi, lo);
    return hipGetLastError();
}

hipError_t launch_row(int n, int batch, bool lift, const float* phi, const float* eps, const float* prm, int layer,
                      const float2* Z, const uint16_t* v, uint16_t* vout, uint16_t* uout, float2* xout,
                      const uint16_t* bhi, const uint16_t* blo, const float2* tw, hipStream_t st) {
    const dim3 g(n / (TPB / n), batch), b(TPB);
#define FNO_ROW(NN)                                                                                               \
    if (lift) hipLaunchKernelGGL((k_row<NN, true>), g, b, 0, st, phi, eps, prm, layer, Z, v, vout, uout, xout, bhi, \
                                 blo, tw);                                                                         \
    else hipLaunchKernelGGL((k_row<NN, false>), g, b, 0, st, phi, eps, prm, layer, Z, v, vout, uout, xout, bhi, blo, \
                            tw);
    switch (n) {
        case 64: FNO_ROW(64) break;
        case 128: FNO_ROW(128) break;
        case 256: FNO_ROW(256) break;
        default: return hipErrorInvalidValue;
    }
#undef FNO_ROW
    return hipGetLastError();
}

hipError_t launch_col_anal(int n, int planes, const float2* xp, float s, float2* out, const float2* tw,
                           hipStream_t st) {
    FNO_LAUNCH_N(k_col_anal, dim3(planes), dim3(TPB), 0, st, planes, xp, s, out, tw)
    return hipGetLastError();
}

hipError_t launch_col_synth(int n, int planes, const float2* in, float s0, float s1, float2* zout, const float2* tw,
                            hipStream_t st) {
    FNO_LAUNCH_N(k_col_synth, dim3(planes), dim3(TPB), 0, st, planes, in, s0, s1, zout, tw)
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* wr, const float* wi, uint16_t* wpk, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(NMODE), dim3(TPB), 0, st, wr, wi, wpk);
    return hipGetLastError();
}

hipError_t launch_pointwise(int n, int batch, bool act, const float* w, const uint16_t* v, const float* pw,
                            const float* pb, uint16_t* vout, uint16_t* uout, hipStream_t st) {
    const int npts = n * n;
    hipLaunchKernelGGL(k_pointwise, dim3((npts + TPB - 1) / TPB, batch), dim3(TPB), 0, st, npts, act ? 1 : 0, w, v,
                       pw, pb, vout, uout);
    return hipGetLastError();
}

hipError_t launch_project(int n, int batch, const uint16_t* v4, const float* prm, float* out_raw, float* part,
                          hipStream_t st) {
    const int npts = n * n;
    hipLaunchKernelGGL(k_project, dim3(npts / TPB, batch), dim3(TPB), 0, st, npts, v4, prm, out_raw, part);
    return hipGetLastError();
}

hipError_t launch_finish(int n, int batch, const float* phi, const float* out_raw, const float* part,
                         const float* target, float* pred, float* gpred, float* lpart, float* gpart, hipStream_t st) {
    const int npts = n * n;
    hipLaunchKernelGGL(k_finish, dim3(npts / TPB, batch), dim3(TPB), 0, st, npts, batch, phi, out_raw, part, target,
                       pred, gpred, lpart, gpart);
    return hipGetLastError();
}

hipError_t launch_center(int n, int batch, const float* gpred, const float* gpart, float* gout, hipStream_t st) {
    hipLaunchKernelGGL(k_center, dim3(n * n / TPB, batch), dim3(TPB), 0, st, n * n, gpred, gpart, gout);
    return hipGetLastError();
}

hipError_t launch_project_bwd(int n, int batch, const uint16_t* v4, const float* prm, const float* gout, float* gv,
                              float* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_project_bwd, dim3(GRED64), dim3(64), 0, st, n * n, batch, v4, prm, gout, gv, partials);
    return hipGetLastError();
}

hipError_t launch_pointwise_bwd(int n, int batch, bool act, const float* gout, const uint16_t* u, const uint16_t* v,
                                const float* pw, float* gu, float* gv, float* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_pointwise_bwd, dim3(GRED64), dim3(64), 0, st, n * n, batch, act ? 1 : 0, gout, u, v, pw, gu,
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
