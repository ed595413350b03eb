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
    __shared__ float q[H * C + H + H + 1];
    __shared__ float red[TPB / 64];
    for (int i = threadIdx.x; i < H * C + H + H + 1; i += TPB) q[i] = prm[P_Q1 + i];
    __syncthreads();
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

// projection (workgroups of 64 threads, one point each per chunk of 64 points):
// g_out = gpred - mean(gpred); recompute pre/h; gv4[c] = sum_k Q1[k][c] g_pre[k];
// partials: Q1 (g_pre v4), q1 (g_pre), Q2 (g_out h), q2 (g_out).  Thread t owns row k = t
// of Q1 and q1[t], Q2[t]; thread 0 also q2.
__global__ void __launch_bounds__(64) k_project_bwd(int npts, int batch, const uint16_t* v4, const float* prm,
                                                    const float* gpred, const float* gpart, float* gv,
                                                    float* partials) {
    constexpr int Q = 64;
    __shared__ float q[H * C + H + H + 1];
    __shared__ float gp_s[H * Q];
    __shared__ float h_s[H * Q];
    __shared__ float x_s[C * Q];
    __shared__ float go_s[Q];
    const int t = threadIdx.x;
    for (int i = t; i < H * C + H + H + 1; i += Q) q[i] = prm[P_Q1 + i];
    const int nwf = npts / TPB;   // workgroups per sample of the finish pass (its partial sums)
    const int per = npts / Q, chunks = batch * per;
    float aQ1[C];
#pragma unroll
    for (int c = 0; c < C; ++c) aQ1[c] = 0.f;
    float aq1 = 0.f, aQ2 = 0.f, aq2 = 0.f;
    __syncthreads();
    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int b = ch / per;
        const int p = (ch - b * per) * Q + t;
        float gmean = 0.f;
        for (int w = 0; w < nwf; ++w) gmean += gpart[(size_t)b * nwf + w];
        gmean /= (float)npts;
        const float go = gpred[(size_t)b * npts + p] - gmean;
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

// lifting: partials Lw[c][0] (g phi), Lw[c][1] (g eps), Lb[c] (g)
__global__ void __launch_bounds__(TPB) k_lift_bwd(int npts, int batch, const float* gv0, const float* phi,
                                                  const float* eps, float* partials) {
    constexpr int Q = 64;
    __shared__ float g_s[C * Q];
    __shared__ float f_s[Q];
    __shared__ float e_s;
    const int t = threadIdx.x;
    const int nwg = npts / TPB, chunks = batch * nwg;
    const int c = t < 2 * C ? t >> 1 : t - 2 * C;
    const int kind = t < 2 * C ? (t & 1) : 2;   // 0: phi, 1: eps, 2: bias
    float acc = 0.f;
    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int b = ch / nwg;
        const int p = (ch - b * nwg) * TPB + t;
        const size_t base = (size_t)b * C * npts + p;
        for (int qq = 0; qq < TPB / Q; ++qq) {
            __syncthreads();
            if ((t / Q) == qq) {
                const int pt = t - qq * Q;
#pragma unroll
                for (int cc = 0; cc < C; ++cc) g_s[cc * Q + pt] = gv0[base + (size_t)cc * npts];
                f_s[pt] = phi[(size_t)b * npts + p];
            }
            if (t == 0) e_s = eps[b];
            __syncthreads();
            if (t < 3 * C)
                for (int pt = 0; pt < Q; ++pt) {
                    const float g = g_s[c * Q + pt];
                    acc += kind == 0 ? g * f_s[pt] : (kind == 1 ? g * e_s : g);
                }
        }
    }
    if (t < 3 * C) partials[(size_t)blockIdx.x * PART_LIFT + t] = acc;
}

// dst[j] = scale * sum_r partials[r][j] (rows in order)
__global__ void __launch_bounds__(TPB) k_reduce(const float* partials, int nrows, int cnt, float scale, float* dst) {
    const int j = blockIdx.x * TPB + threadIdx.x;
    if (j >= cnt) return;
    float s = 0.f;
    for (int r = 0; r < nrows; ++r) s += partials[(size_t)r * cnt + j];
    dst[j] = scale * s;
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

hipError_t launch_project_bwd(int n, int batch, const uint16_t* v4, const float* prm, const float* gpred,
                              const float* gpart, float* gv, float* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_project_bwd, dim3(GRED), dim3(64), 0, st, n * n, batch, v4, prm, gpred, gpart, gv, partials);
    return hipGetLastError();
}

hipError_t launch_pointwise_bwd(int n, int batch, bool act, const float* gout, const uint16_t* u, const uint16_t* v,
                                const float* pw, float* gu, float* gv, float* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_pointwise_bwd, dim3(GRED), dim3(64), 0, st, n * n, batch, act ? 1 : 0, gout, u, v, pw, gu,
                       gv, partials);
    return hipGetLastError();
}

hipError_t launch_lift_bwd(int n, int batch, const float* gv0, const float* phi, const float* eps, float* partials,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_lift_bwd, dim3(GRED), dim3(TPB), 0, st, n * n, batch, gv0, phi, eps, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const float* partials, int nrows, int cnt, float scale, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3((cnt + TPB - 1) / TPB), dim3(TPB), 0, st, partials, nrows, cnt, scale, dst);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* prm, const float* grad, float* m, float* v, float lr, float c1,
                       float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + TPB - 1) / TPB)), dim3(TPB), 0, st, count, prm, grad, m, v, lr,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace fno
