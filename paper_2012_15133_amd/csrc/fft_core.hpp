// Line FFT building blocks for gfx950: complex arithmetic, register radix-2/4/8/16
// butterflies and a Stockham autosort schedule exchanging through LDS.
//
// A line of length N (power of two, 8..1024) is owned by P = N / E threads of
// one workgroup; thread t keeps E complex values in registers (E = 4, 8 or 16).  On entry and on
// exit v[m] is element t + P*m of the line (natural order in both domains), so
// the first pass can load straight from HBM with coalesced accesses and the last
// pass result can be used in registers (pointwise work, spectral symbols) without
// another trip through LDS.  Between passes the values go through LDS.
//
// Each pass with radix R and span Ns (product of the earlier radices) does
// N/R butterflies; butterfly b reads elements b + r*N/R (r = 0..R-1), scales
// input r by exp(dir 2 pi i r (b mod Ns) / (Ns R)), runs a length-R DFT and
// writes output r to position (b / Ns) * Ns * R + (b mod Ns) + r * Ns.
// This is the Stockham formulation of the Cooley-Tukey FFT.
//
// The per-thread steps are __host__ __device__ so that a host program can run
// the schedule thread by thread (the CPU tests do) with the same code.
#pragma once

#include <hip/hip_runtime.h>

namespace spfc {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__host__ __device__ inline cpx<T> mk(T a, T b) {
    cpx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ inline cpx<T> scale(cpx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T>
__host__ __device__ inline cpx<T> conj(cpx<T> a) { return mk<T>(a.x, -a.y); }
// a * (s i), s = +1 or -1
template <int S, typename T>
__host__ __device__ inline cpx<T> mul_si(cpx<T> a) {
    return S > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ------------------------------------------------------------------ schedule

// Plan<N, E>: E values per thread (E in {2, 4, 8, 16}, E <= N), P = N / E threads per
// line.  Radices: E while at least E remain, then the leftover factor as the last pass.
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int default_E(int N) { return N >= 16 ? 16 : N; }

template <int N, int EE = default_E(N)>
struct Plan {
    static_assert(N >= 8 && N <= 4096 && (N & (N - 1)) == 0, "line length must be a power of two >= 8");
    static_assert(EE == 2 || EE == 4 || EE == 8 || EE == 16, "values per thread must be 2, 4, 8 or 16");
    static_assert(EE <= N, "values per thread exceed the line length");
    static constexpr int Nl = N;
    static constexpr int E = EE;
    static constexpr int P = N / E;
    static constexpr int nE = ilog2(N) / ilog2(E);              // full radix-E passes
    static constexpr int rest = 1 << (ilog2(N) - nE * ilog2(E));  // leftover radix (1 = none)
    static constexpr int NP = nE + (rest > 1 ? 1 : 0);
    static constexpr int radix(int p) { return p < nE ? E : rest; }
    static constexpr int span(int p) {
        int s = 1;
        for (int q = 0; q < p; ++q) s *= radix(q);
        return s;
    }
};

// ------------------------------------------------------------------ small DFTs
// DIR = -1: X[k] = sum x[n] exp(-2 pi i n k / R); DIR = +1: exp(+...).  In place,
// natural order in and out.

template <int DIR, typename T>
__host__ __device__ inline void dft2(cpx<T>& a, cpx<T>& b) {
    cpx<T> t = a - b;
    a = a + b;
    b = t;
}

template <int DIR, typename T>
__host__ __device__ inline void dft4(cpx<T>& x0, cpx<T>& x1, cpx<T>& x2, cpx<T>& x3) {
    cpx<T> t0 = x0 + x2, t1 = x0 - x2, t2 = x1 + x3, t3 = mul_si<DIR>(x1 - x3);
    x0 = t0 + t2;
    x2 = t0 - t2;
    x1 = t1 + t3;
    x3 = t1 - t3;
}

template <int DIR, typename T>
__host__ __device__ inline void dft8(cpx<T> (&x)[8]) {
    // n = 2 n1 + n2: two length-4 DFTs over n1, twiddle exp(DIR 2 pi i n2 k1 / 8), length-2 over n2.
    const T h = T(0.70710678118654752440);
    cpx<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    cpx<T> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = mk<T>(h * o1.x - T(DIR) * h * o1.y, T(DIR) * h * o1.x + h * o1.y);   // * h (1 + DIR i)
    o2 = mul_si<DIR>(o2);                                                      // * DIR i
    o3 = mk<T>(-h * o3.x - T(DIR) * h * o3.y, T(DIR) * h * o3.x - h * o3.y);  // * h (-1 + DIR i)
    x[0] = e0 + o0; x[4] = e0 - o0;
    x[1] = e1 + o1; x[5] = e1 - o1;
    x[2] = e2 + o2; x[6] = e2 - o2;
    x[3] = e3 + o3; x[7] = e3 - o3;
}

template <int DIR, typename T>
__host__ __device__ inline void dft16(cpx<T> (&x)[16]) {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle exp(DIR 2 pi i n2 k1 / 16), DFT4 over n2.
    const T c1 = T(0.92387953251128675613);  // cos(pi/8)
    const T s1 = T(0.38268343236508977173);  // sin(pi/8)
    const T h = T(0.70710678118654752440);   // cos(pi/4)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<DIR>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2]);
    // now x[4 k1 + n2] = Y[n2][k1]; apply W16^(n2 k1) with W16 = exp(DIR 2 pi i / 16)
    const T cs[10] = {T(1), c1, h, s1, T(0), -s1, -h, -c1, T(-1), -c1};   // cos(pi j / 8)
    const T sn[10] = {T(0), s1, h, c1, T(1), c1, h, s1, T(0), -s1};       // sin(pi j / 8)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) {
            const int j = n2 * k1;
            cpx<T> w = mk<T>(cs[j], T(DIR) * sn[j]);
            x[4 * k1 + n2] = x[4 * k1 + n2] * w;
        }
    }
    cpx<T> y[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cpx<T> a0 = x[4 * k1], a1 = x[4 * k1 + 1], a2 = x[4 * k1 + 2], a3 = x[4 * k1 + 3];
        dft4<DIR>(a0, a1, a2, a3);
        y[k1] = a0;
        y[k1 + 4] = a1;
        y[k1 + 8] = a2;
        y[k1 + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = y[i];
}

template <int R, int DIR, typename T>
__host__ __device__ inline void dftR(cpx<T> (&a)[R]) {
    if constexpr (R == 2) {
        dft2<DIR>(a[0], a[1]);
    } else if constexpr (R == 4) {
        dft4<DIR>(a[0], a[1], a[2], a[3]);
    } else if constexpr (R == 8) {
        dft8<DIR>(a);
    } else {
        static_assert(R == 16, "radix must be 2, 4, 8 or 16");
        dft16<DIR>(a);
    }
}

// ------------------------------------------------------------------ passes
// Twiddles: pass p (span Ns, radix R) scales input r of butterfly k by
// w^j, j = r k N / (Ns R) < N, w = exp(-2 pi i / N) (conjugated for DIR = +1).
// A workgroup stages two short tables in LDS, T2[b] = w^b (b < M) and
// T1[a] = w^(a M) (a < N / M), M = 2^floor(log2(N) / 2), and forms
// w^j = T1[j / M] T2[j mod M] with one complex product (for r = 1; the other inputs'
// twiddles are its powers): about 2 sqrt(N) staged values
// per workgroup instead of a full table of N - 1 (at 1024 points in FP64 that table was
// 16 KB of loads per workgroup, as much as the line data of the real-space pass).
template <int N>
struct TwSplit {
    static constexpr int S = ilog2(N) / 2;
    static constexpr int M = 1 << S;       // entries of T2 (stored first)
    static constexpr int A = N / M;        // entries of T1 (stored after T2)
    static constexpr int size = M + A;     // <= N for N >= 4
};

// build_twiddles fills [T2 | T1] from a natural table tw[j] = exp(-2 pi i j / (N tws)).
template <typename T, typename PL>
__host__ __device__ inline void build_twiddles(cpx<T>* dst, const cpx<T>* __restrict__ tw, int tws, int tid,
                                               int nthreads) {
    using TS = TwSplit<PL::Nl>;
    for (int j = tid; j < TS::size; j += nthreads)
        dst[j] = j < TS::M ? tw[(size_t)j * tws] : tw[(size_t)(j - TS::M) * TS::M * tws];
}

template <typename T, typename PL, int DIR, int C, int PASS>
__host__ __device__ inline void pass_compute(cpx<T> (&v)[C][PL::E], int t, const cpx<T>* __restrict__ ptw) {
    constexpr int E = PL::E, P = PL::P;
    constexpr int R = PL::radix(PASS), Ns = PL::span(PASS), NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        cpx<T> w[R];
        if constexpr (Ns > 1) {
            // w^(r j1), j1 = k N / (Ns R): the first from the tables, the others as powers
            // of it (R - 2 more complex products, about r ulp each, instead of R - 2 more
            // pairs of LDS reads)
            using TS = TwSplit<PL::Nl>;
            const int k = (t + P * u) & (Ns - 1);
            const int j = k * (PL::Nl / (Ns * R));
            const cpx<T> q = ptw[TS::M + (j >> TS::S)] * ptw[j & (TS::M - 1)];
            w[1] = DIR > 0 ? conj(q) : q;
#pragma unroll
            for (int r = 2; r < R; ++r) w[r] = w[r - 1] * w[1];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            cpx<T> a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                a[r] = v[c][u + r * NB];
                if constexpr (Ns > 1) {
                    if (r > 0) a[r] = a[r] * w[r];
                }
            }
            dftR<R, DIR>(a);
#pragma unroll
            for (int r = 0; r < R; ++r) v[c][u + r * NB] = a[r];
        }
    }
}

// LDS line stride: N plus one element of padding per 16, which breaks the
// power-of-two strides of the stores into different banks.
template <int N>
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
template <int N>
struct LdsLine {
    static constexpr int size = N + N / 16;
};

// LDS index of element i of a line in the exchanges between passes.  With 4 or 8 values
// per thread (lines of 64 or more) an XOR swizzle of the low five bits by the bits above
// log2(E), which puts the strided stores and loads of every pass on distinct banks (both
// for 32 and for 64 four-byte banks, bank by bank over each wave's access); with 16 the
// padded index already does.  Each map is a bijection of [0, N).
template <int N, int E>
__host__ __device__ constexpr int xch_index(int i) {
    if constexpr ((E == 4 || E == 8) && N >= 64) return i ^ ((i >> ilog2(E)) & 31);
    else return lds_pad<N>(i);
}

// The exchange stores and loads of lines C0 .. C0 + CN - 1 of v, through buffer lines
// 0 .. CN - 1.
template <typename T, typename PL, int C, int PASS, int C0 = 0, int CN = C>
__host__ __device__ inline void pass_store(const cpx<T> (&v)[C][PL::E], cpx<T>* lds, int t) {
    constexpr int N = PL::Nl, E = PL::E, P = PL::P;
    constexpr int R = PL::radix(PASS), Ns = PL::span(PASS), NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int b = t + P * u;
        const int base = (b / Ns) * Ns * R + (b & (Ns - 1));
#pragma unroll
        for (int c = C0; c < C0 + CN; ++c) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                lds[(c - C0) * LdsLine<N>::size + xch_index<N, E>(base + r * Ns)] = v[c][u + r * NB];
        }
    }
}

template <typename T, typename PL, int C, int PASS, int C0 = 0, int CN = C>
__host__ __device__ inline void pass_load(cpx<T> (&v)[C][PL::E], const cpx<T>* lds, int t) {
    constexpr int N = PL::Nl, E = PL::E, P = PL::P;
    constexpr int R = PL::radix(PASS), NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int b = t + P * u;
#pragma unroll
        for (int c = C0; c < C0 + CN; ++c) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[c][u + r * NB] = lds[(c - C0) * LdsLine<N>::size + xch_index<N, E>(b + r * (N / R))];
        }
    }
}

// natural-order store / load of the whole line (element t + P m)
template <typename T, typename PL, int C>
__host__ __device__ inline void line_store(const cpx<T> (&v)[C][PL::E], cpx<T>* lds, int t) {
    constexpr int N = PL::Nl;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int m = 0; m < PL::E; ++m) lds[c * LdsLine<N>::size + lds_pad<N>(t + PL::P * m)] = v[c][m];
}

// The exchange before pass PASS, CH of the C lines at a time through CH line buffers.
template <typename T, typename PL, int C, int PASS, int CH, int C0 = 0>
__device__ inline void pass_exchange(cpx<T> (&v)[C][PL::E], cpx<T>* lds, int t) {
    if constexpr (C0 < C) {
        constexpr int CN = C - C0 < CH ? C - C0 : CH;
        __syncthreads();
        pass_store<T, PL, C, PASS - 1, C0, CN>(v, lds, t);
        __syncthreads();
        pass_load<T, PL, C, PASS, C0, CN>(v, lds, t);
        pass_exchange<T, PL, C, PASS, CH, C0 + CN>(v, lds, t);
    }
}

// Whole transform of C lines on the device: all threads of the workgroup must call it
// (it contains workgroup barriers).  lds points at this thread group's
// CH * LdsLine<N>::size elements: the lines go through the exchanges between passes CH at
// a time (CH = C: all at once; fewer line buffers cost more barriers).
// ptw: the two twiddle tables of this line length (TwSplit, in LDS).
template <typename T, typename PL, int DIR, int C, int PASS = 0, int CH = C>
__device__ inline void fft_run(cpx<T> (&v)[C][PL::E], cpx<T>* lds, int t, const cpx<T>* __restrict__ ptw) {
    if constexpr (PASS > 0) pass_exchange<T, PL, C, PASS, CH>(v, lds, t);
    pass_compute<T, PL, DIR, C, PASS>(v, t, ptw);
    if constexpr (PASS + 1 < PL::NP) fft_run<T, PL, DIR, C, PASS + 1, CH>(v, lds, t, ptw);
}

// Stage this line length's two twiddle tables in LDS from the global natural table
// (spacing tws); every thread of the workgroup takes part.  The first pass reads
// no twiddles and the barrier before the second pass orders these writes.
template <typename T, typename PL>
__device__ inline void stage_twiddles(cpx<T>* lds_tw, const cpx<T>* __restrict__ tw, int tws) {
    build_twiddles<T, PL>(lds_tw, tw, tws, threadIdx.x, blockDim.x);
}

// stage_twiddles in two halves: the loads into registers (issued early, ahead of a
// kernel's field loads) and the LDS stores (after them).  A workgroup has at least the
// P threads of one line, so `per` entries per thread cover the tables.
template <typename T, typename PL>
struct TwStage {
    using TS = TwSplit<PL::Nl>;
    static constexpr int per = (TS::size + PL::P - 1) / PL::P;
    cpx<T> v[per];
    __device__ inline void load(const cpx<T>* __restrict__ tw, int tws) {
#pragma unroll
        for (int i = 0; i < per; ++i) {
            const int j = threadIdx.x + i * (int)blockDim.x;
            const int jj = j < TS::size ? j : 0;
            v[i] = jj < TS::M ? tw[(size_t)jj * tws] : tw[(size_t)(jj - TS::M) * TS::M * tws];
        }
    }
    __device__ inline void store(cpx<T>* lds_tw) const {
#pragma unroll
        for (int i = 0; i < per; ++i) {
            const int j = threadIdx.x + i * (int)blockDim.x;
            if (j < TS::size) lds_tw[j] = v[i];
        }
    }
};

// Workgroup index remapped so that consecutive line blocks run on the same XCD
// (workgroups are dealt to the 8 XCDs round-robin).  Bijective on [0, nblocks).
__device__ inline int xcd_block(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

}  // namespace spfc
